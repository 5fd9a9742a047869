// Serving runtime of libah: a request loop over a packed collection resident
// in HBM.  Jobs (one primer pair over a subset of the genomes) are split into
// parts of whole genomes; compile threads specialise each new pair's scan
// kernel off the request path; lane threads, each driving its own device
// stream, take the next part of the active jobs in round-robin order, carve
// the part's buffers from the caller's pool (the HBM budget), run gather ->
// scan -> Tm -> pairing -> remap on their stream, wait for it and copy the
// part's records to host memory: straight into a pinned result arena
// allocated once at start, or, when the arena is full, through a pinned
// staging buffer per lane into ordinary host memory.
// Pool memory is held only while a part is in flight, so every admitted part
// completes and frees it: admission by memory cannot deadlock.  Parts of
// several jobs are in flight on the device together, and a new job starts as
// soon as a lane and pool memory are free.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ah.h"
#include "ah_dev.h"
#include "ah_internal.h"

namespace {

#define AH_HIP(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return ah::set_error(AH_ERR_HIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                           __LINE__);                                                        \
  } while (0)

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// First-fit allocator over the caller's pool (offsets; 256-byte granules).
class Pool {
 public:
  explicit Pool(uint64_t bytes) : bytes_(bytes) {
    if (bytes) free_[0] = bytes;
  }
  bool alloc(uint64_t size, uint64_t* off) {
    size = align256(std::max<uint64_t>(size, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < size) continue;
      *off = it->first;
      const uint64_t rest = it->second - size, next = it->first + size;
      free_.erase(it);
      if (rest) free_[next] = rest;
      in_use_ += size;
      high_ = std::max(high_, in_use_);
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t size) {
    size = align256(std::max<uint64_t>(size, 1));
    in_use_ -= size;
    auto it = free_.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t bytes() const { return bytes_; }
  uint64_t in_use() const { return in_use_; }
  uint64_t high() const { return high_; }

 private:
  uint64_t bytes_, in_use_ = 0, high_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

struct Part {
  uint32_t g0 = 0, g1 = 0;  // indices into the job's genome list
  uint64_t bases = 0;
  uint64_t words = 0;       // window words of its genomes
  uint32_t max_len = 1;
  uint64_t hcap = 0, acap = 0;
  uint64_t n_hits = 0, n_amps = 0;       // records of a done part
  uint64_t arena_off = ~0ull, arena_bytes = 0;  // their place in the host arena, or
  std::vector<ah_hit> hits;              // host copies when the arena was full
  std::vector<ah_amplicon> amps;
  bool done = false;
  bool in_arena() const { return arena_off != ~0ull; }
};

struct Job {
  uint64_t id = 0;
  std::string fwd, rev;
  ah_primer_pair pair{};
  ah_window win{};
  ah_tm_params tm{};
  std::vector<uint32_t> ids;
  std::vector<Part> parts;
  size_t next = 0;                 // next part never dispatched
  std::deque<uint32_t> redo;       // parts to run again with exact capacities
  uint32_t done_parts = 0, in_flight = 0, retries = 0;
  int32_t status = AH_OK;
  bool queued = false, finished = false;
  double t_submit = 0, t_ready = -1, t_start = -1, t_done = -1;
  uint64_t bases = 0, hits = 0, amps = 0;
  bool has_work() const { return status == AH_OK && (next < parts.size() || !redo.empty()); }
};

// Byte sizes of a part's device buffers (one pool block while it runs).
struct PartSizes {
  uint64_t total, res, hits, amps, ids, off, len, scan_ws, pair_ws;
};

PartSizes part_sizes(const Part& p, const ah_primer_pair* pair) {
  PartSizes s{};
  const uint32_t n = p.g1 - p.g0;
  s.res = align256(2 * sizeof(ah_result));
  s.hits = align256(p.hcap * sizeof(ah_hit));
  s.amps = align256(p.acap * sizeof(ah_amplicon));
  s.ids = align256((uint64_t)n * 4);
  s.off = align256(((uint64_t)n + 1) * 8);
  s.len = align256((uint64_t)n * 4);
  s.scan_ws = align256(ah::scan_workspace_for(n, p.words, pair, 1, p.hcap));
  s.pair_ws = align256(ah_pair_workspace_bytes(p.hcap, 1));
  s.total = s.res + s.hits + s.amps + s.ids + s.off + s.len + s.scan_ws + s.pair_ws;
  return s;
}

}  // namespace

struct ah_server {
  ah_genomes res{};
  std::vector<uint32_t> len;
  ah_server_config cfg{};
  uintptr_t base = 0;
  int dev = 0;
  Pool pool{0};
  char* arena = nullptr;  // pinned host memory for part records
  Pool arena_pool{0};
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_lane, cv_done, cv_compile;
  bool stop = false;
  uint64_t next_id = 1;
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<uint64_t> active;     // jobs with parts to dispatch, round robin
  std::deque<uint64_t> compile_q;  // jobs whose kernel is not ready yet
  std::deque<uint64_t> finished_q; // finished, not yet returned by wait
  ah_server_stats stats{};
  std::vector<std::thread> threads;
  // Failure injection for tests (AH_SERVER_FAIL_PART=n at creation): the
  // n-th part run (0-based, any lane) fails right after its first launch.
  int64_t inject_fail = -1;
  std::atomic<uint64_t> part_runs{0};

  double sim_now = -1.0;  // the simulated clock of ah_sched_simulate (>= 0 there)
  double now() const {
    if (sim_now >= 0.0) return sim_now;
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // Frees a part's records (mu held).
  void drop_records(Part& q) {
    if (q.in_arena()) arena_pool.release(q.arena_off, q.arena_bytes);
    q.arena_off = ~0ull;
    std::vector<ah_hit>().swap(q.hits);
    std::vector<ah_amplicon>().swap(q.amps);
    q.done = false;
  }

  // Called with mu held.
  void finish(Job& j) {
    if (j.finished) return;
    j.finished = true;
    if (j.queued) {  // a failed job may still sit in the round robin
      active.erase(std::remove(active.begin(), active.end(), j.id), active.end());
      j.queued = false;
    }
    j.t_done = now();
    finished_q.push_back(j.id);
    stats.jobs_finished++;
    cv_done.notify_all();
  }

  void compile_loop() {
    (void)hipSetDevice(dev);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_compile.wait(lk, [&] { return stop || !compile_q.empty(); });
      if (stop) return;
      const uint64_t id = compile_q.front();
      compile_q.pop_front();
      Job* j = jobs.at(id).get();
      lk.unlock();
      const ah_status s = ah_scan_prepare(&j->pair, 1, res.nmask != nullptr);
      lk.lock();
      j->t_ready = now();
      if (s != AH_OK) {
        j->status = s;
        finish(*j);
        continue;
      }
      if (j->has_work()) {
        j->queued = true;
        active.push_back(id);
        cv_lane.notify_all();
      } else {
        finish(*j);
      }
    }
  }

  // Amplicon capacity from the sites a part actually has: random + and -
  // sites at the measured density, paired within the window.
  uint64_t amp_capacity(uint64_t nh, const Part& p, double win) const {
    const double b = std::max<double>((double)p.bases, 1.0);
    const double e = (double)nh * (double)nh * win / (4.0 * b);
    return (uint64_t)std::min(std::ceil(cfg.capacity_scale * e), 1e12) +
           4ull * (p.g1 - p.g0) + 256;
  }

  // Runs part p of job j on `st` in the pool block at `blk`.  hr[0..1] get the
  // part's results; when both fit, the records are copied to host memory.  The
  // amplicon buffer is resized from the sites found before pairing (an extra
  // pool block when the planned one is too small), and pairing alone is run
  // again when it overflows, so only an overflow of sites (or no pool memory
  // for the extra block) sends the whole part back for another run.
  ah_status run_part(Job& j, Part& p, const PartSizes& z, uint64_t blk, hipStream_t st,
                     ah_result* hr, void*& stage, size_t& stage_bytes, double* t_gpu,
                     double* t_copy) {
    const double t0 = now();
    const uint32_t n = p.g1 - p.g0;
    uintptr_t q = base + blk;
    ah_result* d_res = (ah_result*)q;
    ah_hit* hits = (ah_hit*)(q += z.res);
    ah_amplicon* amps = (ah_amplicon*)(q += z.hits);
    uint32_t* ids = (uint32_t*)(q += z.amps);
    uint64_t* off = (uint64_t*)(q += z.ids);
    uint32_t* len_v = (uint32_t*)(q += z.off);
    void* scan_ws = (void*)(q += z.len);
    void* pair_ws = (void*)(q += z.scan_ws);
    struct Extra {  // an extra amplicon block, returned to the pool on exit
      ah_server* srv;
      uint64_t off = ~0ull, bytes = 0;
      ~Extra() {
        if (off == ~0ull) return;
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->pool.release(off, bytes);
        srv->cv_lane.notify_all();
      }
    } extra{this};
    // Whatever way this returns, nothing it queued on `st` is still running
    // when the pool block (released by the caller) or the extra block
    // (released by `extra`, destroyed after this) can be handed to another
    // lane.  On the success paths the stream has already been synchronised.
    struct SyncOnExit {
      hipStream_t st;
      ~SyncOnExit() { (void)hipStreamSynchronize(st); }
    } sync_on_exit{st};
    uint64_t acap = p.acap;
    auto take_extra = [&](uint64_t cap) -> bool {
      std::lock_guard<std::mutex> lk(mu);
      if (extra.off != ~0ull) pool.release(extra.off, extra.bytes);
      extra.off = ~0ull;
      const uint64_t bytes = align256(cap * sizeof(ah_amplicon));
      uint64_t o;
      if (!pool.alloc(bytes, &o)) return false;
      extra.off = o;
      extra.bytes = bytes;
      amps = (ah_amplicon*)(base + o);
      acap = cap;
      return true;
    };
    AH_HIP(hipMemcpyAsync(ids, j.ids.data() + p.g0, (size_t)n * 4, hipMemcpyHostToDevice, st));
    AH_HIP(ah::launch_gather_view(ids, n, res.word_off, res.len, off, len_v, st));
    if (inject_fail >= 0 && part_runs.fetch_add(1) == (uint64_t)inject_fail)
      return ah::set_error(AH_ERR_HIP, "injected failure after the first launch of a part");
    ah_genomes view = res;
    view.word_off = off;
    view.len = len_v;
    view.n = n;
    view.max_len = std::max<uint32_t>(p.max_len, 1);
    ah_status s = ah_scan_primers(&view, &j.pair, 1, hits, p.hcap, &d_res[0], scan_ws, z.scan_ws, st);
    if (s) return s;
    s = ah_tm(&view, &j.pair, 1, &j.tm, hits, &d_res[0], p.hcap, st);
    if (s) return s;
    AH_HIP(hipMemcpyAsync(&hr[0], &d_res[0], sizeof(ah_result), hipMemcpyDeviceToHost, st));
    AH_HIP(hipStreamSynchronize(st));
    hr[1] = ah_result{0, 0, AH_OK, 0};
    if (hr[0].status != AH_OK) return AH_OK;  // run again with the exact site count
    const uint64_t want = amp_capacity(hr[0].count, p, (double)j.win.max_len - j.win.min_len + 1.0);
    if (want > acap && !take_extra(want)) {
      hr[1].status = AH_ERR_OVERFLOW;  // run again, planning the larger buffer
      hr[1].required = want;
      return AH_OK;
    }
    for (int pass = 0; pass < 2; ++pass) {
      s = ah_pair_amplicons(hits, &d_res[0], p.hcap, &j.pair, &j.win, 1, amps, acap, &d_res[1],
                            pair_ws, z.pair_ws, st);
      if (s) return s;
      AH_HIP(hipMemcpyAsync(&hr[1], &d_res[1], sizeof(ah_result), hipMemcpyDeviceToHost, st));
      AH_HIP(hipStreamSynchronize(st));
      if (hr[1].status == AH_OK || pass == 1 || !take_extra(hr[1].required)) break;
    }
    if (hr[1].status != AH_OK) return AH_OK;  // run again with the exact amplicon count
    AH_HIP(ah::launch_remap(hits, &d_res[0], amps, &d_res[1], ids, ah::cu_count_current() * 4, st));
    AH_HIP(hipStreamSynchronize(st));
    const double t1 = now();
    *t_gpu = t1 - t0;
    struct CopyClock {
      ah_server* srv;
      double t1;
      double* out;
      ~CopyClock() { *out = srv->now() - t1; }
    } copy_clock{this, t1, t_copy};
    const size_t hb = hr[0].count * sizeof(ah_hit), ab = hr[1].count * sizeof(ah_amplicon);
    p.n_hits = hr[0].count;
    p.n_amps = hr[1].count;
    uint64_t aoff = 0;
    bool in_arena = false;
    if (hb + ab > 0 && arena) {
      std::lock_guard<std::mutex> lk(mu);
      in_arena = arena_pool.alloc(hb + ab, &aoff);
      if (!in_arena) stats.host_fallbacks++;
    }
    if (in_arena) {  // straight into the arena
      p.arena_off = aoff;
      p.arena_bytes = hb + ab;
      hipError_t e = hb ? hipMemcpyAsync(arena + aoff, hits, hb, hipMemcpyDeviceToHost, st)
                        : hipSuccess;
      if (e == hipSuccess && ab)
        e = hipMemcpyAsync(arena + aoff + hb, amps, ab, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        arena_pool.release(aoff, hb + ab);
        p.arena_off = ~0ull;
        return ah::set_error(AH_ERR_HIP, "record copy: %s", hipGetErrorString(e));
      }
      return AH_OK;
    }
    if (hb + ab > stage_bytes) {
      const size_t want = std::max<size_t>(hb + ab, 2 * stage_bytes + (1u << 20));
      if (stage) AH_HIP(hipHostFree(stage));
      stage = nullptr;
      stage_bytes = 0;
      AH_HIP(hipHostMalloc(&stage, want, hipHostMallocDefault));
      stage_bytes = want;
    }
    if (hb) AH_HIP(hipMemcpyAsync(stage, hits, hb, hipMemcpyDeviceToHost, st));
    if (ab) AH_HIP(hipMemcpyAsync((char*)stage + hb, amps, ab, hipMemcpyDeviceToHost, st));
    AH_HIP(hipStreamSynchronize(st));
    p.hits.assign((const ah_hit*)stage, (const ah_hit*)stage + hr[0].count);
    p.amps.assign((const ah_amplicon*)((char*)stage + hb),
                  (const ah_amplicon*)((char*)stage + hb) + hr[1].count);
    return AH_OK;
  }

  // ---- scheduling: the decisions the lanes take with mu held.  They touch
  // only the jobs, the round robin, the pool and the statistics, so the
  // host-only simulation (ah_sched_simulate) drives the same code with
  // simulated part runs.

  // The next part to run: the job at the front of the round robin, once its
  // buffers (size_of(job, part) bytes) fit in the pool.  Returns true with
  // the part taken (its block allocated, the round robin advanced), false
  // when nothing is runnable or the front part's buffers do not fit yet.
  template <class SizeFn>
  bool take_next(SizeFn size_of, Job*& j, uint32_t& pi, uint64_t& blk, uint64_t& bytes) {
    while (!active.empty()) {
      Job* cand = jobs.at(active.front()).get();
      if (!cand->has_work()) {  // failed meanwhile, or nothing left to start
        cand->queued = false;
        active.pop_front();
        if (cand->in_flight == 0 &&
            (cand->status != AH_OK || cand->done_parts == cand->parts.size()))
          finish(*cand);
        continue;
      }
      const uint32_t cpi = cand->redo.empty() ? (uint32_t)cand->next : cand->redo.front();
      const uint64_t need = size_of(*cand, cpi);
      if (need > pool.bytes()) {
        cand->status = ah::set_error(AH_ERR_LIMIT, "a part needs %llu bytes > pool %llu",
                                     (unsigned long long)need, (unsigned long long)pool.bytes());
        continue;  // dropped on the next pass
      }
      if (!pool.alloc(need, &blk)) {
        stats.admission_waits++;
        return false;  // a finished part frees pool memory
      }
      j = cand;
      pi = cpi;
      bytes = need;
      active.pop_front();
      if (!j->redo.empty() && j->redo.front() == pi) j->redo.pop_front();
      else j->next++;
      j->in_flight++;
      if (j->t_start < 0) j->t_start = now();
      if (j->has_work()) active.push_back(j->id);
      else j->queued = false;
      stats.parts_run++;
      return true;
    }
    return false;
  }

  // After part pi of job j ran with status s and results hr[0..1]: its block
  // returns to the pool, an overflow sends the part back with the exact
  // counts, and the job finishes once none of its parts is left.
  void settle(Job& jr, uint32_t pi, uint64_t blk, uint64_t bytes, ah_status s,
              const ah_result* hr) {
    Job* j = &jr;
    Part& p = j->parts[pi];
    pool.release(blk, bytes);
    j->in_flight--;
    if (s != AH_OK) {
      if (j->status == AH_OK) j->status = s;
    } else if (hr[0].status != AH_OK || hr[1].status != AH_OK) {
      // the exact counts are known now: run the part again with them
      if (hr[0].required >= 0xffffffffull) {
        if (j->status == AH_OK)
          j->status = ah::set_error(AH_ERR_LIMIT, "a part of job %llu has %llu sites",
                                    (unsigned long long)j->id,
                                    (unsigned long long)hr[0].required);
      } else if (hr[0].required <= p.hcap && hr[1].required <= p.acap) {
        // a rerun with the same buffers would overflow again
        if (j->status == AH_OK)
          j->status = ah::set_error(AH_ERR_LIMIT,
                                    "a part of job %llu overflows buffers sized for its "
                                    "counts (%llu sites, %llu amplicons)",
                                    (unsigned long long)j->id,
                                    (unsigned long long)hr[0].required,
                                    (unsigned long long)hr[1].required);
      } else {
        p.hcap = std::max<uint64_t>(p.hcap, hr[0].required);
        p.acap = std::max<uint64_t>(p.acap, hr[1].required);
        j->redo.push_back(pi);
        j->retries++;
        stats.retries++;
        if (!j->queued) {
          j->queued = true;
          active.push_back(j->id);
        }
      }
    } else {
      p.done = true;
      j->done_parts++;
      j->hits += p.n_hits;
      j->amps += p.n_amps;
    }
    if (j->in_flight == 0 && (j->status != AH_OK || j->done_parts == j->parts.size())) {
      if (j->status != AH_OK)
        for (Part& q : j->parts) drop_records(q);  // a failed job returns no records
      finish(*j);
    }
  }

  void lane_loop() {
    (void)hipSetDevice(dev);
    hipStream_t st = nullptr;
    void* stage = nullptr;  // pinned staging for the device -> host record copies
    size_t stage_bytes = 0;
    const hipError_t ce = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    std::unique_lock<std::mutex> lk(mu);
    if (ce != hipSuccess) return;
    auto size_of = [](const Job& j, uint32_t pi) { return part_sizes(j.parts[pi], &j.pair).total; };
    for (;;) {
      Job* j = nullptr;
      uint32_t pi = 0;
      uint64_t blk = 0, bytes = 0;
      while (!stop && !take_next(size_of, j, pi, blk, bytes)) cv_lane.wait(lk);
      if (stop) break;
      Part& p = j->parts[pi];
      const PartSizes z = part_sizes(p, &j->pair);
      lk.unlock();

      const double t_run = now();
      ah_result hr[2] = {};
      double t_gpu = 0, t_copy = 0;
      const ah_status s =
          run_part(*j, p, z, blk, st, hr, stage, stage_bytes, &t_gpu, &t_copy);

      lk.lock();
      stats.lane_busy_s += now() - t_run;
      stats.gpu_s += t_gpu;
      stats.copy_s += t_copy;
      settle(*j, pi, blk, bytes, s, hr);
      cv_lane.notify_all();
    }
    lk.unlock();
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (stage) (void)hipHostFree(stage);
  }
};

extern "C" {

ah_status ah_server_create(const ah_genomes* resident, const uint32_t* h_len,
                           const ah_server_config* cfg, void* d_pool, size_t pool_bytes,
                           ah_server** out) {
  ah::clear_error();
  if (!resident || !cfg || !out || (resident->n > 0 && !h_len))
    return ah::set_error(AH_ERR_INVALID_ARG, "resident, h_len, cfg and out are required");
  if (resident->n > 0 && (!resident->words || !resident->word_off || !resident->len))
    return ah::set_error(AH_ERR_INVALID_ARG, "resident: words, word_off and len are required");
  if (cfg->n_lanes < 1 || cfg->n_lanes > 16 || cfg->n_compilers < 1 || cfg->n_compilers > 32)
    return ah::set_error(AH_ERR_INVALID_ARG, "n_lanes must be 1..16 and n_compilers 1..32");
  if (cfg->part_bases == 0 || cfg->max_part_hits == 0 || !(cfg->capacity_scale >= 0.0))
    return ah::set_error(AH_ERR_INVALID_ARG, "part_bases and max_part_hits must be >= 1, "
                         "capacity_scale >= 0");
  if (!d_pool || pool_bytes < 4096)
    return ah::set_error(AH_ERR_INVALID_ARG, "a device pool of at least 4 KiB is required");
  auto s = std::make_unique<ah_server>();
  AH_HIP(hipGetDevice(&s->dev));
  s->res = *resident;
  s->len.assign(h_len, h_len + resident->n);
  s->cfg = *cfg;
  s->base = ((uintptr_t)d_pool + 255) & ~(uintptr_t)255;
  const uint64_t lost = s->base - (uintptr_t)d_pool;
  s->pool = Pool((pool_bytes - lost) & ~255ull);
  s->t0 = std::chrono::steady_clock::now();
  s->stats.pool_bytes = s->pool.bytes();
  if (const char* e = getenv("AH_SERVER_FAIL_PART")) s->inject_fail = atoll(e);
  if (cfg->host_pool_bytes) {
    void* a = nullptr;
    AH_HIP(hipHostMalloc(&a, cfg->host_pool_bytes, hipHostMallocDefault));
    s->arena = (char*)a;
    s->arena_pool = Pool(cfg->host_pool_bytes & ~255ull);
  }
  ah_server* srv = s.get();
  for (uint32_t i = 0; i < cfg->n_compilers; ++i)
    s->threads.emplace_back([srv] { srv->compile_loop(); });
  for (uint32_t i = 0; i < cfg->n_lanes; ++i) s->threads.emplace_back([srv] { srv->lane_loop(); });
  *out = s.release();
  return AH_OK;
}

ah_status ah_server_submit(ah_server* srv, const ah_job* job, uint64_t* job_id) {
  ah::clear_error();
  if (!srv || !job) return ah::set_error(AH_ERR_INVALID_ARG, "server and job are required");
  ah_status st = ah::check_tm(&job->pair, 1, &job->tm);
  if (st) return st;
  if (job->window.min_len > job->window.max_len)
    return ah::set_error(AH_ERR_INVALID_ARG, "window: min_len > max_len");
  auto j = std::make_unique<Job>();
  j->fwd = job->pair.fwd;
  j->rev = job->pair.rev;
  j->pair = job->pair;
  j->pair.fwd = j->fwd.c_str();
  j->pair.rev = j->rev.c_str();
  j->win = job->window;
  j->tm = job->tm;
  const uint32_t N = srv->res.n;
  if (job->genomes) {
    j->ids.assign(job->genomes, job->genomes + job->n_genomes);
    for (size_t i = 0; i < j->ids.size(); ++i)
      if (j->ids[i] >= N || (i > 0 && j->ids[i] <= j->ids[i - 1]))
        return ah::set_error(AH_ERR_INVALID_ARG, "genome list must be strictly ascending ids < %u",
                             N);
  } else {
    j->ids.resize(N);
    for (uint32_t g = 0; g < N; ++g) j->ids[g] = g;
  }
  // parts: whole genomes, at most part_bases bases and about max_part_hits
  // expected sites each
  const auto& cfg = srv->cfg;
  const double rate = 2.0 * (ah::site_probability(j->fwd, j->pair.k, j->pair.clamp) +
                             ah::site_probability(j->rev, j->pair.k, j->pair.clamp));
  const double scale = cfg.capacity_scale;
  double cut = (double)cfg.part_bases;
  if (rate * scale > 0) cut = std::min(cut, (double)cfg.max_part_hits / (rate * scale));
  const uint64_t part_bases = std::max<uint64_t>((uint64_t)cut, 1);
  const double win = (double)j->win.max_len - (double)j->win.min_len + 1.0;
  auto close = [&](Part& p) {
    const uint32_t n = p.g1 - p.g0;
    const double eh = scale * rate * (double)p.bases;
    const double ea = scale * (rate / 2) * (rate / 2) * win * (double)p.bases;
    p.hcap = std::min<uint64_t>((uint64_t)std::ceil(eh) + 16ull * n + 1024, 0xfffffffeull);
    p.acap = (uint64_t)std::min(std::ceil(ea), 1e12) + 4ull * n + 256;
    j->parts.push_back(p);
  };
  Part cur;
  for (uint32_t i = 0; i < (uint32_t)j->ids.size(); ++i) {
    const uint32_t L = srv->len[j->ids[i]];
    if (cur.g1 > cur.g0 && cur.bases + L > part_bases) {
      close(cur);
      cur = Part();
      cur.g0 = cur.g1 = i;
    }
    cur.g1 = i + 1;
    cur.bases += L;
    cur.words += ((uint64_t)L + 31) / 32;
    cur.max_len = std::max(cur.max_len, L);
    j->bases += L;
  }
  if (cur.g1 > cur.g0) close(cur);

  std::lock_guard<std::mutex> lk(srv->mu);
  j->id = srv->next_id++;
  j->t_submit = srv->now();
  const uint64_t id = j->id;
  Job* jp = j.get();
  srv->jobs[id] = std::move(j);
  srv->stats.jobs_submitted++;
  if (jp->parts.empty()) {
    jp->t_ready = jp->t_start = jp->t_submit;
    srv->finish(*jp);
  } else {
    srv->compile_q.push_back(id);
    srv->cv_compile.notify_one();
  }
  if (job_id) *job_id = id;
  return AH_OK;
}

ah_status ah_server_wait(ah_server* srv, double timeout_s, ah_job_status* out) {
  ah::clear_error();
  if (!srv || !out) return ah::set_error(AH_ERR_INVALID_ARG, "server and status are required");
  std::unique_lock<std::mutex> lk(srv->mu);
  const auto until = std::chrono::steady_clock::now() +
                     std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                         std::chrono::duration<double>(std::max(timeout_s, 0.0)));
  if (!srv->cv_done.wait_until(lk, until, [&] { return !srv->finished_q.empty(); }))
    return AH_ERR_AGAIN;
  const uint64_t id = srv->finished_q.front();
  srv->finished_q.pop_front();
  const Job& j = *srv->jobs.at(id);
  *out = ah_job_status{};
  out->job = id;
  out->status = j.status;
  out->n_parts = (uint32_t)j.parts.size();
  out->hits = j.hits;
  out->amplicons = j.amps;
  out->bases = j.bases;
  out->t_submit = j.t_submit;
  out->t_ready = j.t_ready;
  out->t_start = j.t_start;
  out->t_done = j.t_done;
  out->retries = j.retries;
  return AH_OK;
}

ah_status ah_server_part(ah_server* srv, uint64_t job_id, uint32_t part, ah_job_part* out) {
  ah::clear_error();
  if (!srv || !out) return ah::set_error(AH_ERR_INVALID_ARG, "server and out are required");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(job_id);
  if (it == srv->jobs.end() || !it->second->finished)
    return ah::set_error(AH_ERR_INVALID_ARG, "job %llu is not a finished, unreleased job",
                         (unsigned long long)job_id);
  const Job& j = *it->second;
  if (j.status != AH_OK)
    return ah::set_error((ah_status)j.status, "job %llu failed", (unsigned long long)job_id);
  if (part >= j.parts.size()) return ah::set_error(AH_ERR_INVALID_ARG, "job has %zu parts", j.parts.size());
  const Part& p = j.parts[part];
  if (p.in_arena()) {
    out->hits = (const ah_hit*)(srv->arena + p.arena_off);
    out->amplicons = (const ah_amplicon*)(srv->arena + p.arena_off + p.n_hits * sizeof(ah_hit));
  } else {
    out->hits = p.hits.data();
    out->amplicons = p.amps.data();
  }
  out->n_hits = p.n_hits;
  out->n_amplicons = p.n_amps;
  out->first_genome = p.g0;
  out->n_genomes = p.g1 - p.g0;
  return AH_OK;
}

ah_status ah_server_release(ah_server* srv, uint64_t job_id) {
  ah::clear_error();
  if (!srv) return ah::set_error(AH_ERR_INVALID_ARG, "server is required");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(job_id);
  if (it == srv->jobs.end() || !it->second->finished)
    return ah::set_error(AH_ERR_INVALID_ARG, "job %llu is not a finished, unreleased job",
                         (unsigned long long)job_id);
  for (Part& p : it->second->parts) srv->drop_records(p);
  for (auto q = srv->finished_q.begin(); q != srv->finished_q.end(); ++q)
    if (*q == job_id) {
      srv->finished_q.erase(q);
      break;
    }
  srv->jobs.erase(it);
  srv->cv_lane.notify_all();
  return AH_OK;
}

void ah_server_stats_get(ah_server* srv, ah_server_stats* out) {
  if (!srv || !out) return;
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->stats;
  out->pool_bytes = srv->pool.bytes();
  out->pool_in_use = srv->pool.in_use();
  out->pool_high_water = srv->pool.high();
  out->host_pool_bytes = srv->arena_pool.bytes();
  out->host_pool_high_water = srv->arena_pool.high();
}

double ah_server_now(ah_server* srv) { return srv ? srv->now() : 0.0; }

void ah_server_destroy(ah_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_lane.notify_all();
  srv->cv_compile.notify_all();
  srv->cv_done.notify_all();
  for (std::thread& t : srv->threads) t.join();
  if (srv->arena) (void)hipHostFree(srv->arena);
  delete srv;
}

ah_status ah_sched_simulate(const ah_sched_job* jobs, uint32_t n_jobs, const ah_sched_part* parts,
                            uint32_t n_parts, uint32_t n_lanes, uint64_t pool_bytes,
                            ah_sched_event* events, uint64_t max_events, uint64_t* n_events,
                            ah_job_status* done) {
  ah::clear_error();
  if ((n_jobs && !jobs) || (n_parts && !parts) || !n_events || (n_jobs && !done) ||
      (max_events && !events))
    return ah::set_error(AH_ERR_INVALID_ARG, "ah_sched_simulate: null argument");
  if (n_lanes < 1 || n_lanes > 16)
    return ah::set_error(AH_ERR_INVALID_ARG, "n_lanes must be 1..16");
  std::vector<uint32_t> order(n_jobs);
  for (uint32_t i = 0; i < n_jobs; ++i) {
    if ((uint64_t)jobs[i].first_part + jobs[i].n_parts > n_parts || !(jobs[i].arrival >= 0.0))
      return ah::set_error(AH_ERR_INVALID_ARG, "job %u: parts out of range or bad arrival", i);
    order[i] = i;
  }
  for (uint32_t q = 0; q < n_parts; ++q)
    if (!(parts[q].seconds >= 0.0))
      return ah::set_error(AH_ERR_INVALID_ARG, "part %u: bad run time", q);
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return jobs[a].arrival < jobs[b].arrival; });
  ah_server srv;  // no device, no threads: only the scheduling state
  srv.pool = Pool(pool_bytes & ~255ull);
  srv.stats.pool_bytes = srv.pool.bytes();
  srv.sim_now = 0.0;
  std::vector<uint32_t> overflows_left(n_parts);
  for (uint32_t q = 0; q < n_parts; ++q) overflows_left[q] = parts[q].overflows;
  struct Lane {
    bool busy = false;
    double until = 0.0;
    Job* j = nullptr;
    uint32_t pi = 0, spec = 0;
    uint64_t blk = 0, bytes = 0;
  };
  std::vector<Lane> lanes(n_lanes);
  std::vector<uint32_t> runs(n_parts, 0);
  auto spec_of = [&](const Job& j, uint32_t pi) { return jobs[j.id - 1].first_part + pi; };
  auto size_of = [&](const Job& j, uint32_t pi) { return parts[spec_of(j, pi)].bytes; };
  uint64_t ne = 0;
  size_t next_arrival = 0;
  std::unique_lock<std::mutex> lk(srv.mu);  // the decisions expect it held
  for (;;) {
    double t = std::numeric_limits<double>::infinity();
    if (next_arrival < order.size()) t = jobs[order[next_arrival]].arrival;
    for (const Lane& l : lanes)
      if (l.busy) t = std::min(t, l.until);
    if (t == std::numeric_limits<double>::infinity()) break;
    srv.sim_now = t;
    for (Lane& l : lanes) {  // part runs that end now
      if (!l.busy || l.until > t) continue;
      ah_result hr[2] = {};
      Part& p = l.j->parts[l.pi];
      if (overflows_left[l.spec] > 0) {  // the run reports more sites than it had room for
        overflows_left[l.spec]--;
        hr[0].status = AH_ERR_OVERFLOW;
        hr[0].required = p.hcap + 1;
      }
      srv.settle(*l.j, l.pi, l.blk, l.bytes, AH_OK, hr);
      l.busy = false;
    }
    while (next_arrival < order.size() && jobs[order[next_arrival]].arrival <= t) {
      const uint32_t i = order[next_arrival++];
      auto j = std::make_unique<Job>();
      j->id = (uint64_t)i + 1;
      j->t_submit = j->t_ready = t;
      for (uint32_t q = 0; q < jobs[i].n_parts; ++q) {
        Part p;
        p.hcap = 1;  // an overflow asks for one more
        p.acap = 1;
        j->parts.push_back(p);
      }
      Job* jp = j.get();
      srv.jobs[jp->id] = std::move(j);
      srv.stats.jobs_submitted++;
      if (jp->has_work()) {
        jp->queued = true;
        srv.active.push_back(jp->id);
      } else {
        jp->t_start = t;
        srv.finish(*jp);
      }
    }
    for (uint32_t li = 0; li < n_lanes; ++li) {  // idle lanes take the next parts
      Lane& l = lanes[li];
      if (l.busy) continue;
      if (!srv.take_next(size_of, l.j, l.pi, l.blk, l.bytes)) break;
      l.spec = spec_of(*l.j, l.pi);
      l.busy = true;
      l.until = t + parts[l.spec].seconds;
      if (ne < max_events) {
        ah_sched_event& e = events[ne];
        e.t_start = t;
        e.t_end = l.until;
        e.lane = li;
        e.job = (uint32_t)(l.j->id - 1);
        e.part = l.pi;
        e.run = runs[l.spec];
        e.block = l.blk;
        e.bytes = l.bytes;
        e.pool_in_use = srv.pool.in_use();
      }
      ++ne;
      runs[l.spec]++;
    }
  }
  *n_events = ne;
  for (uint32_t i = 0; i < n_jobs; ++i) {
    ah_job_status& d = done[i];
    memset(&d, 0, sizeof d);
    auto it = srv.jobs.find((uint64_t)i + 1);
    if (it == srv.jobs.end()) continue;
    const Job& j = *it->second;
    d.job = i;
    d.status = j.finished ? j.status : AH_ERR_AGAIN;
    d.n_parts = (uint32_t)j.parts.size();
    d.t_submit = j.t_submit;
    d.t_ready = j.t_ready;
    d.t_start = j.t_start;
    d.t_done = j.t_done;
    d.retries = j.retries;
  }
  return ne > max_events ? ah::set_error(AH_ERR_OVERFLOW, "%llu events > %llu given",
                                         (unsigned long long)ne, (unsigned long long)max_events)
                         : AH_OK;
}

}  // extern "C"
