// Streaming executor of libah: a packed collection in host memory goes to the
// GPU chunk by chunk (whole genomes, one contiguous copy per chunk) into a ring
// of staging slots, on the caller's copy streams, while earlier chunks run the
// scan -> Tm -> pairing sequence on the compute stream.  Built on the public
// entry points: every chunk is an ordinary collection to them; afterwards one
// small kernel rewrites the chunk's genome ids and hit indices to
// collection-wide ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
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

constexpr uint32_t kMaxSlots = 16;

struct Chunk {
  uint32_t first, count;  // genomes [first, first + count)
  uint64_t w0, w1;        // packed words [w0, w1)
  uint32_t max_len;
};

// Smallest genome span: a genome of length 0 still holds the halo, rounded to
// an even word count.
constexpr uint64_t kMinGenomeWords = (AH_HALO_WORDS + 1) & ~1ull;

uint32_t max_genomes_per_slot(uint64_t chunk_words) {
  const uint64_t m = chunk_words / kMinGenomeWords;
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(m, 1), 0xffffffffull);
}

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

struct Layout {
  uint64_t slot_words, slot_nmask, slot_off;  // bytes per slot of each part
  uint64_t slots, g_len, g_off, res, scan_ws, pair_ws, total;
  uint32_t max_g;
};

Layout layout(const ah_host_genomes* hg, const ah_stream_config* cfg, const ah_primer_pair* pairs,
              uint32_t n_pairs, uint64_t hit_capacity) {
  Layout L{};
  L.max_g = max_genomes_per_slot(cfg->chunk_words);
  L.slot_words = align256(cfg->chunk_words * 8);
  L.slot_nmask = hg->nmask ? align256(cfg->chunk_words * 4) : 0;
  L.slot_off = align256(((uint64_t)L.max_g + 1) * 8);
  L.slots = (L.slot_words + L.slot_nmask + L.slot_off) * cfg->n_slots;
  L.g_len = align256((uint64_t)std::max<uint32_t>(hg->n, 1) * 4);
  L.g_off = align256(((uint64_t)hg->n + 1) * 8);
  L.res = align256(2 * sizeof(ah_result));
  L.scan_ws =
      align256(ah::scan_workspace_for(L.max_g, cfg->chunk_words, pairs, n_pairs, hit_capacity));
  L.pair_ws = align256(ah_pair_workspace_bytes(hit_capacity, n_pairs));
  L.total = L.slots + L.g_len + L.g_off + L.res + L.scan_ws + L.pair_ws + 256;
  return L;
}

ah_status check_args(const ah_host_genomes* hg, const ah_stream_config* cfg) {
  if (!hg || !cfg) return ah::set_error(AH_ERR_INVALID_ARG, "genomes and cfg are required");
  if (cfg->n_slots < 2 || cfg->n_slots > kMaxSlots)
    return ah::set_error(AH_ERR_INVALID_ARG, "n_slots %u outside 2..%u", cfg->n_slots, kMaxSlots);
  if (cfg->chunk_words < kMinGenomeWords || (cfg->chunk_words & 1))
    return ah::set_error(AH_ERR_INVALID_ARG, "chunk_words must be even and >= %llu",
                         (unsigned long long)kMinGenomeWords);
  if (hg->n > 0 && (!hg->words || !hg->word_off || !hg->len))
    return ah::set_error(AH_ERR_INVALID_ARG, "genomes: words, word_off and len are required");
  return AH_OK;
}

// Consecutive genomes grouped into chunks of at most chunk_words words.
ah_status plan_chunks(const ah_host_genomes* hg, uint64_t chunk_words, uint32_t max_g,
                      std::vector<Chunk>& out) {
  out.clear();
  Chunk cur{0, 0, hg->word_off[0], hg->word_off[0], 1};
  for (uint32_t g = 0; g < hg->n; ++g) {
    const uint64_t w = hg->word_off[g + 1] - hg->word_off[g];
    if (w > chunk_words)
      return ah::set_error(AH_ERR_LIMIT, "genome %u spans %llu packed words > chunk_words %llu", g,
                           (unsigned long long)w, (unsigned long long)chunk_words);
    if (cur.count > 0 && (cur.w1 - cur.w0 + w > chunk_words || cur.count == max_g)) {
      out.push_back(cur);
      cur = Chunk{g, 0, hg->word_off[g], hg->word_off[g], 1};
    }
    cur.count++;
    cur.w1 = hg->word_off[g + 1];
    cur.max_len = std::max(cur.max_len, hg->len[g]);
  }
  if (cur.count > 0) out.push_back(cur);
  return AH_OK;
}

struct Slot {
  uint32_t* words;
  uint32_t* nmask;
  uint64_t* off;
  hipEvent_t copied;
};

// Waits for every stream the call used before returning (on success and on
// every error path), so that no copy or kernel of the call outlives it.
struct Drain {
  hipStream_t compute;
  const std::vector<hipStream_t>& copies;
  std::vector<Slot>& slots;
  ~Drain() {
    for (hipStream_t s : copies) (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(compute);
    for (Slot& s : slots)
      if (s.copied) (void)hipEventDestroy(s.copied);
  }
};

}  // namespace

extern "C" {

size_t ah_stream_workspace_bytes(const ah_host_genomes* hg, const ah_stream_config* cfg,
                                 const ah_primer_pair* pairs, uint32_t n_pairs,
                                 uint64_t hit_capacity) {
  if (!hg || !cfg || cfg->n_slots < 2 || cfg->n_slots > kMaxSlots) return 0;
  return (size_t)layout(hg, cfg, pairs, n_pairs, hit_capacity).total;
}

ah_status ah_stream_query(const ah_host_genomes* hg, const ah_stream_config* cfg,
                          const ah_primer_pair* pairs, const ah_window* windows, uint32_t n_pairs,
                          const ah_tm_params* tm, ah_hit* d_hits, uint64_t hit_capacity,
                          ah_result* d_hit_res, ah_amplicon* d_amp, uint64_t amp_capacity,
                          ah_result* d_amp_res, void* d_work, size_t work_bytes, void* stream,
                          void* const* copy_streams, uint32_t n_copy_streams) {
  ah::clear_error();
  ah_status s = check_args(hg, cfg);
  if (s) return s;
  if (!tm || !windows || !d_hit_res || !d_amp_res)
    return ah::set_error(AH_ERR_INVALID_ARG, "tm, windows and both results are required");
  if (hit_capacity > 0 && !d_hits) return ah::set_error(AH_ERR_INVALID_ARG, "d_hits is NULL");
  if (amp_capacity > 0 && !d_amp) return ah::set_error(AH_ERR_INVALID_ARG, "d_amp is NULL");
  if (hit_capacity >= (1ull << 32)) return ah::set_error(AH_ERR_LIMIT, "hit capacity must be < 2^32");
  if (n_copy_streams > 0 && !copy_streams)
    return ah::set_error(AH_ERR_INVALID_ARG, "copy_streams is NULL");
  s = ah::check_tm(pairs, n_pairs, tm);
  if (s) return s;
  // the minimum layout; the scan workspace comes last and takes whatever the
  // caller gave beyond it (a longer candidate list)
  const Layout L = layout(hg, cfg, nullptr, n_pairs, hit_capacity);
  if (!d_work || work_bytes < L.total)
    return ah::set_error(AH_ERR_WORKSPACE, "stream workspace: %zu bytes given, %llu needed",
                         work_bytes, (unsigned long long)L.total);
  std::vector<Chunk> chunks;
  if (hg->n > 0) {
    s = plan_chunks(hg, cfg->chunk_words, L.max_g, chunks);
    if (s) return s;
  }

  hipStream_t compute = (hipStream_t)stream;
  std::vector<hipStream_t> copies;
  for (uint32_t i = 0; i < n_copy_streams; ++i) copies.push_back((hipStream_t)copy_streams[i]);
  if (copies.empty()) copies.push_back(compute);

  // carve the workspace
  uintptr_t p = ((uintptr_t)d_work + 255) & ~(uintptr_t)255;
  std::vector<Slot> slots(cfg->n_slots);
  for (Slot& sl : slots) {
    sl.words = (uint32_t*)p;
    p += L.slot_words;
    sl.nmask = L.slot_nmask ? (uint32_t*)p : nullptr;
    p += L.slot_nmask;
    sl.off = (uint64_t*)p;
    p += L.slot_off;
    sl.copied = nullptr;
  }
  uint32_t* d_len = (uint32_t*)p;
  p += L.g_len;
  uint64_t* d_off = (uint64_t*)p;
  p += L.g_off;
  ah_result* d_cres = (ah_result*)p;  // [0] hits, [1] amplicons of the current chunk
  p += L.res;
  void* pair_ws = (void*)p;
  p += L.pair_ws;
  void* scan_ws = (void*)p;
  const size_t scan_bytes = (size_t)((uintptr_t)d_work + work_bytes - p);

  Drain drain{compute, copies, slots};
  for (Slot& sl : slots) AH_HIP(hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming));

  ah_result total_h{0, 0, AH_OK, 0}, total_a{0, 0, AH_OK, 0};
  if (hg->n > 0) {
    AH_HIP(hipMemcpyAsync(d_len, hg->len, (size_t)hg->n * 4, hipMemcpyHostToDevice, compute));
    AH_HIP(hipMemcpyAsync(d_off, hg->word_off, ((size_t)hg->n + 1) * 8, hipMemcpyHostToDevice,
                          compute));
    // the offsets must be on the device before any chunk is rebased; the
    // host arrays may be pageable, so finish the copies here
    AH_HIP(hipStreamSynchronize(compute));
  }

  auto enqueue_copy = [&](size_t c) -> ah_status {
    const Chunk& ch = chunks[c];
    Slot& sl = slots[c % slots.size()];
    hipStream_t cs = copies[c % copies.size()];
    const uint64_t nw = ch.w1 - ch.w0;
    AH_HIP(hipMemcpyAsync(sl.words, hg->words + 2 * ch.w0, nw * 8, hipMemcpyHostToDevice, cs));
    if (sl.nmask)
      AH_HIP(hipMemcpyAsync(sl.nmask, hg->nmask + ch.w0, nw * 4, hipMemcpyHostToDevice, cs));
    AH_HIP(hipEventRecord(sl.copied, cs));
    return AH_OK;
  };

  const size_t n_chunks = chunks.size();
  for (size_t c = 0; c < std::min<size_t>(slots.size(), n_chunks); ++c) {
    s = enqueue_copy(c);
    if (s) return s;
  }
  const int grid = ah::cu_count_current() * 4;
  bool hits_overflowed = false;
  for (size_t c = 0; c < n_chunks; ++c) {
    const Chunk& ch = chunks[c];
    Slot& sl = slots[c % slots.size()];
    AH_HIP(hipStreamWaitEvent(compute, sl.copied, 0));
    AH_HIP(ah::launch_rebase(d_off + ch.first, ch.count, sl.off, compute));
    ah_genomes view{};
    view.words = sl.words;
    view.nmask = sl.nmask;
    view.word_off = sl.off;
    view.len = d_len + ch.first;
    view.n = ch.count;
    view.max_len = std::max<uint32_t>(ch.max_len, 1);
    const uint64_t hoff = total_h.count, aoff = total_a.count;
    const uint64_t hcap = hit_capacity - hoff, acap = amp_capacity - aoff;
    ah_hit* hits = hcap ? d_hits + hoff : nullptr;
    ah_amplicon* amps = acap ? d_amp + aoff : nullptr;
    s = ah_scan_primers(&view, pairs, n_pairs, hits, hcap, &d_cres[0], scan_ws, scan_bytes, compute);
    if (s) return s;
    s = ah_tm(&view, pairs, n_pairs, tm, hits, &d_cres[0], hcap, compute);
    if (s) return s;
    s = ah_pair_amplicons(hits, &d_cres[0], hcap, pairs, windows, n_pairs, amps, acap, &d_cres[1],
                          pair_ws, L.pair_ws, compute);
    if (s) return s;
    ah_result cr[2];
    AH_HIP(hipMemcpyAsync(cr, d_cres, sizeof cr, hipMemcpyDeviceToHost, compute));
    AH_HIP(hipStreamSynchronize(compute));  // chunk c is done: its slot is free
    if (c + slots.size() < n_chunks) {
      s = enqueue_copy(c + slots.size());
      if (s) return s;
    }
    if (total_h.count + cr[0].count > 0xffffffffull)
      return ah::set_error(AH_ERR_LIMIT, "more than 2^32 - 1 hits");
    AH_HIP(ah::launch_stream_fixup(hits, cr[0].count, amps, cr[1].count, ch.first,
                                   (uint32_t)total_h.count, grid, compute));
    if (cr[0].status != AH_OK) hits_overflowed = true;
    total_h.count += cr[0].count;
    total_h.required += cr[0].required;
    total_a.count += cr[1].count;
    total_a.required += cr[1].required;
    if (cr[1].status != AH_OK) total_a.status = AH_ERR_OVERFLOW;
  }
  if (hits_overflowed) {
    total_h.status = AH_ERR_OVERFLOW;
    total_a.status = AH_ERR_OVERFLOW;  // amplicons of the clipped chunks are missing
  }
  AH_HIP(hipMemcpyAsync(d_hit_res, &total_h, sizeof total_h, hipMemcpyHostToDevice, compute));
  AH_HIP(hipMemcpyAsync(d_amp_res, &total_a, sizeof total_a, hipMemcpyHostToDevice, compute));
  AH_HIP(hipStreamSynchronize(compute));
  return AH_OK;
}

}  // extern "C"
