// Offline-compiled kernels of libah: packing, prefix scans, the canonical-order
// radix sort of hit records, nearest-neighbour melting temperature and
// amplicon calling.  The site scan itself is specialised per primer set at
// run time (scan_core.hip).
#include <math.h>

#include <mutex>

#include "ah_internal.h"

namespace ah {
namespace {

typedef unsigned long long u64;
typedef uint32_t u32;

__device__ __forceinline__ u64 grid_threads() { return (u64)gridDim.x * blockDim.x; }
__device__ __forceinline__ u64 global_tid() { return (u64)blockIdx.x * blockDim.x + threadIdx.x; }

// Exclusive scan of one value per thread across a 256-thread workgroup.
__device__ __forceinline__ u64 block_exclusive_scan(u64 v, u64* lds4, u64& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  u64 x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    u64 y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds4[w] = x;
  __syncthreads();
  u64 before = 0;
  for (int i = 0; i < w; ++i) before += lds4[i];
  total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  __syncthreads();
  return before + x - v;
}

__device__ __forceinline__ u64 block_sum(u64 v, u64* lds4) {
  u64 t;
  block_exclusive_scan(v, lds4, t);
  return t;
}

// ---------------------------------------------------------------- packing --
// One thread per packed word: bit b of word t of genome g is base b*S + t.
__global__ __launch_bounds__(kBlock) void k_pack(const uint8_t* __restrict__ ascii,
                                                 const u64* __restrict__ ascii_off, u32 n,
                                                 const u64* __restrict__ word_off,
                                                 uint2* __restrict__ words, u32* __restrict__ len,
                                                 u32* __restrict__ nmask,
                                                 u64* __restrict__ non_acgt) {
  const u64 W = word_off[n];
  for (u64 w = global_tid(); w < W; w += grid_threads()) {
    u32 lo = 0, hi = n;
    while (hi - lo > 1) {
      const u32 mid = (lo + hi) >> 1;
      if (word_off[mid] <= w) lo = mid; else hi = mid;
    }
    const u32 g = lo;
    const u64 a0 = ascii_off[g];
    const u64 nb = ascii_off[g + 1] - a0;
    const u64 S = (nb + 31) >> 5;
    const u64 t = w - word_off[g];
    u32 h = 0, l = 0, nm = 0;
#pragma unroll 8
    for (int b = 0; b < 32; ++b) {
      const u64 p = (u64)b * S + t;
      u32 code = 0, isn = 0;
      if (p < nb) {
        const u32 c = ascii[a0 + p] | 0x20u;  // fold case
        if (c == 'a') code = 0;
        else if (c == 'c') code = 1;
        else if (c == 'g') code = 2;
        else if (c == 't') code = 3;
        else isn = 1;
      }
      h |= (code >> 1) << b;
      l |= (code & 1u) << b;
      nm |= isn << b;
    }
    words[w] = make_uint2(h, l);
    if (nmask) nmask[w] = nm;
    if (t == 0) len[g] = (u32)nb;
    if (non_acgt && t < S && nm) atomicAdd(&non_acgt[g], (u64)__popc(nm));
  }
}

__global__ void k_zero_u64(u64* p, u32 n) {
  for (u64 i = global_tid(); i < n; i += grid_threads()) p[i] = 0;
}

// ----------------------------------------------------------- ah_result ----
__global__ void k_result_init(ah_result* r) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    r->count = 0;
    r->required = 0;
    r->status = AH_OK;
    r->reserved = 0;
  }
}

__global__ void k_tile_counts(const u32* __restrict__ len, u32 n, u32 tile_words,
                              u64* __restrict__ counts) {
  for (u64 i = global_tid(); i < n; i += grid_threads()) {
    const u64 S = ((u64)len[i] + 31) >> 5;
    counts[i] = (S + tile_words - 1) / tile_words;
  }
}

// Small collections (n <= kSmallPrefix): tile counts and their exclusive
// prefix (n + 1 entries) in one workgroup of 1024 threads, and the result
// reset, in one launch.
constexpr int kSmallBlock = 1024;

__global__ __launch_bounds__(kSmallBlock) void k_tile_prefix_small(const u32* __restrict__ len, u32 n,
                                                                   u32 tile_words,
                                                                   u64* __restrict__ prefix,
                                                                   ah_result* r, u32* __restrict__ zero,
                                                                   u32 n_zero, u64* __restrict__ zero64,
                                                                   u32 n_zero64) {
  __shared__ u64 wsum[kSmallBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (u32 i = threadIdx.x; i < n_zero; i += kSmallBlock) zero[i] = 0u;
  for (u32 i = threadIdx.x; i < n_zero64; i += kSmallBlock) zero64[i] = 0ull;
  if (threadIdx.x == 0) {
    r->count = 0;
    r->required = 0;
    r->status = AH_OK;
    r->reserved = 0;
  }
  u64 run = 0;
  for (u32 base = 0; base < n; base += kSmallBlock) {
    const u32 i = base + threadIdx.x;
    u64 v = 0;
    if (i < n) {
      const u64 S = ((u64)len[i] + 31) >> 5;
      v = (S + tile_words - 1) / tile_words;
    }
    u64 x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const u64 y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    u64 before = 0, total = 0;
    for (int q = 0; q < kSmallBlock / 64; ++q) {
      before += q < w ? wsum[q] : 0u;
      total += wsum[q];
    }
    if (i < n) prefix[i] = run + before + x - v;
    run += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) prefix[n] = run;
}

// ------------------------------------------------------- prefix scans ----
template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T* __restrict__ in, u64 n_host,
                                                        const u64* __restrict__ n_dev,
                                                        u64* __restrict__ partial) {
  __shared__ u64 lds4[4];
  const u64 n = n_dev ? *n_dev : n_host;
  const u64 chunk = (n + gridDim.x - 1) / gridDim.x;
  const u64 beg = (u64)blockIdx.x * chunk;
  const u64 end = beg + chunk < n ? beg + chunk : n;
  u64 s = 0;
  for (u64 i = beg + threadIdx.x; i < end; i += blockDim.x) s += (u64)in[i];
  s = block_sum(s, lds4);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_scan_partials(u64* partial) {
  __shared__ u64 lds4[4];
  u64 total;
  const u64 v = partial[threadIdx.x];
  const u64 e = block_exclusive_scan(v, lds4, total);
  partial[threadIdx.x] = e;
  if (threadIdx.x == 0) partial[kScanGrid] = total;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_down(const T* __restrict__ in, u64* __restrict__ out,
                                                      u64 n_host, const u64* __restrict__ n_dev,
                                                      const u64* __restrict__ partial) {
  __shared__ u64 lds4[4];
  const u64 n = n_dev ? *n_dev : n_host;
  const u64 chunk = (n + gridDim.x - 1) / gridDim.x;
  const u64 beg = (u64)blockIdx.x * chunk;
  const u64 end = beg + chunk < n ? beg + chunk : n;
  u64 run = partial[blockIdx.x];
  for (u64 base = beg; base < end; base += blockDim.x) {
    const u64 i = base + threadIdx.x;
    const u64 v = i < end ? (u64)in[i] : 0;
    u64 tot;
    const u64 e = block_exclusive_scan(v, lds4, tot);
    if (i < end) out[i] = run + e;
    run += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partial[kScanGrid];
}

// ------------------------------------------------------------ radix sort --
// LSD radix sort of the hit records by their canonical key, D = 8 or 9 bits
// a pass (9 when that saves a pass).  Every pass splits the n records into
// the same G <= kSortGrid contiguous chunks, one per workgroup, and each
// pass is one scatter kernel: it derives its chunk's output offsets from all
// G chunk histograms of its digit itself (no prefix-scan launches) and,
// while placing the items, counts their next digit per destination chunk
// (no histogram launches).  The keys and the first histograms come from the
// scan's emit pass, which uses the same chunking; the last scatter writes
// the records: one launch per pass.  The counts
// are stored digit-major (hist[digit * hs + chunk], hs >= G a multiple of 4
// from the capacity: SortBuffers::hstride), so that the
// thread of a digit reads its G counts with 16-byte loads, all in flight at
// once: the counts were written by another kernel and miss the caches.

__device__ __forceinline__ u32 sort_chunks(u64 n, u64& chunk) {
  u64 c = (n + kSortGrid - 1) / kSortGrid;
  c = (c + kBlock - 1) / kBlock * kBlock;
  chunk = c < kSortChunkMin ? kSortChunkMin : c;
  return (u32)((n + chunk - 1) / chunk);
}

// Digit counts of this chunk (h: 2^D LDS counters) into the digit-major table.
template <int D>
__device__ __forceinline__ void store_hist(const u32* h, u32* __restrict__ hist, u32 hs) {
  for (u32 d = threadIdx.x; d < (1u << D); d += blockDim.x) hist[(u64)d * hs + blockIdx.x] = h[d];
}

// Stable scatter: items keep their order within a digit (chunk, then round,
// then wave, then lane).  With `out` set (last pass) the records themselves
// are written in sorted order instead of keys and indices.  Otherwise each
// item also counts its next digit into `hist_next`, in the column of the
// chunk its new position falls in (the next pass's histograms, with no
// histogram launch), and the workgroup zeroes its own column of
// `hist_clear`, which the pass after next counts into (the previous pass
// read it and has finished).
// No-op observer of the records the last pass writes.
struct NoWritten {
  __device__ void operator()(u64, const ah_hit&) const {}
};

// One pass of the sort by one block (chunk blockIdx.x); in the last pass
// (out != null) written(dst, record) is called for every record written.
template <int D, class Written>
__device__ __forceinline__ void scatter_pass(
    const u64* __restrict__ kin, const u32* __restrict__ iin, u64* __restrict__ kout,
    u32* __restrict__ iout, u64 n, int shift, const u32* __restrict__ hist,
    u32* __restrict__ hist_next, u32* __restrict__ hist_clear, u32 hs,
    const ah_hit* __restrict__ staged, ah_hit* __restrict__ out, const Written& written) {
  constexpr u32 NB = 1u << D, R = NB / kBlock;  // digits, digits per thread
  __shared__ u64 run[NB];
  __shared__ u32 wcnt[4][NB];
  __shared__ u64 lds4[4];
  u64 chunk;
  const u32 G = sort_chunks(n, chunk);
  if (blockIdx.x >= G) return;
  const u64 beg = (u64)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
  u64 pk[4];
  u32 pi[4];
  ah_hit ph[4];
  // the keys (and, in the last pass, the records) of four rounds are loaded
  // together, one round's latency; the first four are in flight while the
  // counts are read
  auto load4 = [&](u64 base) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const u64 j = base + (u64)q * blockDim.x + threadIdx.x;
      pk[q] = j < end ? kin[j] : 0;
      pi[q] = j < end ? iin[j] : 0u;
    }
    if (out) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const u64 j = base + (u64)q * blockDim.x + threadIdx.x;
        if (j < end) ph[q] = staged[pi[q]];
      }
    }
  };
  load4(beg);
  // this chunk's first slot per digit: records of smaller digits, then those
  // of the same digit in earlier chunks (thread t owns digits R t .. R t + R - 1)
  {
    u64 tot[R], before[R];
#pragma unroll
    for (u32 e = 0; e < R; ++e) {
      const uint4* row = (const uint4*)(hist + (u64)(R * threadIdx.x + e) * hs);
      tot[e] = 0;
      before[e] = 0;
#pragma unroll 16
      for (u32 q = 0; q < kSortGrid / 4; ++q) {
        if (4 * q >= G) break;
        const uint4 v = row[q];
        const u32 c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (u32 f = 0; f < 4; ++f) {
          const u32 w = 4 * q + f;
          tot[e] += w < G ? c[f] : 0u;
          before[e] += w < blockIdx.x ? c[f] : 0u;
        }
      }
    }
    u64 mine = 0;
#pragma unroll
    for (u32 e = 0; e < R; ++e) mine += tot[e];
    u64 all;
    u64 at = block_exclusive_scan(mine, lds4, all);
#pragma unroll
    for (u32 e = 0; e < R; ++e) {
      run[R * threadIdx.x + e] = at + before[e];
      at += tot[e];
    }
  }
  if (hist_clear)
    for (u32 d = threadIdx.x; d < NB; d += blockDim.x) hist_clear[(u64)d * hs + blockIdx.x] = 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (u64 base = beg; base < end; base += blockDim.x) {
    const int r = (int)(((base - beg) / blockDim.x) & 3u);
    if (r == 0 && base != beg) load4(base);
    for (int q = 0; q < 4; ++q)
      for (u32 d = threadIdx.x; d < NB; d += blockDim.x) wcnt[q][d] = 0;
    __syncthreads();
    const u64 i = base + threadIdx.x;
    const bool valid = i < end;
    u64 key = 0;
    u32 id = 0, d = 0;
    if (valid) {
      key = r == 0 ? pk[0] : r == 1 ? pk[1] : r == 2 ? pk[2] : pk[3];
      id = r == 0 ? pi[0] : r == 1 ? pi[1] : r == 2 ? pi[2] : pi[3];
      d = (u32)((key >> shift) & (NB - 1u));
    }
    // lanes of this wave with the same digit, and this lane's rank among them
    u64 peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < D; ++bit) {
      const bool on = (d >> bit) & 1u;
      const u64 bal = __ballot(valid && on);
      peers &= on ? bal : ~bal;
    }
    const u64 below = peers & ((1ull << lane) - 1ull);
    const u32 rank = (u32)__popcll(below);
    if (valid && rank == 0) wcnt[w][d] = (u32)__popcll(peers);
    __syncthreads();
    if (valid) {
      u64 dst = run[d] + rank;
      for (int q = 0; q < w; ++q) dst += wcnt[q][d];
      if (out) {
        const ah_hit rec = r == 0 ? ph[0] : r == 1 ? ph[1] : r == 2 ? ph[2] : ph[3];
        out[dst] = rec;
        written(dst, rec);
      } else {
        kout[dst] = key;
        iout[dst] = id;
        if (hist_next)
          atomicAdd(&hist_next[(u64)((key >> (shift + D)) & (NB - 1u)) * hs + dst / chunk], 1u);
      }
    }
    __syncthreads();
    for (u32 e = threadIdx.x; e < NB; e += blockDim.x)
      run[e] += (u64)wcnt[0][e] + wcnt[1][e] + wcnt[2][e] + wcnt[3][e];
    __syncthreads();
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(
    const u64* __restrict__ kin, const u32* __restrict__ iin, u64* __restrict__ kout,
    u32* __restrict__ iout, const u64* __restrict__ n_dev, int shift, const u32* __restrict__ hist,
    u32* __restrict__ hist_next, u32* __restrict__ hist_clear, u32 hs,
    const ah_hit* __restrict__ staged, ah_hit* __restrict__ out) {
  scatter_pass<D>(kin, iin, kout, iout, *n_dev, shift, hist, hist_next, hist_clear, hs, staged, out,
                  NoWritten{});
}

// ------------------------------------------------ melting temperature ----
// SantaLucia (1998) unified nearest-neighbour stacks, indexed by the
// dinucleotide (5' base * 4 + 3' base) read on the oligo strand.
__constant__ float c_nn_dh[16] = {
    -7.9f, -8.4f, -7.8f, -7.2f,   // AA AC(=GT) AG(=CT) AT
    -8.5f, -8.0f, -10.6f, -7.8f,  // CA CC(=GG) CG CT
    -8.2f, -9.8f, -8.0f, -8.4f,   // GA GC GG GT
    -7.2f, -8.2f, -8.5f, -7.9f};  // TA TC(=GA) TG(=CA) TT(=AA)
__constant__ float c_nn_ds[16] = {
    -22.2f, -22.4f, -21.0f, -20.4f,
    -22.7f, -19.9f, -27.2f, -21.0f,
    -22.2f, -24.4f, -19.9f, -22.4f,
    -21.3f, -22.2f, -22.7f, -22.2f};
constexpr float kInitGcH = 0.1f, kInitGcS = -2.8f, kInitAtH = 2.3f, kInitAtS = 4.1f;

// Error-free transformation of s + x (Knuth's TwoSum); the rounding error is
// accumulated in c.
__device__ __forceinline__ void two_sum(float& s, float& c, float x) {
  const float t = s + x;
  const float bp = t - s;
  const float err = (s - (t - bp)) + (x - bp);
  s = t;
  c += err;
}

__device__ __forceinline__ void init_term(u32 base, float& sh, float& ch, float& ss, float& cs) {
  const bool gc = base == 1u || base == 2u;
  two_sum(sh, ch, gc ? kInitGcH : kInitAtH);
  two_sum(ss, cs, gc ? kInitGcS : kInitAtS);
}

// The genomes and primer tables a Tm evaluation reads.
struct TmJob {
  const uint2* words;
  const u32* nmask;
  const u64* word_off;
  const u32* len;
  const PrimerTab* tabs;
  u32 n_genomes, n_pairs;
};

// ---- exact route for primers with too many pairings to enumerate ----------
// Under salt methods 0-5 the Tm of a pairing (a set of paired positions)
// rises with the ratio N / D of N = -Delta-H and D = -(Delta-S + KL), and D
// is positive for every pairing (the host checks KL against the largest
// Delta-S a pairing can have: two A.T initiations and no stack).  The best
// pairing then follows from Dinkelbach's iteration for a maximum ratio: with
// lambda the best ratio found so far, one max-sum pass over the positions
// finds the pairing that maximises N - lambda D, and it becomes the best
// while its ratio is higher.  The ratio rises at every step over a finite
// set, and a pass that finds nothing higher proves lambda the maximum.
//
// The pass runs over the primer's positions 5'->3' with a state per number
// e of in-set positions turned into mismatches so far (e <= budget), times
// four: S0 nothing paired yet; S1 this position paired, more pairs may
// follow; S2 a gap after a pair; S3 the last pair placed (its right
// initiation counted), nothing pairs after it.  A stack counts when a pair
// follows S1; the left initiation when a pair leaves S0.  Only positions of
// eq0 (the representative's pairs) can pair, and those outside afree (clamp
// or non-degenerate) must.  A term (h, s) weighs -h + lambda s; the constant
// lambda KL is left out.  Each state keeps its pairing as a position mask.
constexpr int kDpE = AH_MAX_K + 1;

// Delta-H / (Delta-S + KL) of pairing eq (bit 2j: position j paired) of
// oligo o, in double precision; equal to N / D above.
__device__ double pairing_ratio(u64 eq, u64 o, double KL, const float* s_dh, const float* s_ds) {
  double h = 0.0, s = 0.0;
  for (u64 st = eq & (eq >> 2); st; st &= st - 1) {
    const u32 j2 = (u32)__ffsll((long long)st) - 1u;
    const u32 ix = (u32)(((o >> j2) & 3u) << 2) | (u32)((o >> (j2 + 2u)) & 3u);
    h += (double)s_dh[ix];
    s += (double)s_ds[ix];
  }
  if (eq) {
    const u32 ends[2] = {(u32)__ffsll((long long)eq) - 1u, 63u - (u32)__clzll((long long)eq)};
    for (u32 i = 0; i < 2; ++i) {
      const u32 b = (u32)(o >> ends[i]) & 3u;
      const bool gc = b == 1u || b == 2u;
      h += (double)(gc ? kInitGcH : kInitAtH);
      s += (double)(gc ? kInitGcS : kInitAtS);
    }
  }
  return h / (s + KL);
}

// The pairing of highest Tm among eq0 with at most `budget` positions of
// afree unpaired (bit 2j: position j paired); o: the representative oligo.
// Not inlined: the enumeration route's kernels keep their own registers.
__device__ __noinline__ u64 tm_dp_pairing(u64 o, u64 eq0, u64 afree, u32 budget, u32 L, double KL,
                                          const float* s_dh, const float* s_ds) {
  const double kNeg = -__builtin_inf();
  double v[4][kDpE];
  u32 m[4][kDpE];
  u64 best = eq0;
  double rbest = pairing_ratio(eq0, o, KL, s_dh, s_ds);
  budget = min(budget, (u32)(kDpE - 1));
  for (int it = 0; it < 64; ++it) {
    const double lam = rbest;
    for (u32 e = 0; e <= budget; ++e)
      for (u32 q = 0; q < 4; ++q) {
        v[q][e] = kNeg;
        m[q][e] = 0u;
      }
    v[0][0] = 0.0;
    for (u32 j = 0; j < L; ++j) {
      const u32 j2 = 2u * j;
      const bool can_pair = ((eq0 >> j2) & 1u) != 0u;
      const bool is_free = ((afree >> j2) & 1u) != 0u;
      const u32 b = (u32)(o >> j2) & 3u;
      const bool gc = b == 1u || b == 2u;
      const double wi = -(double)(gc ? kInitGcH : kInitAtH) + lam * (double)(gc ? kInitGcS : kInitAtS);
      double ws = kNeg;
      if (j > 0u && can_pair && ((eq0 >> (j2 - 2u)) & 1u) != 0u) {
        const u32 ix = (((u32)(o >> (j2 - 2u)) & 3u) << 2) | b;
        ws = -(double)s_dh[ix] + lam * (double)s_ds[ix];
      }
      const u32 bit = 1u << j;
      // descending e: an unpaired free position reads e - 1 before it is
      // rewritten, every other transition reads e itself
      for (int e = (int)budget; e >= 0; --e) {
        double n[4] = {kNeg, kNeg, kNeg, kNeg};
        u32 q[4] = {0u, 0u, 0u, 0u};
        if (can_pair) {
          double p = v[0][e] + wi;
          u32 pm = m[0][e];
          if (v[1][e] + ws > p) { p = v[1][e] + ws; pm = m[1][e]; }
          if (v[2][e] > p) { p = v[2][e]; pm = m[2][e]; }
          n[1] = p;
          q[1] = pm | bit;
          n[3] = p + wi;
          q[3] = pm | bit;
        }
        if (!can_pair || is_free) {
          const int eu = can_pair ? e - 1 : e;
          if (eu >= 0) {
            n[0] = v[0][eu];
            q[0] = m[0][eu];
            n[2] = v[1][eu];
            q[2] = m[1][eu];
            if (v[2][eu] > n[2]) { n[2] = v[2][eu]; q[2] = m[2][eu]; }
            if (v[3][eu] > n[3]) { n[3] = v[3][eu]; q[3] = m[3][eu]; }
          }
        }
        for (u32 s = 0; s < 4; ++s) {
          v[s][e] = n[s];
          m[s][e] = q[s];
        }
      }
    }
    double fb = kNeg;
    u32 fm = 0u;
    for (u32 e = 0; e <= budget; ++e) {
      if (v[0][e] > fb) { fb = v[0][e]; fm = 0u; }
      if (v[3][e] > fb) { fb = v[3][e]; fm = m[3][e]; }
    }
    u64 eq = 0;
    for (u32 j = 0; j < L; ++j) eq |= (u64)((fm >> j) & 1u) << (2u * j);
    const double r = pairing_ratio(eq, o, KL, s_dh, s_ds);
    if (!(r > rbest)) break;
    rbest = r;
    best = eq;
  }
  return best;
}

__device__ __forceinline__ u64 wave_incl_scan(u64 v) {
  const u32 lane = threadIdx.x & 63u;
  u64 x = v;
#pragma unroll
  for (u32 o = 1; o < 64; o <<= 1) {
    const u64 y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ u64 wave_sum(u64 v) {
#pragma unroll
  for (u32 o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// A site's representative pairing and the sums every other pairing of it
// starts from.  Under the model only paired positions enter Delta-H, Delta-S
// and the initiation terms, so every oligo with the same set of paired
// positions has the same Tm.  Representative oligo: the template's base at
// each degenerate position whose set holds it ("in-set"), any member
// elsewhere (those positions mismatch for every oligo).  Other compatible
// pairings come from turning at most k - mm in-set, non-clamp positions into
// mismatches, which any other member of their set does.
//
// Salt methods 6 and 7 also depend on the oligo's G+C count, so oligos that
// pair alike differ: each pairing takes the best choice at its unpaired
// degenerate positions, a member other than the template's base (any member
// where that base is not in the set): G or C if one is allowed when G+C
// raises Tm (rB < 0), else G or C only if every allowed member is.  gp: G+C
// bits (bit 2j) of the representative, which is the oligo at paired
// positions; gu: of the best choice at unpaired ones.
struct TmRep {
  u64 o;       // representative oligo, 2 bits per position
  u64 eq0;     // its paired positions (bit 2j)
  u64 afree;   // in-set, non-clamp positions a pairing may unpair
  u64 st0;     // its stacks (bit 2j: positions j, j + 1 paired)
  u64 gp, gu;  // G+C bits (salt methods 6 and 7)
  float sh0, ch0, ss0, cs0;  // its stack sums, compensated
  u32 budget;  // positions of afree a pairing may unpair
  u32 nfree;   // positions in afree
  bool ok;     // some oligo of the primer is compatible with the site
};

// Site record h (a genome and pair of this call); T: its primer's table;
// S: the segment words of the site's genome, wbase: its first word; s_dh /
// s_ds: the stack tables in LDS.
__device__ __forceinline__ TmRep tm_rep(const TmJob& J, const ah_hit& h, u64 S, u64 wbase,
                                        const float* s_dh, const float* s_ds,
                                        const PrimerTab* T) {
  const uint2* __restrict__ words = J.words;
  const u32* __restrict__ nmask = J.nmask;
  TmRep r;
  const u32 L = T->L;
  const u32 strand = (h.strand_primer >> 1) & 1u;
  const u32 b = h.pos / (u32)S;  // S <= 2^27: 32-bit division
  const u64 w0 = wbase + (h.pos - (u64)b * S);
  // ow: the base an oligo must carry at each primer position to pair with
  // the template (2 bits per position, primer 5'->3'); nb: positions
  // opposite a non-ACGT template base, which pair with nothing.  The
  // oligo's position runs against the window on the - strand; it carries
  // the complement of the window's base on the - strand of a site, and on
  // the + strand of a decoy site (the decoy's + pattern is the primer's
  // complement: the primer against the reversed genome's - strand).
  const u32 cflip = strand ^ T->decoy;
  // All 32 words a primer can span are loaded at once, unconditionally:
  // the window word is t < S and every genome carries 31 halo words, so
  // words t .. t + 31 lie inside its allocation (and its mask's).
  uint2 wv[32];
#pragma unroll
  for (u32 j = 0; j < 32; ++j) wv[j] = words[w0 + j];
  u64 ow = 0;
#pragma unroll
  for (u32 j = 0; j < 32; ++j) {
    const u32 c = (((wv[j].x >> b) & 1u) << 1) | ((wv[j].y >> b) & 1u);
    const u32 jj = strand ? L - 1u - j : j;
    if (j < L) ow |= (u64)(cflip ? 3u - c : c) << (2u * jj);
  }
  u64 nb = 0;
  if (nmask) {
    u32 nmv[32];
#pragma unroll
    for (u32 j = 0; j < 32; ++j) nmv[j] = nmask[w0 + j];
#pragma unroll
    for (u32 j = 0; j < 32; ++j) {
      const u32 jj = strand ? L - 1u - j : j;
      if (j < L) nb |= (u64)((nmv[j] >> b) & 1u) << (2u * jj);
    }
  }
  const u64 lanes = T->lanes & ~nb;
  const u64 clampm = T->clampm;
  const u64 stackm = T->stackm;
  const u32 k = T->k;
  const bool recip = T->recip != 0u;
  const bool want_gc = T->rB < 0.0;
  u64 o = T->fixed, afree = 0, degm = 0, gu_deg = 0;
  for (u32 d = 0; d < T->nd; ++d) {
    const u32 pos2 = 2u * T->dpos[d];
    const u32 t = (u32)(ow >> pos2) & 3u;
    const u32 mem = T->mem[d];
    bool in_set = false;
    for (u32 q = 0; q < T->nmem[d]; ++q) in_set |= ((mem >> (2u * q)) & 3u) == t;
    in_set &= ((nb >> pos2) & 1u) == 0u;
    o |= (u64)(in_set ? t : (mem & 3u)) << pos2;
    if (in_set && ((clampm >> pos2) & 1u) == 0u) afree |= 1ull << pos2;
    if (recip) {
      bool any_gc = false, all_gc = true;
      for (u32 q = 0; q < T->nmem[d]; ++q) {
        const u32 m = (mem >> (2u * q)) & 3u;
        if (in_set && m == t) continue;
        const bool gc = ((m ^ (m >> 1)) & 1u) != 0u;  // C = 1, G = 2
        any_gc |= gc;
        all_gc &= gc;
      }
      degm |= 1ull << pos2;
      if (want_gc ? any_gc : all_gc) gu_deg |= 1ull << pos2;
    }
  }
  const u64 allpos = T->lanes;
  r.o = o;
  r.afree = afree;
  r.gp = (o ^ (o >> 1)) & allpos;
  r.gu = (r.gp & ~degm) | gu_deg;
  const u64 x = o ^ ow;
  r.eq0 = ~(x | (x >> 1)) & lanes;  // paired positions of the representative
  const u32 mism0 = L - (u32)__popcll(r.eq0);
  // The representative's stacks are summed once.  Another pairing turns
  // positions of it into mismatches, which only removes the stacks on
  // either side of each: its sums are the representative's minus those
  // (compensated sums throughout).
  r.st0 = r.eq0 & (r.eq0 >> 2) & stackm;
  float sh0 = 0.f, ch0 = 0.f, ss0 = 0.f, cs0 = 0.f;
  for (u64 st = r.st0; st; st &= st - 1) {
    const u32 j2 = (u32)__ffsll((long long)st) - 1u;
    const u32 ix = (u32)(((o >> j2) & 3u) << 2) | (u32)((o >> (j2 + 2u)) & 3u);
    two_sum(sh0, ch0, s_dh[ix]);
    two_sum(ss0, cs0, s_ds[ix]);
  }
  r.sh0 = sh0;
  r.ch0 = ch0;
  r.ss0 = ss0;
  r.cs0 = cs0;
  r.ok = mism0 <= k && (r.eq0 & clampm) == clampm;
  r.nfree = (u32)__popcll(afree);
  r.budget = r.ok ? min(k - mism0, r.nfree) : 0u;
  return r;
}

// The Tm of pairing eq (a subset of r.eq0) of site r, in degrees before the
// shift of salt methods 1-4.
__device__ __forceinline__ float tm_pairing(const TmRep& r, const PrimerTab* T, u64 eq,
                                            const float* s_dh, const float* s_ds) {
  float sh = r.sh0, ch = r.ch0, ss = r.ss0, cs = r.cs0;
  for (u64 st = r.st0 & ~(eq & (eq >> 2)); st; st &= st - 1) {  // the stacks eq breaks
    const u32 j2 = (u32)__ffsll((long long)st) - 1u;
    const u32 ix = (u32)(((r.o >> j2) & 3u) << 2) | (u32)((r.o >> (j2 + 2u)) & 3u);
    two_sum(sh, ch, -s_dh[ix]);
    two_sum(ss, cs, -s_ds[ix]);
  }
  if (eq) {
    const u32 lo = (u32)__ffsll((long long)eq) - 1u;
    const u32 hi = 63u - (u32)__clzll((long long)eq);
    init_term((u32)(r.o >> lo) & 3u, sh, ch, ss, cs);
    init_term((u32)(r.o >> hi) & 3u, sh, ch, ss, cs);
  }
  const float den = (float)((double)ss + (double)cs + T->KL);
  float tm = 1000.0f * (sh + ch) / den - 273.15f;
  if (T->recip) {  // 1/T += rA + rB fGC, with this pairing's best G+C count
    const u64 allpos = T->lanes;
    const u32 gc = (u32)__popcll(eq & r.gp) + (u32)__popcll(allpos & ~eq & r.gu);
    const double inv = 1.0 / ((double)tm + 273.15) + T->rA + T->rB * (double)gc / (double)T->L;
    tm = (float)(1.0 / inv - 273.15);
  }
  return tm;
}

// C(n, r) for n <= 32.  Each partial product is a binomial below 2^30 and
// each step's product below 2^35, so double precision carries them exactly
// (and a correctly rounded division of an exact multiple is exact), without
// the 64-bit integer division the device does in software.
__device__ __forceinline__ u64 binom(u32 n, u32 r) {
  if (r > n) return 0;
  double c = 1.0;
  for (u32 i = 1; i <= r; ++i) c = c * (double)(n - r + i) / (double)i;
  return (u64)c;
}

// Extra pairings of a site with nfree positions to choose from and budget
// of them to unpair: every nonempty subset of at most budget positions.
__device__ __forceinline__ u64 extra_pairings(u32 nfree, u32 budget) {
  u64 p = 0;
  for (u32 e = 1; e <= budget; ++e) p += binom(nfree, e);
  return p;
}

// The q-th of those subsets, as positions of afree (bit 2j), q <
// extra_pairings(nfree, budget): subsets by size 1, 2, ..., each size in
// colexicographic order (the combinatorial number system).
__device__ __forceinline__ u64 unrank_pairing(u64 q, u64 afree, u32 nfree, u32 budget) {
  u32 e = 1;
  for (; e < budget; ++e) {
    const u64 c = binom(nfree, e);
    if (q < c) break;
    q -= c;
  }
  u32 sel = 0, n = nfree;
  for (u32 i = e; i >= 1; --i) {
    u32 c = n - 1u;  // the largest c < n with C(c, i) <= q (C(i - 1, i) = 0)
    u64 bc = binom(c, i);
    while (bc > q) bc = binom(--c, i);
    sel |= 1u << c;
    q -= bc;
    n = c;
  }
  u64 sub = 0, m = afree;  // the sel-th positions of afree
  for (u32 j = 0; m; ++j, m &= m - 1ull)
    if ((sel >> j) & 1u) sub |= m & (0ull - m);
  return sub;
}

__device__ __forceinline__ u64 shfl64(u64 v, int src) {
  const u32 lo = (u32)__shfl((int)(u32)v, src, 64), hi = (u32)__shfl((int)(u32)(v >> 32), src, 64);
  return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ float shflf(float v, int src) { return __shfl(v, src, 64); }

// A float as an int that orders like it (for LDS atomic max; NaN never
// stored).
__device__ __forceinline__ int tm_key(float v) {
  const int b = __float_as_int(v);
  return b >= 0 ? b : b ^ 0x7fffffff;
}
__device__ __forceinline__ float tm_unkey(int k) {
  return __int_as_float(k >= 0 ? k : k ^ 0x7fffffff);
}

// The Tm of each lane's site record h (valid: the lane has one; every lane
// of the wave calls this together).  T2: the lane's pair's two primer
// tables; s_best: 64 ints of LDS for this wave.  The representative pairing
// is evaluated by its own lane.  The other pairings of all the wave's sites
// are then dealt out over the 64 lanes in turn (a site with many pairings no
// longer holds the wave while the others idle): lane l takes pairings l,
// l + 64, ... of the wave's list, finds the site each belongs to and its
// subset, and its Tm goes to the site's slot by an atomic max.  A wave whose
// sites have at most kTmLaneMax extra pairings each keeps them in their own
// lanes (a round of the dealing costs more than a few pairings).  Primers
// that take the exact route (kExact and the table's dp) find their best
// pairing by tm_dp_pairing in their own lane instead.
constexpr u64 kTmLaneMax = 4;
template <bool kExact>
__device__ __forceinline__ float tm_wave(const TmJob& J, const ah_hit& h, bool valid, u64 S,
                                         u64 wbase, const float* s_dh, const float* s_ds,
                                         const PrimerTab* T2, int* s_best) {
  const int lane = (int)(threadIdx.x & 63u);
  const PrimerTab* T = &T2[h.strand_primer & 1u];
  TmRep r{};
  float best = __int_as_float(0x7fc00000);  // NaN: no compatible oligo
  u64 own = 0;                                // this site's extra pairings
  constexpr int kNoTm = (int)0x80000000;      // below every tm_key
  if (valid) {
    r = tm_rep(J, h, S, wbase, s_dh, s_ds, T);
    if (r.ok) {
      best = tm_pairing(r, T, r.eq0, s_dh, s_ds);
      if (kExact && T->dp != 0u) {
        if (r.budget) {  // too many pairings to enumerate: the exact route
          const float v = tm_pairing(
              r, T, tm_dp_pairing(r.o, r.eq0, r.afree, r.budget, T->L, T->KL, s_dh, s_ds), s_dh,
              s_ds);
          best = best >= v ? best : v;
        }
      } else {
        own = extra_pairings(r.nfree, r.budget);
      }
    }
  }
  u64 most = own;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const u64 y = ((u64)(u32)__shfl_xor((int)(u32)(most >> 32), o, 64) << 32) |
                  (u32)__shfl_xor((int)(u32)most, o, 64);
    most = y > most ? y : most;
  }
  if (most <= kTmLaneMax) {
    // every e-subset of the free positions, e <= budget (Gosper's next
    // combination over nfree bits, deposited onto the position mask)
    for (u32 e = 1; own && e <= r.budget; ++e) {
      u64 comb = (1ull << e) - 1ull;
      while (comb < (1ull << r.nfree)) {  // nfree <= 32
        u64 sub = 0, m = r.afree, c = comb;
        while (c) {
          if (c & 1ull) sub |= m & (0ull - m);
          m &= m - 1ull;
          c >>= 1;
        }
        const float v = tm_pairing(r, T, r.eq0 & ~sub, s_dh, s_ds);
        best = (best == best && best >= v) ? best : v;
        const u64 low = comb & (0ull - comb);
        const u64 nx = comb + low;
        if (nx == 0) break;
        comb = (((nx ^ comb) >> 2) >> (__ffsll((long long)low) - 1)) | nx;  // low: a power of two
      }
    }
    return valid ? best + (float)T->tshift : best;  // salt methods 1-4 (NaN stays NaN)
  }
  const u64 incl = wave_incl_scan(own);
  const u64 total = shfl64(incl, 63);
  {
    s_best[lane] = kNoTm;
    for (u64 g0 = 0; g0 < total; g0 += 64) {
      const u64 g = g0 + (u64)lane;
      // the site of pairing g: the first lane whose inclusive count exceeds g
      int site = 0;
      for (int step = 32; step > 0; step >>= 1) {
        const u64 v = shfl64(incl, site + step - 1);
        if (v <= g) site += step;
      }
      site = site < 63 ? site : 63;
      TmRep q;
      q.o = shfl64(r.o, site);
      q.eq0 = shfl64(r.eq0, site);
      q.afree = shfl64(r.afree, site);
      q.st0 = shfl64(r.st0, site);
      q.gp = shfl64(r.gp, site);
      q.gu = shfl64(r.gu, site);
      q.sh0 = shflf(r.sh0, site);
      q.ch0 = shflf(r.ch0, site);
      q.ss0 = shflf(r.ss0, site);
      q.cs0 = shflf(r.cs0, site);
      q.nfree = (u32)__shfl((int)r.nfree, site, 64);
      q.budget = (u32)__shfl((int)r.budget, site, 64);
      const PrimerTab* Tq = (const PrimerTab*)shfl64((u64)(uintptr_t)T, site);
      const u64 first = shfl64(incl - own, site);
      if (g < total) {
        const u64 sub = unrank_pairing(g - first, q.afree, q.nfree, q.budget);
        const float v = tm_pairing(q, Tq, q.eq0 & ~sub, s_dh, s_ds);
        if (v == v) atomicMax(&s_best[site], tm_key(v));
      }
    }
    const int kb = s_best[lane];
    if (own && kb != kNoTm) {
      const float v = tm_unkey(kb);
      best = (best == best && best >= v) ? best : v;
    }
  }
  return valid ? best + (float)T->tshift : best;  // salt methods 1-4 (NaN stays NaN)
}

// Whether record h names a genome and pair of this call (a record never
// written by a scan of it is left alone rather than followed).
__device__ __forceinline__ bool tm_record_ok(const TmJob& J, const ah_hit& h) {
  return h.genome < J.n_genomes && h.pair < J.n_pairs;
}

// Sets the tm of records i = i0 + lane of hits (i < n), for the whole wave
// at once (i0: the wave's first index, the same in every lane).
template <bool kExact>
__device__ __forceinline__ void tm_records(const TmJob& J, ah_hit* __restrict__ hits, u64 i0,
                                           u64 n, const float* s_dh, const float* s_ds,
                                           int* s_best) {
  const u64 i = i0 + (threadIdx.x & 63u);
  ah_hit h{};
  bool valid = false;
  if (i < n) {
    h = hits[i];
    valid = tm_record_ok(J, h);
  }
  const u32 g = valid ? h.genome : 0u, pair = valid ? (u32)h.pair : 0u;
  const u64 S = valid ? ((u64)J.len[g] + 31) >> 5 : 1u, wbase = valid ? J.word_off[g] : 0u;
  const float v = tm_wave<kExact>(J, h, valid, S, wbase, s_dh, s_ds, &J.tabs[pair * 2u], s_best);
  if (valid) {
    h.tm = v;
    hits[i] = h;
  }
}

// Loads the stack tables into LDS (every thread of the block calls this).
__device__ __forceinline__ void tm_tables(float* s_dh, float* s_ds) {
  if (threadIdx.x < 16) {
    s_dh[threadIdx.x] = c_nn_dh[threadIdx.x];
    s_ds[threadIdx.x] = c_nn_ds[threadIdx.x];
  }
  __syncthreads();
}

template <bool kExact>
__global__ __launch_bounds__(kBlock) void k_tm(TmJob J, ah_hit* __restrict__ hits,
                                               const ah_result* __restrict__ nhits, u64 cap) {
  // the stack tables in LDS: lanes index them divergently, once per stack
  __shared__ float s_dh[16], s_ds[16];
  __shared__ int s_best[kBlock];  // per wave: the best pairing of each lane's site
  tm_tables(s_dh, s_ds);
  const u64 cnt = nhits->count;
  const u64 n = cnt < cap ? cnt : cap;
  // a wave takes 64 consecutive records at a time (the stride is whole waves)
  for (u64 i0 = global_tid() - (threadIdx.x & 63u); i0 < n; i0 += grid_threads())
    tm_records<kExact>(J, hits, i0, n, s_dh, s_ds, s_best + (threadIdx.x & ~63u));
}

// ----------------------------------------------------------- pairing ----
// Four kernels over the same partition of the sorted hits into G <= kPairGrid
// contiguous chunks, one per workgroup; each kernel derives its chunk's
// offsets from the previous kernel's per-chunk totals itself.
//   mark:    kept minus sites of the fwd and rev primer per chunk;
//   compact: the minus sites into two lists ordered like the hits;
//   count:   amplicons started by each leader + site (their minus-site
//            ranges kept for the writer), and per chunk;
//   write:   the amplicons at their offsets, and the result.
constexpr u64 kPairChunkMin = kBlock;

__device__ __forceinline__ u32 pair_chunks(u64 n, u64& chunk) {
  u64 c = (n + kPairGrid - 1) / kPairGrid;
  c = (c + kBlock - 1) / kBlock * kBlock;
  chunk = c < kPairChunkMin ? kPairChunkMin : c;
  return (u32)((n + chunk - 1) / chunk);
}

__device__ __forceinline__ u64 pair_n(const ah_result* nhits, u64 cap) {
  const u64 c = nhits->count;
  return c < cap ? c : cap;
}

// Sum of part[w] over w < upto (and over all w < G into *total), G <= kPairGrid.
__device__ __forceinline__ u64 chunk_prefix(const u64* __restrict__ part, u32 G, u32 upto,
                                            u64* lds4, u64* total) {
  u64 b = 0, t = 0;
  for (u32 w = threadIdx.x; w < G; w += blockDim.x) {
    const u64 v = part[w];
    t += v;
    b += w < upto ? v : 0u;
  }
  if (total) *total = block_sum(t, lds4);
  return block_sum(b, lds4);
}

__device__ __forceinline__ bool kept(const ah_hit& h, const PairTab* tabs) {
  const PairTab& p = tabs[h.pair];
  return !p.filter_tm || h.tm >= p.min_tm;  // NaN fails the filter
}

// 1: fwd-primer (bit 0) and rev-primer (bit 1) kept minus site
__device__ __forceinline__ u32 minus_kind(const ah_hit& h, const PairTab* tabs) {
  if (!((h.strand_primer >> 1) & 1u) || !kept(h, tabs)) return 0u;
  return (h.strand_primer & 1u) ? 2u : 1u;
}

__global__ __launch_bounds__(kBlock) void k_pair_mark(const ah_hit* __restrict__ hits,
                                                      const ah_result* __restrict__ nhits, u64 hcap,
                                                      const PairTab* __restrict__ tabs,
                                                      u64* __restrict__ cf, u64* __restrict__ cr) {
  __shared__ u64 lds4[4];
  const u64 n = pair_n(nhits, hcap);
  u64 chunk;
  if (blockIdx.x >= pair_chunks(n, chunk)) return;
  const u64 beg = (u64)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
  u64 f = 0, r = 0;
  for (u64 i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const u32 k = minus_kind(hits[i], tabs);
    f += k & 1u;
    r += k >> 1;
  }
  f = block_sum(f, lds4);
  r = block_sum(r, lds4);
  if (threadIdx.x == 0) {
    cf[blockIdx.x] = f;
    cr[blockIdx.x] = r;
  }
}

// mtot = {fwd list length, rev list length}, written by workgroup 0.
__global__ __launch_bounds__(kBlock) void k_pair_compact(
    const ah_hit* __restrict__ hits, const ah_result* __restrict__ nhits, u64 hcap,
    const PairTab* __restrict__ tabs, const u64* __restrict__ cf, const u64* __restrict__ cr,
    u64* __restrict__ kf, u32* __restrict__ pf, u32* __restrict__ xf, u64* __restrict__ kr,
    u32* __restrict__ pr, u32* __restrict__ xr, u32* __restrict__ pre_f, u32* __restrict__ pre_r,
    u64* __restrict__ mtot) {
  __shared__ u64 lds4[4];
  const u64 n = pair_n(nhits, hcap);
  u64 chunk;
  const u32 G = pair_chunks(n, chunk);
  if (blockIdx.x >= (G ? G : 1u)) return;  // workgroup 0 runs even for no hits
  const u64 beg = (u64)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
  // the first round's records and both lists' chunk counts, loaded together
  ah_hit h{};
  if (beg + threadIdx.x < end) h = hits[beg + threadIdx.x];
  u64 bf = 0, tf = 0, br = 0, tr = 0;
  for (u32 w = threadIdx.x; w < G; w += blockDim.x) {
    const u64 vf = cf[w], vr = cr[w];
    tf += vf;
    tr += vr;
    bf += w < blockIdx.x ? vf : 0u;
    br += w < blockIdx.x ? vr : 0u;
  }
  bf = block_sum(bf, lds4);
  br = block_sum(br, lds4);
  tf = block_sum(tf, lds4);
  tr = block_sum(tr, lds4);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    mtot[0] = tf;
    mtot[1] = tr;
  }
  for (u64 base = beg; base < end; base += blockDim.x) {
    const u64 i = base + threadIdx.x;
    u32 k = 0;
    if (base != beg) h = i < end ? hits[i] : ah_hit{};
    if (i < end) k = minus_kind(h, tabs);
    u64 sf, sr;
    const u64 ef = block_exclusive_scan(k & 1u, lds4, sf);
    const u64 er = block_exclusive_scan(k >> 1, lds4, sr);
    if (i < end) {  // minus sites of each list before hit i: a search hint
      pre_f[i] = (u32)(bf + ef);
      pre_r[i] = (u32)(br + er);
    }
    const u64 key = ((u64)h.pair << 32) | h.genome;
    if (k == 1u) {
      const u64 j = bf + ef;
      kf[j] = key; pf[j] = h.pos; xf[j] = (u32)i;
    } else if (k == 2u) {
      const u64 j = br + er;
      kr[j] = key; pr[j] = h.pos; xr[j] = (u32)i;
    }
    bf += sf;
    br += sr;
  }
}

// First index in [0, m) whose (key, pos) is >= (key0, pos0), found by
// exponential search from a hint h (few probes when the answer is near h, as
// it is for a hit's own minus sites).
__device__ __forceinline__ u64 lower_from(const u64* __restrict__ K, const u32* __restrict__ P,
                                          u64 m, u64 key0, u64 pos0, u64 h) {
  auto less = [&](u64 x) { return K[x] < key0 || (K[x] == key0 && (u64)P[x] < pos0); };
  if (h > m) h = m;
  u64 lo, hi;
  if (h < m && less(h)) {  // the answer lies in (h, m]
    lo = h + 1;
    hi = lo;
    u64 step = 1;
    while (hi < m && less(hi)) {
      lo = hi + 1;
      hi = lo + step;
      step <<= 1;
    }
    if (hi > m) hi = m;
  } else {  // the answer lies in [0, h]
    hi = h;
    lo = 0;
    u64 step = 1;
    while (hi > 0) {
      const u64 p = hi >= step ? hi - step : 0;
      if (less(p)) {
        lo = p + 1;
        break;
      }
      hi = p;
      step <<= 1;
    }
  }
  while (lo < hi) {
    const u64 mid = (lo + hi) >> 1;
    if (less(mid)) lo = mid + 1; else hi = mid;
  }
  return lo;
}

struct Range {
  u64 beg, end;
};

// Minus-site ranges for a + site at `pos` of (pair, genome) `key` whose
// amplicon length b.pos + lb - pos lies in [min_len, max_len]; `hint`: the
// list's sites before the + site.
__device__ __forceinline__ Range minus_range(const u64* K, const u32* P, u64 m, u64 key, u64 pos,
                                             u32 lb, const PairTab& t, u64 hint) {
  const long long lo = (long long)pos + (long long)t.min_len - (long long)lb;
  const long long hi = (long long)pos + (long long)t.max_len - (long long)lb;
  Range r{0, 0};
  if (hi < 0) return r;
  r.beg = lower_from(K, P, m, key, lo < 0 ? 0 : (u64)lo, hint);
  r.end = lower_from(K, P, m, key, (u64)hi + 1, r.beg);
  if (r.end < r.beg) r.end = r.beg;
  return r;
}

__device__ __forceinline__ bool plus_kept(const ah_hit& h, const PairTab* tabs) {
  return !((h.strand_primer >> 1) & 1u) && kept(h, tabs);
}

__device__ __forceinline__ bool same_site(const ah_hit& a, const ah_hit& b) {
  return a.pair == b.pair && a.genome == b.genome && a.pos == b.pos;
}

// A leader is the first kept + site of its (pair, genome, pos) group; it owns
// every amplicon that starts there (the fwd and rev + sites of that pos).
// Hit i and its neighbours (i itself stands in for a missing one), loaded
// unconditionally so that the three loads are in flight together.
struct Nbr {
  ah_hit prev, cur, next;
};

__device__ __forceinline__ Nbr load_nbr(const ah_hit* hits, u64 n, u64 i) {
  return Nbr{hits[i > 0 ? i - 1 : i], hits[i], hits[i + 1 < n ? i + 1 : i]};
}

// Sites of the group hit i leads: 0 (not a leader), 1 or 2 (a[0], a[1]).
__device__ __forceinline__ int group_of(const Nbr& b, u64 n, u64 i, const PairTab* tabs,
                                        ah_hit& a0, ah_hit& a1) {
  a0 = b.cur;
  a1 = b.next;
  if (!plus_kept(a0, tabs)) return 0;
  if (i > 0 && plus_kept(b.prev, tabs) && same_site(b.prev, a0)) return 0;
  if (i + 1 < n && plus_kept(a1, tabs) && same_site(a1, a0)) return 2;
  return 1;
}

__global__ __launch_bounds__(kBlock) void k_pair_count(
    const ah_hit* __restrict__ hits, const ah_result* __restrict__ nhits, u64 hcap,
    const PairTab* __restrict__ tabs, const u64* __restrict__ kf, const u32* __restrict__ pf,
    const u64* __restrict__ kr, const u32* __restrict__ pr, const u32* __restrict__ pre_f,
    const u32* __restrict__ pre_r, const u64* __restrict__ mtot, u32* __restrict__ cnt,
    u64* __restrict__ cc, uint4* __restrict__ rng) {
  __shared__ u64 lds4[4];
  const u64 n = pair_n(nhits, hcap);
  u64 chunk;
  if (blockIdx.x >= pair_chunks(n, chunk)) return;
  const u64 mf = mtot[0], mr = mtot[1];
  const u64 beg = (u64)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
  u64 sum = 0;
  for (u64 i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const u32 hf = pre_f[i], hr = pre_r[i];  // in flight with the records
    ah_hit a[2];
    const int ng = group_of(load_nbr(hits, n, i), n, i, tabs, a[0], a[1]);
    u64 c = 0;
    for (int q = 0; q < ng; ++q) {
      const PairTab t = tabs[a[q].pair];
      const u64 key = ((u64)a[q].pair << 32) | a[q].genome;
      const Range rf = minus_range(kf, pf, mf, key, a[q].pos, t.lf, t, hf);
      const Range rr = minus_range(kr, pr, mr, key, a[q].pos, t.lr, t, hr);
      c += (rf.end - rf.beg) + (rr.end - rr.beg);
      // the ranges, for the writer (list indices < cap < 2^32)
      rng[2 * i + q] = make_uint4((u32)rf.beg, (u32)rf.end, (u32)rr.beg, (u32)rr.end);
    }
    cnt[i] = (u32)c;
    sum += c;
  }
  sum = block_sum(sum, lds4);
  if (threadIdx.x == 0) cc[blockIdx.x] = sum;
}

__global__ __launch_bounds__(kBlock) void k_pair_write(
    const ah_hit* __restrict__ hits, const ah_result* __restrict__ nhits, u64 hcap,
    const PairTab* __restrict__ tabs, const u64* __restrict__ kf, const u32* __restrict__ pf,
    const u32* __restrict__ xf, const u64* __restrict__ kr, const u32* __restrict__ pr,
    const u32* __restrict__ xr, const uint4* __restrict__ rng, const u32* __restrict__ cnt,
    const u64* __restrict__ cc, ah_amplicon* __restrict__ amp, u64 cap,
    ah_result* __restrict__ res, int need_all) {
  __shared__ u64 lds4[4];
  if (need_all && nhits->status != AH_OK) {  // some sites are missing: no amplicons
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      res->count = 0;
      res->required = 0;
      res->status = AH_ERR_OVERFLOW;
      res->reserved = 0;
    }
    return;
  }
  const u64 n = pair_n(nhits, hcap);
  u64 chunk;
  const u32 G = pair_chunks(n, chunk);
  if (blockIdx.x >= (G ? G : 1u)) return;  // workgroup 0 writes the result even for no hits
  const u64 beg = (u64)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
  // a round's counts, records and ranges; the first round's are in flight
  // with the chunk counts
  u32 ci = 0;
  Nbr nb;
  uint4 g2[2];
  auto load = [&](u64 rb) {
    const u64 i = rb + threadIdx.x;
    ci = 0;
    if (i < end) {
      ci = cnt[i];
      nb = load_nbr(hits, n, i);
      g2[0] = rng[2 * i];
      g2[1] = rng[2 * i + 1];
    }
  };
  if (beg < end) load(beg);
  u64 total;
  u64 run = chunk_prefix(cc, G, blockIdx.x, lds4, &total);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    res->required = total;
    res->count = total < cap ? total : cap;
    res->status = total > cap ? AH_ERR_OVERFLOW : AH_OK;
    res->reserved = 0;
  }
  for (u64 rb = beg; rb < end; rb += blockDim.x) {
    const u64 i = rb + threadIdx.x;
    if (rb != beg) load(rb);
    u64 rt;
    const u64 base = run + block_exclusive_scan(ci, lds4, rt);
    run += rt;
    if (ci == 0) continue;
    ah_hit a[2];
    const int ng = group_of(nb, n, i, tabs, a[0], a[1]);
    if (ng == 0) continue;
    if (base >= cap) continue;
    // up to four lists, each ordered by end: (a primer, b primer)
    Range r[4];
    u32 orient[4], lb[4], plus_idx[4];
    const u32* P[4];
    const u32* X[4];
    int nl = 0;
    for (int q = 0; q < ng; ++q) {
      const PairTab t = tabs[a[q].pair];
      const u32 ap = a[q].strand_primer & 1u;
      const uint4 g4 = g2[q];  // the counting kernel's ranges
      const Range rf{g4.x, g4.y}, rr{g4.z, g4.w};
      r[nl] = rf; lb[nl] = t.lf; P[nl] = pf; X[nl] = xf; plus_idx[nl] = (u32)(i + q);
      orient[nl] = ap ? (u32)AH_RF : (u32)AH_FF; ++nl;
      r[nl] = rr; lb[nl] = t.lr; P[nl] = pr; X[nl] = xr; plus_idx[nl] = (u32)(i + q);
      orient[nl] = ap ? (u32)AH_RR : (u32)AH_FR; ++nl;
    }
    u64 w = base;
    while (w < cap) {
      int best = -1;
      u64 bend = 0;
      for (int q = 0; q < nl; ++q) {
        if (r[q].beg >= r[q].end) continue;
        const u64 e = (u64)P[q][r[q].beg] + lb[q];
        if (best < 0 || e < bend || (e == bend && orient[q] < orient[best])) {
          best = q;
          bend = e;
        }
      }
      if (best < 0) break;
      ah_amplicon A;
      A.genome = a[0].genome;
      A.start = a[0].pos;
      A.end = (u32)bend;
      A.plus_hit = plus_idx[best];
      A.minus_hit = X[best][r[best].beg];
      A.pair = a[0].pair;
      A.orient = (uint8_t)orient[best];
      A.reserved = 0;
      amp[w++] = A;
      ++r[best].beg;
    }
  }
}

// ------------------------------------------------ segmented query tail ----
// ah_query over at most kSegMax segments (pair, genome).  The scan's
// segmented emit has put each segment's records together, in no particular
// order, at seg_off[s] .. seg_off[s + 1] of the staging area.  k_seg_tail, one
// one-wave workgroup per segment, puts the segment in canonical order (its
// keys pos << 2 | strand-primer are distinct), computes every site's Tm,
// counts the amplicons each leader + site starts (the leader, its minus
// ranges and the count as the pairing kernels above define them, inside one
// segment), takes the amplicons of the earlier segments by a decoupled
// look-back over the segments' published counts, and writes its amplicons
// there.  A segment of at most kSegLds records is sorted and searched in LDS
// (at most 64 in registers); a longer one by its workgroup alone in global
// memory: stable LSD radix passes between the staging area and the output,
// an odd number of them so that the last lands in the output.
struct SegArgs {
  ah_hit* staged;          // the segments' records (the long path sorts through it)
  ah_hit* out;             // the records in canonical order
  const u32* seg_cnt;      // records of each segment
  const u64* seg_off;      // first record of each segment
  u32 n_seg, n_genomes;    // segment s = pair * n_genomes + genome
  const ah_result* hres;   // the sites' result: nothing is done on an overflow
  int key_bits;            // bits of pos << 2 | strand-primer
  TmJob tj;
  const PairTab* ptabs;
  u32* pcf;                // long segments: kept fwd- / rev- minus sites up to
  u32* pcr;                // each record (inclusive), by record index
  u32* cnt;                // amplicons each record leads (0: not a leader)
  uint4* rng;              // a leader's minus ranges, one per record
  u64* lb;                 // look-back words, one per segment (cleared before the scan)
  ah_amplicon* amp;
  u64 acap;
  ah_result* ares;
  u64 hcap;                // capacity of out (the sites)
};

__device__ __forceinline__ u64 seg_key(const ah_hit& h) {
  return ((u64)h.pos << 2) | (u64)(h.strand_primer & 3u);
}

// strand-primer (bits 0-1: primer, strand) and kept (bit 2): a kept + site
// has (kind & 6) == 4, a kept fwd-primer minus site is 6, a rev-primer one 7.
__device__ __forceinline__ u32 seg_kind(const ah_hit& h, const PairTab& p) {
  const bool k = !p.filter_tm || h.tm >= p.min_tm;  // NaN fails the filter
  return (h.strand_primer & 3u) | (k ? 4u : 0u);
}
__device__ __forceinline__ bool plus_kind(u32 k) { return (k & 6u) == 4u; }

// First index in [0, m) whose position is >= x.
template <class PosF>
__device__ __forceinline__ u32 seg_lower(const PosF& P, u32 m, u64 x) {
  u32 lo = 0, hi = m;
  while (lo < hi) {
    const u32 mid = (lo + hi) >> 1;
    if ((u64)P(mid) < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Records [x, y) of the minus sites whose amplicon with a + site at pos
// (end = their pos + lb) has a length in [min_len, max_len].
template <class PosF>
__device__ __forceinline__ uint2 seg_range(const PosF& P, u32 m, u32 pos, u32 lb, const PairTab& t) {
  const long long lo = (long long)pos + (long long)t.min_len - (long long)lb;
  const long long hi = (long long)pos + (long long)t.max_len - (long long)lb;
  if (hi < 0) return make_uint2(0u, 0u);
  const u32 a = seg_lower(P, m, lo < 0 ? 0ull : (u64)lo);
  const u32 b = seg_lower(P, m, (u64)hi + 1ull);
  return make_uint2(a, b < a ? a : b);
}

// Wanted sites in [r.x, r.y) from inclusive counts pc.
template <class C>
__device__ __forceinline__ u32 seg_count(const C* pc, uint2 r) {
  return (r.y ? (u32)pc[r.y - 1] : 0u) - (r.x ? (u32)pc[r.x - 1] : 0u);
}

// One wave per segment: the segment kernels run workgroups of one wave, so
// that a segment of a few sites does not hold three idle waves (and their
// registers), and every segment of the query is resident at once.
constexpr u32 kSegBlock = 64;


// Leaders of the sorted segment at records base .. base + m: the amplicons
// each starts (cnt) and its minus ranges (rng: fwd-primer x, y and
// rev-primer z, w, the same for both + sites of a group, which share the
// position); returns the segment's total.  The last record a lane handled
// leaves its count and ranges in c_last / r_last (for a segment of at most
// one record per lane, this lane's own).
template <class PosF, class KindF, class C>
__device__ __forceinline__ u64 seg_leaders(const SegArgs& A, const PairTab& pt, u64 base, u32 m,
                                           const PosF& P, const KindF& K, const C* pcf,
                                           const C* pcr, u32& c_last, uint4& r_last) {
  u64 sum = 0;
  c_last = 0;
  r_last = make_uint4(0u, 0u, 0u, 0u);
  for (u32 i = threadIdx.x; i < m; i += kSegBlock) {
    u32 c = 0;
    const u32 k = K(i), pos = P(i);
    if (plus_kind(k) && !(i > 0 && plus_kind(K(i - 1)) && P(i - 1) == pos)) {
      const u32 ng = (i + 1 < m && plus_kind(K(i + 1)) && P(i + 1) == pos) ? 2u : 1u;
      const uint2 rf = seg_range(P, m, pos, pt.lf, pt), rr = seg_range(P, m, pos, pt.lr, pt);
      c = ng * (seg_count(pcf, rf) + seg_count(pcr, rr));
      r_last = make_uint4(rf.x, rf.y, rr.x, rr.y);
      A.rng[base + i] = r_last;
    }
    A.cnt[base + i] = c;
    c_last = c;
    sum += c;
  }
  return wave_sum(sum);
}

// Look-back words: (state << 62) | value, state 1: the segment's own
// amplicons, 2: those of it and every earlier segment; kLbErr marks a
// prefix that a wait gave up on.
constexpr u64 kLbAgg = 1ull << 62, kLbIncl = 2ull << 62, kLbErr = 1ull << 61;
constexpr u64 kLbVal = (1ull << 61) - 1ull;
constexpr u32 kLbPolls = 1u << 20;  // polls of one window before a wait gives up

__device__ __forceinline__ u64 lb_load(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Amplicons of segments 0 .. s - 1, with kLbErr set when a wait gave up
// (every lane returns the same).  Segment s publishes its own count `agg`
// first, then reads the words of the 64 segments before the ones it has
// summed at once, back to the nearest inclusive word, and publishes its
// inclusive count.  A workgroup waits only on lower segments, whose
// workgroups were dispatched before it.
__device__ __forceinline__ u64 seg_lookback(u64* lb, u32 s, u64 agg) {
  const u32 lane = threadIdx.x & 63u;
  if (s == 0) {
    if (lane == 0) lb_store(&lb[0], kLbIncl | agg);
    return 0;
  }
  if (lane == 0) lb_store(&lb[s], kLbAgg | agg);
  u64 acc = 0, err = 0;
  long long j = (long long)s - 1;
  u32 polls = 0;
  for (;;) {
    const long long idx = j - (long long)lane;
    const u64 w = idx >= 0 ? lb_load(&lb[idx]) : kLbIncl;
    const u64 incl = __ballot((w >> 62) == 2u);
    const u32 first = incl ? (u32)__ffsll((long long)incl) - 1u : 64u;  // lane 0 reads j
    const u64 need = first >= 63u ? ~0ull : (2ull << first) - 1ull;
    const u64 ready = __ballot((w >> 62) != 0u);
    if ((ready & need) != need) {  // a word the sum needs is not published yet
      if (++polls > kLbPolls) {
        err = kLbErr;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    acc += wave_sum(lane <= first ? (w & kLbVal) : 0ull);
    if (__ballot(lane <= first && (w & kLbErr) != 0ull)) err = kLbErr;
    if (first < 64u) break;
    j -= 64;
  }
  if (lane == 0) lb_store(&lb[s], kLbIncl | err | ((acc + agg) & kLbVal));
  return acc | err;
}

// Bitonic sort of a[0 .. n2) (n2 a power of two) by the one-wave workgroup.
__device__ __forceinline__ void lds_bitonic(u64* a, u32 n2) {
  for (u32 k = 2; k <= n2; k <<= 1)
    for (u32 j = k >> 1; j > 0; j >>= 1) {
      for (u32 p = threadIdx.x; p < n2 / 2; p += kSegBlock) {
        const u32 i = ((p & ~(j - 1u)) << 1) | (p & (j - 1u));  // bit j of i clear
        const u32 l = i | j;
        const u64 x = a[i], y = a[l];
        if ((x > y) == ((i & k) == 0u)) {
          a[i] = y;
          a[l] = x;
        }
      }
      __syncthreads();
    }
}

constexpr u32 kSegIdxBits = 10;  // record index inside a sorted LDS key
static_assert((1u << kSegIdxBits) == kSegLds, "LDS keys carry the record index");

// Writes the amplicons leader i starts, from slot `at` on (below acap), in
// (end, orient) order: up to four lists (each + site of the group with the
// fwd- and the rev- sites of its ranges), each ordered by end.
template <class PosF, class KindF>
__device__ __forceinline__ void seg_write(const SegArgs& A, const PairTab& pt, const ah_hit* o,
                                          u64 base, u32 i, u32 m, u64 at, u64 acap,
                                          ah_amplicon* __restrict__ amp, const PosF& P,
                                          const KindF& K, uint4 g) {
  const u32 pos = P(i);
  const u32 ng = (i + 1 < m && plus_kind(K(i + 1)) && P(i + 1) == pos) ? 2u : 1u;
  u32 cur[4], hi[4], want[4], lb[4], orient[4], plus[4];
  int nl = 0;
  for (u32 q = 0; q < ng; ++q) {
    const u32 ap = K(i + q) & 1u;  // the + site's primer
    cur[nl] = g.x; hi[nl] = g.y; want[nl] = 6u; lb[nl] = pt.lf; plus[nl] = i + q;
    orient[nl] = ap ? (u32)AH_RF : (u32)AH_FF;
    ++nl;
    cur[nl] = g.z; hi[nl] = g.w; want[nl] = 7u; lb[nl] = pt.lr; plus[nl] = i + q;
    orient[nl] = ap ? (u32)AH_RR : (u32)AH_FR;
    ++nl;
  }
  for (int q = 0; q < nl; ++q)
    while (cur[q] < hi[q] && K(cur[q]) != want[q]) ++cur[q];
  const ah_hit lead = o[i];
  u64 w = at;
  while (w < acap) {
    int best = -1;
    u64 bend = 0;
    for (int q = 0; q < nl; ++q) {
      if (cur[q] >= hi[q]) continue;
      const u64 e = (u64)P(cur[q]) + lb[q];
      if (best < 0 || e < bend || (e == bend && orient[q] < orient[best])) {
        best = q;
        bend = e;
      }
    }
    if (best < 0) break;
    ah_amplicon a;
    a.genome = lead.genome;
    a.start = pos;
    a.end = (u32)bend;
    a.plus_hit = (u32)(base + plus[best]);
    a.minus_hit = (u32)(base + cur[best]);
    a.pair = lead.pair;
    a.orient = (uint8_t)orient[best];
    a.reserved = 0;
    amp[w++] = a;
    ++cur[best];
    while (cur[best] < hi[best] && K(cur[best]) != want[best]) ++cur[best];
  }
}

// The amplicon result from the query's total (kLbErr: a look-back wait gave
// up, reported as AH_ERR_HIP), written by the last segment's workgroup.
__device__ __forceinline__ void seg_result(const SegArgs& A, u64 total) {
  const u64 n = total & kLbVal;
  A.ares->required = n;
  A.ares->count = n < A.acap ? n : A.acap;
  A.ares->status = (total & kLbErr) ? AH_ERR_HIP : (n > A.acap ? AH_ERR_OVERFLOW : AH_OK);
  A.ares->reserved = 0;
}

// Segment blockIdx.x: canonical order, Tm, leaders, amplicons.
template <bool kExact>
__global__ __launch_bounds__(kSegBlock) void k_seg_tail(SegArgs A) {
  __shared__ u64 keys[kSegLds];  // also the long path's digit counters
  __shared__ u32 spos[kSegLds];
  __shared__ unsigned short pcf[kSegLds], pcr[kSegLds];
  __shared__ unsigned char kind[kSegLds];
  __shared__ float s_dh[16], s_ds[16];
  __shared__ PrimerTab s_tab[2];  // the pair's primer tables, read throughout the Tm
  __shared__ int s_best[kSegBlock];  // the best pairing of each lane's site
  const u32 t = threadIdx.x, s = blockIdx.x;
  // the segment's constants, loaded together: its sites, first slot, pair
  // tables and genome (every site of segment s is on genome s mod n)
  const int status = A.hres->status;
  const u32 m = A.seg_cnt[s];
  const u64 base = A.seg_off[s];
  const u32 pair = s / A.n_genomes, g = s % A.n_genomes;
  const PairTab pt = A.ptabs[pair];
  const u64 S = ((u64)A.tj.len[g] + 31) >> 5, wbase = A.tj.word_off[g];
  static_assert(sizeof(PrimerTab) % 4 == 0, "primer tables copy as words");
  for (u32 i = t; i < 2 * sizeof(PrimerTab) / 4; i += kSegBlock)
    ((u32*)s_tab)[i] = ((const u32*)(A.tj.tabs + 2 * pair))[i];
  tm_tables(s_dh, s_ds);  // its barrier also covers the copy
  const bool sites_ok = status == AH_OK;
  if (!sites_ok) {  // the sites overflowed: the pairing needs all of them
    if (s == 0 && t == 0) {
      A.ares->count = 0;
      A.ares->required = 0;
      A.ares->status = AH_ERR_OVERFLOW;
      A.ares->reserved = 0;
    }
    // The sites found still go out in canonical order with their Tm, as the
    // separate calls write them, when they fit (a full candidate list left
    // them incomplete); past the capacity none were staged.
    if (m == 0 || A.seg_off[A.n_seg] > A.hcap) return;
  }
  if (m == 0) {
    const u64 before = seg_lookback(A.lb, s, 0ull);
    if (s + 1 == A.n_seg && t == 0) seg_result(A, before);
    return;
  }
  const bool tiny = m <= kSegBlock, small = m <= kSegLds;
  ah_hit* o = A.out + base;
  if (tiny) {
    // one site per lane: a bitonic network over the wave's registers, then
    // each lane takes the record of its sorted place from the lane that
    // loaded it
    ah_hit h{};
    u64 key = ~0ull;
    if (t < m) {
      h = A.staged[base + t];
      key = (seg_key(h) << 6) | t;
    }
    for (u32 k = 2; k <= kSegBlock; k <<= 1)
      for (u32 j = k >> 1; j > 0; j >>= 1) {
        const u64 y = __shfl_xor(key, j, 64);
        const bool keep_min = ((t & j) == 0u) == ((t & k) == 0u);
        key = keep_min ? (y < key ? y : key) : (y > key ? y : key);
      }
    u32 hv[4];
    __builtin_memcpy(hv, &h, sizeof hv);
    const int from = (int)(key & 63u);
#pragma unroll
    for (int q = 0; q < 4; ++q) hv[q] = __shfl(hv[q], from, 64);
    ah_hit r;
    __builtin_memcpy(&r, hv, sizeof r);
    const float tmv = tm_wave<kExact>(A.tj, r, t < m, S, wbase, s_dh, s_ds, s_tab, s_best);
    if (t < m) {
      r.tm = tmv;
      o[t] = r;
      spos[t] = r.pos;
      kind[t] = (unsigned char)seg_kind(r, pt);
    }
  } else if (small) {
    // keys with the record index below them, padded to a power of two
    u32 n2 = 1;
    while (n2 < m) n2 <<= 1;
    for (u32 e = t; e < n2; e += kSegBlock)
      keys[e] = e < m ? (seg_key(A.staged[base + e]) << kSegIdxBits) | e : ~0ull;
    __syncthreads();
    lds_bitonic(keys, n2);
  } else {
    // stable LSD passes, an odd number, staging <-> output
    u32* hist = (u32*)keys;  // [256] digit counts, then first slots
    const int bits = A.key_bits;
    int np = (bits + 7) / 8;
    if ((np & 1) == 0) ++np;
    const int D = (bits + np - 1) / np;
    const u32 mask = (1u << D) - 1u;
    ah_hit* src = A.staged + base;
    ah_hit* dst = A.out + base;
    const u32 lane = t & 63u;
    for (int p = 0; p < np; ++p) {
      const int shift = p * D;
#pragma unroll
      for (u32 q = 0; q < 4; ++q) hist[q * 64 + t] = 0;
      __syncthreads();
      for (u32 i = t; i < m; i += kSegBlock)
        atomicAdd(&hist[(u32)(seg_key(src[i]) >> shift) & mask], 1u);
      __syncthreads();
      {  // exclusive prefix of the 256 counts: lane t owns digits 4t .. 4t + 3
        u32 c[4];
        u64 own = 0;
#pragma unroll
        for (u32 q = 0; q < 4; ++q) {
          c[q] = hist[4 * t + q];
          own += c[q];
        }
        u64 at = wave_incl_scan(own) - own;
#pragma unroll
        for (u32 q = 0; q < 4; ++q) {
          hist[4 * t + q] = (u32)at;
          at += c[q];
        }
      }
      __syncthreads();
      for (u32 r0 = 0; r0 < m; r0 += kSegBlock) {
        const u32 i = r0 + t;
        const bool valid = i < m;
        ah_hit h{};
        u32 d = 0;
        if (valid) {
          h = src[i];
          d = (u32)(seg_key(h) >> shift) & mask;
        }
        // this lane's rank among the lanes with the same digit
        u64 peers = __ballot(valid);
        for (int bit = 0; bit < D; ++bit) {
          const bool on = (d >> bit) & 1u;
          const u64 bal = __ballot(valid && on);
          peers &= on ? bal : ~bal;
        }
        const u32 rank = (u32)__popcll(peers & ((1ull << lane) - 1ull));
        if (valid) dst[hist[d] + rank] = h;
        __syncthreads();
        if (valid && rank == 0) hist[d] += (u32)__popcll(peers);
        __syncthreads();
      }
      ah_hit* x = src;
      src = dst;
      dst = x;
    }
    // src == A.out + base: the passes are odd in number
  }
  // the Tm of every site, written with the record to its place
  if (!tiny)
    for (u32 r0 = 0; r0 < m; r0 += kSegBlock) {  // the whole wave, 64 records at a time
      const u32 i = r0 + t;
      ah_hit h{};
      if (i < m) h = small ? A.staged[base + (u32)(keys[i] & (kSegLds - 1u))] : o[i];
      const float tmv = tm_wave<kExact>(A.tj, h, i < m, S, wbase, s_dh, s_ds, s_tab, s_best);
      if (i < m) {
        h.tm = tmv;
        o[i] = h;
        if (small) {
          spos[i] = h.pos;
          kind[i] = (unsigned char)seg_kind(h, pt);
        }
      }
    }
  __syncthreads();
  if (!sites_ok) return;  // the sites are in place; no pairing
  // kept fwd- (low half) and rev- (high half) minus sites up to each record
  u64 carry = 0;
  for (u32 r0 = 0; r0 < m; r0 += kSegBlock) {
    const u32 i = r0 + t;
    const u32 k = i < m ? (small ? (u32)kind[i] : seg_kind(o[i], pt)) : 0u;
    const u64 v = (k == 6u ? 1ull : 0ull) | (k == 7u ? 1ull << 32 : 0ull);
    const u64 incl = wave_incl_scan(v);
    const u64 inc = carry + incl;
    if (i < m) {
      if (small) {
        pcf[i] = (unsigned short)(inc & 0xffffffffull);
        pcr[i] = (unsigned short)(inc >> 32);
      } else {
        A.pcf[base + i] = (u32)(inc & 0xffffffffull);
        A.pcr[base + i] = (u32)(inc >> 32);
      }
    }
    carry += __shfl(incl, 63, 64);
  }
  __syncthreads();
  u64 sum;
  u32 c_own;
  uint4 r_own;
  if (small)
    sum = seg_leaders(A, pt, base, m, [&](u32 i) { return spos[i]; },
                      [&](u32 i) { return (u32)kind[i]; }, pcf, pcr, c_own, r_own);
  else
    sum = seg_leaders(A, pt, base, m, [&](u32 i) { return o[i].pos; },
                      [&](u32 i) { return seg_kind(o[i], pt); }, A.pcf + base, A.pcr + base,
                      c_own, r_own);
  const u64 before = seg_lookback(A.lb, s, sum);
  if (s + 1 == A.n_seg && t == 0) seg_result(A, (before & kLbErr) | ((before & kLbVal) + sum));
  if ((before & kLbErr) || sum == 0 || before >= A.acap) return;
  __syncthreads();  // this wave's counts and ranges are in place
  u64 at0 = before;
  for (u32 r0 = 0; r0 < m; r0 += kSegBlock) {
    const u32 i = r0 + t;
    // one record per lane: the count and ranges are still in this lane's registers
    const u32 c = tiny ? c_own : (i < m ? A.cnt[base + i] : 0u);
    const u64 incl = wave_incl_scan(c);
    const u64 at = at0 + incl - c;
    at0 += __shfl(incl, 63, 64);
    if (c && at < A.acap) {
      const uint4 g = tiny ? r_own : A.rng[base + i];
      if (small)
        seg_write(A, pt, o, base, i, m, at, A.acap, A.amp, [&](u32 j) { return spos[j]; },
                  [&](u32 j) { return (u32)kind[j]; }, g);
      else
        seg_write(A, pt, o, base, i, m, at, A.acap, A.amp, [&](u32 j) { return o[j].pos; },
                  [&](u32 j) { return seg_kind(o[j], pt); }, g);
    }
  }
}

// ----------------------------------------------------- amplicon FASTA ----
// The main output of the tool is a FASTA file of the predicted amplicons with
// their coordinates, orientation and maximum Tm (Section 2.1,
// "Visualization"); amplitypes are the per-genome patterns of copy numbers
// and sequence variants (Section 3.3, "Amplicon Pattern Visualization").
// Record of amplicon i:
//   >g<genome>:<start>-<end> pair=<pair> orient=<FR|RF|FF|RR> tm=<tm+>,<tm->
//   <sequence>
// tm+ / tm- are the Tm of its + and - sites with two decimals (nan when no
// compatible oligo).  The sequence is the top strand [start, end) for FR, FF
// and RR and its reverse complement for RF, so that the copies of one target
// read alike on either strand; a non-ACGT genome base is N.
// Sequence hash: mix(n ^ sum_k (c_k + 1) P^k mod 2^64) over its n bases
// (A0 C1 G2 T3 N4), P = 0x100000001B3, mix = the SplitMix64 finaliser.
// Amplitype of (pair, genome): the sum mod 2^64 of mix(h + 0x9E3779B97F4A7C15)
// over the sequence hashes h of its FR and RF amplicons, and their count: an
// order-free multiset hash, equal for two genomes with the same sequences in
// the same copy numbers.
constexpr u64 kSeqP = 0x100000001B3ull;
constexpr u64 kGolden = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ u32 dec_digits(u32 v) {
  u32 d = 1;
  while (v >= 10u) {
    v /= 10u;
    ++d;
  }
  return d;
}

__device__ __forceinline__ char* put_dec(char* o, u32 v) {
  const u32 d = dec_digits(v);
  for (u32 i = d; i > 0; --i) {
    o[i - 1] = (char)('0' + v % 10u);
    v /= 10u;
  }
  return o + d;
}

__device__ __forceinline__ char* put_str(char* o, const char* s) {
  while (*s) *o++ = *s++;
  return o;
}

// Tm x 100 rounded half to even, as a magnitude and a sign; false for NaN.
// |Tm| < 2^31 / 100 for every finite value this library computes.
__device__ __forceinline__ bool tm_centi(float v, u32& a, bool& neg) {
  if (!(v == v)) return false;
  const double r = rint((double)v * 100.0);
  neg = r < 0;
  a = (u32)(neg ? -r : r);
  return true;
}

__device__ __forceinline__ u32 tm_len(float v) {
  u32 a;
  bool neg;
  if (!tm_centi(v, a, neg)) return 3;  // "nan"
  return (neg ? 1u : 0u) + dec_digits(a / 100u) + 3u;
}

__device__ __forceinline__ char* put_tm(char* o, float v) {
  u32 a;
  bool neg;
  if (!tm_centi(v, a, neg)) return put_str(o, "nan");
  if (neg) *o++ = '-';
  o = put_dec(o, a / 100u);
  *o++ = '.';
  *o++ = (char)('0' + (a % 100u) / 10u);
  *o++ = (char)('0' + a % 10u);
  return o;
}

__device__ __forceinline__ u32 fasta_header_len(const ah_amplicon& A, const ah_hit* hits) {
  // ">g" ":" "-" " pair=" " orient=XX" " tm=" "," "\n"
  return 2u + dec_digits(A.genome) + 1u + dec_digits(A.start) + 1u + dec_digits(A.end) + 6u +
         dec_digits(A.pair) + 10u + 4u + tm_len(hits[A.plus_hit].tm) + 1u +
         tm_len(hits[A.minus_hit].tm) + 1u;
}

// 1: record lengths (header + sequence + newline) and per-chunk sums; the
// amplitype tables are zeroed for the writer.
__global__ __launch_bounds__(kBlock) void k_fasta_len(
    const ah_amplicon* __restrict__ amp, const ah_result* __restrict__ namp, u64 acap,
    const ah_hit* __restrict__ hits, u32* __restrict__ rec_len, u64* __restrict__ cc,
    u64* __restrict__ atype, u32* __restrict__ atype_n, u64 n_groups) {
  __shared__ u64 lds4[4];
  for (u64 q = global_tid(); q < n_groups; q += grid_threads()) {
    if (atype) atype[q] = 0;
    if (atype_n) atype_n[q] = 0;
  }
  const u64 n = pair_n(namp, acap);
  u64 chunk;
  if (blockIdx.x >= pair_chunks(n, chunk)) return;
  const u64 beg = (u64)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
  u64 sum = 0;
  for (u64 i = beg + threadIdx.x; i < end; i += blockDim.x) {
    const ah_amplicon A = amp[i];
    const u32 l = fasta_header_len(A, hits) + (A.end - A.start) + 1u;
    rec_len[i] = l;
    sum += l;
  }
  sum = block_sum(sum, lds4);
  if (threadIdx.x == 0) cc[blockIdx.x] = sum;
}

// 2: each record's first byte, and the result.
__global__ __launch_bounds__(kBlock) void k_fasta_offsets(
    const ah_result* __restrict__ namp, u64 acap, const u32* __restrict__ rec_len,
    const u64* __restrict__ cc, u64* __restrict__ rec_at, u64 tcap, ah_result* __restrict__ res) {
  __shared__ u64 lds4[4];
  const u64 n = pair_n(namp, acap);
  u64 chunk;
  const u32 G = pair_chunks(n, chunk);
  if (blockIdx.x >= (G ? G : 1u)) return;  // workgroup 0 writes the result even for none
  u64 total;
  u64 run = chunk_prefix(cc, G, blockIdx.x, lds4, &total);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    res->required = total;
    res->count = total < tcap ? total : tcap;
    res->status = total > tcap ? AH_ERR_OVERFLOW : AH_OK;
    res->reserved = 0;
  }
  const u64 beg = (u64)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
  for (u64 rb = beg; rb < end; rb += blockDim.x) {
    const u64 i = rb + threadIdx.x;
    const u32 li = i < end ? rec_len[i] : 0u;
    u64 rt;
    const u64 at = run + block_exclusive_scan(li, lds4, rt);
    if (i < end) rec_at[i] = at;
    run += rt;
  }
}

// 3: one wave per amplicon (grid-stride): lane 0 writes the header, the
// lanes the bases (lane j takes bases j, j + 64, ...: its word index steps by
// 64 words, wrapping into the next segment, with no division per base), and
// the wave sums the lanes' shares of the sequence hash.
__global__ __launch_bounds__(kBlock) void k_fasta_write(
    const uint2* __restrict__ words, const u32* __restrict__ nmask, const u64* __restrict__ word_off,
    const u32* __restrict__ glen, u32 n_genomes, const ah_amplicon* __restrict__ amp,
    const ah_result* __restrict__ namp, u64 acap, const ah_hit* __restrict__ hits,
    const u32* __restrict__ rec_len, const u64* __restrict__ rec_at, char* __restrict__ text,
    u64 tcap, u64* __restrict__ seq_hash, u64* __restrict__ atype, u32* __restrict__ atype_n,
    u32 n_pairs) {
  const u64 n = pair_n(namp, acap);
  const u32 lane = threadIdx.x & 63u;
  const u64 wid = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const u64 nw = ((u64)gridDim.x * blockDim.x) >> 6;
  // P^lane and Q = P^64 for the lane-parallel sequence hash
  u64 p_lane = 1;
  for (u32 e = 0; e < lane; ++e) p_lane *= kSeqP;
  u64 Q = kSeqP;
  for (int e = 0; e < 6; ++e) Q *= Q;
  for (u64 ai = wid; ai < n; ai += nw) {
    const ah_amplicon A = amp[ai];
    if (A.genome >= n_genomes) continue;  // not written by a pairing of these genomes
    const u64 at = rec_at[ai];
    const u32 len = A.end - A.start;
    const u32 rl = rec_len[ai];
    const u32 hl = rl - len - 1u;
    const bool fits = at + rl <= tcap;
    if (fits && lane == 0) {
      char* o = text + at;
      o = put_str(o, ">g");
      o = put_dec(o, A.genome);
      *o++ = ':';
      o = put_dec(o, A.start);
      *o++ = '-';
      o = put_dec(o, A.end);
      o = put_str(o, " pair=");
      o = put_dec(o, A.pair);
      o = put_str(o, A.orient == AH_FR ? " orient=FR" : A.orient == AH_RF ? " orient=RF"
                     : A.orient == AH_FF ? " orient=FF" : " orient=RR");
      o = put_str(o, " tm=");
      o = put_tm(o, hits[A.plus_hit].tm);
      *o++ = ',';
      o = put_tm(o, hits[A.minus_hit].tm);
      *o++ = '\n';
      text[at + rl - 1u] = '\n';
    }
    const int S = (int)(((u64)glen[A.genome] + 31u) >> 5);  // len up to 2^32 - 1
    const uint2* w = words + word_off[A.genome];
    const u32* nm = nmask ? nmask + word_off[A.genome] : nullptr;
    const bool rc = A.orient == AH_RF;
    // base x = b * S + t of this lane's first position; then x moves by 64
    const int x0 = rc ? (int)A.end - 1 - (int)lane : (int)A.start + (int)lane;
    int b = x0 / S, t = x0 - b * S;
    char* out = text + at + hl;
    u64 acc = 0, qp = 1;
    for (u32 k = lane; k < len; k += 64u) {
      const uint2 v = w[t];
      u32 c = (((v.x >> b) & 1u) << 1) | ((v.y >> b) & 1u);
      if (nm && ((nm[t] >> b) & 1u)) c = 4u;
      else if (rc) c = 3u - c;
      if (fits) out[k] = "ACGTN"[c];
      acc += (u64)(c + 1u) * qp;
      qp *= Q;
      if (rc) {
        t -= 64;
        while (t < 0) {
          t += S;
          --b;
        }
      } else {
        t += 64;
        while (t >= S) {
          t -= S;
          ++b;
        }
      }
    }
    acc *= p_lane;
    for (u32 o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) {
      const u64 h = mix64(acc ^ (u64)len);
      if (seq_hash) seq_hash[ai] = h;
      if ((A.orient == AH_FR || A.orient == AH_RF) && atype && A.pair < n_pairs) {
        const u64 gq = (u64)A.pair * n_genomes + A.genome;
        atomicAdd(&atype[gq], mix64(h + kGolden));
        if (atype_n) atomicAdd(&atype_n[gq], 1u);
      }
    }
  }
}

// ---- streaming: per-chunk offsets and id fix-up ---------------------------
// out[i] = off[i] - off[0] for i = 0..n: the word offsets of a run of genomes
// relative to the first, for a chunk staged on its own.
__global__ void k_rebase(const u64* __restrict__ off, u32 n, u64* __restrict__ out) {
  const u64 base = off[0];
  for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x)
    out[i] = off[i] - base;
}

// Chunk-local ids to collection ids: genome += gbase on hits and amplicons,
// hit indices of amplicons += hbase.
__global__ __launch_bounds__(kBlock) void k_stream_fixup(ah_hit* __restrict__ hits, u64 nh,
                                                         ah_amplicon* __restrict__ amp, u64 na,
                                                         u32 gbase, u32 hbase) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += stride) hits[i].genome += gbase;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += stride) {
    amp[i].genome += gbase;
    amp[i].plus_hit += hbase;
    amp[i].minus_hit += hbase;
  }
}

// ---- serving: subset views and id remapping ------------------------------
// View of genomes ids[0..n) of a packed collection: their word offsets and
// lengths gathered (out_off[n] = end of the last genome's words, for tidiness;
// the scan and Tm read only the first n).
__global__ void k_gather_view(const u32* __restrict__ ids, u32 n, const u64* __restrict__ off,
                              const u32* __restrict__ len, u64* __restrict__ out_off,
                              u32* __restrict__ out_len) {
  for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const u32 g = ids[i];
    out_off[i] = off[g];
    out_len[i] = len[g];
    if (i + 1 == n) out_off[n] = off[g + 1];
  }
}

// View indices to collection ids on a part's hits and amplicons; the record
// counts are read from the device results (count = records written).
__global__ __launch_bounds__(kBlock) void k_remap(ah_hit* __restrict__ hits,
                                                  const ah_result* __restrict__ hres,
                                                  ah_amplicon* __restrict__ amp,
                                                  const ah_result* __restrict__ ares,
                                                  const u32* __restrict__ ids) {
  const u64 nh = hres->count, na = ares->count;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += stride)
    hits[i].genome = ids[hits[i].genome];
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += stride)
    amp[i].genome = ids[amp[i].genome];
}

// ---- the query in one call (ah_query): the sort's passes also carry the
// melting temperature and the first step of the pairing.
//
// First pass: blocks [0, kSortGrid) run the pass; blocks from kSortGrid on
// compute the Tm of every staged record (the order is irrelevant to it, and
// the last pass copies the records, Tm included, into place) and clear the
// pairing's per-chunk counts.
template <int D, bool kExact>
__global__ __launch_bounds__(kBlock) void k_sort_scatter_tm(
    const u64* __restrict__ kin, const u32* __restrict__ iin, u64* __restrict__ kout,
    u32* __restrict__ iout, const u64* __restrict__ n_dev, int shift, const u32* __restrict__ hist,
    u32* __restrict__ hist_next, u32* __restrict__ hist_clear, u32 hs, TmJob J,
    ah_hit* __restrict__ staged, u64* __restrict__ cf, u64* __restrict__ cr) {
  if (blockIdx.x < (u32)kSortGrid) {
    scatter_pass<D>(kin, iin, kout, iout, *n_dev, shift, hist, hist_next, hist_clear, hs, nullptr,
                    nullptr, NoWritten{});
    return;
  }
  __shared__ float s_dh[16], s_ds[16];
  __shared__ int s_best[kBlock];  // per wave: the best pairing of each lane's site
  tm_tables(s_dh, s_ds);
  const u64 n = *n_dev;
  const u64 t = (u64)(blockIdx.x - kSortGrid) * kBlock + threadIdx.x;
  const u64 stride = (u64)(gridDim.x - kSortGrid) * kBlock;
  for (u64 c = t; c < (u64)kPairGrid; c += stride) {
    cf[c] = 0;
    cr[c] = 0;
  }
  for (u64 i0 = t - (threadIdx.x & 63u); i0 < n; i0 += stride)
    tm_records<kExact>(J, staged, i0, n, s_dh, s_ds, s_best + (threadIdx.x & ~63u));
}

// Last pass: as a record reaches its place, the kept minus sites of the fwd
// and rev primer are counted per chunk of the pairing (what k_pair_mark counts
// from the sorted records), summed in LDS per block first.
struct MarkWritten {
  const PairTab* tabs;
  u32* lf;  // LDS, [kPairGrid]
  u32* lr;
  u64 pchunk;
  __device__ void operator()(u64 dst, const ah_hit& rec) const {
    const u32 k = minus_kind(rec, tabs);
    if (k) atomicAdd(&((k & 1u) ? lf : lr)[dst / pchunk], 1u);
  }
};

template <int D>
__global__ __launch_bounds__(kBlock) void k_sort_scatter_mark(
    const u64* __restrict__ kin, const u32* __restrict__ iin, const u64* __restrict__ n_dev,
    int shift, const u32* __restrict__ hist, u32 hs, const ah_hit* __restrict__ staged,
    ah_hit* __restrict__ out, const PairTab* __restrict__ tabs, u64* __restrict__ cf,
    u64* __restrict__ cr) {
  __shared__ u32 lf[kPairGrid], lr[kPairGrid];
  const u64 n = *n_dev;
  u64 pchunk;
  const u32 PG = pair_chunks(n, pchunk);
  for (u32 c = threadIdx.x; c < PG; c += blockDim.x) {
    lf[c] = 0;
    lr[c] = 0;
  }
  __syncthreads();
  scatter_pass<D>(kin, iin, nullptr, nullptr, n, shift, hist, nullptr, nullptr, hs, staged, out,
                  MarkWritten{tabs, lf, lr, pchunk});
  __syncthreads();
  for (u32 c = threadIdx.x; c < PG; c += blockDim.x) {
    if (lf[c]) atomicAdd(&cf[c], (u64)lf[c]);
    if (lr[c]) atomicAdd(&cr[c], (u64)lr[c]);
  }
}

template <int D, bool kExact>
void sort_passes_fused(ah_hit* staged, ah_hit* out, const u64* n_dev, KeyBits kb,
                       const SortBuffers& sb, const TmJob& J, const PairTab* ptabs, u64* cf,
                       u64* cr, int tm_blocks, hipStream_t st) {
  const int bits = kb.total();
  const int passes = (bits + D - 1) / D;  // at least 2 (the caller checks)
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const bool last = p + 1 == passes;
    u32* next = last ? nullptr : sb.hist[(p + 1) % 3];
    u32* clear = p + 2 < passes ? sb.hist[(p + 2) % 3] : nullptr;
    if (p == 0) {
      k_sort_scatter_tm<D, kExact><<<kSortGrid + tm_blocks, kBlock, 0, st>>>(
          (const u64*)sb.keys[cur], sb.idx[cur], (u64*)sb.keys[cur ^ 1], sb.idx[cur ^ 1], n_dev, 0,
          sb.hist[0], next, clear, sb.hstride, J, staged, cf, cr);
    } else if (last) {
      k_sort_scatter_mark<D><<<kSortGrid, kBlock, 0, st>>>(
          (const u64*)sb.keys[cur], sb.idx[cur], n_dev, p * D, sb.hist[p % 3], sb.hstride, staged,
          out, ptabs, cf, cr);
    } else {
      k_sort_scatter<D><<<kSortGrid, kBlock, 0, st>>>(
          (const u64*)sb.keys[cur], sb.idx[cur], (u64*)sb.keys[cur ^ 1], sb.idx[cur ^ 1], n_dev,
          p * D, sb.hist[p % 3], next, clear, sb.hstride, staged, nullptr);
    }
    cur ^= 1;
  }
}
}  // namespace

// --------------------------------------------------- scan scratch array --
// Workspace of ah_scan_primers_noalloc: one array per device, part of the
// library's code object (so it exists as soon as the library's kernels are
// loaded on a device and lives until the process ends).  Host code never uses
// the array's name as an address: scan_scratch() looks the device address up
// once per device, with that device current, and hands out that address.
static __device__ __align__(256) unsigned char scratch[AH_SCAN_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kScratchDevices] = {};
}  // namespace

hipError_t scan_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *ptr = g_scratch[dev];
  return hipSuccess;
}

// ---------------------------------------------------------- launchers ----
hipError_t launch_pack(const uint8_t* ascii, const uint64_t* ascii_off, uint32_t n,
                       const uint64_t* word_off, uint32_t* words, uint32_t* len, uint32_t* nmask,
                       uint64_t* non_acgt, int grid, hipStream_t st) {
  if (non_acgt) {
    k_zero_u64<<<(n + kBlock - 1) / kBlock > 0 ? (n + kBlock - 1) / kBlock : 1, kBlock, 0, st>>>(
        (u64*)non_acgt, n);
  }
  k_pack<<<grid, kBlock, 0, st>>>(ascii, (const u64*)ascii_off, n, (const u64*)word_off,
                                  (uint2*)words, len, nmask, (u64*)non_acgt);
  return hipGetLastError();
}

hipError_t launch_result_init(ah_result* res, hipStream_t st) {
  k_result_init<<<1, 64, 0, st>>>(res);
  return hipGetLastError();
}

hipError_t launch_tile_prefix_small(const uint32_t* len, uint32_t n, uint32_t tile_words,
                                    uint64_t* prefix, ah_result* res, hipStream_t st,
                                    uint32_t* zero, uint32_t n_zero, uint64_t* zero64,
                                    uint32_t n_zero64) {
  k_tile_prefix_small<<<1, kSmallBlock, 0, st>>>(len, n, tile_words, (u64*)prefix, res, zero,
                                                 zero ? n_zero : 0u, (u64*)zero64,
                                                 zero64 ? n_zero64 : 0u);
  return hipGetLastError();
}

hipError_t launch_tile_counts(const uint32_t* len, uint32_t n, uint32_t tile_words, uint64_t* counts,
                              hipStream_t st) {
  const int grid = (int)((n + kBlock - 1) / kBlock) > 0 ? (int)((n + kBlock - 1) / kBlock) : 1;
  k_tile_counts<<<grid < 4096 ? grid : 4096, kBlock, 0, st>>>(len, n, tile_words, (u64*)counts);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan(const uint64_t* in, uint64_t* out, uint64_t n_host,
                                 const uint64_t* n_dev, uint64_t* tmp, hipStream_t st) {
  k_scan_reduce<u64><<<kScanGrid, kBlock, 0, st>>>((const u64*)in, n_host, (const u64*)n_dev, (u64*)tmp);
  k_scan_partials<<<1, kBlock, 0, st>>>((u64*)tmp);
  k_scan_down<u64><<<kScanGrid, kBlock, 0, st>>>((const u64*)in, (u64*)out, n_host, (const u64*)n_dev,
                                                 (const u64*)tmp);
  return hipGetLastError();
}

template <int D>
void sort_passes(const ah_hit* staged, ah_hit* out, const u64* n_dev, KeyBits kb,
                 const SortBuffers& sb, hipStream_t st) {
  const int bits = kb.total();
  const int passes = (bits + D - 1) / D;
  // three histogram tables in rotation: pass p reads H[p % 3], counts pass
  // p + 1's digits into H[(p + 1) % 3] and clears H[(p + 2) % 3]; the keys
  // and H[0] come from the scan's emit pass
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const bool last = p + 1 == passes;
    u32* next = last ? nullptr : sb.hist[(p + 1) % 3];
    u32* clear = p + 2 < passes ? sb.hist[(p + 2) % 3] : nullptr;
    k_sort_scatter<D><<<kSortGrid, kBlock, 0, st>>>(
        (const u64*)sb.keys[cur], sb.idx[cur], (u64*)sb.keys[cur ^ 1], sb.idx[cur ^ 1], n_dev, p * D,
        sb.hist[p % 3], next, clear, sb.hstride, staged, last ? out : nullptr);
    cur ^= 1;
  }
}

hipError_t launch_sort_hits(const ah_hit* staged, ah_hit* out, const uint64_t* n_dev, KeyBits kb,
                            const SortBuffers& sb, hipStream_t st) {
  if (sort_digit_bits(kb) == 9)
    sort_passes<9>(staged, out, (const u64*)n_dev, kb, sb, st);
  else
    sort_passes<8>(staged, out, (const u64*)n_dev, kb, sb, st);
  return hipGetLastError();
}

bool sort_fusable(const KeyBits& kb) {
  const int d = sort_digit_bits(kb);
  return (kb.total() + d - 1) / d >= 2;
}

hipError_t launch_sort_tm_mark(ah_hit* staged, ah_hit* out, const uint64_t* n_dev, KeyBits kb,
                               const SortBuffers& sb, const ah_genomes& g, const PrimerTab* tm_tabs,
                               uint32_t n_pairs, const PairTab* pair_tabs, const PairBuffers& pb,
                               int tm_blocks, bool exact, hipStream_t st) {
  const TmJob J{(const uint2*)g.words, g.nmask, (const u64*)g.word_off, g.len, tm_tabs, g.n, n_pairs};
  auto run = [&](auto d, auto x) {
    sort_passes_fused<decltype(d)::value, decltype(x)::value>(
        staged, out, (const u64*)n_dev, kb, sb, J, pair_tabs, (u64*)pb.cf, (u64*)pb.cr, tm_blocks,
        st);
  };
  using I8 = std::integral_constant<int, 8>;
  using I9 = std::integral_constant<int, 9>;
  if (sort_digit_bits(kb) == 9)
    exact ? run(I9{}, std::true_type{}) : run(I9{}, std::false_type{});
  else
    exact ? run(I8{}, std::true_type{}) : run(I8{}, std::false_type{});
  return hipGetLastError();
}

hipError_t launch_seg_tail(ah_hit* staged, ah_hit* out, uint64_t hcap, const SegBuffers& sg,
                           const ah_result* hres, int key_bits, const ah_genomes& g,
                           const PrimerTab* tm_tabs, uint32_t n_pairs, const PairTab* pair_tabs,
                           const PairBuffers& pb, ah_amplicon* amp, uint64_t acap,
                           ah_result* ares, bool exact, hipStream_t st) {
  SegArgs A;
  A.staged = staged;
  A.out = out;
  A.seg_cnt = sg.cnt;
  A.seg_off = (const u64*)sg.off;
  A.n_seg = sg.n_seg;
  A.n_genomes = sg.n_genomes;
  A.hres = hres;
  A.key_bits = key_bits;
  A.tj = TmJob{(const uint2*)g.words, g.nmask, (const u64*)g.word_off, g.len, tm_tabs, g.n, n_pairs};
  A.ptabs = pair_tabs;
  A.pcf = pb.pre_f;
  A.pcr = pb.pre_r;
  A.cnt = pb.cnt;
  A.rng = (uint4*)pb.rng;
  A.lb = (u64*)sg.lb;
  A.amp = amp;
  A.acap = acap;
  A.hcap = hcap;
  A.ares = ares;
  const u32 grid = sg.n_seg > 0 ? sg.n_seg : 1u;
  if (exact)
    k_seg_tail<true><<<grid, kSegBlock, 0, st>>>(A);
  else
    k_seg_tail<false><<<grid, kSegBlock, 0, st>>>(A);
  return hipGetLastError();
}

hipError_t launch_tm(const ah_genomes& g, const PrimerTab* tabs, uint32_t n_pairs, ah_hit* hits,
                     const ah_result* nhits, uint64_t cap, int grid, bool exact, hipStream_t st) {
  const TmJob J{(const uint2*)g.words, g.nmask, (const u64*)g.word_off, g.len, tabs, g.n, n_pairs};
  if (exact)
    k_tm<true><<<grid, kBlock, 0, st>>>(J, hits, nhits, cap);
  else
    k_tm<false><<<grid, kBlock, 0, st>>>(J, hits, nhits, cap);
  return hipGetLastError();
}

hipError_t launch_pair(const ah_hit* hits, const ah_result* nhits, uint64_t hit_cap,
                       const PairTab* tabs, ah_amplicon* amp, uint64_t cap, ah_result* res,
                       const PairBuffers& pb, hipStream_t st, bool marked, bool need_all) {
  if (!marked)
    k_pair_mark<<<kPairGrid, kBlock, 0, st>>>(hits, nhits, hit_cap, tabs, (u64*)pb.cf, (u64*)pb.cr);
  k_pair_compact<<<kPairGrid, kBlock, 0, st>>>(hits, nhits, hit_cap, tabs, (const u64*)pb.cf,
                                              (const u64*)pb.cr, (u64*)pb.mkey_f, pb.mpos_f,
                                              pb.midx_f, (u64*)pb.mkey_r, pb.mpos_r, pb.midx_r,
                                              pb.pre_f, pb.pre_r, (u64*)pb.mtot);
  k_pair_count<<<kPairGrid, kBlock, 0, st>>>(hits, nhits, hit_cap, tabs, (const u64*)pb.mkey_f,
                                            pb.mpos_f, (const u64*)pb.mkey_r, pb.mpos_r,
                                            pb.pre_f, pb.pre_r, (const u64*)pb.mtot, pb.cnt,
                                            (u64*)pb.cc, (uint4*)pb.rng);
  k_pair_write<<<kPairGrid, kBlock, 0, st>>>(hits, nhits, hit_cap, tabs, (const u64*)pb.mkey_f,
                                            pb.mpos_f, pb.midx_f, (const u64*)pb.mkey_r, pb.mpos_r,
                                            pb.midx_r, (const uint4*)pb.rng, pb.cnt,
                                            (const u64*)pb.cc, amp, cap, res, need_all ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_fasta(const ah_genomes& g, const ah_hit* hits, const ah_amplicon* amp,
                        const ah_result* namp, uint64_t acap, uint32_t n_pairs, char* text,
                        uint64_t tcap, ah_result* res, uint64_t* seq_hash, uint64_t* atype,
                        uint32_t* atype_n, uint32_t* rec_len, uint64_t* rec_at, uint64_t* cc,
                        int waves, hipStream_t st) {
  const u64 n_groups = (u64)n_pairs * g.n;
  k_fasta_len<<<kPairGrid, kBlock, 0, st>>>(amp, namp, acap, hits, rec_len, (u64*)cc, (u64*)atype,
                                           atype_n, n_groups);
  k_fasta_offsets<<<kPairGrid, kBlock, 0, st>>>(namp, acap, rec_len, (const u64*)cc, (u64*)rec_at,
                                               tcap, res);
  const int blocks = (waves + kBlock / 64 - 1) / (kBlock / 64);
  k_fasta_write<<<blocks > 0 ? blocks : 1, kBlock, 0, st>>>(
      (const uint2*)g.words, g.nmask, (const u64*)g.word_off, g.len, g.n, amp, namp, acap, hits,
      rec_len, (const u64*)rec_at, text, tcap, (u64*)seq_hash, (u64*)atype, atype_n, n_pairs);
  return hipGetLastError();
}

hipError_t launch_rebase(const uint64_t* off, uint32_t n, uint64_t* out, hipStream_t st) {
  const uint64_t blocks = ((uint64_t)n + kBlock) / kBlock;
  const unsigned grid = blocks > 1024 ? 1024u : (unsigned)blocks;
  k_rebase<<<grid, kBlock, 0, st>>>((const u64*)off, n, (u64*)out);
  return hipGetLastError();
}

hipError_t launch_stream_fixup(ah_hit* hits, uint64_t nh, ah_amplicon* amp, uint64_t na,
                               uint32_t gbase, uint32_t hbase, int grid, hipStream_t st) {
  if (nh == 0 && na == 0) return hipSuccess;
  k_stream_fixup<<<grid, kBlock, 0, st>>>(hits, nh, amp, na, gbase, hbase);
  return hipGetLastError();
}

hipError_t launch_gather_view(const uint32_t* ids, uint32_t n, const uint64_t* off, const uint32_t* len,
                              uint64_t* out_off, uint32_t* out_len, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = ((uint64_t)n + kBlock - 1) / kBlock;
  const unsigned grid = blocks > 1024 ? 1024u : (unsigned)blocks;
  k_gather_view<<<grid, kBlock, 0, st>>>(ids, n, (const u64*)off, len, (u64*)out_off, out_len);
  return hipGetLastError();
}

hipError_t launch_remap(ah_hit* hits, const ah_result* hres, ah_amplicon* amp, const ah_result* ares,
                        const uint32_t* ids, int grid, hipStream_t st) {
  k_remap<<<grid, kBlock, 0, st>>>(hits, hres, amp, ares, ids);
  return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t* p, uint32_t n, hipStream_t st) {
  k_zero_u64<<<1, 64, 0, st>>>((u64*)p, n);
  return hipGetLastError();
}

}  // namespace ah
