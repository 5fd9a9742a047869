// Binding-site scan core (primer matching, Section 2.1 of AmpliconHunter).
//
// This file is compiled at run time (hipRTC) once per primer set, with a
// generated pattern program appended after it; the build compiles a few such
// specialisations to check that it builds.  A pattern is one primer of a pair
// on one strand.  Two kernels:
//
// * ah_scan_kernel, the filter.  Packed layout (see ah.h): bit b of word t of a
//   genome holds the base at b*S + t, so the window starting at b*S + t reads
//   word t + j at bit b for primer position j and 32 windows advance together.
//   A workgroup stages a tile of 256 x AH_U window words plus the primer halo
//   in LDS; each lane takes AH_U consecutive window words and keeps, in
//   registers, a sliding window of the one-hot planes (A, C, G, T) of the
//   words they read, so each genome word is read from LDS and converted once
//   per lane.  On one-hot planes a primer position with a single base is a
//   single operand, and one 3-input bitwise operation tests two positions.
//   The generated filter of each pattern passes every window with at most k
//   mismatches (pigeonhole blocks, or the exact count for patterns where
//   blocks do not pay); windows that pass are appended to the workgroup's own
//   slice of a candidate list (counted in LDS: no global atomics on the hot
//   path, where same-address device atomics would serialise).
// * ah_verify_kernel: one workgroup per slice; the exact count (every
//   position, the non-ACGT mask, the clamp, window starts inside the genome)
//   of every candidate, which appends the binding sites.  Kept apart from the
//   filter so that its registers do not lower the filter's occupancy.
//
// Macros supplied by the generated program: AH_U (window words per lane, odd
// so that the lanes' LDS reads fall in distinct banks), AH_HALO (longest
// primer - 1), AH_HAS_N (1 if the collection has non-ACGT bases, whose
// positions mismatch every primer position).

typedef unsigned int u32;
typedef unsigned long long u64;

#ifndef AH_BLOCK
#define AH_BLOCK 256
#endif
#define AH_TILE (AH_BLOCK * AH_U)

// Must match ah_hit in ah.h (16 bytes).
struct AhHitRec {
  u32 genome;
  u32 pos;
  unsigned short pair;
  unsigned char strand_primer;
  unsigned char mm;
  float tm;
};

struct AhCtx {
  const uint2* gw;  // this genome's first packed word
  const u32* gn;    // this genome's first non-ACGT mask word (or null)
  u32 g;            // genome
  u32 n;            // bases
  u32 S;            // segment words
  int tail;         // n - 31*S: a window of length L at word t is valid in
                    // every segment iff t + L <= tail
};

// Candidate list: one record per (window word, pattern) with at least one
// window that passed the filter; workgroup b owns records [b * slice, (b + 1)
// * slice).
struct AhCands {
  uint4* out;   // {genome, window word, pattern, window mask}
  u32 slice;    // records per workgroup
};

// This workgroup's candidate count and the windows in them.
__shared__ u32 ah_n_cand;
__shared__ u32 ah_n_win;

// Window starts b*S + t (b = 0..31) that lie inside the genome for a primer
// of length L, as a bit mask over b.
__device__ __forceinline__ u32 ah_valid(const AhCtx& c, u32 t, u32 L) {
  if ((long long)t + (long long)L <= (long long)c.tail) return 0xffffffffu;
  const long long d = (long long)c.n - (long long)L - (long long)t;
  if (d < 0) return 0u;
  if (d >= 31ll * (long long)c.S) return 0xffffffffu;
  const u32 bmax = (u32)(d / (long long)c.S);  // <= 30
  return (2u << bmax) - 1u;
}

// Write one record per set bit of hb from `slot` on (records at or beyond
// cap are dropped); lv[m] has bit b set iff window b has more than m
// mismatches.
template <int NLEV>
__device__ __forceinline__ void ah_emit(const AhCtx& c, AhHitRec* out, u64 cap, u64 slot, u32 t,
                                        u32 hb, const u32* lv, u32 pair, u32 sp) {
  while (hb) {
    const u32 b = __ffs(hb) - 1u;
    hb &= hb - 1u;
    u32 mm = 0;
#pragma unroll
    for (int m = 0; m < NLEV; ++m) mm += (lv[m] >> b) & 1u;
    if (slot < cap) {
      AhHitRec r;
      r.genome = c.g;
      r.pos = b * c.S + t;
      r.pair = (unsigned short)pair;
      r.strand_primer = (unsigned char)sp;
      r.mm = (unsigned char)mm;
      r.tm = __int_as_float(0x7fc00000);
      out[slot] = r;
    }
    ++slot;
  }
}

__device__ __forceinline__ AhCtx ah_ctx(const uint2* words, const u32* nmask,
                                        const u64* __restrict__ word_off,
                                        const u32* __restrict__ len, u32 g) {
  AhCtx c;
  c.g = g;
  c.n = len[g];
  c.S = (c.n + 31u) >> 5;
  c.tail = (int)((long long)c.n - 31ll * (long long)c.S);
  const u64 wbase = word_off[g];
  c.gw = words + wbase;
  c.gn = AH_HAS_N ? nmask + wbase : nullptr;
  return c;
}

// Genome of tile T (binary search over the tile prefix, starting from the
// previous tile's genome when it still applies) and the tile's first word.
__device__ __forceinline__ u32 ah_tile_genome(const u64* __restrict__ tile_prefix, u32 n_genomes,
                                              u64 T, u32& lo) {
  u32 hi = n_genomes;
  if (tile_prefix[lo] > T) lo = 0;
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (tile_prefix[mid] <= T) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void ah_cand(const AhCtx& c, const AhCands& k, u32 t, u32 pattern,
                                        u32 cand) {
  if (t >= c.S) return;  // lanes past the genome's last window word
  const u32 slot = atomicAdd(&ah_n_cand, 1u);
  atomicAdd(&ah_n_win, (u32)__popc(cand));
  if (slot < k.slice) k.out[(u64)blockIdx.x * k.slice + slot] = make_uint4(c.g, t, pattern, cand);
}

// One-hot planes of a packed word: bit b of each is set iff base b*S + t is
// that base (A=00, C=01, G=10, T=11 in (h, l)).
__device__ __forceinline__ void ah_onehot(uint2 v, u32& a, u32& c, u32& g, u32& t) {
  a = ~(v.x | v.y);
  c = ~v.x & v.y;
  g = v.x & ~v.y;
  t = v.x & v.y;
}

typedef __attribute__((address_space(3))) const uint2 ah_lds_uint2;

// Generated: every group of patterns in turn filters the staged tile and
// appends its candidates.
__device__ void ah_groups(ah_lds_uint2* tw, u32 t0, const AhCtx& c, const AhCands& k);
// Generated: exact count of the candidate windows `cand` of pattern `p` at
// window word t, whose words t, t + 1, ... are w[0], w[1], ...; returns the
// binding sites found and, when `emit`, writes their records from `slot` on.
template <class W>
__device__ u32 ah_verify_one(const AhCtx& c, W w, u32 t, u32 p, u32 cand, AhHitRec* out, u64 cap,
                             u64 slot, bool emit);

// Words staged per tile: the tile's window words plus the halo, in 16-byte
// pairs (every genome starts 16-byte aligned).
#define AH_STAGE_PAIRS ((AH_TILE + AH_HALO + 1) / 2)
#define AH_STAGE_PER_THREAD ((AH_STAGE_PAIRS + AH_BLOCK - 1) / AH_BLOCK)

typedef __attribute__((address_space(3))) void ah_lds_void;
typedef __attribute__((address_space(1))) void ah_global_void;

// Copy this wave's share of a tile straight from HBM into LDS (no registers):
// each lane moves 16 bytes; the LDS base is uniform over the wave and the
// hardware places lane i at base + 16 i.
__device__ __forceinline__ void ah_stage(const AhCtx& c, u32 t0, uint4* tw) {
  const u32 last_pair = ((c.S + 31u + 1u) >> 1) - 1u;
  const uint4* gp = (const uint4*)c.gw;
  const u32 wave_base = threadIdx.x & ~63u;
#pragma unroll
  for (int k = 0; k < AH_STAGE_PER_THREAD; ++k) {
    const u32 i = threadIdx.x + (u32)k * AH_BLOCK;
    if (i < AH_STAGE_PAIRS) {
      // a clamped index only ever replaces words that no valid window reads
      const uint4* src = gp + min((t0 >> 1) + i, last_pair);
      __builtin_amdgcn_global_load_lds((ah_global_void*)src,
                                       (ah_lds_void*)(tw + wave_base + (u32)k * AH_BLOCK), 16, 0, 0);
    }
  }
}

extern "C" __global__ __launch_bounds__(AH_BLOCK) void ah_scan_kernel(
    const uint2* __restrict__ words, const u32* __restrict__ nmask,
    const u64* __restrict__ word_off, const u32* __restrict__ len,
    const u64* __restrict__ tile_prefix, u32 n_genomes, uint4* __restrict__ cand_out,
    u32 slice, u32* __restrict__ slice_count, u64* __restrict__ cand_stat) {
  __shared__ uint4 tile[AH_STAGE_PAIRS];
  const u64 n_tiles = tile_prefix[n_genomes];
  const AhCands k{cand_out, slice};
  if (threadIdx.x == 0) {
    ah_n_cand = 0;
    ah_n_win = 0;
  }
  __syncthreads();
  u32 lo = 0;
  for (u64 T = blockIdx.x; T < n_tiles; T += gridDim.x) {
    const u32 g = ah_tile_genome(tile_prefix, n_genomes, T, lo);
    const AhCtx c = ah_ctx(words, nmask, word_off, len, g);
    const u32 t0 = (u32)(T - tile_prefix[g]) * (u32)AH_TILE;
    ah_stage(c, t0, tile);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed
    __syncthreads();                // and everyone's
    ah_groups((ah_lds_uint2*)tile, t0, c, k);
    __syncthreads();                // nobody reads the tile any more
  }
  if (threadIdx.x == 0) {  // every workgroup reports, with or without tiles
    slice_count[blockIdx.x] = min(ah_n_cand, slice);
    if (ah_n_cand) {
      atomicAdd(&cand_stat[0], (u64)ah_n_cand);
      atomicAdd(&cand_stat[1], (u64)ah_n_win);
      if (ah_n_cand > slice) atomicAdd(&cand_stat[2], 1ull);
      atomicMax(&cand_stat[3], (u64)ah_n_cand);
    }
  }
}

extern "C" __global__ __launch_bounds__(AH_BLOCK) void ah_verify_kernel(
    const uint2* __restrict__ words, const u32* __restrict__ nmask,
    const u64* __restrict__ word_off, const u32* __restrict__ len,
    const uint4* __restrict__ cands, u32 slice, const u32* __restrict__ slice_count,
    AhHitRec* __restrict__ out, u64 cap, u64* __restrict__ counter) {
  // One workgroup per slice, in rounds of one candidate per thread: count the
  // round's sites, reserve their records with one atomic for the workgroup
  // (same-address device atomics serialise), then count again and write.
  __shared__ u32 round_sites;
  __shared__ u64 round_base;
  const u32 n = slice_count[blockIdx.x];
  const uint4* mine = cands + (u64)blockIdx.x * slice;
  for (u32 r = 0; r < n; r += AH_BLOCK) {
    if (threadIdx.x == 0) round_sites = 0;
    __syncthreads();
    const u32 i = r + threadIdx.x;
    uint4 e = make_uint4(0, 0, 0, 0);
    AhCtx c{};
    u32 found = 0, off = 0;
    if (i < n) {
      e = mine[i];
      c = ah_ctx(words, nmask, word_off, len, e.x);
      found = ah_verify_one(c, c.gw + e.y, e.y, e.z, e.w, out, cap, 0, false);
      if (found) off = atomicAdd(&round_sites, found);
    }
    __syncthreads();
    if (threadIdx.x == 0 && round_sites) round_base = atomicAdd(counter, (u64)round_sites);
    __syncthreads();
    if (found) ah_verify_one(c, c.gw + e.y, e.y, e.z, e.w, out, cap, round_base + off, true);
    __syncthreads();
  }
}

// ---- generated pattern program follows ----
