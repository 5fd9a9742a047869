// Binding-site scan core (primer matching, Section 2.1 of AmpliconHunter).
//
// This file is compiled at run time (hipRTC) once per primer set, with a
// generated pattern program appended after it; the build compiles a few such
// specialisations to check that it builds.  A pattern is one primer of a pair
// on one strand.  The kernels: the filter, the exact count where the filter
// does not take it, and one of two emit passes:
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
//   path, where same-address device atomics would serialise).  After its
//   last tile each wave (wave mode) or workgroup (tile mode, AH_TILE_COUNT)
//   takes the exact count (every position, the non-ACGT mask, the clamp,
//   window starts inside the genome) of the candidates of its own slice,
//   stored per candidate and summed per slice, while others still filter:
//   the count waits on memory, the filter on the vector ALU.
// * ah_verify_kernel: the same count as a launch of its own after the
//   filter, one workgroup per slice, for tile-mode programs of many
//   patterns (AH_TILE_COUNT 0).
// * ah_emit_kernel: one workgroup per slice; the slice's output offset is the
//   sum of the earlier slices' sites (the sums of the earlier groups of 64
//   slices, then of the earlier slices of its own group; no device atomics),
//   and the candidates with sites are counted again, now writing the site
//   records, their sort keys and the sort's first histograms.  Workgroup 0
//   also writes the result (required = sites found, count = records written)
//   and the candidate-list statistics; a full slice makes the result an
//   overflow whose bound covers both lists.
// * ah_emit_seg_kernel: the same records, written into their (pair, genome)
//   segments at the places the exact count reserved, for the segmented tail
//   of the whole query.
//
// Macros supplied by the generated program: AH_U (window words per lane, odd
// so that the lanes' LDS reads fall in distinct banks), AH_HALO (longest
// primer - 1), AH_HAS_N (1 if the collection has non-ACGT bases, whose
// positions mismatch every primer position), AH_WAVE (1: wave mode, below),
// AH_QUAD_ONE_PAIR (1: the four patterns of every candidate record belong to
// one primer pair), AH_TILE_COUNT (1: in tile mode the filter takes the exact
// count).

typedef unsigned int u32;
typedef unsigned long long u64;

#ifndef AH_BLOCK
#define AH_BLOCK 256
#endif
#define AH_TILE (AH_BLOCK * AH_U)
// Slices per group of the emit pass's offsets (group sums added by the exact
// count, cleared before the filter).  Each group's sum has a 256-byte line of its
// own: atomics to one line serialise.
#define AH_SLICE_GROUP 64
#define AH_GROUP_STRIDE 32
// Candidate slices per workgroup of the filter: one per wave in wave mode.
// The count and emit passes run one workgroup per filter workgroup and read
// its slices in order as one list.
#if AH_WAVE
#define AH_SPW (AH_BLOCK / 64)
#else
#define AH_SPW 1
#endif

// Counts of the AH_SPW slices of workgroup b, and their total.
struct AhSlices {
  u32 n[AH_SPW];
  u32 total;
};
__device__ __forceinline__ AhSlices ah_slices(const u32* __restrict__ slice_count, u32 b) {
  AhSlices r;
  r.total = 0;
#pragma unroll
  for (int q = 0; q < AH_SPW; ++q) {
    r.n[q] = slice_count[b * AH_SPW + q];
    r.total += r.n[q];
  }
  return r;
}
// Index into the candidate list of the i-th candidate of workgroup b's slices.
__device__ __forceinline__ u64 ah_slice_at(const AhSlices& sl, u32 b, u32 slice, u32 i) {
  u32 q = 0;
#pragma unroll
  for (int k = 0; k + 1 < AH_SPW; ++k)
    if (q == (u32)k && i >= sl.n[k]) {  // past slice k (constant indices only)
      i -= sl.n[k];
      q = (u32)k + 1u;
    }
  return (u64)(b * AH_SPW + q) * slice + i;
}

// Must match ah_result in ah.h.
struct AhResult {
  u64 count;
  u64 required;
  int status;
  u32 reserved;
};
#define AH_RES_OVERFLOW (-4)

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

// Candidate list: one 32-byte record per (window word, quad of patterns p0 ..
// p0 + 3) where the filter of at least one of the four passed a window: two
// uint4, {genome, window word, p0, 0} and the four patterns' window masks
// (0 for patterns past the set's last).  Slice s owns records [s * slice,
// (s + 1) * slice).
struct AhCands {
  uint4* out;   // 2 uint4 per record
  u32 slice;    // records per workgroup (per wave in wave mode)
  u64* win;     // wave mode: windows of the candidates a full slice dropped, per slice
};

// This workgroup's candidate count and the windows in them.
__shared__ u32 ah_n_cand;
__shared__ unsigned long long ah_n_lost;  // windows of the candidates a full slice dropped

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
  c.S = (u32)(((u64)c.n + 31u) >> 5);  // n may be up to 2^32 - 1
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

__device__ __forceinline__ void ah_cand(const AhCtx& c, const AhCands& k, u32 t, u32 p0, u32 m0,
                                        u32 m1, u32 m2, u32 m3) {
  if (t >= c.S) return;  // lanes past the genome's last window word
  const u32 slot = atomicAdd(&ah_n_cand, 1u);
  if (slot < k.slice) {
    uint4* o = k.out + 2 * ((u64)blockIdx.x * k.slice + slot);
    o[0] = make_uint4(c.g, t, p0, 0u);
    o[1] = make_uint4(m0, m1, m2, m3);
  } else {
    atomicAdd(&ah_n_lost, (unsigned long long)(__popc(m0) + __popc(m1) + __popc(m2) + __popc(m3)));
  }
}

// Wave mode: append the lanes' candidates of the quad of patterns p0 .. p0 +
// 3 to slice s, owned by this wave alone; cnt (wave-uniform: every lane
// calls this) counts the records offered so far, kept or not, and the new
// count is returned.  Slots come from a ballot over the wave, so nothing on
// this path touches LDS (an LDS access here would also wait for the wave's
// copy of its next tile to land).
__device__ __forceinline__ u32 ah_wcand(const AhCtx& c, const AhCands& k, u32 t, u32 p0, u32 m0,
                                        u32 m1, u32 m2, u32 m3, u32 cnt, u32 s) {
  const bool ok = (m0 | m1 | m2 | m3) != 0u && t < c.S;  // t >= S: past the genome, or lane 63
  const u64 m = __ballot(ok);
  if (ok) {
    const u32 slot = cnt + __builtin_amdgcn_mbcnt_hi((u32)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((u32)m, 0u));
    if (slot < k.slice) {
      uint4* o = k.out + 2 * ((u64)s * k.slice + slot);
      o[0] = make_uint4(c.g, t, p0, 0u);
      o[1] = make_uint4(m0, m1, m2, m3);
    } else {
      atomicAdd(&k.win[s],
                (unsigned long long)(__popc(m0) + __popc(m1) + __popc(m2) + __popc(m3)));
    }
  }
  return cnt + (u32)__popcll(m);
}

// Bit planes of a packed word: bit b of the one-hot planes a/c/g/t is set iff
// base b*S + t is that base (A=00, C=01, G=10, T=11 in (h, l)); h, l and
// x = h ^ l hold the two-base classes.  Planes a filter never reads cost
// nothing (the compiler drops them).
__device__ __forceinline__ void ah_planes(uint2 v, u32& a, u32& c, u32& g, u32& t, u32& h, u32& l,
                                          u32& x) {
  a = ~(v.x | v.y);
  c = ~v.x & v.y;
  g = v.x & ~v.y;
  t = v.x & v.y;
  h = v.x;
  l = v.y;
  x = v.x ^ v.y;
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
// Generated: the primer pair of pattern p.
__device__ u32 ah_pat_pair(u32 p);

// Exact count of candidate record `at` (the windows of its four patterns):
// its sites go to cand_sites[at] and the running sums; with seg_cnt set they
// are also counted per segment (pair, genome) at seg_cnt[pair * seg_n +
// genome], and when every record's patterns share a pair (AH_QUAD_ONE_PAIR)
// one device atomic per candidate reserves its sites' places in the segment:
// cand_sites[at] then keeps the first place + 1 (0: no sites) for the
// segmented emit instead of the count.
__device__ __forceinline__ void ah_verify_cand(const uint2* __restrict__ words,
                                               const u32* __restrict__ nmask,
                                               const u64* __restrict__ word_off,
                                               const u32* __restrict__ len,
                                               const uint4* __restrict__ cands, u64 at,
                                               u32* __restrict__ cand_sites,
                                               u32* __restrict__ seg_cnt, u32 seg_n,
                                               u64& my_sites, u64& my_win) {
  const uint4 e = cands[2 * at], mk = cands[2 * at + 1];
  const AhCtx c = ah_ctx(words, nmask, word_off, len, e.x);
  const u32 m[4] = {mk.x, mk.y, mk.z, mk.w};
  u32 found = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (m[q]) {
      const u32 f = ah_verify_one(c, c.gw + e.y, e.y, e.z + (u32)q, m[q], nullptr, 0, 0, false);
      if (!AH_QUAD_ONE_PAIR && seg_cnt && f)
        atomicAdd(&seg_cnt[ah_pat_pair(e.z + (u32)q) * seg_n + e.x], f);
      found += f;
      my_win += (u64)__popc(m[q]);
    }
  if (AH_QUAD_ONE_PAIR && seg_cnt)
    cand_sites[at] = found ? atomicAdd(&seg_cnt[ah_pat_pair(e.z) * seg_n + e.x], found) + 1u : 0u;
  else
    cand_sites[at] = found;
  my_sites += found;
}

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

#if AH_WAVE
// ---- wave mode (AH_WAVE = 1): every wave of the workgroup scans wave tiles
// of its own, with no workgroup barrier.  A wave tile is 63 x AH_U window
// words: lane i < 63 filters the AH_U words [i AH_U, (i + 1) AH_U) of it and
// lane 63 only holds the words after the tile.  The wave stages 64 x AH_U
// words (plus one when the tile starts at an odd word, to keep 16-byte copies
// aligned) in its own LDS slice; each lane converts its own words to one-hot
// planes once, and reads the planes of the words past its range (at most
// AH_U, since AH_U >= the longest primer - 1) from the next lane's registers
// with ds_bpermute, which moves data between the lanes of a wave without
// using the vector ALU.  Once every lane holds its planes, the LDS slice is
// free: the copy of the wave's next tile is issued then and lands while the
// steps run from registers.
#define AH_WTILE (63u * (u32)AH_U)
#define AH_WSTAGE_PAIRS (32 * AH_U + 1)
#define AH_WSTAGE_ROUNDS ((AH_WSTAGE_PAIRS + 63) / 64)

// s_waitcnt immediates (gfx9 family: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8; a field at its maximum does not wait)
#define AH_WAIT_VMCNT0 0x0F70
#define AH_WAIT_LGKMCNT0 0xC07F

// Copy wave tile words [t0 & ~1, (t0 & ~1) + 2 AH_WSTAGE_PAIRS) of genome c into
// this wave's LDS slice, 16 bytes per lane and instruction (the hardware puts
// lane i at base + 16 i); indices past the genome's allocation are clamped
// (only lanes whose windows lie past the genome read them).
__device__ __forceinline__ void ah_wstage(const AhCtx& c, u32 t0, uint4* my, u32 lane) {
  const u32 last_pair = ((c.S + 31u + 1u) >> 1) - 1u;
  const uint4* gp = (const uint4*)c.gw + (t0 >> 1);
  const u32 room = last_pair - (t0 >> 1);
#pragma unroll
  for (int k = 0; k < AH_WSTAGE_ROUNDS; ++k) {
    const u32 i = lane + 64u * (u32)k;
    if (i < AH_WSTAGE_PAIRS)
      __builtin_amdgcn_global_load_lds((ah_global_void*)(gp + min(i, room)),
                                       (ah_lds_void*)(my + 64u * (u32)k), 16, 0, 0);
  }
}

// The next stage of a wave: genome context and first window word of the
// wave's next tile (valid = 0 when the wave has none).
struct AhNext {
  AhCtx c;
  u32 t0;
  u32 valid;
};

// Generated: every group of patterns in turn converts this lane's words of
// the staged wave tile and filters them, appending candidates to slice s
// (cnt of them so far; returns the new count); the last group issues the copy
// of the next tile (`nx`) into `my` once its words are in registers.
__device__ u32 ah_wgroups(ah_lds_uint2* tw, u32 t0, const AhCtx& c, const AhCands& k, u32 lane,
                          uint4* my, const AhNext& nx, u32 cnt, u32 s);

// Wave tile of round r for wave `wv` of workgroup b: with a grid that is a
// multiple of the 8 XCDs (workgroups are placed on them round robin), the
// waves of one XCD take consecutive tiles, so the words a tile shares with the
// next (the last lane's) are read from the same L2.
__device__ __forceinline__ u64 ah_wtile(u64 r, u32 b, u32 wv) {
  const u64 V = (u64)gridDim.x * 4u;
  if ((gridDim.x & 7u) == 0u) {
    const u32 vx = (gridDim.x >> 3) * 4u;
    return r * V + (u64)(b & 7u) * vx + (u64)(b >> 3) * 4u + wv;
  }
  return r * V + (u64)b * 4u + wv;
}

extern "C" __global__ __launch_bounds__(AH_BLOCK) void ah_scan_kernel(
    const uint2* __restrict__ words, const u32* __restrict__ nmask,
    const u64* __restrict__ word_off, const u32* __restrict__ len,
    const u64* __restrict__ tile_prefix, u32 n_genomes, uint4* __restrict__ cand_out,
    u32 slice, u32* __restrict__ slice_count, u32* __restrict__ slice_total,
    u64* __restrict__ slice_win, u64* __restrict__ group_sites, u32* __restrict__ cand_sites,
    u64* __restrict__ slice_sites, u32* __restrict__ hist_a, u32* __restrict__ hist_b,
    u64 hist_words, u32* __restrict__ seg_cnt, u32 seg_n) {
  // Each wave owns candidate slice s = 4 b + wave (slice records each).  After
  // its last tile the wave also counts the sites of its own candidates exactly
  // (as a workgroup does in tile mode), while the other waves still
  // filter; the emit pass reads the four slices of a workgroup as one list.
  // The grid clears the sort's first two histogram tables (the emit pass
  // counts into the first, the first sort pass into the second); the group
  // sums were cleared before this launch.
  __shared__ uint4 tiles[AH_BLOCK / 64][AH_WSTAGE_PAIRS];
  for (u64 e = (u64)blockIdx.x * AH_BLOCK + threadIdx.x; e < hist_words;
       e += (u64)gridDim.x * AH_BLOCK) {
    hist_a[e] = 0u;
    hist_b[e] = 0u;
  }
  const u64 n_tiles = tile_prefix[n_genomes];
  const AhCands k{cand_out, slice, slice_win};
  const u32 wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const u32 lane = threadIdx.x & 63u;
  const u32 s = blockIdx.x * (AH_BLOCK / 64) + wv;
  uint4* my = tiles[wv];
  if (lane == 0) slice_win[s] = 0;  // windows of dropped candidates, added by ah_wcand
  __builtin_amdgcn_s_waitcnt(AH_WAIT_VMCNT0);  // the zero is in place before any atomic on it
  u32 cnt = 0;
  u32 lo = 0;
  u64 r = 0;
  u64 T = ah_wtile(r, blockIdx.x, wv);
  AhNext cur;
  cur.valid = T < n_tiles ? 1u : 0u;
  if (cur.valid) {
    const u32 g = ah_tile_genome(tile_prefix, n_genomes, T, lo);
    cur.c = ah_ctx(words, nmask, word_off, len, g);
    cur.t0 = (u32)(T - tile_prefix[g]) * AH_WTILE;
    ah_wstage(cur.c, cur.t0, my, lane);
  }
  while (cur.valid) {
    AhNext nx;
    const u64 Tn = ah_wtile(++r, blockIdx.x, wv);
    nx.valid = Tn < n_tiles ? 1u : 0u;
    if (nx.valid) {
      const u32 g = ah_tile_genome(tile_prefix, n_genomes, Tn, lo);
      nx.c = ah_ctx(words, nmask, word_off, len, g);
      nx.t0 = (u32)(Tn - tile_prefix[g]) * AH_WTILE;
    }
    __builtin_amdgcn_s_waitcnt(AH_WAIT_VMCNT0);  // this wave's copies have landed
    cnt = ah_wgroups((ah_lds_uint2*)my + (cur.t0 & 1u), cur.t0, cur.c, k, lane, my, nx, cnt, s);
    cur = nx;
  }
  // the exact count of this wave's candidates (records written by its own
  // lanes: the fence orders their stores before the loads)
  __threadfence_block();
  const u32 nk = min(cnt, slice);
  u64 my_sites = 0, my_win = 0;
  for (u32 i = lane; i < nk; i += 64u)
    ah_verify_cand(words, nmask, word_off, len, cand_out, (u64)s * slice + i, cand_sites, seg_cnt,
                   seg_n, my_sites, my_win);
  for (u32 o = 32; o > 0; o >>= 1) {
    my_sites += __shfl_xor(my_sites, o, 64);
    my_win += __shfl_xor(my_win, o, 64);
  }
  if (lane == 0) {  // every wave reports its slice, with or without tiles
    slice_count[s] = nk;
    slice_total[s] = cnt;
    slice_sites[s] = my_sites;
    if (my_sites) atomicAdd(&group_sites[(blockIdx.x / AH_SLICE_GROUP) * AH_GROUP_STRIDE], my_sites);
    atomicAdd(&slice_win[s], my_win);
  }
}
#else
extern "C" __global__ __launch_bounds__(AH_BLOCK) void ah_scan_kernel(
    const uint2* __restrict__ words, const u32* __restrict__ nmask,
    const u64* __restrict__ word_off, const u32* __restrict__ len,
    const u64* __restrict__ tile_prefix, u32 n_genomes, uint4* __restrict__ cand_out,
    u32 slice, u32* __restrict__ slice_count, u32* __restrict__ slice_total,
    u64* __restrict__ slice_win, u64* __restrict__ group_sites, u32* __restrict__ cand_sites,
    u64* __restrict__ slice_sites, u32* __restrict__ hist_a, u32* __restrict__ hist_b,
    u64 hist_words, u32* __restrict__ seg_cnt, u32 seg_n) {
  // The workgroup's candidates go to its slice.  With AH_TILE_COUNT, after
  // its last tile it counts their sites exactly, while other workgroups
  // still filter, and the grid clears the sort's first two histogram tables
  // (the emit pass counts into the first, the first sort pass into the
  // second); the group sums were cleared before this launch.  Without it
  // ah_verify_kernel does both after the filter: a program of many patterns
  // keeps every workgroup filtering to the end, so nothing would overlap the
  // count, which then runs at the filter's occupancy.
  __shared__ uint4 tile[AH_STAGE_PAIRS];
#if AH_TILE_COUNT
  __shared__ u64 s_sites, s_win;
  for (u64 e = (u64)blockIdx.x * AH_BLOCK + threadIdx.x; e < hist_words;
       e += (u64)gridDim.x * AH_BLOCK) {
    hist_a[e] = 0u;
    hist_b[e] = 0u;
  }
#endif
  const u64 n_tiles = tile_prefix[n_genomes];
  const AhCands k{cand_out, slice, nullptr};
  if (threadIdx.x == 0) {
    ah_n_cand = 0;
    ah_n_lost = 0;
#if AH_TILE_COUNT
    s_sites = 0;
    s_win = 0;
#endif
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
#if AH_TILE_COUNT
  // the exact count of the workgroup's candidates (records written by its
  // own threads: the fence and the barrier order their stores before the
  // loads)
  __threadfence_block();
  __syncthreads();
  const u32 nk = min(ah_n_cand, slice);
  u64 my_sites = 0, my_win = 0;
  for (u32 i = threadIdx.x; i < nk; i += AH_BLOCK)
    ah_verify_cand(words, nmask, word_off, len, cand_out, (u64)blockIdx.x * slice + i, cand_sites,
                   seg_cnt, seg_n, my_sites, my_win);
  if (my_sites) atomicAdd(&s_sites, my_sites);
  if (my_win) atomicAdd(&s_win, my_win);
  __syncthreads();
  if (threadIdx.x == 0) {  // every workgroup reports, with or without tiles
    slice_count[blockIdx.x] = nk;
    slice_total[blockIdx.x] = ah_n_cand;
    slice_win[blockIdx.x] = ah_n_lost + s_win;  // dropped candidates' windows and the kept ones'
    slice_sites[blockIdx.x] = s_sites;
    if (s_sites) atomicAdd(&group_sites[(blockIdx.x / AH_SLICE_GROUP) * AH_GROUP_STRIDE], s_sites);
  }
#else
  if (threadIdx.x == 0) {  // every workgroup reports, with or without tiles
    slice_count[blockIdx.x] = min(ah_n_cand, slice);
    slice_total[blockIdx.x] = ah_n_cand;
    slice_win[blockIdx.x] = ah_n_lost;  // ah_verify_kernel adds the kept ones
  }
#endif
}
#endif

extern "C" __global__ __launch_bounds__(AH_BLOCK) void ah_verify_kernel(
    const uint2* __restrict__ words, const u32* __restrict__ nmask,
    const u64* __restrict__ word_off, const u32* __restrict__ len,
    const uint4* __restrict__ cands, u32 slice, const u32* __restrict__ slice_count,
    u32* __restrict__ cand_sites, u64* __restrict__ slice_sites, u64* __restrict__ group_sites,
    u64* __restrict__ slice_win, u32* __restrict__ hist_a, u32* __restrict__ hist_b,
    u64 hist_words, u32* __restrict__ seg_cnt, u32 seg_n) {
  // Tile mode with AH_TILE_COUNT 0 (programs of many patterns): sites of each
  // candidate of a workgroup's slice after the filter, their sum, and the
  // candidates' windows (added to those of the candidates a full slice
  // dropped).  The grid also clears the sort's first two histogram tables
  // (the emit pass counts into the first, the first sort pass into the
  // second).  With seg_cnt set, the sites are also counted per segment
  // (pair, genome) at seg_cnt[pair * seg_n + genome]; when every record's
  // patterns share a pair, one device atomic per candidate reserves its
  // sites' places in the segment, and cand_sites keeps the first place + 1
  // (0: no sites) for the segmented emit instead of the count.
  for (u64 e = (u64)blockIdx.x * AH_BLOCK + threadIdx.x; e < hist_words;
       e += (u64)gridDim.x * AH_BLOCK) {
    hist_a[e] = 0u;
    hist_b[e] = 0u;
  }
  __shared__ u64 s_sites, s_win;
  if (threadIdx.x == 0) {
    s_sites = 0;
    s_win = 0;
  }
  __syncthreads();
  const AhSlices sl = ah_slices(slice_count, blockIdx.x);
  u64 my_sites = 0, my_win = 0;
  for (u32 i = threadIdx.x; i < sl.total; i += AH_BLOCK)
    ah_verify_cand(words, nmask, word_off, len, cands, ah_slice_at(sl, blockIdx.x, slice, i),
                   cand_sites, seg_cnt, seg_n, my_sites, my_win);
  if (my_sites) atomicAdd(&s_sites, my_sites);
  atomicAdd(&s_win, my_win);
  __syncthreads();
  if (threadIdx.x == 0) {
    slice_sites[blockIdx.x] = s_sites;
    if (s_sites) atomicAdd(&group_sites[(blockIdx.x / AH_SLICE_GROUP) * AH_GROUP_STRIDE], s_sites);
    slice_win[blockIdx.x * AH_SPW] += s_win;  // the statistics sum over every slice
  }
}

// Exclusive prefix of one value per thread over the workgroup; *total gets
// the sum.  Two barriers; `tmp` holds AH_BLOCK / 64 entries.
__device__ __forceinline__ u64 ah_block_scan(u64 v, u64* tmp, u64* total) {
  const u32 lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  u64 x = v;
#pragma unroll
  for (u32 o = 1; o < 64; o <<= 1) {
    const u64 y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63u) tmp[w] = x;
  __syncthreads();
  u64 before = 0, all = 0;
#pragma unroll
  for (u32 q = 0; q < AH_BLOCK / 64; ++q) {
    before += q < w ? tmp[q] : 0ull;
    all += tmp[q];
  }
  *total = all;
  __syncthreads();
  return before + x - v;
}

extern "C" __global__ __launch_bounds__(AH_BLOCK) void ah_emit_kernel(
    const uint2* __restrict__ words, const u32* __restrict__ nmask,
    const u64* __restrict__ word_off, const u32* __restrict__ len,
    const uint4* __restrict__ cands, u32 slice, const u32* __restrict__ slice_count,
    const u32* __restrict__ slice_total, const u64* __restrict__ slice_win,
    const u32* __restrict__ cand_sites, const u64* __restrict__ slice_sites,
    const u64* __restrict__ group_sites, AhHitRec* __restrict__ out, u64 cap,
    AhResult* __restrict__ res, u64* __restrict__ n_out, u64* __restrict__ cand_stat,
    u64* __restrict__ sort_keys, u32* __restrict__ sort_idx, u32* __restrict__ sort_hist,
    u32 sort_hs, u32 sort_dmask, u32 sort_gshift, u32 sort_qshift, u32 sort_grid,
    u32 sort_chunk_min) {
  __shared__ u64 tmp[AH_BLOCK / 64];
  const u32 G = gridDim.x;
  // this slice's first record: the sites of the earlier groups of slices,
  // then of the earlier slices of its own group
  const u32 ng = (G + AH_SLICE_GROUP - 1) / AH_SLICE_GROUP, my = blockIdx.x / AH_SLICE_GROUP;
  u64 mine_before = 0, mine_all = 0;
  for (u32 q = threadIdx.x; q < ng; q += AH_BLOCK) {
    const u64 v = group_sites[q * AH_GROUP_STRIDE];
    mine_all += v;
    mine_before += q < my ? v : 0ull;
  }
  for (u32 w = my * AH_SLICE_GROUP * AH_SPW + threadIdx.x; w < blockIdx.x * AH_SPW; w += AH_BLOCK)
    mine_before += slice_sites[w];  // sites per slice (AH_SPW slices per workgroup)
  u64 slot, found;
  ah_block_scan(mine_before, tmp, &slot);
  ah_block_scan(mine_all, tmp, &found);
  // The emit pass starts the radix sort that puts the records in canonical
  // order: for each record it writes, the key (pair << qshift | genome <<
  // gshift | pos << 2 | strand-primer) and index, and counts the sort's first
  // digit (key & dmask) per chunk of the written order into hist[digit * hs
  // + chunk] (cleared by the filter or the count).  The sort partitions the
  // min(found, cap) records into chunks of ceil(n / sort_grid) rounded up to
  // whole workgroups, at least sort_chunk_min.  sort_keys == null: no keys
  // (a scan run on its own).
  u64 chunk;
  {
    const u64 nrec = found < cap ? found : cap;
    u64 ch = (nrec + sort_grid - 1) / sort_grid;
    ch = (ch + AH_BLOCK - 1) / AH_BLOCK * AH_BLOCK;
    chunk = ch < sort_chunk_min ? sort_chunk_min : ch;
  }
  if (blockIdx.x == 0) {
    // candidate-list statistics: candidates, their windows, full slices, most
    // of one slice
    const u32 GS = G * AH_SPW;  // slices
    u64 c = 0, wn = 0, full = 0, mx = 0;
    for (u32 w = threadIdx.x; w < GS; w += AH_BLOCK) {
      const u64 t = slice_total[w];
      c += t;
      wn += slice_win[w];
      full += t > slice_count[w] ? 1ull : 0ull;
      mx = t > mx ? t : mx;
    }
    u64 sc, sw, sf;
    ah_block_scan(c, tmp, &sc);
    ah_block_scan(wn, tmp, &sw);
    ah_block_scan(full, tmp, &sf);
    // maximum: through the shuffle tree of each wave, then the waves
    for (u32 o = 32; o > 0; o >>= 1) {
      const u64 y = __shfl_xor(mx, o, 64);
      mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & 63u) == 0) tmp[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (u32 q = 0; q < AH_BLOCK / 64; ++q) mx = tmp[q] > mx ? tmp[q] : mx;
      const u64 cnt = found < cap ? found : cap;
      res->count = cnt;
      res->required = found;
      res->status = found > cap ? AH_RES_OVERFLOW : 0;
      if (n_out) *n_out = cnt;
      cand_stat[0] = sc;
      cand_stat[1] = sw;
      cand_stat[2] = sf;
      cand_stat[3] = mx;
      if (sf > 0) {  // dropped candidates: sites <= windows, list >= slices x most
        const u64 list = (u64)GS * mx;
        const u64 bound = sw > list ? sw : list;
        if (bound > res->required) res->required = bound;
        res->status = AH_RES_OVERFLOW;
      }
    }
    __syncthreads();  // thread 0 has read tmp before the loop below reuses it
  }
  // the slices' candidates with sites, in order, written from `slot` on
  const AhSlices sl = ah_slices(slice_count, blockIdx.x);
  const u32 n = sl.total;
  for (u32 r = 0; r < n; r += AH_BLOCK) {
    const u32 i = r + threadIdx.x;
    const u64 at = i < n ? ah_slice_at(sl, blockIdx.x, slice, i) : 0ull;
    const u32 f = i < n ? cand_sites[at] : 0u;
    u64 rt;
    const u64 off = ah_block_scan(f, tmp, &rt);
    if (f) {
      const uint4 e = cands[2 * at], mk = cands[2 * at + 1];
      const AhCtx c = ah_ctx(words, nmask, word_off, len, e.x);
      const u32 m[4] = {mk.x, mk.y, mk.z, mk.w};
      u64 q_slot = slot + off;  // the quad's patterns in order
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (m[q]) q_slot += ah_verify_one(c, c.gw + e.y, e.y, e.z + (u32)q, m[q], out, cap, q_slot, true);
      if (sort_keys) {  // keys of the records just written (read back by their writer)
        const u64 end = slot + off + f < cap ? slot + off + f : cap;
        for (u64 q = slot + off; q < end; ++q) {
          const AhHitRec h = out[q];
          const u64 key = ((u64)h.pair << sort_qshift) | ((u64)h.genome << sort_gshift) |
                          ((u64)h.pos << 2) | (u64)(h.strand_primer & 3u);
          sort_keys[q] = key;
          sort_idx[q] = (u32)q;
          atomicAdd(&sort_hist[(u64)(key & sort_dmask) * sort_hs + q / chunk], 1u);
        }
      }
    }
    slot += rt;
  }
}

// Segmented emit (the whole query in one call): the records go straight to
// their segment (pair, genome), whose first slot is the sum of the sites of
// the earlier segments (seg_cnt from the exact count, at most AH_SEG_MAX
// segments), at the place inside it that the count reserved
// (AH_QUAD_ONE_PAIR) or one taken here with a device atomic on
// seg_fill[segment] (cleared before the filter).  The order inside a segment
// is left to the segment sort that follows.  Workgroup 0 also writes the
// segments' first slots (seg_off, n_seg + 1 entries), the result and the
// candidate-list statistics, as the slice-order emit does.  Nothing is
// written when the sites overflow the capacity.
#define AH_SEG_MAX 4096
extern "C" __global__ __launch_bounds__(AH_BLOCK) void ah_emit_seg_kernel(
    const uint2* __restrict__ words, const u32* __restrict__ nmask,
    const u64* __restrict__ word_off, const u32* __restrict__ len,
    const uint4* __restrict__ cands, u32 slice, const u32* __restrict__ slice_count,
    const u32* __restrict__ slice_total, const u64* __restrict__ slice_win,
    const u32* __restrict__ cand_sites, const u32* __restrict__ seg_cnt, u32 n_seg, u32 seg_n,
    u64* __restrict__ seg_off, u32* __restrict__ seg_fill, AhHitRec* __restrict__ out, u64 cap,
    AhResult* __restrict__ res, u64* __restrict__ cand_stat) {
  __shared__ u64 s_off[AH_SEG_MAX + 1];
  __shared__ u64 tmp[AH_BLOCK / 64];
  // this thread's first candidate, in flight while the slots are summed
  const AhSlices sl = ah_slices(slice_count, blockIdx.x);
  u64 at0 = 0;
  u32 f0 = 0;
  uint4 e0 = make_uint4(0u, 0u, 0u, 0u), mk0 = e0;
  if (threadIdx.x < sl.total) {
    at0 = ah_slice_at(sl, blockIdx.x, slice, threadIdx.x);
    f0 = cand_sites[at0];
    e0 = cands[2 * at0];
    mk0 = cands[2 * at0 + 1];
  }
  // the segments' first slots: thread i sums a run of `per` segments
  const u32 per = (n_seg + AH_BLOCK - 1) / AH_BLOCK;
  const u32 s0 = threadIdx.x * per;
  u32 v[AH_SEG_MAX / AH_BLOCK];
  u64 mine = 0;
#pragma unroll
  for (u32 q = 0; q < AH_SEG_MAX / AH_BLOCK; ++q) {
    v[q] = q < per && s0 + q < n_seg ? seg_cnt[s0 + q] : 0u;
    mine += v[q];
  }
  u64 found;
  u64 run = ah_block_scan(mine, tmp, &found);
#pragma unroll
  for (u32 q = 0; q < AH_SEG_MAX / AH_BLOCK; ++q)
    if (q < per && s0 + q < n_seg) {
      s_off[s0 + q] = run;
      run += v[q];
    }
  if (threadIdx.x == 0) s_off[n_seg] = found;
  __syncthreads();
  if (blockIdx.x == 0) {
    for (u32 q = threadIdx.x; q <= n_seg; q += AH_BLOCK) seg_off[q] = s_off[q];
    // candidate-list statistics: candidates, their windows, full slices,
    // most of one slice
    const u32 GS = gridDim.x * AH_SPW;
    u64 c = 0, wn = 0, full = 0, mx = 0;
    for (u32 w = threadIdx.x; w < GS; w += AH_BLOCK) {
      const u64 t = slice_total[w];
      c += t;
      wn += slice_win[w];
      full += t > slice_count[w] ? 1ull : 0ull;
      mx = t > mx ? t : mx;
    }
    u64 sc, sw, sf;
    ah_block_scan(c, tmp, &sc);
    ah_block_scan(wn, tmp, &sw);
    ah_block_scan(full, tmp, &sf);
    for (u32 o = 32; o > 0; o >>= 1) {
      const u64 y = __shfl_xor(mx, o, 64);
      mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & 63u) == 0) tmp[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (u32 q = 0; q < AH_BLOCK / 64; ++q) mx = tmp[q] > mx ? tmp[q] : mx;
      res->count = found < cap ? found : cap;
      res->required = found;
      res->status = found > cap ? AH_RES_OVERFLOW : 0;
      cand_stat[0] = sc;
      cand_stat[1] = sw;
      cand_stat[2] = sf;
      cand_stat[3] = mx;
      if (sf > 0) {  // dropped candidates: sites <= windows, list >= slices x most
        const u64 list = (u64)GS * mx;
        const u64 bound = sw > list ? sw : list;
        if (bound > res->required) res->required = bound;
        res->status = AH_RES_OVERFLOW;
      }
    }
  }
  if (found > cap) return;
  for (u32 i = threadIdx.x; i < sl.total; i += AH_BLOCK) {
    u64 at = at0;
    u32 f = f0;
    uint4 e = e0, mk = mk0;
    if (i != threadIdx.x) {
      at = ah_slice_at(sl, blockIdx.x, slice, i);
      f = cand_sites[at];
      e = cands[2 * at];
      mk = cands[2 * at + 1];
    }
    if (!f) continue;
    const AhCtx c = ah_ctx(words, nmask, word_off, len, e.x);
    const u32 m[4] = {mk.x, mk.y, mk.z, mk.w};
#if AH_QUAD_ONE_PAIR
    {  // f - 1: the first place the exact count reserved in the segment
      u64 slot = s_off[ah_pat_pair(e.z) * seg_n + e.x] + (f - 1u);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (m[q]) slot += ah_verify_one(c, c.gw + e.y, e.y, e.z + (u32)q, m[q], out, cap, slot, true);
      continue;
    }
#endif
    // one reservation when the quad's patterns with windows share a pair
    u32 pq = 0xffffffffu;
    bool one = true;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (m[q]) {
        const u32 pp = ah_pat_pair(e.z + (u32)q);
        one &= pq == 0xffffffffu || pq == pp;
        pq = pp;
      }
    if (one) {
      const u32 sg = pq * seg_n + e.x;
      u64 slot = s_off[sg] + atomicAdd(&seg_fill[sg], f);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (m[q]) slot += ah_verify_one(c, c.gw + e.y, e.y, e.z + (u32)q, m[q], out, cap, slot, true);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (m[q]) {
          const u32 fq = ah_verify_one(c, c.gw + e.y, e.y, e.z + (u32)q, m[q], nullptr, 0, 0, false);
          if (!fq) continue;
          const u32 sg = ah_pat_pair(e.z + (u32)q) * seg_n + e.x;
          const u64 slot = s_off[sg] + atomicAdd(&seg_fill[sg], fq);
          ah_verify_one(c, c.gw + e.y, e.y, e.z + (u32)q, m[q], out, cap, slot, true);
        }
    }
  }
}

// ---- generated pattern program follows ----
