// Binding-site scan core (primer matching, Section 2.1 of AmpliconHunter).
//
// This file is compiled at run time (hipRTC) once per primer set, with a
// generated pattern program appended after it: one device function per
// pattern (fwd / rev primer on the + / - strand) in which every primer
// position is a single bitwise test of 32 packed genome positions against
// that position's IUPAC set, followed by the bit-sliced count of mismatches
// (exactly the threshold "at most k").  The build also compiles it offline
// with a sample program to check that it builds.
//
// Packed layout (see ah.h): bit b of word t of a genome holds the base at
// b*S + t, so the window starting at b*S + t reads word t + j at bit b for
// primer position j: 32 windows advance together with no shifts.  A lane
// block stages a tile of AH_TILE window words plus the halo in LDS (double
// buffered: the next tile's loads are in flight while this one is scanned);
// each lane reads the AH_HALO + 1 words of one window word at a time.
//
// Macros supplied by the generated program: AH_U (window words per lane),
// AH_HALO (longest primer - 1), AH_HAS_N (1 if the collection has non-ACGT
// bases, whose positions mismatch every primer position).

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
  AhHitRec* out;
  u64 cap;
  u64* counter;
  const uint2* gw;  // this genome's first packed word
  const u32* gn;    // this genome's first non-ACGT mask word (or null)
  u32 g;            // genome
  u32 n;            // bases
  u32 S;            // segment words
  int tail;         // n - 31*S: a window of length L at word t is valid in
                    // every segment iff t + L <= tail
};

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

// Append one record per set bit of hb; lv[m] has bit b set iff window b has
// more than m mismatches.
template <int NLEV>
__device__ __forceinline__ void ah_emit(const AhCtx& c, u32 t, u32 hb, const u32* lv, u32 pair,
                                        u32 sp) {
  u64 slot = atomicAdd(c.counter, (u64)__popc(hb));
  while (hb) {
    const u32 b = __ffs(hb) - 1u;
    hb &= hb - 1u;
    u32 mm = 0;
#pragma unroll
    for (int m = 0; m < NLEV; ++m) mm += (lv[m] >> b) & 1u;
    if (slot < c.cap) {
      AhHitRec r;
      r.genome = c.g;
      r.pos = b * c.S + t;
      r.pair = (unsigned short)pair;
      r.strand_primer = (unsigned char)sp;
      r.mm = (unsigned char)mm;
      r.tm = __int_as_float(0x7fc00000);
      c.out[slot] = r;
    }
    ++slot;
  }
}

// Genome context of tile T (g from a binary search over the tile prefix,
// starting from the previous tile's genome when it still applies).
__device__ __forceinline__ AhCtx ah_tile_ctx(const u64* __restrict__ tile_prefix, u32 n_genomes,
                                             const uint2* words, const u32* nmask,
                                             const u64* __restrict__ word_off,
                                             const u32* __restrict__ len, u64 T, u32& lo,
                                             AhHitRec* out, u64 cap, u64* counter, u32& t0) {
  u32 hi = n_genomes;
  if (tile_prefix[lo] > T) lo = 0;
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (tile_prefix[mid] <= T) lo = mid; else hi = mid;
  }
  AhCtx c;
  c.out = out;
  c.cap = cap;
  c.counter = counter;
  c.g = lo;
  c.n = len[lo];
  c.S = (c.n + 31u) >> 5;
  c.tail = (int)((long long)c.n - 31ll * (long long)c.S);
  const u64 wbase = word_off[lo];
  c.gw = words + wbase;
  c.gn = AH_HAS_N ? nmask + wbase : nullptr;
  t0 = (u32)(T - tile_prefix[lo]) * (u32)AH_TILE;
  return c;
}

typedef __attribute__((address_space(3))) const uint2 ah_lds_uint2;

// Generated: for every group of patterns in turn, every lane walks its window
// words of the staged tile (reading the group's longest primer's worth of
// words from LDS), prefilters each pattern of the group and runs the exact
// count where a lane has a candidate window.  One group's code runs over the
// whole tile before the next group's.
__device__ void ah_groups(ah_lds_uint2* tw, u32 t0, const AhCtx& c);

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
    const u64* __restrict__ tile_prefix, u32 n_genomes, AhHitRec* __restrict__ out, u64 cap,
    u64* __restrict__ counter) {
  __shared__ uint4 tiles[2][AH_STAGE_PAIRS];
  const u64 n_tiles = tile_prefix[n_genomes];
  u64 T = blockIdx.x;
  if (T >= n_tiles) return;
  u32 lo = 0, t0;
  AhCtx c = ah_tile_ctx(tile_prefix, n_genomes, words, nmask, word_off, len, T, lo, out, cap,
                        counter, t0);
  ah_stage(c, t0, tiles[0]);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int buf = 0;
  for (;;) {
    // the next tile streams into the other buffer while this one is scanned
    const u64 Tn = T + gridDim.x;
    u32 lon = lo, t0n = 0;
    AhCtx cn = c;
    if (Tn < n_tiles) {
      cn = ah_tile_ctx(tile_prefix, n_genomes, words, nmask, word_off, len, Tn, lon, out, cap,
                       counter, t0n);
      ah_stage(cn, t0n, tiles[buf ^ 1]);
    }
    ah_groups((ah_lds_uint2*)tiles[buf], t0, c);
    if (Tn >= n_tiles) break;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed
    __syncthreads();                // and everyone's; nobody still reads `buf`
    buf ^= 1;
    T = Tn;
    lo = lon;
    t0 = t0n;
    c = cn;
  }
}

// ---- generated pattern program follows ----
