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
// owns AH_U consecutive window words and keeps AH_U + AH_HALO words in
// registers.
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
  u32 g;  // genome
  u32 n;  // bases
  u32 S;  // segment words
};

// Window starts b*S + t (b = 0..31) that lie inside the genome for a primer
// of length L, as a bit mask over b.
__device__ __forceinline__ u32 ah_valid(const AhCtx& c, u32 t, u32 L) {
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

// Generated: evaluates every pattern of the primer set on one window word.
__device__ void ah_patterns(const u32* h, const u32* l, const u32* nm, const AhCtx& c, u32 t);

extern "C" __global__ __launch_bounds__(AH_BLOCK) void ah_scan_kernel(
    const uint2* __restrict__ words, const u32* __restrict__ nmask,
    const u64* __restrict__ word_off, const u32* __restrict__ len,
    const u64* __restrict__ tile_prefix, u32 n_genomes, AhHitRec* __restrict__ out, u64 cap,
    u64* __restrict__ counter) {
  const u64 n_tiles = tile_prefix[n_genomes];
  for (u64 T = blockIdx.x; T < n_tiles; T += gridDim.x) {
    u32 lo = 0, hi = n_genomes;
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
    const u64 wbase = word_off[lo];
    const u32 nw = c.S + 31u;
    const u32 t0 = (u32)(T - tile_prefix[lo]) * (u32)AH_TILE + threadIdx.x * (u32)AH_U;
    if (t0 >= c.S) continue;
    u32 h[AH_U + AH_HALO], l[AH_U + AH_HALO], nm[AH_U + AH_HALO];
#pragma unroll
    for (int i = 0; i < AH_U + AH_HALO; ++i) {
      const u32 wi = t0 + (u32)i;
      uint2 v = make_uint2(0u, 0u);
      if (wi < nw) v = words[wbase + wi];
      h[i] = v.x;
      l[i] = v.y;
      nm[i] = (AH_HAS_N && wi < nw) ? nmask[wbase + wi] : 0u;
    }
#pragma unroll
    for (int u = 0; u < AH_U; ++u)
      if (t0 + (u32)u < c.S) ah_patterns(h + u, l + u, nm + u, c, t0 + (u32)u);
  }
}

// ---- generated pattern program follows ----
