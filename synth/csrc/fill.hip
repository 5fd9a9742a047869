// GPU realisation of a synthetic-collection plan (input generation only; no
// scan, melting-temperature or pairing arithmetic).  Computes the same bytes
// as synth/fill.py from the same counter-based SplitMix64 draws:
//   draw(key, i) = MIX(key + (i + 1) * GAMMA)
// with MIX the SplitMix64 finaliser (Steele, Lea & Flood, 2014).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned long long u64;

constexpr u64 GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ u64 mix64(u64 z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ u64 draw(u64 key, u64 i) { return mix64(key + (i + 1) * GAMMA); }

// Background: byte i of genome g from the genome's stream key and thresholds.
__global__ void k_background(uint8_t* __restrict__ out, const u64* __restrict__ off, uint32_t n,
                             const u64* __restrict__ keys, const uint32_t* __restrict__ thr) {
  const u64 total = off[n];
  const u64 stride = (u64)gridDim.x * blockDim.x * 16;
  for (u64 p0 = ((u64)blockIdx.x * blockDim.x + threadIdx.x) * 16; p0 < total; p0 += stride) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (off[mid] <= p0) lo = mid; else hi = mid;
    }
    uint32_t g = lo;
    for (int q = 0; q < 16; ++q) {
      const u64 p = p0 + q;
      if (p >= total) break;
      while (p >= off[g + 1]) ++g;
      const u64 i = p - off[g];
      const uint32_t u = (uint32_t)(draw(keys[g], i) >> 32);
      const uint32_t c = (u >= thr[3 * g]) + (u >= thr[3 * g + 1]) + (u >= thr[3 * g + 2]);
      out[p] = (uint8_t)("ACGT"[c]);
    }
  }
}

__device__ __forceinline__ uint8_t comp(uint8_t b) {
  return b == 'A' ? 'T' : b == 'C' ? 'G' : b == 'G' ? 'C' : 'A';
}

__device__ __forceinline__ uint32_t code_of(uint8_t b) {
  return b == 'A' ? 0u : b == 'C' ? 1u : b == 'G' ? 2u : 3u;
}

// Planted copies: one thread per (copy, offset); copy c covers flat indices
// [coff[c], coff[c+1]).
__global__ void k_plant(uint8_t* __restrict__ out, const u64* __restrict__ coff, uint32_t m,
                        const u64* __restrict__ dest, const uint8_t* __restrict__ strand,
                        const u64* __restrict__ tstart, const uint32_t* __restrict__ tlen,
                        const uint8_t* __restrict__ tbytes, const u64* __restrict__ mkeys,
                        uint32_t t_mut) {
  const u64 total = coff[m];
  for (u64 f = (u64)blockIdx.x * blockDim.x + threadIdx.x; f < total;
       f += (u64)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = m;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (coff[mid] <= f) lo = mid; else hi = mid;
    }
    const uint32_t c = lo;
    const u64 o = f - coff[c];
    const uint32_t L = tlen[c];
    uint8_t b = strand[c] ? comp(tbytes[tstart[c] + (L - 1 - o)]) : tbytes[tstart[c] + o];
    const u64 r = draw(mkeys[c], o);
    if ((uint32_t)(r >> 32) < t_mut) {
      const uint32_t orig = code_of(b);
      const uint32_t choice = (uint32_t)(((r & 0xFFFFFFFFull) * 3ull) >> 32);
      const uint32_t repl = choice + (choice >= orig ? 1u : 0u);
      b = (uint8_t)("ACGT"[repl]);
    }
    out[dest[c] + o] = b;
  }
}

__global__ void k_nruns(uint8_t* __restrict__ out, const u64* __restrict__ pos,
                        const uint32_t* __restrict__ len, uint32_t r) {
  for (u64 i = blockIdx.x; i < r; i += gridDim.x)
    for (uint32_t j = threadIdx.x; j < len[i]; j += blockDim.x) out[pos[i] + j] = 'N';
}

}  // namespace

extern "C" {

int synth_fill_background(uint8_t* out, const uint64_t* off, uint32_t n, const uint64_t* keys,
                          const uint32_t* thr, void* stream) {
  k_background<<<4096, 256, 0, (hipStream_t)stream>>>(out, (const u64*)off, n, (const u64*)keys, thr);
  return (int)hipGetLastError();
}

int synth_fill_plants(uint8_t* out, const uint64_t* coff, uint32_t m, const uint64_t* dest,
                      const uint8_t* strand, const uint64_t* tstart, const uint32_t* tlen,
                      const uint8_t* tbytes, const uint64_t* mkeys, uint32_t t_mut, void* stream) {
  if (m == 0) return 0;
  k_plant<<<4096, 256, 0, (hipStream_t)stream>>>(out, (const u64*)coff, m, (const u64*)dest, strand,
                                                 (const u64*)tstart, tlen, tbytes, (const u64*)mkeys,
                                                 t_mut);
  return (int)hipGetLastError();
}

int synth_fill_nruns(uint8_t* out, const uint64_t* pos, const uint32_t* len, uint32_t r, void* stream) {
  if (r == 0) return 0;
  k_nruns<<<1024, 256, 0, (hipStream_t)stream>>>(out, (const u64*)pos, len, r);
  return (int)hipGetLastError();
}

}  // extern "C"
