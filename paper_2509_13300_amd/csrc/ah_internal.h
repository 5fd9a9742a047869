// Internal declarations shared by the host runtime (ah_host.cpp) and the
// offline-compiled kernels (ah_kernels.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ah.h"

namespace ah {

constexpr int kBlock = 256;        // threads per workgroup for every kernel
constexpr int kSortGrid = 256;     // workgroups (chunks) of the radix-sort passes
constexpr int kSortDigits = 512;   // most digit values of a radix-sort pass (9 bits)
constexpr int kPairGrid = 1024;    // workgroups (chunks) of the pairing kernels
constexpr int kScanGrid = 256;     // workgroups of the generic prefix scan
constexpr int kScanU = 19;         // default window words per lane (odd) in the scan kernel

// Per-primer table used by the Tm kernel (one per pair and primer).  Oligos
// are 2-bit codes (A=0 C=1 G=2 T=3), position j of the primer (5'->3') at
// bits 2j..2j+1; the masks below have bit 2j set for the positions they name.
struct PrimerTab {
  uint64_t fixed;     // codes of the non-degenerate positions (0 at degenerate ones)
  uint64_t lanes;     // positions 0..L-1
  uint64_t clampm;    // clamp positions L-c..L-1 (the primer's 3' end)
  uint64_t stackm;    // positions 0..L-2 (left base of each stack)
  uint64_t deg;       // oligos in the expansion
  double KL;          // FP64: salt entropy + R ln C (+ symmetry), cal/(K mol)
  double tshift;      // salt methods 1-4: degrees added to Tm
  double rA, rB;      // salt methods 6, 7: 1/T += rA + rB * (G+C count) / L
  uint32_t recip;     // 1: apply rA, rB
  uint32_t L, k, nd;
  uint32_t decoy;     // 1: the site is the primer against the reversed genome
  uint32_t dp;        // 1: exact best pairing (ratio iteration), not enumeration
  uint8_t dpos[32];   // degenerate positions, 5'->3'
  uint8_t nmem[32];   // number of members of each degenerate position
  uint8_t mem[32];    // members, 2 bits each, in A<C<G<T order
};

// Per-pair table used by the pairing kernels.
struct PairTab {
  uint32_t lf, lr;        // primer lengths
  uint32_t min_len, max_len;
  int32_t filter_tm;
  float min_tm;
};

// Sort-key field widths for hit records: key = pair | genome | pos | strand | primer.
struct KeyBits {
  int qb, gb, pb;
  int total() const { return qb + gb + pb + 2; }
};

// ---- launch wrappers (ah_kernels.hip); all asynchronous on `st` ----------
hipError_t launch_pack(const uint8_t* ascii, const uint64_t* ascii_off, uint32_t n,
                       const uint64_t* word_off, uint32_t* words, uint32_t* len,
                       uint32_t* nmask, uint64_t* non_acgt, int grid, hipStream_t st);
hipError_t launch_result_init(ah_result* res, hipStream_t st);
hipError_t launch_tile_counts(const uint32_t* len, uint32_t n, uint32_t tile_words, uint64_t* counts,
                              hipStream_t st);
// Exclusive prefix sum of in[0..n) into out[0..n]; out[n] = total.  n is
// n_host when n_dev is null, else *n_dev (device).  tmp: kScanGrid + 1 u64.
hipError_t launch_exclusive_scan(const uint64_t* in, uint64_t* out, uint64_t n_host,
                                 const uint64_t* n_dev, uint64_t* tmp, hipStream_t st);
// Radix sort of staged hit records into canonical order.
struct SortBuffers {
  uint64_t* keys[2];
  uint32_t* idx[2];
  uint32_t* hist[3];   // kSortDigits x hstride digit counts each (one row per digit)
  uint32_t hstride;    // columns: the most chunks a sort of `capacity` records uses
};
// Column stride of the sort histograms for a capacity: the most chunks of
// kSortChunkMin records (at most kSortGrid), a multiple of 4.  Every chunk
// reads all G x 2^D counts, so short lists take few, longer chunks (512
// measured faster than 256 and 1024 at ~16k hits).
constexpr uint32_t kSortChunkMin = 512;
inline uint32_t sort_hist_stride(uint64_t capacity) {
  const uint64_t g = (capacity + kSortChunkMin - 1) / kSortChunkMin;
  const uint64_t c = g < (uint64_t)kSortGrid ? g : (uint64_t)kSortGrid;
  return (uint32_t)((c + 3) / 4 * 4 > 0 ? (c + 3) / 4 * 4 : 4);
}
// Bits per digit of the radix sort of keys of `kb` (9 when that saves a pass).
inline int sort_digit_bits(const KeyBits& kb) {
  const int bits = kb.total();
  return (bits + 8) / 9 < (bits + 7) / 8 ? 9 : 8;
}
// The sort of the staged records.  The scan's emit pass has written their
// keys and indices (keys[0], idx[0]) and counted the first digit into
// hist[0]; its verify pass has cleared hist[0] and hist[1].
hipError_t launch_sort_hits(const ah_hit* staged, ah_hit* out, const uint64_t* n_dev,
                            KeyBits kb, const SortBuffers& sb, hipStream_t st);
// exact: some primer table has dp set (the kernels' exact-route variant).
hipError_t launch_tm(const ah_genomes& g, const PrimerTab* tabs, uint32_t n_pairs, ah_hit* hits,
                     const ah_result* nhits, uint64_t cap, int grid, bool exact, hipStream_t st);
struct PairBuffers {
  uint64_t* cf;         // [kPairGrid] kept fwd-primer minus sites per chunk
  uint64_t* cr;         // [kPairGrid] rev-primer
  uint64_t* cc;         // [kPairGrid] amplicons per chunk
  uint64_t* mtot;       // [2] lengths of the two minus-site lists
  uint64_t* mkey_f;     // [cap] (pair << 32 | genome) of compacted - sites
  uint32_t* mpos_f;     // [cap]
  uint32_t* midx_f;     // [cap]
  uint64_t* mkey_r;
  uint32_t* mpos_r;
  uint32_t* midx_r;
  uint32_t* cnt;        // [cap] amplicons started by each leader + site
  uint32_t* pre_f;      // [cap] fwd-list minus sites before each hit (search hint)
  uint32_t* pre_r;      // [cap] rev-list
  uint32_t* rng;        // [cap x 8] a leader's minus-site ranges (count -> write)
};
// marked: the per-chunk counts of kept minus sites are in place already (the
// sort of ah_query took them), so the pairing starts with the compaction.
// need_all: when the sites' result is not AH_OK (some sites are missing),
// write no amplicons and an overflow result with count and required 0.
hipError_t launch_pair(const ah_hit* hits, const ah_result* nhits, uint64_t hit_cap,
                       const PairTab* tabs, ah_amplicon* amp, uint64_t cap, ah_result* res,
                       const PairBuffers& pb, hipStream_t st, bool marked = false,
                       bool need_all = false);
// The sort of ah_query: as launch_sort_hits, with the melting temperature of
// the staged records computed in tm_blocks extra blocks of the first pass and
// the pairing's per-chunk counts of kept minus sites (k_pair_mark) taken by
// the last pass.  Needs at least two passes (sort_fusable).
bool sort_fusable(const KeyBits& kb);
hipError_t launch_sort_tm_mark(ah_hit* staged, ah_hit* out, const uint64_t* n_dev, KeyBits kb,
                               const SortBuffers& sb, const ah_genomes& g, const PrimerTab* tm_tabs,
                               uint32_t n_pairs, const PairTab* pair_tabs,
                               const PairBuffers& pb, int tm_blocks, bool exact, hipStream_t st);

// The tail of ah_query over at most kSegMax segments (pair, genome), after
// the scan's segmented emit has put each segment's sites at
// off[s] .. off[s + 1] of the staging area in no particular order: one
// launch, a workgroup of one wave per segment, sorts the segment into
// canonical order (in LDS up to kSegLds sites), computes the Tm of every
// site, counts the amplicons each leader + site starts, takes the amplicons
// of the earlier segments by a look-back over lb, and writes its own.
// key_bits: bits of pos << 2 | strand-primer; hcap: the capacity of out.
// When the sites overflowed, the amplicon result is an overflow with count
// and required 0 and no amplicon is written; the sites found still go to
// out in canonical order with their Tm when they fit in hcap (a full
// candidate list), as the separate calls write them.
constexpr uint32_t kSegMax = 4096;  // AH_SEG_MAX of the scan core
constexpr uint32_t kSegLds = 1024;
struct SegBuffers {
  uint32_t* cnt;   // [n_seg] sites per segment, then
  uint32_t* fill;  // [n_seg] places taken so far, then
  uint64_t* lb;    // [n_seg] look-back words (the three cleared together before the filter)
  uint64_t* off;   // [n_seg + 1] first site of each segment
  uint32_t n_seg, n_genomes;
};
hipError_t launch_seg_tail(ah_hit* staged, ah_hit* out, uint64_t hcap, const SegBuffers& sg,
                           const ah_result* hres, int key_bits, const ah_genomes& g,
                           const PrimerTab* tm_tabs, uint32_t n_pairs, const PairTab* pair_tabs,
                           const PairBuffers& pb, ah_amplicon* amp, uint64_t acap,
                           ah_result* ares, bool exact, hipStream_t st);

// Amplicon FASTA records, sequence hashes and amplitypes (see ah.h); rec_len
// [acap], rec_at [acap] and cc [kPairGrid] are workspace; `waves` writers.
hipError_t launch_fasta(const ah_genomes& g, const ah_hit* hits, const ah_amplicon* amp,
                        const ah_result* namp, uint64_t acap, uint32_t n_pairs, char* text,
                        uint64_t tcap, ah_result* res, uint64_t* seq_hash, uint64_t* atype,
                        uint32_t* atype_n, uint32_t* rec_len, uint64_t* rec_at, uint64_t* cc,
                        int waves, hipStream_t st);

// Streaming: word offsets of genomes off[0..n] relative to off[0], and the
// chunk-local -> collection id fix-up of a chunk's hits and amplicons.
hipError_t launch_rebase(const uint64_t* off, uint32_t n, uint64_t* out, hipStream_t st);
hipError_t launch_stream_fixup(ah_hit* hits, uint64_t nh, ah_amplicon* amp, uint64_t na,
                               uint32_t gbase, uint32_t hbase, int grid, hipStream_t st);

// Serving: a gathered view of genomes ids[0..n) of a packed collection
// (out_off [n + 1], out_len [n]), and view index -> collection id on a part's
// records (counts read from the device results).
hipError_t launch_gather_view(const uint32_t* ids, uint32_t n, const uint64_t* off, const uint32_t* len,
                              uint64_t* out_off, uint32_t* out_len, hipStream_t st);
hipError_t launch_remap(ah_hit* hits, const ah_result* hres, ah_amplicon* amp, const ah_result* ares,
                        const uint32_t* ids, int grid, hipStream_t st);

// Scan: zero n u64 (graph-capturable, no memset node).
hipError_t launch_zero_u64(uint64_t* p, uint32_t n, hipStream_t st);
// Tile counts of n <= kSmallPrefix genomes, their exclusive prefix
// (prefix[n] = total), the reset of `res` and the clearing of
// zero[0 .. n_zero) and zero64[0 .. n_zero64) (each when set), in one launch.
constexpr uint32_t kSmallPrefix = 4096;
hipError_t launch_tile_prefix_small(const uint32_t* len, uint32_t n, uint32_t tile_words,
                                    uint64_t* prefix, ah_result* res, hipStream_t st,
                                    uint32_t* zero = nullptr, uint32_t n_zero = 0,
                                    uint64_t* zero64 = nullptr, uint32_t n_zero64 = 0);

// Recommended scan workspace for n genomes holding at most `window_words`
// window words in total (pairs may be null: the minimum).
size_t scan_workspace_for(uint32_t n, uint64_t window_words, const ah_primer_pair* pairs,
                          uint32_t n_pairs, uint64_t capacity);

// Device address of the current device's scratch array
// (AH_SCAN_SCRATCH_BYTES bytes, the workspace of ah_scan_primers_noalloc),
// looked up on the first call on each device.
hipError_t scan_scratch(void** ptr);

// Chance that a window of independent uniform bases is a site of `primer` on
// one strand (clamp positions match, at most k others mismatch): the serving
// form sizes buffers from it, and ah_query picks its tail.
double site_probability(const std::string& primer, uint32_t k, uint32_t clamp);

// Validation of a Tm request exactly as ah_tm does it, with no device work.
ah_status check_tm(const ah_primer_pair* pairs, uint32_t n_pairs, const ah_tm_params* p);

// Error reporting shared by the host sources: records the message returned by
// ah_last_error() on this thread and returns s.
ah_status set_error(ah_status s, const char* fmt, ...);
void clear_error();
int cu_count_current();

}  // namespace ah
