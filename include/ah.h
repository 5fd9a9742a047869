/*
 * libah -- genome-wide scan for degenerate-primer binding sites, nearest-
 * neighbour melting temperature and amplicon calling on AMD MI355X (gfx950).
 *
 * The operations follow AmpliconHunter (Howard-Stone & Mandoiu,
 * arXiv 2509.13300), Section 2.1: primer matching with up to k mismatches and
 * an optional 3'-clamp, melting-temperature scoring of every binding site as
 * the maximum over the compatible oligonucleotides of the degenerate primer,
 * and amplicon calling by pairing opposite-strand sites within a length
 * window, labelled FR / RF / FF / RR.
 *
 * Conventions for every call:
 *  - Device pointers (prefix d_) are owned by the caller and must stay valid
 *    until the work enqueued on `stream` has finished.  Host pointers are
 *    borrowed for the duration of the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously; the calls never synchronise the stream,
 *    so a whole scan -> Tm -> pairing sequence can be captured in a hipGraph.
 *  - Arguments and primers are validated synchronously; on any error nothing
 *    is enqueued and the status is returned.  Errors discovered on the device
 *    (output capacity exceeded) are written to a device-resident ah_result.
 *  - The first call with a new primer set specialises and compiles the scan
 *    kernel for it and uploads small per-set tables (cached per device and
 *    per primer set until ah_release_caches); later calls with the same set
 *    allocate nothing.
 *  - No C++ exception crosses this interface.
 */
#ifndef AH_H
#define AH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ah_status {
  AH_OK = 0,
  AH_ERR_INVALID_ARG = -1,    /* null pointer, bad size, bad parameter value */
  AH_ERR_INVALID_PRIMER = -2, /* a character outside the IUPAC nucleotide codes */
  AH_ERR_LIMIT = -3,          /* primer length, k, clamp or key-width limit exceeded */
  AH_ERR_OVERFLOW = -4,       /* (device) more records than the output capacity */
  AH_ERR_WORKSPACE = -5,      /* workspace smaller than the *_workspace_bytes query */
  AH_ERR_HIP = -6,            /* a HIP runtime call failed */
  AH_ERR_JIT = -7,            /* specialising the scan kernel failed */
  AH_ERR_AGAIN = -8           /* nothing to return yet (server wait timed out) */
} ah_status;

enum {
  AH_MIN_PRIMER_LEN = 5,   /* the paper's server limit: primers of at least 5 bp */
  AH_MAX_PRIMER_LEN = 32,  /* one packed word of window positions */
  AH_MAX_K = 15,
  AH_HALO_WORDS = 31       /* packed words appended to each genome (AH_MAX_PRIMER_LEN - 1) */
};

/* Orientation codes of an amplicon (Section 2.1, "Amplicon analysis", item 1). */
enum { AH_FR = 0, AH_RF = 1, AH_FF = 2, AH_RR = 3 };

/* ---------------------------------------------------------------------------
 * Packed genome collection (Section 1 / 2.1: genomes are the FASTA input).
 *
 * Layout of genome g with n bases: S = ceil(n / 32) segment words plus
 * AH_HALO_WORDS halo words, rounded up to an even number of words so that
 * every genome starts 16-byte aligned, starting at word word_off[g].  Word t is a pair of
 * uint32 (h, l) stored consecutively in `words`; bit b of word t holds the
 * base at position b*S + t as the 2-bit code A=00, C=01, G=10, T=11 (h the
 * high bit, l the low bit; the complement of a base is the bitwise NOT of
 * both planes).  Positions >= n read as A and are never reported.  `nmask`,
 * when not NULL, holds one uint32 per word with bit b set iff that base was
 * not A/C/G/T (such bases match no primer position).
 *
 * ah_scan_primers and ah_tm read word_off[g] and len[g] for g < n only, so a
 * view of any subset of a packed collection (words and nmask shared,
 * word_off and len gathered for the chosen genomes, in any order) is valid
 * for them; hits then name genomes by their index in the view.
 * ------------------------------------------------------------------------- */
typedef struct ah_genomes {
  const uint32_t* words;    /* device, 2 uint32 per word                        */
  const uint32_t* nmask;    /* device, 1 uint32 per word, or NULL              */
  const uint64_t* word_off; /* device, [n + 1]; word_off[g] = first word of g   */
  const uint32_t* len;      /* device, [n] bases per genome                    */
  uint32_t n;               /* host: number of genomes                         */
  uint32_t max_len;         /* host: an upper bound on every len[g] (>= 1)     */
} ah_genomes;

/* Host-side layout query.  Fills h_word_off[0..n] (may be NULL) for genomes of
 * lengths h_len[0..n-1] and returns the total number of words.  The words
 * buffer needs 8 bytes per word, the nmask buffer 4 bytes per word.  A genome
 * has at most 2^32 - 1 bases (positions and lengths are 32-bit): for a longer
 * one it returns UINT64_MAX, writes nothing and sets ah_last_error. */
uint64_t ah_pack_layout(const uint64_t* h_len, uint32_t n, uint64_t* h_word_off);

/* FASTA text in host memory -> the records' sequence bytes (Section 2.1: the
 * input is genomes in FASTA).  A record starts at a line whose first byte is
 * '>'; its name is the rest of that line (trailing blanks and '\r'
 * removed).  Its sequence is every byte of the lines up to the next record,
 * line breaks, '\r', blanks and tabs removed: case and IUPAC codes are kept
 * (ah_pack_genomes folds case and masks the non-ACGT bytes).  Each record is
 * its own linear sequence; a genome of several contigs is several records.
 * ah_fasta_count gives the number of records and of sequence bytes;
 * ah_fasta_read writes the bytes to seq (host, seq_capacity bytes), record r
 * at [seq_off[r], seq_off[r + 1]) (seq_off: n_records + 1 entries), and its
 * name's byte span in the text to name_span[2r], name_span[2r + 1].  The text
 * is read by up to 16 threads.  Errors: AH_ERR_INVALID_ARG (null argument,
 * sequence bytes before the first '>' line), AH_ERR_LIMIT (more records or
 * bytes than given room for). */
ah_status ah_fasta_count(const char* text, uint64_t bytes, uint64_t* n_records,
                         uint64_t* seq_bytes);
ah_status ah_fasta_read(const char* text, uint64_t bytes, uint8_t* seq, uint64_t seq_capacity,
                        uint64_t* seq_off, uint64_t* name_span, uint64_t max_records);

/* Pack ASCII genomes into the layout above.  Genome g is
 * d_ascii[d_ascii_off[g] .. d_ascii_off[g+1]); upper or lower case A/C/G/T are
 * bases, every other byte is a non-ACGT base.  d_word_off must hold the
 * offsets from ah_pack_layout (which refuses genomes longer than 2^32 - 1
 * bases).  Writes d_words, d_len, and, when not NULL, d_nmask and
 * d_non_acgt[g] (number of non-ACGT bytes of genome g).  If any genome has
 * non-ACGT bytes the scan needs d_nmask.
 * Errors: AH_ERR_INVALID_ARG (null required pointer), AH_ERR_HIP. */
ah_status ah_pack_genomes(const uint8_t* d_ascii, const uint64_t* d_ascii_off, uint32_t n,
                          const uint64_t* d_word_off, uint32_t* d_words, uint32_t* d_len,
                          uint32_t* d_nmask, uint64_t* d_non_acgt, void* stream);

/* ---------------------------------------------------------------------------
 * Primer pairs and binding sites (Section 2.1, "Primer matching").
 * ------------------------------------------------------------------------- */
typedef struct ah_primer_pair {
  const char* fwd;    /* IUPAC codes 5'->3' (case-insensitive), 5..32 nt    */
  const char* rev;    /* IUPAC codes 5'->3'                                  */
  uint32_t k;         /* maximum mismatches per site, <= AH_MAX_K            */
  uint32_t clamp;     /* 3'-terminal primer bases that must match (0 = none) */
  uint32_t flags;     /* 0 or AH_PAIR_DECOY                                   */
} ah_primer_pair;

/* Decoy pair (Section 2.1, "Amplicon analysis": off-target amplification
 * estimated from decoys made by reversing the genome sequences).  A pair with
 * this flag stands for the same primers run on every genome reversed (not
 * reverse-complemented), scanned in the same pass as the other pairs, over
 * the genomes as given.  Scanning reverse(G) for a primer P is scanning G
 * for the position-wise complement of P as an ordinary primer (its 3' clamp
 * stays at the window end the clamp rule expects), so a decoy pair's sites
 * and amplicons are reported in G's coordinates: a decoy-frame site at pos
 * p on strand s of a genome of n bases is reported at pos n - p - L on
 * strand 1 - s; a decoy-frame amplicon [a, b) is reported as [n - b, n - a)
 * with FR and RF exchanged (FF and RR stay).  Its melting temperatures are
 * those of the given primers against the reversed genome.  Counts, lengths,
 * mismatches and Tm are the decoy run's. */
#define AH_PAIR_DECOY 1u

/* One binding site.  pos is the 0-based leftmost top-strand coordinate of the
 * window for both strands.  strand_primer: bit 1 = strand (0 = the primer
 * sequence itself is on the top strand, 1 = its reverse complement is),
 * bit 0 = primer (0 = fwd, 1 = rev).  mm = mismatching positions.  tm is
 * filled by ah_tm (NaN before). */
typedef struct ah_hit {
  uint32_t genome;
  uint32_t pos;
  uint16_t pair;
  uint8_t strand_primer;
  uint8_t mm;
  float tm;
} ah_hit;

/* Device-resident result of an asynchronous call.  required = records found;
 * count = records written = min(required, capacity); status = AH_OK or
 * AH_ERR_OVERFLOW (then the buffer contents are unspecified and the call can
 * be repeated with capacity >= required, giving the same records). */
typedef struct ah_result {
  uint64_t count;
  uint64_t required;
  int32_t status;
  uint32_t reserved;
} ah_result;

/* Find every window of every genome where a primer of a pair, or its reverse
 * complement, has at most k mismatching positions (a genome base outside the
 * position's IUPAC set is a mismatch; substitutions only) and no mismatch in
 * the clamp (the primer's 3'-most `clamp` bases).  Output: d_hits sorted by
 * (pair, genome, pos, strand, primer) -- a canonical order independent of
 * scheduling -- and *d_res.  Needs a device workspace (caller-owned,
 * 256-byte aligned); ah_scan_workspace_bytes gives the recommended size.
 * Part of it holds the list of candidate windows that pass the scan's filter
 * (at least max(capacity, 2^16) records; all extra workspace lengthens it).
 * The list is split evenly over the filter's workgroups; if one finds more
 * candidates than its share holds, the sites are incomplete: the result is
 * AH_ERR_OVERFLOW and `required` is an upper bound on the sites, large
 * enough that a call with capacity >= required succeeds.
 * Errors: AH_ERR_INVALID_ARG, AH_ERR_INVALID_PRIMER, AH_ERR_LIMIT (primer
 * length outside 5..32, k > AH_MAX_K, clamp > primer length, sort key wider
 * than 64 bits), AH_ERR_WORKSPACE, AH_ERR_JIT, AH_ERR_HIP. */
ah_status ah_scan_primers(const ah_genomes* genomes, const ah_primer_pair* pairs,
                          uint32_t n_pairs, ah_hit* d_hits, uint64_t capacity,
                          ah_result* d_res, void* d_work, size_t work_bytes, void* stream);
/* ah_scan_primers for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid allocation):
 * the same sites in the same order, with the workspace taken from a scratch
 * array of AH_SCAN_SCRATCH_BYTES bytes that the library holds on each device
 * (part of its code object, so it is reserved on a device with the library's
 * kernels and kept until the process ends).  The call allocates nothing: the
 * primer set's kernels must already be compiled and loaded on the current
 * device (by ah_scan_prepare, or an earlier ah_scan_primers call with the same
 * set and shape), else AH_ERR_INVALID_ARG; profiling events (ah_profile_*) are
 * not recorded for it.  Its candidate list is the part of the array that the
 * fixed parts for n genomes and `capacity` sites leave; AH_ERR_WORKSPACE if
 * those parts do not fit with at least max(capacity, 2^16) candidates.
 * Every call on a device uses that device's one array, and nothing in it has
 * to start at any value: calls that overlap in time on one device (different
 * streams, or host threads) race and give unspecified results; enqueue them
 * on one stream or synchronise between them.  Errors: those of
 * ah_scan_primers, AH_ERR_WORKSPACE as above. */
enum { AH_SCAN_SCRATCH_BYTES = 64 << 20 };
ah_status ah_scan_primers_noalloc(const ah_genomes* genomes, const ah_primer_pair* pairs,
                                  uint32_t n_pairs, ah_hit* d_hits, uint64_t capacity,
                                  ah_result* d_res, void* stream);

/* Recommended workspace: the fixed parts for `capacity` sites plus a
 * candidate list of twice the records that the filters of `pairs` are
 * expected to pass on random bases, over at most n x ceil(max_len / 32)
 * window words, plus 2^16 records.  pairs may be NULL (the minimum). */
size_t ah_scan_workspace_bytes(const ah_genomes* genomes, const ah_primer_pair* pairs,
                               uint32_t n_pairs, uint64_t capacity);

/* ---------------------------------------------------------------------------
 * Melting temperature (Section 2.1, "Melting temperature filtering"; the
 * paper exposes the ion concentrations and the salt-correction method).
 * Nearest-neighbour model: SantaLucia (1998) unified stacks, initiation per
 * duplex end, C = max(dnac1,dnac2) - min(dnac1,dnac2)/2 (dnac1 if selfcomp).
 * A stack with a mismatched pair contributes nothing and initiation is taken
 * at the outermost paired positions.  Salt correction (saltcorr), with the
 * sodium equivalent [Na+] = Na + K + Tris/2 + 120 sqrt(Mg - dNTPs) mM for
 * methods 1-6:
 *   0 none;
 *   1 Schildkraut & Lifson (1965): Tm + 16.6 log10[Na+];
 *   2 Wetmur (1991): Tm + 16.6 log10([Na+] / (1 + 0.7 [Na+]));
 *   3 SantaLucia et al. (1996): Tm + 12.5 log10[Na+];
 *   4 SantaLucia (1998): Tm + 11.7 log10[Na+];
 *   5 SantaLucia (1998): Delta-S + 0.368 (N-1) ln[Na+]  (the default);
 *   6 Owczarzy et al. (2004): 1/T + (4.29 fGC - 3.95) 1e-5 ln[Na+]
 *     + 9.40e-6 ln^2[Na+];
 *   7 Owczarzy et al. (2008), magnesium, on the monovalent ions
 *     Na + K + Tris/2 and the Mg left free by dNTPs (1:1, Ka 3e4 per M).
 * fGC is the oligo's G+C fraction, so under 6 and 7 the maximum runs over
 * oligos that pair the site alike too (the best member at each unpaired
 * degenerate position).  Concentrations in M inside the logarithms.  Sums
 * are FP32 with compensation; the salt and logarithm terms are FP64.
 * ------------------------------------------------------------------------- */
typedef struct ah_tm_params {
  double dnac1_nM, dnac2_nM, Na_mM, K_mM, Tris_mM, Mg_mM, dNTPs_mM;
  int32_t saltcorr; /* 0-7, see above; AH_ERR_INVALID_ARG otherwise or when the
                       method's ion concentration is not positive */
  int32_t selfcomp; /* 1: symmetry correction -1.4 cal/(K mol) and C = dnac1 */
} ah_tm_params;

/* For each of the min(count, capacity) hits in d_hits (as written by
 * ah_scan_primers with the same genomes and pairs), set tm to the maximum
 * melting temperature over the oligos of the site's primer that have at most
 * k mismatches against the site and none in the clamp.  `capacity` is the
 * size of d_hits.  Oligos that pair a site at the same positions have the
 * same nearest-neighbour sums, so a site costs one evaluation per set of
 * paired positions: at most sum_{e <= min(k, nd)} C(nd, e) for a primer with
 * nd degenerate positions outside the clamp, whatever its degeneracy.  Up to
 * AH_TM_MAX_PAIRINGS of them are enumerated.  Above that, under salt methods
 * 0-5 (where Tm rises with Delta-H / (Delta-S + R ln C + salt entropy)), the
 * best set is found exactly by Dinkelbach's iteration for a maximum ratio,
 * each step a pass over the positions with the mismatches spent as state: a
 * few passes of L x (k + 1) x 4 states per site.  It needs R ln C plus the
 * salt entropy below -8.2 cal/(K mol), so that no set of pairs can make the
 * denominator non-negative.  Methods 6 and 7 also depend on the oligo's G+C
 * count and stay at the enumeration bound.  A request outside these limits
 * is refused with AH_ERR_LIMIT before any device work (the paper's web
 * server caps degeneracy at 10,000, Section 2.2; its command-line tool has
 * no cap).  Errors: AH_ERR_INVALID_ARG, AH_ERR_INVALID_PRIMER, AH_ERR_LIMIT,
 * AH_ERR_HIP. */
enum { AH_TM_MAX_PAIRINGS = 65536 };
ah_status ah_tm(const ah_genomes* genomes, const ah_primer_pair* pairs, uint32_t n_pairs,
                const ah_tm_params* params, ah_hit* d_hits, const ah_result* d_nhits,
                uint64_t capacity, void* stream);

/* Melting temperature of one duplex, on the host in double precision (Section
 * 2.1, "Melting temperature filtering": the nearest-neighbour Tm of an oligo
 * against the template at a binding site).  oligo: A/C/G/T (case-insensitive),
 * 5'->3', 2..AH_TM_DUPLEX_MAX_LEN bases.  opposite: the template bases written
 * opposite each oligo base (same length, template read 3'->5'); position j
 * pairs iff opposite[j] is the complement of oligo[j] (any other byte, N
 * included, pairs with nothing).  Same model, conditions and salt methods as
 * ah_tm (fGC of methods 6 and 7: the oligo's G+C fraction), all in double
 * precision; a duplex in which no pair forms has zero enthalpy: -273.15.
 * Writes *tm_c in degrees Celsius.  Borrowed host strings; no device work.
 * Errors: AH_ERR_INVALID_ARG (null argument, lengths differ, bad salt method
 * or concentrations), AH_ERR_INVALID_PRIMER (oligo byte not A/C/G/T),
 * AH_ERR_LIMIT (length outside 2..AH_TM_DUPLEX_MAX_LEN). */
enum { AH_TM_DUPLEX_MAX_LEN = 4096 };
ah_status ah_tm_duplex(const char* oligo, const char* opposite, const ah_tm_params* params,
                       double* tm_c);

/* ---------------------------------------------------------------------------
 * Amplicon calling (Section 2.1, "Amplicon calling" and "Amplicon analysis").
 * ------------------------------------------------------------------------- */
typedef struct ah_window {
  uint32_t min_len;  /* inclusive bounds on end - start                   */
  uint32_t max_len;
  int32_t filter_tm; /* 1: drop sites with tm < min_tm before pairing     */
  float min_tm;
} ah_window;

/* [start, end): start = pos of the + site, end = pos of the - site plus the
 * length of that site's primer.  plus_hit / minus_hit index d_hits. */
typedef struct ah_amplicon {
  uint32_t genome;
  uint32_t start;
  uint32_t end;
  uint32_t plus_hit;
  uint32_t minus_hit;
  uint16_t pair;
  uint8_t orient; /* AH_FR, AH_RF, AH_FF, AH_RR */
  uint8_t reserved;
} ah_amplicon;

/* Pair every kept + site with every kept - site of the same pair and genome
 * whose amplicon length end - start lies in [min_len, max_len] of that pair's
 * window; all such pairs are reported (FF and RR included).  d_hits must be
 * in the canonical order written by ah_scan_primers.  Output sorted by
 * (pair, genome, start, end, orient).  capacity 0 counts without writing.
 * Errors: AH_ERR_INVALID_ARG, AH_ERR_INVALID_PRIMER, AH_ERR_LIMIT,
 * AH_ERR_WORKSPACE, AH_ERR_HIP. */
ah_status ah_pair_amplicons(const ah_hit* d_hits, const ah_result* d_nhits, uint64_t hit_capacity,
                            const ah_primer_pair* pairs, const ah_window* windows,
                            uint32_t n_pairs, ah_amplicon* d_amp, uint64_t capacity,
                            ah_result* d_res, void* d_work, size_t work_bytes, void* stream);
size_t ah_pair_workspace_bytes(uint64_t hit_capacity, uint32_t n_pairs);

/* The whole query in one call (Section 2.1: primer matching, melting
 * temperature, amplicon calling): ah_scan_primers, ah_tm and
 * ah_pair_amplicons of `pairs` (with `windows` and Tm parameters `tm`) on
 * `stream`, with the same outputs byte for byte (sites in d_hits and
 * *d_hit_res, Tm included; amplicons in d_amp and *d_amp_res) and the same
 * workspaces (ah_scan_workspace_bytes for hit_capacity, and
 * ah_pair_workspace_bytes), except that the amplicons need every site: when
 * the sites overflow, no amplicon is written and *d_amp_res is
 * AH_ERR_OVERFLOW with count and required 0 (run again with the sites'
 * `required` first).  Knowing the whole query lets the library fold steps
 * together.  Up to 4,096 segments (n_pairs x genomes, each a pair on one
 * genome), the scan puts the sites of each segment together and one
 * workgroup per segment sorts them into canonical order (in LDS up to 1,024
 * sites), computes their Tm, counts the amplicons each + site starts, takes
 * its first amplicon slot from the counts of the earlier segments and
 * writes its amplicons, in one launch.  With more segments, when a pair is
 * expected to give more than 512 sites on the longest genome (random bases,
 * both primers and strands: one workgroup per segment would take too long),
 * or with AH_QUERY_SEGMENTED=0 in the environment (=1 forces the segmented
 * tail), the sites go through the radix sort instead, the Tm is computed by
 * extra workgroups of its first pass and the pairing's per-chunk counts of
 * kept minus sites are taken by its last.
 * Errors: those of the three calls. */
ah_status ah_query(const ah_genomes* genomes, const ah_primer_pair* pairs, const ah_window* windows,
                   uint32_t n_pairs, const ah_tm_params* tm, ah_hit* d_hits, uint64_t hit_capacity,
                   ah_result* d_hit_res, ah_amplicon* d_amp, uint64_t amp_capacity,
                   ah_result* d_amp_res, void* d_scan_work, size_t scan_work_bytes,
                   void* d_pair_work, size_t pair_work_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batched form: many primer pairs in one pass over the genomes (the paper's
 * future work, Section 4: analysing several primer pairs simultaneously so that
 * the genomes are not re-read for each pair).  ah_scan_primers, ah_tm and
 * ah_pair_amplicons already take n_pairs pairs; the scan then reads each
 * genome tile from HBM once and runs every pair's patterns on it, group by
 * group.  The calls below choose the kernel shape for a primer set.
 * ------------------------------------------------------------------------- */

/* Scan kernel shape: window words per lane (odd, 3..31; a tile of 256 x
 * words_per_lane window words plus the primer halo is staged in LDS, and each
 * lane filters words_per_lane consecutive window words from registers) and
 * primer patterns per group (four per pair: each primer on each strand; a
 * group's code runs over the whole staged tile before the next group's). */
typedef struct ah_scan_tuning {
  uint32_t words_per_lane;
  uint32_t patterns_per_group;
} ah_scan_tuning;

/* Time candidate shapes of the scan kernel for this primer set on `genomes`
 * (every candidate is compiled concurrently on host threads, run `repeats`
 * times after a warm-up, timed with HIP events on `stream`), keep the fastest
 * for later calls with the same set on this device, and return it.  The output
 * buffers are used as scratch (results unspecified afterwards).  Synchronises
 * `stream`.  With the environment variable AH_VERBOSE=1 it writes a line to
 * stderr as each candidate is compiled and timed.  Errors: as ah_scan_primers. */
ah_status ah_autotune_scan(const ah_genomes* genomes, const ah_primer_pair* pairs, uint32_t n_pairs,
                           ah_hit* d_hits, uint64_t capacity, ah_result* d_res, void* d_work,
                           size_t work_bytes, void* stream, uint32_t repeats,
                           ah_scan_tuning* chosen, double* best_ms);
/* Specialise, compile and load the scan kernel for this primer set on the
 * current device now (has_nmask: whether the genomes will carry a non-ACGT
 * mask), so that a later ah_scan_primers call finds it cached.  Safe to call
 * from several host threads at once (compilations run concurrently).
 * Errors: AH_ERR_INVALID_PRIMER, AH_ERR_LIMIT, AH_ERR_JIT, AH_ERR_HIP. */
ah_status ah_scan_prepare(const ah_primer_pair* pairs, uint32_t n_pairs, int has_nmask);
/* Set (tuning != NULL) or forget (NULL) the shape used for this primer set on
 * the current device; AH_ERR_INVALID_ARG for an unsupported shape. */
ah_status ah_set_scan_tuning(const ah_primer_pair* pairs, uint32_t n_pairs,
                             const ah_scan_tuning* tuning);
/* Shape that ah_scan_primers will use for this primer set. */
ah_status ah_get_scan_tuning(const ah_primer_pair* pairs, uint32_t n_pairs, ah_scan_tuning* tuning);

/* ---------------------------------------------------------------------------
 * Amplicon sequences (Section 2.1, "Visualization": the main output is a
 * FASTA file of the predicted amplicon sequences with their coordinates,
 * orientation and maximum Tm) and amplitypes (Section 3.3, "Amplicon Pattern
 * Visualization": per genome, the combination of copy numbers and sequence
 * variants).
 * ------------------------------------------------------------------------- */

/* FASTA text of the amplicons d_amp[0 .. min(d_namp->count, amp_capacity))
 * (as written by ah_pair_amplicons over d_hits of the same genomes), one
 * record per amplicon in their order:
 *   >g<genome>:<start>-<end> pair=<pair> orient=<FR|RF|FF|RR> tm=<tm+>,<tm->
 *   <sequence>
 * tm+ / tm-: the Tm of the amplicon's + and - sites, two decimals (round half
 * to even), "nan" without a compatible oligo.  The sequence is the top strand
 * [start, end) for FR, FF and RR and its reverse complement for RF (copies of
 * one target read alike on either strand); a masked non-ACGT base is N.
 * d_text (device, text_capacity bytes) receives the records back to back;
 * *d_text_res: required = total bytes, count = min(required, capacity),
 * AH_ERR_OVERFLOW when they do not fit (contents then unspecified).
 * d_seq_hash [amp_capacity] (optional): each amplicon's sequence hash
 * mix(n ^ sum_k (c_k + 1) P^k mod 2^64) over its n bases c_k (A0 C1 G2 T3
 * N4), P = 0x100000001B3, mix = the SplitMix64 finaliser (Steele, Lea & Flood
 * 2014).  d_amplitype / d_amplitype_n [n_pairs x n_genomes] (optional, index
 * pair * n_genomes + genome): the amplitype of each (pair, genome), the sum
 * mod 2^64 of mix(h + 0x9E3779B97F4A7C15) over the hashes h of its FR and RF
 * amplicons, and their number; equal for two genomes with the same sequences
 * in the same copy numbers, 0 / 0 for none.  Workspace:
 * ah_fasta_workspace_bytes.  Errors: AH_ERR_INVALID_ARG, AH_ERR_WORKSPACE,
 * AH_ERR_HIP. */
size_t ah_fasta_workspace_bytes(uint64_t amp_capacity);
ah_status ah_amplicon_fasta(const ah_genomes* genomes, const ah_hit* d_hits,
                            const ah_amplicon* d_amp, const ah_result* d_namp,
                            uint64_t amp_capacity, uint32_t n_pairs, char* d_text,
                            uint64_t text_capacity, ah_result* d_text_res, uint64_t* d_seq_hash,
                            uint64_t* d_amplitype, uint32_t* d_amplitype_n, void* d_work,
                            size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Streaming form: a packed collection held in host memory is copied to the GPU
 * in chunks of whole genomes on the caller's copy streams while the previous
 * chunks are scanned, scored and paired on the compute stream.  The paper
 * reads genomes from disk and names that I/O as a large part of its run time
 * (Section 4); here the host-to-HBM copy of the 2-bit packed form (0.25 B per
 * base) is the only transfer, and it overlaps the device work.
 * ------------------------------------------------------------------------- */

/* A packed collection in host memory, laid out as ah_pack_layout and
 * ah_pack_genomes lay it out on the device: words holds 2 x word_off[n]
 * uint32 (h, l of each word), nmask word_off[n] uint32 or NULL.  words and
 * nmask should be pinned (hipHostMalloc, or a torch tensor created with
 * pin_memory=True): from pageable memory the copies do not overlap.
 * word_off (n + 1) and len (n) are host arrays.  All borrowed for the call. */
typedef struct ah_host_genomes {
  const uint32_t* words;
  const uint32_t* nmask;
  const uint64_t* word_off;
  const uint32_t* len;
  uint32_t n;
} ah_host_genomes;

/* chunk_words: packed words per staging slot; consecutive genomes are grouped
 * into chunks of at most this many words, and every genome must fit in one
 * (word_off[g + 1] - word_off[g] <= chunk_words, else AH_ERR_LIMIT).
 * n_slots (2..16): staging slots on the device; while one chunk is processed
 * the copies of up to n_slots - 1 later chunks are in flight. */
typedef struct ah_stream_config {
  uint64_t chunk_words;
  uint32_t n_slots;
  uint32_t reserved; /* 0 */
} ah_stream_config;

/* Device workspace for ah_stream_query: the staging slots, the collection's
 * offsets and lengths, and the pairing and scan workspaces of one chunk.
 * Returns the recommended size (the scan's candidate list sized for the
 * filters of `pairs` over a chunk, as ah_scan_workspace_bytes does); with
 * pairs NULL, the minimum.  Any size from the minimum up is accepted; extra
 * bytes lengthen the candidate list. */
size_t ah_stream_workspace_bytes(const ah_host_genomes* genomes, const ah_stream_config* cfg,
                                 const ah_primer_pair* pairs, uint32_t n_pairs,
                                 uint64_t hit_capacity);

/* Scan, Tm and pairing of `pairs` over a host-resident packed collection,
 * streamed chunk by chunk.  Chunk c's copy runs on copy_streams[c %
 * n_copy_streams] (the compute stream when n_copy_streams is 0); everything
 * else runs on `stream`.  The call blocks until every chunk is done (it reads
 * each chunk's counts to place the next chunk's output); results are then
 * complete in d_hits / d_amp and their ah_result records.
 *
 * Output: the chunks' outputs concatenated in chunk order, genome ids and the
 * amplicons' hit indices rewritten to collection-wide ones.  Each chunk is in
 * canonical order, so for one pair the output is byte-identical to a call of
 * ah_scan_primers / ah_tm / ah_pair_amplicons on the resident collection; for
 * several pairs it is that output ordered by (genome chunk, pair, ...).
 * Overflow: when the hits exceed hit_capacity, both results report
 * AH_ERR_OVERFLOW, d_hit_res->required is the exact total, and the amplicons
 * are incomplete (retry with hit_capacity >= required); when only the
 * amplicons exceed amp_capacity, d_amp_res->required is the exact total.
 * Errors: those of the three calls, AH_ERR_LIMIT (a genome larger than a
 * slot, or more than 2^32 - 1 hits), AH_ERR_WORKSPACE, AH_ERR_HIP. */
ah_status ah_stream_query(const ah_host_genomes* genomes, const ah_stream_config* cfg,
                          const ah_primer_pair* pairs, const ah_window* windows, uint32_t n_pairs,
                          const ah_tm_params* tm, ah_hit* d_hits, uint64_t hit_capacity,
                          ah_result* d_hit_res, ah_amplicon* d_amp, uint64_t amp_capacity,
                          ah_result* d_amp_res, void* d_work, size_t work_bytes, void* stream,
                          void* const* copy_streams, uint32_t n_copy_streams);

/* ---------------------------------------------------------------------------
 * Serving form: a request loop over a collection resident in HBM, in the
 * spirit of the paper's web server answering primer-pair queries against
 * fixed reference databases (Section 2.2, Performance Optimization) and of the
 * planned searches over subsets of those databases (Section 4).  Jobs (one
 * primer pair over a subset of the resident genomes) are admitted as they
 * arrive: each job is split into parts
 * of whole genomes; lane threads, each driving its own device stream, take the
 * next part of the active jobs in turn, so parts of different jobs run on the
 * device at the same time and a job that arrives while others run starts as
 * soon as a lane and memory are free.  Every part's device buffers are carved
 * from a caller-given device pool (the HBM budget) while it runs: a part is
 * started only when its buffers fit, and its records are copied to host
 * memory when it ends, so the pool only ever holds running parts (admission
 * cannot deadlock).  Capacities come from the pair's expected random-site
 * rate; a part that overflows is run again with the exact counts, so results
 * never depend on the estimate, on the mix of other jobs or on the lane that
 * ran them.
 * ------------------------------------------------------------------------- */
typedef struct ah_server ah_server;

typedef struct ah_server_config {
  uint32_t n_lanes;       /* device streams, each driven by a host thread (1..16) */
  uint32_t n_compilers;   /* host threads that specialise scan kernels for new pairs (1..32) */
  uint64_t part_bases;    /* bases per part at most (whole genomes; >= 1) */
  uint64_t max_part_hits; /* parts are also cut so that their expected sites stay below this */
  double capacity_scale;  /* capacity = scale x expected records + a per-genome reserve */
  uint64_t host_pool_bytes; /* pinned host arena for part records (0: none); parts whose
                               records do not fit go through a staging buffer instead */
} ah_server_config;

/* One request.  Strings and the genome list are copied at submission. */
typedef struct ah_job {
  ah_primer_pair pair;
  ah_window window;
  ah_tm_params tm;
  const uint32_t* genomes; /* host, strictly ascending ids into the resident collection, or NULL = all */
  uint32_t n_genomes;
  uint32_t reserved;       /* 0 */
} ah_job;

/* A finished job.  Times are seconds on the server's clock (ah_server_now). */
typedef struct ah_job_status {
  uint64_t job;
  int32_t status;          /* AH_OK or the error that ended the job */
  uint32_t n_parts;
  uint64_t hits;           /* sites, all parts */
  uint64_t amplicons;      /* all parts */
  uint64_t bases;          /* bases of the job's genomes */
  double t_submit, t_ready, t_start, t_done; /* ready: kernel compiled; start: first part on a lane */
  uint32_t retries;        /* parts run again after an overflow */
  uint32_t reserved;
} ah_job_status;

/* Output of one part (host memory owned by the server: the pinned arena or
 * ordinary memory, valid until the job is released).  Genome ids are ids of the resident collection; plus_hit and
 * minus_hit index this part's hits.  The parts of a job cover its genomes in
 * ascending order, so their concatenation is the job's canonical output. */
typedef struct ah_job_part {
  const ah_hit* hits;
  uint64_t n_hits;
  const ah_amplicon* amplicons;
  uint64_t n_amplicons;
  uint32_t first_genome;   /* index into the job's genome list */
  uint32_t n_genomes;
} ah_job_part;

typedef struct ah_server_stats {
  uint64_t jobs_submitted, jobs_finished, parts_run, retries;
  uint64_t pool_bytes, pool_in_use, pool_high_water;
  uint64_t admission_waits; /* times a lane found the next part's buffers not fitting yet */
                            /* pool_in_use / pool_high_water: device bytes of running parts */
  double lane_busy_s;       /* summed over lanes: time from a part's launch to its completion */
  uint64_t host_pool_bytes, host_pool_high_water;
  uint64_t host_fallbacks;  /* parts whose records did not fit in the host arena */
  double gpu_s;             /* summed over parts: launch to results on the host (last run) */
  double copy_s;            /* summed over parts: copying records to host memory */
} ah_server_stats;

/* Start a server on the current device over `resident` (device views stay
 * borrowed until ah_server_destroy; h_len: host copy of the genome lengths,
 * copied; resident->word_off must hold the n + 1 offsets of ah_pack_layout).
 * d_pool / pool_bytes: device memory that the server carves all per-part
 * buffers from (caller-owned; no other device memory is allocated per job
 * apart from small per-pair tables cached by ah_tm / ah_pair_amplicons).  A
 * part that needs more than the whole pool ends its job with AH_ERR_LIMIT.
 * Errors: AH_ERR_INVALID_ARG, AH_ERR_HIP. */
ah_status ah_server_create(const ah_genomes* resident, const uint32_t* h_len,
                           const ah_server_config* cfg, void* d_pool, size_t pool_bytes,
                           ah_server** server);
/* Queue a job; returns at once with its id.  The pair and the Tm parameters
 * are checked as ah_tm checks them.  Errors: AH_ERR_INVALID_ARG (bad genome
 * list, window or Tm parameters), AH_ERR_INVALID_PRIMER, AH_ERR_LIMIT. */
ah_status ah_server_submit(ah_server* server, const ah_job* job, uint64_t* job_id);
/* Wait up to timeout_s for the next finished job (in order of completion);
 * AH_ERR_AGAIN if none finished in time. */
ah_status ah_server_wait(ah_server* server, double timeout_s, ah_job_status* status);
/* Output of part `part` of a finished job. */
ah_status ah_server_part(ah_server* server, uint64_t job_id, uint32_t part, ah_job_part* out);
/* Drop a finished job and its records; its part pointers become invalid. */
ah_status ah_server_release(ah_server* server, uint64_t job_id);
void ah_server_stats_get(ah_server* server, ah_server_stats* stats);
double ah_server_now(ah_server* server);
/* Stop accepting parts, let the lanes finish the parts they run, join every
 * thread and free the server (jobs not finished are dropped). */
void ah_server_destroy(ah_server* server);

/* ---------------------------------------------------------------------------
 * Utilities.
 * ------------------------------------------------------------------------- */
const char* ah_status_str(int status);
/* Message of the last error on the calling thread ("" if none). */
const char* ah_last_error(void);
/* Drop the cached specialised kernels and per-set device tables. */
void ah_release_caches(void);
/* Number of scan-kernel specialisations compiled so far and their total
 * compile time in milliseconds. */
void ah_jit_stats(uint64_t* n_compiled, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* AH_H */
