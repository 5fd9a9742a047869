/*
 * libah introspection helpers (host only; no GPU needed).  They expose the
 * primer compiler and the per-primer-set scan specialisation described in
 * ah.h (primer matching, Section 2.1 of AmpliconHunter, arXiv 2509.13300) so
 * that both can be checked without running a kernel.
 */
#ifndef AH_DEV_H
#define AH_DEV_H

#include "ah.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Validate a primer set exactly as ah_scan_primers does (IUPAC codes, length
 * 5..32, k <= AH_MAX_K, clamp <= primer length); no device work.  Returns
 * AH_OK or the error ah_scan_primers would return (message in
 * ah_last_error()). */
ah_status ah_validate_pairs(const ah_primer_pair* pairs, uint32_t n_pairs);

/* Validate a Tm request exactly as ah_tm does (the pairs, the salt method
 * and its ion concentrations, the strand concentration, and for a primer
 * above AH_TM_MAX_PAIRINGS what the exact route needs); no device work.
 * Returns AH_OK or the error ah_tm would return (message in
 * ah_last_error()). */
ah_status ah_validate_tm(const ah_primer_pair* pairs, uint32_t n_pairs, const ah_tm_params* params);

/* Source text of the specialised scan program for a primer set (has_nmask:
 * whether the collection carries a non-ACGT mask).  Copies at most
 * buf_bytes - 1 characters plus a terminating NUL into buf (buf may be NULL)
 * and returns the full size including the NUL, or 0 if the set is invalid. */
size_t ah_scan_program_source(const ah_primer_pair* pairs, uint32_t n_pairs, int has_nmask,
                              char* buf, size_t buf_bytes);

/* Compile (but do not load) the specialised scan program for gfx950 and
 * report the code-object size.  Errors: as ah_validate_pairs, AH_ERR_JIT. */
ah_status ah_scan_program_compile(const ah_primer_pair* pairs, uint32_t n_pairs, int has_nmask,
                                  size_t* code_bytes);

/* Kernel timing with HIP events recorded on the launching stream.  While
 * enabled, every launch of the named kernels is bracketed by a pair of
 * events: "scan" (the filter of the specialised site scan), "verify" (its
 * exact count of the candidates), "tm", "pair" (the amplicon
 * writer), "sort" (all radix-sort passes of one call), "pack".  Queries wait
 * for the recorded events and return the launch count and summed device time
 * since the last reset.  Not for use inside hipGraph capture. */
void ah_profile_enable(int on);
void ah_profile_reset(void);
ah_status ah_profile_query(const char* name, uint64_t* launches, double* total_ms);

/* Statistics of the filter stage of the last ah_scan_primers call that used
 * this workspace (the same n genomes and capacity): out[0] candidate records,
 * out[1] windows in them, out[2] workgroups whose share of the candidate list
 * was full, out[3] most candidates of one workgroup.  Synchronises the device. */
ah_status ah_scan_candidate_stats(const void* d_work, size_t work_bytes, uint32_t n_genomes,
                                  uint64_t capacity, uint64_t out[4]);

/* Candidate records that the list of a scan workspace of work_bytes holds
 * for n genomes and a hit capacity, with the workspace starting base_offset
 * (mod 256) bytes past a 256-byte boundary.  Host arithmetic only. */
uint64_t ah_scan_candidate_capacity(size_t base_offset, size_t work_bytes, uint32_t n_genomes,
                                    uint64_t capacity);

/* Host-only simulation of the serving scheduler (ah_server_*): the lanes'
 * own admission, round-robin and retry decisions, driven by simulated part
 * runs on a simulated clock instead of device work.  Job i (the jobs need
 * not be sorted) arrives at jobs[i].arrival with the parts
 * parts[first_part .. first_part + n_parts) in that order; part q holds
 * parts[q].bytes of the pool while it runs for parts[q].seconds, and its
 * first parts[q].overflows runs report an output overflow (the part then runs
 * again, as the server reruns a part with exact counts).  n_lanes lanes
 * (1..16) share a pool of pool_bytes.  events[e] (up to max_events; the
 * number of part runs in *n_events) lists every run in start order; done[i]
 * gives job i's status (AH_OK, AH_ERR_LIMIT for a part larger than the pool),
 * times (t_submit, t_start, t_done), parts and reruns.  Errors:
 * AH_ERR_INVALID_ARG, AH_ERR_OVERFLOW (more runs than max_events; the
 * statuses are still complete). */
typedef struct ah_sched_part {
  uint64_t bytes;
  double seconds;
  uint32_t overflows;
  uint32_t reserved;
} ah_sched_part;
typedef struct ah_sched_job {
  double arrival;
  uint32_t first_part;
  uint32_t n_parts;
} ah_sched_job;
typedef struct ah_sched_event {
  double t_start, t_end;
  uint32_t lane, job, part, run; /* run: 0 for a part's first run */
  uint64_t block, bytes;         /* its pool block (offset) and size */
  uint64_t pool_in_use;          /* pool bytes in use once it was admitted */
} ah_sched_event;
ah_status ah_sched_simulate(const ah_sched_job* jobs, uint32_t n_jobs, const ah_sched_part* parts,
                            uint32_t n_parts, uint32_t n_lanes, uint64_t pool_bytes,
                            ah_sched_event* events, uint64_t max_events, uint64_t* n_events,
                            ah_job_status* done);

#ifdef __cplusplus
}
#endif
#endif /* AH_DEV_H */
