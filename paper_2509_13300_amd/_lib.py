"""ctypes binding of libah (include/ah.h): argument marshalling only.

Every function here forwards to the C entry point of the same name; all the
work runs in libah's HIP kernels.  Device buffers are torch tensors (their
data pointers are passed through) and streams are torch streams.  There is
no fallback: if libah.so is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libah.so")

AH_OK, AH_ERR_INVALID_ARG, AH_ERR_INVALID_PRIMER, AH_ERR_LIMIT = 0, -1, -2, -3
AH_ERR_OVERFLOW, AH_ERR_WORKSPACE, AH_ERR_HIP, AH_ERR_JIT, AH_ERR_AGAIN = -4, -5, -6, -7, -8
AH_FR, AH_RF, AH_FF, AH_RR = 0, 1, 2, 3
HALO_WORDS = 31

HIT_DTYPE = np.dtype([("genome", "<u4"), ("pos", "<u4"), ("pair", "<u2"),
                      ("strand_primer", "u1"), ("mm", "u1"), ("tm", "<f4")])
AMP_DTYPE = np.dtype([("genome", "<u4"), ("start", "<u4"), ("end", "<u4"), ("plus_hit", "<u4"),
                      ("minus_hit", "<u4"), ("pair", "<u2"), ("orient", "u1"), ("reserved", "u1")])
assert HIT_DTYPE.itemsize == 16 and AMP_DTYPE.itemsize == 24


class AhError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status} ({message})")
        self.status = status


class ah_genomes(ctypes.Structure):
    _fields_ = [("words", ctypes.c_void_p), ("nmask", ctypes.c_void_p),
                ("word_off", ctypes.c_void_p), ("len", ctypes.c_void_p),
                ("n", ctypes.c_uint32), ("max_len", ctypes.c_uint32)]


AH_PAIR_DECOY = 1


class ah_primer_pair(ctypes.Structure):
    _fields_ = [("fwd", ctypes.c_char_p), ("rev", ctypes.c_char_p),
                ("k", ctypes.c_uint32), ("clamp", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class ah_result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("required", ctypes.c_uint64),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


class ah_tm_params(ctypes.Structure):
    _fields_ = [("dnac1_nM", ctypes.c_double), ("dnac2_nM", ctypes.c_double),
                ("Na_mM", ctypes.c_double), ("K_mM", ctypes.c_double),
                ("Tris_mM", ctypes.c_double), ("Mg_mM", ctypes.c_double),
                ("dNTPs_mM", ctypes.c_double), ("saltcorr", ctypes.c_int32),
                ("selfcomp", ctypes.c_int32)]


class ah_scan_tuning(ctypes.Structure):
    _fields_ = [("words_per_lane", ctypes.c_uint32), ("patterns_per_group", ctypes.c_uint32)]


class ah_window(ctypes.Structure):
    _fields_ = [("min_len", ctypes.c_uint32), ("max_len", ctypes.c_uint32),
                ("filter_tm", ctypes.c_int32), ("min_tm", ctypes.c_float)]


class ah_host_genomes(ctypes.Structure):
    _fields_ = [("words", ctypes.c_void_p), ("nmask", ctypes.c_void_p),
                ("word_off", ctypes.c_void_p), ("len", ctypes.c_void_p), ("n", ctypes.c_uint32)]


class ah_stream_config(ctypes.Structure):
    _fields_ = [("chunk_words", ctypes.c_uint64), ("n_slots", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ah_server_config(ctypes.Structure):
    _fields_ = [("n_lanes", ctypes.c_uint32), ("n_compilers", ctypes.c_uint32),
                ("part_bases", ctypes.c_uint64), ("max_part_hits", ctypes.c_uint64),
                ("capacity_scale", ctypes.c_double), ("host_pool_bytes", ctypes.c_uint64)]


class ah_job(ctypes.Structure):
    _fields_ = [("pair", ah_primer_pair), ("window", ah_window), ("tm", ah_tm_params),
                ("genomes", ctypes.c_void_p), ("n_genomes", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ah_sched_part(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_uint64), ("seconds", ctypes.c_double),
                ("overflows", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ah_sched_job(ctypes.Structure):
    _fields_ = [("arrival", ctypes.c_double), ("first_part", ctypes.c_uint32),
                ("n_parts", ctypes.c_uint32)]


class ah_sched_event(ctypes.Structure):
    _fields_ = [("t_start", ctypes.c_double), ("t_end", ctypes.c_double),
                ("lane", ctypes.c_uint32), ("job", ctypes.c_uint32), ("part", ctypes.c_uint32),
                ("run", ctypes.c_uint32), ("block", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("pool_in_use", ctypes.c_uint64)]


class ah_job_status(ctypes.Structure):
    _fields_ = [("job", ctypes.c_uint64), ("status", ctypes.c_int32), ("n_parts", ctypes.c_uint32),
                ("hits", ctypes.c_uint64), ("amplicons", ctypes.c_uint64),
                ("bases", ctypes.c_uint64), ("t_submit", ctypes.c_double),
                ("t_ready", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("retries", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ah_job_part(ctypes.Structure):
    _fields_ = [("hits", ctypes.c_void_p), ("n_hits", ctypes.c_uint64),
                ("amplicons", ctypes.c_void_p), ("n_amplicons", ctypes.c_uint64),
                ("first_genome", ctypes.c_uint32), ("n_genomes", ctypes.c_uint32)]


class ah_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "jobs_submitted", "jobs_finished", "parts_run", "retries", "pool_bytes", "pool_in_use",
        "pool_high_water", "admission_waits")] + [("lane_busy_s", ctypes.c_double)] + [
        (n, ctypes.c_uint64) for n in ("host_pool_bytes", "host_pool_high_water", "host_fallbacks")] + [
        ("gpu_s", ctypes.c_double), ("copy_s", ctypes.c_double)]


# Every symbol declared in include/ah.h and include/ah_dev.h.
EXPORTS = (
    "ah_pack_layout", "ah_pack_genomes", "ah_scan_primers", "ah_scan_workspace_bytes", "ah_tm",
    "ah_pair_amplicons", "ah_pair_workspace_bytes", "ah_status_str", "ah_last_error",
    "ah_release_caches", "ah_jit_stats", "ah_validate_pairs", "ah_scan_program_source",
    "ah_scan_program_compile", "ah_profile_enable", "ah_profile_reset", "ah_profile_query",
    "ah_autotune_scan", "ah_set_scan_tuning", "ah_get_scan_tuning", "ah_scan_prepare",
    "ah_stream_workspace_bytes", "ah_stream_query", "ah_server_create", "ah_server_submit",
    "ah_server_wait", "ah_server_part", "ah_server_release", "ah_server_stats_get",
    "ah_server_now", "ah_server_destroy", "ah_scan_candidate_stats", "ah_scan_candidate_capacity",
    "ah_fasta_workspace_bytes", "ah_amplicon_fasta", "ah_fasta_count", "ah_fasta_read",
    "ah_tm_duplex", "ah_validate_tm", "ah_scan_primers_noalloc", "ah_sched_simulate",
    "ah_query",
)

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2509_13300_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    st = ctypes.c_int
    P = ctypes.POINTER
    L.ah_pack_layout.argtypes = [vp, u32, vp]
    L.ah_pack_layout.restype = u64
    L.ah_pack_genomes.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp, vp]
    L.ah_pack_genomes.restype = st
    L.ah_scan_primers.argtypes = [P(ah_genomes), P(ah_primer_pair), u32, vp, u64, vp, vp, sz, vp]
    L.ah_scan_primers.restype = st
    L.ah_scan_primers_noalloc.argtypes = [P(ah_genomes), P(ah_primer_pair), u32, vp, u64, vp, vp]
    L.ah_scan_primers_noalloc.restype = st
    L.ah_scan_workspace_bytes.argtypes = [P(ah_genomes), P(ah_primer_pair), u32, u64]
    L.ah_scan_workspace_bytes.restype = sz
    L.ah_tm.argtypes = [P(ah_genomes), P(ah_primer_pair), u32, P(ah_tm_params), vp, vp, u64, vp]
    L.ah_tm.restype = st
    L.ah_query.argtypes = [P(ah_genomes), P(ah_primer_pair), P(ah_window), u32, P(ah_tm_params),
                           vp, u64, vp, vp, u64, vp, vp, sz, vp, sz, vp]
    L.ah_query.restype = st
    L.ah_tm_duplex.argtypes = [ctypes.c_char_p, ctypes.c_char_p, P(ah_tm_params),
                               P(ctypes.c_double)]
    L.ah_tm_duplex.restype = st
    L.ah_pair_amplicons.argtypes = [vp, vp, u64, P(ah_primer_pair), P(ah_window), u32, vp, u64, vp,
                                    vp, sz, vp]
    L.ah_pair_amplicons.restype = st
    L.ah_fasta_count.argtypes = [ctypes.c_char_p, u64, P(ctypes.c_uint64), P(ctypes.c_uint64)]
    L.ah_fasta_count.restype = st
    L.ah_fasta_read.argtypes = [ctypes.c_char_p, u64, vp, u64, vp, vp, u64]
    L.ah_fasta_read.restype = st
    L.ah_fasta_workspace_bytes.argtypes = [u64]
    L.ah_fasta_workspace_bytes.restype = sz
    L.ah_amplicon_fasta.argtypes = [P(ah_genomes), vp, vp, vp, u64, u32, vp, u64, vp, vp, vp, vp,
                                    vp, sz, vp]
    L.ah_amplicon_fasta.restype = st
    L.ah_pair_workspace_bytes.argtypes = [u64, u32]
    L.ah_pair_workspace_bytes.restype = sz
    L.ah_status_str.argtypes = [ctypes.c_int]
    L.ah_status_str.restype = ctypes.c_char_p
    L.ah_last_error.argtypes = []
    L.ah_last_error.restype = ctypes.c_char_p
    L.ah_release_caches.argtypes = []
    L.ah_release_caches.restype = None
    L.ah_jit_stats.argtypes = [P(ctypes.c_uint64), P(ctypes.c_double)]
    L.ah_jit_stats.restype = None
    L.ah_validate_pairs.argtypes = [P(ah_primer_pair), u32]
    L.ah_validate_pairs.restype = st
    L.ah_validate_tm.argtypes = [P(ah_primer_pair), u32, P(ah_tm_params)]
    L.ah_validate_tm.restype = st
    L.ah_sched_simulate.argtypes = [P(ah_sched_job), u32, P(ah_sched_part), u32, u32, u64,
                                    P(ah_sched_event), u64, P(ctypes.c_uint64), P(ah_job_status)]
    L.ah_sched_simulate.restype = st
    L.ah_scan_program_source.argtypes = [P(ah_primer_pair), u32, ctypes.c_int, ctypes.c_char_p, sz]
    L.ah_scan_program_source.restype = sz
    L.ah_scan_program_compile.argtypes = [P(ah_primer_pair), u32, ctypes.c_int, P(ctypes.c_size_t)]
    L.ah_scan_program_compile.restype = st
    L.ah_profile_enable.argtypes = [ctypes.c_int]
    L.ah_profile_enable.restype = None
    L.ah_profile_reset.argtypes = []
    L.ah_profile_reset.restype = None
    L.ah_profile_query.argtypes = [ctypes.c_char_p, P(ctypes.c_uint64), P(ctypes.c_double)]
    L.ah_profile_query.restype = st
    L.ah_autotune_scan.argtypes = [P(ah_genomes), P(ah_primer_pair), u32, vp, u64, vp, vp, sz, vp,
                                   u32, P(ah_scan_tuning), P(ctypes.c_double)]
    L.ah_autotune_scan.restype = st
    L.ah_set_scan_tuning.argtypes = [P(ah_primer_pair), u32, P(ah_scan_tuning)]
    L.ah_set_scan_tuning.restype = st
    L.ah_get_scan_tuning.argtypes = [P(ah_primer_pair), u32, P(ah_scan_tuning)]
    L.ah_get_scan_tuning.restype = st
    L.ah_scan_prepare.argtypes = [P(ah_primer_pair), u32, ctypes.c_int]
    L.ah_scan_prepare.restype = st
    L.ah_stream_workspace_bytes.argtypes = [P(ah_host_genomes), P(ah_stream_config),
                                            P(ah_primer_pair), u32, u64]
    L.ah_stream_workspace_bytes.restype = sz
    L.ah_stream_query.argtypes = [P(ah_host_genomes), P(ah_stream_config), P(ah_primer_pair),
                                  P(ah_window), u32, P(ah_tm_params), vp, u64, vp, vp, u64, vp, vp,
                                  sz, vp, P(vp), u32]
    L.ah_stream_query.restype = st
    L.ah_server_create.argtypes = [P(ah_genomes), vp, P(ah_server_config), vp, sz, P(vp)]
    L.ah_server_create.restype = st
    L.ah_server_submit.argtypes = [vp, P(ah_job), P(ctypes.c_uint64)]
    L.ah_server_submit.restype = st
    L.ah_server_wait.argtypes = [vp, ctypes.c_double, P(ah_job_status)]
    L.ah_server_wait.restype = st
    L.ah_server_part.argtypes = [vp, u64, u32, P(ah_job_part)]
    L.ah_server_part.restype = st
    L.ah_server_release.argtypes = [vp, u64]
    L.ah_server_release.restype = st
    L.ah_server_stats_get.argtypes = [vp, P(ah_server_stats)]
    L.ah_server_stats_get.restype = None
    L.ah_server_now.argtypes = [vp]
    L.ah_server_now.restype = ctypes.c_double
    L.ah_server_destroy.argtypes = [vp]
    L.ah_server_destroy.restype = None
    L.ah_scan_candidate_stats.argtypes = [vp, sz, u32, u64, P(ctypes.c_uint64)]
    L.ah_scan_candidate_stats.restype = st
    L.ah_scan_candidate_capacity.argtypes = [sz, sz, u32, u64]
    L.ah_scan_candidate_capacity.restype = u64
    _lib = L
    return L


def _check(status: int, where: str):
    if status != AH_OK:
        msg = lib().ah_last_error().decode(errors="replace")
        raise AhError(status, where, msg or lib().ah_status_str(status).decode())


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch

        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _pair_flags(p) -> int:
    return AH_PAIR_DECOY if getattr(p, "decoy", False) else 0


def primer_pairs(pairs: Sequence) -> ctypes.Array:
    """Marshal objects with fwd, rev, k, clamp (and optionally decoy)
    attributes, or (fwd, rev, k, clamp[, flags]) tuples."""
    arr = (ah_primer_pair * len(pairs))()
    keep = []
    for i, p in enumerate(pairs):
        if hasattr(p, "fwd"):
            fwd, rev, k, clamp, flags = p.fwd, p.rev, p.k, p.clamp, _pair_flags(p)
        else:
            fwd, rev, k, clamp = p[:4]
            flags = p[4] if len(p) > 4 else 0
        f, r = fwd.encode(), rev.encode()
        keep += [f, r]
        arr[i] = ah_primer_pair(f, r, int(k), int(clamp), int(flags))
    arr._keep = keep
    return arr


def windows(pairs: Sequence, filter_tm: bool = False, min_tm: float = 50.0) -> ctypes.Array:
    arr = (ah_window * len(pairs))()
    for i, p in enumerate(pairs):
        arr[i] = ah_window(int(p.min_len), int(p.max_len), 1 if filter_tm else 0, float(min_tm))
    return arr


def tm_params(dnac1=250.0, dnac2=0.0, Na=50.0, K=0.0, Tris=0.0, Mg=1.5, dNTPs=0.0, saltcorr=5,
              selfcomp=False) -> ah_tm_params:
    return ah_tm_params(dnac1, dnac2, Na, K, Tris, Mg, dNTPs, int(saltcorr), 1 if selfcomp else 0)


# ------------------------------------------------------------ entry points --
def ah_pack_layout(lengths) -> np.ndarray:
    lengths = np.ascontiguousarray(lengths, dtype=np.uint64)
    out = np.zeros(lengths.size + 1, dtype=np.uint64)
    total = lib().ah_pack_layout(lengths.ctypes.data, lengths.size, out.ctypes.data)
    if total == 0xFFFFFFFFFFFFFFFF:
        raise AhError(AH_ERR_INVALID_ARG, "ah_pack_layout", lib().ah_last_error().decode())
    return out


def ah_pack_genomes(ascii, ascii_off, n, word_off, words, len_, nmask=None, non_acgt=None,
                    stream=None):
    _check(lib().ah_pack_genomes(_ptr(ascii), _ptr(ascii_off), int(n), _ptr(word_off), _ptr(words),
                                 _ptr(len_), _ptr(nmask), _ptr(non_acgt), _stream(stream)),
           "ah_pack_genomes")


def _pairs_arg(pairs):
    """(array or None, count): a pair list, or an int for a count alone."""
    if isinstance(pairs, int):
        return None, pairs
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    return pp, len(pp)


def ah_scan_workspace_bytes(genomes: ah_genomes, pairs, capacity: int) -> int:
    """Recommended scan workspace; `pairs` may be an int (the minimum)."""
    pp, n = _pairs_arg(pairs)
    return int(lib().ah_scan_workspace_bytes(ctypes.byref(genomes), pp, n, capacity))


def ah_scan_primers(genomes: ah_genomes, pairs, hits, capacity: int, res, work, stream=None):
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    _check(lib().ah_scan_primers(ctypes.byref(genomes), pp, len(pp), _ptr(hits), int(capacity),
                                 _ptr(res), _ptr(work), 0 if work is None else work.numel(),
                                 _stream(stream)), "ah_scan_primers")


def ah_scan_primers_noalloc(genomes: ah_genomes, pairs, hits, capacity: int, res, stream=None):
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    _check(lib().ah_scan_primers_noalloc(ctypes.byref(genomes), pp, len(pp), _ptr(hits),
                                         int(capacity), _ptr(res), _stream(stream)),
           "ah_scan_primers_noalloc")


def ah_query(genomes: ah_genomes, pairs, wins, params: ah_tm_params, hits, hit_capacity: int,
             hit_res, amps, amp_capacity: int, amp_res, scan_work, pair_work, stream=None):
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    _check(lib().ah_query(ctypes.byref(genomes), pp, wins, len(pp), ctypes.byref(params),
                          _ptr(hits), int(hit_capacity), _ptr(hit_res), _ptr(amps),
                          int(amp_capacity), _ptr(amp_res), _ptr(scan_work),
                          0 if scan_work is None else scan_work.numel(), _ptr(pair_work),
                          0 if pair_work is None else pair_work.numel(), _stream(stream)),
           "ah_query")


def ah_tm(genomes: ah_genomes, pairs, params: ah_tm_params, hits, nhits, capacity: int,
          stream=None):
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    _check(lib().ah_tm(ctypes.byref(genomes), pp, len(pp), ctypes.byref(params), _ptr(hits),
                       _ptr(nhits), int(capacity), _stream(stream)), "ah_tm")


def ah_tm_duplex(oligo: str, opposite: str, params: ah_tm_params) -> float:
    out = ctypes.c_double()
    _check(lib().ah_tm_duplex(oligo.encode(), opposite.encode(), ctypes.byref(params),
                              ctypes.byref(out)), "ah_tm_duplex")
    return out.value


def ah_pair_workspace_bytes(hit_capacity: int, n_pairs: int) -> int:
    return int(lib().ah_pair_workspace_bytes(int(hit_capacity), int(n_pairs)))


def ah_pair_amplicons(hits, nhits, hit_capacity: int, pairs, wins, amp, capacity: int, res, work,
                      stream=None):
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    _check(lib().ah_pair_amplicons(_ptr(hits), _ptr(nhits), int(hit_capacity), pp, wins, len(pp),
                                   _ptr(amp), int(capacity), _ptr(res), _ptr(work),
                                   0 if work is None else work.numel(), _stream(stream)),
           "ah_pair_amplicons")


def fasta_read(text: bytes, pinned: bool = False):
    """Records of FASTA text: (sequence bytes, offsets [n + 1] int64, names
    [n] str).  The bytes are a numpy uint8 array, or with ``pinned`` a torch
    uint8 tensor in pinned host memory, written there directly."""
    n = ctypes.c_uint64()
    q = ctypes.c_uint64()
    _check(lib().ah_fasta_count(text, len(text), ctypes.byref(n), ctypes.byref(q)), "ah_fasta_count")
    if pinned:
        import torch

        seq = torch.empty(max(1, q.value), dtype=torch.uint8, pin_memory=True)
        dst = seq.data_ptr()
    else:
        seq = np.empty(max(1, q.value), dtype=np.uint8)
        dst = seq.ctypes.data
    off = np.empty(n.value + 1, dtype=np.uint64)
    span = np.empty(max(1, 2 * n.value), dtype=np.uint64)
    _check(lib().ah_fasta_read(text, len(text), dst, q.value, off.ctypes.data, span.ctypes.data,
                               n.value), "ah_fasta_read")
    names = [text[int(span[2 * r]):int(span[2 * r + 1])].decode(errors="replace")
             for r in range(n.value)]
    return seq[: q.value], off.astype(np.int64), names


def ah_fasta_workspace_bytes(amp_capacity: int) -> int:
    return int(lib().ah_fasta_workspace_bytes(int(amp_capacity)))


def ah_amplicon_fasta(genomes: ah_genomes, hits, amps, namp, amp_capacity: int, n_pairs: int,
                      text, text_res, seq_hash, amplitype, amplitype_n, work, stream=None):
    _check(lib().ah_amplicon_fasta(ctypes.byref(genomes), _ptr(hits), _ptr(amps), _ptr(namp),
                                   int(amp_capacity), int(n_pairs), _ptr(text),
                                   0 if text is None else text.numel(), _ptr(text_res),
                                   _ptr(seq_hash), _ptr(amplitype), _ptr(amplitype_n), _ptr(work),
                                   0 if work is None else work.numel(), _stream(stream)),
           "ah_amplicon_fasta")


def ah_validate_pairs(pairs) -> int:
    pp = primer_pairs(pairs)
    return int(lib().ah_validate_pairs(pp, len(pp)))


def ah_validate_tm(pairs, params: ah_tm_params) -> int:
    pp = primer_pairs(pairs)
    return int(lib().ah_validate_tm(pp, len(pp), ctypes.byref(params)))


def ah_sched_simulate(jobs, n_lanes: int, pool_bytes: int, max_events: int = 1 << 16):
    """jobs: [(arrival_s, [(bytes, seconds, overflows), ...]), ...].  Returns
    (events as dicts in start order, per-job status dicts)."""
    parts = [q for _, ps in jobs for q in ps]
    pa = (ah_sched_part * max(len(parts), 1))()
    for i, (b, sec, ov) in enumerate(parts):
        pa[i] = ah_sched_part(int(b), float(sec), int(ov), 0)
    ja = (ah_sched_job * max(len(jobs), 1))()
    at = 0
    for i, (arr, ps) in enumerate(jobs):
        ja[i] = ah_sched_job(float(arr), at, len(ps))
        at += len(ps)
    ev = (ah_sched_event * max_events)()
    n = ctypes.c_uint64()
    done = (ah_job_status * max(len(jobs), 1))()
    _check(lib().ah_sched_simulate(ja, len(jobs), pa, len(parts), int(n_lanes), int(pool_bytes),
                                   ev, max_events, ctypes.byref(n), done), "ah_sched_simulate")
    evs = [{f: getattr(ev[i], f) for f, _ in ah_sched_event._fields_} for i in range(n.value)]
    sts = [{f: getattr(done[i], f) for f, _ in ah_job_status._fields_} for i in range(len(jobs))]
    return evs, sts


def ah_last_error() -> str:
    return lib().ah_last_error().decode(errors="replace")


def ah_scan_program_source(pairs, has_nmask: bool = False) -> str:
    pp = primer_pairs(pairs)
    n = lib().ah_scan_program_source(pp, len(pp), int(has_nmask), None, 0)
    if n == 0:
        raise AhError(AH_ERR_INVALID_ARG, "ah_scan_program_source", ah_last_error())
    buf = ctypes.create_string_buffer(n)
    lib().ah_scan_program_source(pp, len(pp), int(has_nmask), buf, n)
    return buf.value.decode()


def ah_scan_program_compile(pairs, has_nmask: bool = False) -> int:
    pp = primer_pairs(pairs)
    size = ctypes.c_size_t(0)
    _check(lib().ah_scan_program_compile(pp, len(pp), int(has_nmask), ctypes.byref(size)),
           "ah_scan_program_compile")
    return int(size.value)


def ah_jit_stats():
    n, ms = ctypes.c_uint64(0), ctypes.c_double(0)
    lib().ah_jit_stats(ctypes.byref(n), ctypes.byref(ms))
    return int(n.value), float(ms.value)


def ah_release_caches():
    lib().ah_release_caches()


def ah_profile_enable(on: bool = True):
    lib().ah_profile_enable(1 if on else 0)


def ah_profile_reset():
    lib().ah_profile_reset()


def ah_profile_query(name: str):
    """(launches, total device ms) of a library kernel since the last reset."""
    n, ms = ctypes.c_uint64(0), ctypes.c_double(0)
    _check(lib().ah_profile_query(name.encode(), ctypes.byref(n), ctypes.byref(ms)),
           "ah_profile_query")
    return int(n.value), float(ms.value)


def ah_autotune_scan(genomes: ah_genomes, pairs, hits, capacity: int, res, work, stream=None,
                     repeats: int = 3):
    """Time candidate scan shapes for the set; returns ((words_per_lane,
    patterns_per_group), best ms)."""
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    t = ah_scan_tuning()
    ms = ctypes.c_double(0)
    _check(lib().ah_autotune_scan(ctypes.byref(genomes), pp, len(pp), _ptr(hits), int(capacity),
                                  _ptr(res), _ptr(work), 0 if work is None else work.numel(),
                                  _stream(stream), int(repeats), ctypes.byref(t), ctypes.byref(ms)),
           "ah_autotune_scan")
    return (int(t.words_per_lane), int(t.patterns_per_group)), float(ms.value)


def ah_set_scan_tuning(pairs, tuning=None):
    pp = primer_pairs(pairs)
    t = None if tuning is None else ctypes.byref(ah_scan_tuning(int(tuning[0]), int(tuning[1])))
    _check(lib().ah_set_scan_tuning(pp, len(pp), t), "ah_set_scan_tuning")


def ah_get_scan_tuning(pairs):
    pp = primer_pairs(pairs)
    t = ah_scan_tuning()
    _check(lib().ah_get_scan_tuning(pp, len(pp), ctypes.byref(t)), "ah_get_scan_tuning")
    return int(t.words_per_lane), int(t.patterns_per_group)


def ah_scan_prepare(pairs, has_nmask: bool = False):
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    _check(lib().ah_scan_prepare(pp, len(pp), int(has_nmask)), "ah_scan_prepare")


def prepare_many(sets, has_nmask: bool = False, threads: int = 16):
    """Compile the scan kernels of several primer sets concurrently."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    dev = torch.cuda.current_device()

    def one(ps):
        torch.cuda.set_device(dev)
        ah_scan_prepare(ps, has_nmask)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, sets))


class HostGenomes:
    """Host view of a packed collection for the streaming calls.  ``words`` and
    ``nmask`` are host tensors (pinned for overlapped copies); word_off and
    len are kept here as numpy arrays so that they outlive the call."""

    def __init__(self, words, word_off, lengths, nmask=None):
        self.words, self.nmask = words, nmask
        self.word_off = np.ascontiguousarray(word_off, dtype=np.uint64)
        self.len = np.ascontiguousarray(lengths, dtype=np.uint32)
        self.n = int(self.len.size)

    def view(self) -> ah_host_genomes:
        h = ah_host_genomes()
        h.words = _ptr(self.words)
        h.nmask = _ptr(self.nmask)
        h.word_off = self.word_off.ctypes.data
        h.len = self.len.ctypes.data if self.n else None
        h.n = self.n
        return h


def stream_config(chunk_words: int, n_slots: int = 3) -> ah_stream_config:
    c = ah_stream_config()
    c.chunk_words = int(chunk_words)
    c.n_slots = int(n_slots)
    return c


def ah_stream_workspace_bytes(hg: HostGenomes, cfg: ah_stream_config, pairs,
                              hit_capacity: int) -> int:
    pp, n = _pairs_arg(pairs)
    return int(lib().ah_stream_workspace_bytes(ctypes.byref(hg.view()), ctypes.byref(cfg), pp,
                                               int(n), int(hit_capacity)))


def ah_stream_query(hg: HostGenomes, cfg: ah_stream_config, pairs, wins, params: ah_tm_params,
                    hits, hit_capacity: int, hit_res, amp, amp_capacity: int, amp_res, work,
                    stream=None, copy_streams=()):
    pp = pairs if isinstance(pairs, ctypes.Array) else primer_pairs(pairs)
    cs = (ctypes.c_void_p * max(1, len(copy_streams)))(*[_stream(s) for s in copy_streams])
    _check(lib().ah_stream_query(ctypes.byref(hg.view()), ctypes.byref(cfg), pp, wins, len(pp),
                                 ctypes.byref(params), _ptr(hits), int(hit_capacity), _ptr(hit_res),
                                 _ptr(amp), int(amp_capacity), _ptr(amp_res), _ptr(work),
                                 0 if work is None else work.numel(), _stream(stream), cs,
                                 len(copy_streams)), "ah_stream_query")


def server_config(n_lanes: int = 4, n_compilers: int = 8, part_bases: int = 1 << 32,
                  max_part_hits: int = 1 << 25, capacity_scale: float = 2.0,
                  host_pool_bytes: int = 0) -> ah_server_config:
    return ah_server_config(int(n_lanes), int(n_compilers), int(part_bases), int(max_part_hits),
                            float(capacity_scale), int(host_pool_bytes))


def ah_server_create(genomes: ah_genomes, lengths, cfg: ah_server_config, pool) -> int:
    lens = np.ascontiguousarray(lengths, dtype=np.uint32)
    out = ctypes.c_void_p()
    _check(lib().ah_server_create(ctypes.byref(genomes), lens.ctypes.data if lens.size else None,
                                  ctypes.byref(cfg), _ptr(pool), pool.numel(), ctypes.byref(out)),
           "ah_server_create")
    return int(out.value)


def ah_server_submit(server: int, pair, genomes=None, tm: Optional[ah_tm_params] = None,
                     filter_tm: bool = False, min_tm: float = 50.0) -> int:
    job = ah_job()
    f, r = pair.fwd.encode(), pair.rev.encode()
    job.pair = ah_primer_pair(f, r, int(pair.k), int(pair.clamp), _pair_flags(pair))
    job.window = ah_window(int(pair.min_len), int(pair.max_len), 1 if filter_tm else 0,
                           float(min_tm))
    job.tm = tm if tm is not None else tm_params()
    ids = None
    if genomes is not None:
        ids = np.ascontiguousarray(genomes, dtype=np.uint32)
        job.genomes = ids.ctypes.data if ids.size else None
        job.n_genomes = ids.size
        if not ids.size:  # an empty list, not "all genomes"
            job.genomes = ctypes.cast(ctypes.pointer(ctypes.c_uint32(0)), ctypes.c_void_p).value
    jid = ctypes.c_uint64()
    _check(lib().ah_server_submit(server, ctypes.byref(job), ctypes.byref(jid)), "ah_server_submit")
    return int(jid.value)


def ah_server_wait(server: int, timeout_s: float) -> Optional[dict]:
    st = ah_job_status()
    rc = lib().ah_server_wait(server, float(timeout_s), ctypes.byref(st))
    if rc == AH_ERR_AGAIN:
        return None
    _check(rc, "ah_server_wait")
    return {name: getattr(st, name) for name, _ in ah_job_status._fields_ if name != "reserved"}


def ah_server_part(server: int, job: int, part: int) -> ah_job_part:
    out = ah_job_part()
    _check(lib().ah_server_part(server, int(job), int(part), ctypes.byref(out)), "ah_server_part")
    return out


def ah_server_release(server: int, job: int):
    _check(lib().ah_server_release(server, int(job)), "ah_server_release")


def ah_server_stats_get(server: int) -> dict:
    st = ah_server_stats()
    lib().ah_server_stats_get(server, ctypes.byref(st))
    return {name: getattr(st, name) for name, _ in ah_server_stats._fields_}


def ah_server_now(server: int) -> float:
    return float(lib().ah_server_now(server))


def ah_server_destroy(server: int):
    lib().ah_server_destroy(server)


def ah_scan_candidate_stats(work, n_genomes: int, capacity: int) -> dict:
    out = (ctypes.c_uint64 * 4)()
    _check(lib().ah_scan_candidate_stats(_ptr(work), work.numel(), int(n_genomes), int(capacity),
                                         out), "ah_scan_candidate_stats")
    return {"records": int(out[0]), "windows": int(out[1]), "full_slices": int(out[2]),
            "max_per_workgroup": int(out[3])}


def ah_scan_candidate_capacity(work_bytes: int, n_genomes: int, capacity: int,
                               base_offset: int = 0) -> int:
    """Candidate records a scan workspace of work_bytes holds (host arithmetic)."""
    return int(lib().ah_scan_candidate_capacity(int(base_offset), int(work_bytes),
                                                int(n_genomes), int(capacity)))
