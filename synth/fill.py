"""CPU realisation of a plan: ASCII bytes of each genome (numpy).

Per base i of genome g (source id s): u = top 32 bits of draw(S_BASES|s, i);
the base is A, C, G or T as u falls below the genome's first, second or third
cumulative threshold, else T.  Planted copies then overwrite their span: the
template (reverse-complemented for strand 1) with each offset o substituted
when the top 32 bits of draw(S_MUT|copy, o) fall below T_MUT, the replacement
being the ((low 32 bits * 3) >> 32)-th of the three other bases in ACGT order.
Runs of 'N' are written last.
"""
from __future__ import annotations

import numpy as np

from . import rng
from .plan import BASES, T_MUT, Plan

_LUT = np.frombuffer(BASES, dtype=np.uint8)
_COMP = np.zeros(256, dtype=np.uint8)
for _a, _b in zip(b"ACGT", b"TGCA"):
    _COMP[_a] = _b
_CODE = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _CODE[_c] = _i


def oriented_template(plan: Plan, tid: int, strand: int) -> np.ndarray:
    t = np.frombuffer(plan.templates[tid], dtype=np.uint8)
    return _COMP[t[::-1]] if strand else t.copy()


def mutated_copy(plan: Plan, copy_index: int) -> np.ndarray:
    """Bytes written by planted copy ``copy_index`` (index into the plan arrays)."""
    cid = int(plan.copy_ids()[copy_index])
    t = oriented_template(plan, int(plan.plant_template[copy_index]),
                          int(plan.plant_strand[copy_index]))
    m = rng.draws(rng.stream_key(plan.seed, rng.S_MUT | cid), np.arange(t.size))
    hit = (m >> np.uint64(32)) < np.uint64(T_MUT)
    if np.any(hit):
        orig = _CODE[t[hit]].astype(np.int64)
        choice = (((m[hit] & np.uint64(0xFFFFFFFF)) * np.uint64(3)) >> np.uint64(32)).astype(np.int64)
        repl = choice + (choice >= orig)  # skip the original base
        t = t.copy()
        t[hit] = _LUT[repl]
    return t


def genome_bytes(plan: Plan, g: int) -> np.ndarray:
    plan.check()
    n = int(plan.lengths[g])
    key = rng.stream_key(plan.seed, rng.S_BASES | plan.source_id(g))
    u = (rng.draws(key, np.arange(n)) >> np.uint64(32)).astype(np.uint32)
    th = plan.thresholds[g]
    code = (u >= th[0]).astype(np.uint8) + (u >= th[1]) + (u >= th[2])
    seq = _LUT[code]
    for c in np.flatnonzero(plan.plant_genome == g):
        t = mutated_copy(plan, int(c))
        p = int(plan.plant_pos[c])
        seq[p:p + t.size] = t
    for r in np.flatnonzero(plan.nrun_genome == g):
        p, ln = int(plan.nrun_pos[r]), int(plan.nrun_len[r])
        seq[p:p + ln] = ord("N")
    return seq


def genome_range_bytes(plan: Plan, g: int, lo: int, hi: int) -> np.ndarray:
    """Bytes [lo, hi) of genome ``g``, equal to ``genome_bytes(plan, g)[lo:hi]``
    without building the whole genome (for genomes of billions of bases)."""
    plan.check()
    n = int(plan.lengths[g])
    lo, hi = max(0, int(lo)), min(n, int(hi))
    key = rng.stream_key(plan.seed, rng.S_BASES | plan.source_id(g))
    u = (rng.draws(key, np.arange(lo, hi, dtype=np.int64)) >> np.uint64(32)).astype(np.uint32)
    th = plan.thresholds[g]
    code = (u >= th[0]).astype(np.uint8) + (u >= th[1]) + (u >= th[2])
    seq = _LUT[code]
    for c in np.flatnonzero(plan.plant_genome == g):
        p = int(plan.plant_pos[c])
        t = mutated_copy(plan, int(c))
        a, b = max(p, lo), min(p + t.size, hi)
        if a < b:
            seq[a - lo:b - lo] = t[a - p:b - p]
    for r in np.flatnonzero(plan.nrun_genome == g):
        p, ln = int(plan.nrun_pos[r]), int(plan.nrun_len[r])
        a, b = max(p, lo), min(p + ln, hi)
        if a < b:
            seq[a - lo:b - lo] = ord("N")
    return seq


def collection_bytes(plan: Plan) -> np.ndarray:
    """All genomes concatenated (offsets from ``plan.offsets``)."""
    out = np.empty(plan.total_bp, dtype=np.uint8)
    off = plan.offsets
    for g in range(plan.n):
        out[off[g]:off[g + 1]] = genome_bytes(plan, g)
    return out


def genome_str(plan: Plan, g: int) -> str:
    return genome_bytes(plan, g).tobytes().decode()
