"""Amplicon sequences as FASTA and amplitypes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* The tool's main output is a FASTA file of the predicted amplicon sequences
  with their coordinates, orientation and maximum Tm (Section 2.1,
  "Visualization").
* An amplitype is a genome's combination of amplicon copy numbers and
  sequence variants (Section 3.3, "Amplicon Pattern Visualization").

Readings (R23-R25):
  R23 the sequence of an amplicon [start, end) is the top strand for FR, FF
      and RR and its reverse complement for RF, so that the copies of one
      target on either strand read alike; a byte other than A/C/G/T (case
      folded) is written N.
  R24 record layout: ">g<genome>:<start>-<end> pair=<pair> orient=<label>
      tm=<tm+>,<tm->" then the sequence on one line; Tm with two decimals
      (rounded half to even on the value times 100), "nan" for a site with no
      compatible oligo.
  R25 an amplitype is the multiset of the sequences of a genome's FR and RF
      amplicons; it is compared through an order-free multiset hash: the sum
      mod 2^64 of mix(h + 0x9E3779B97F4A7C15) over the sequence hashes h,
      where h = mix(n ^ sum_k (c_k + 1) P^k mod 2^64) over the n bases c_k
      (A0 C1 G2 T3 N4), P = 0x100000001B3 and mix is the SplitMix64
      finaliser (Steele, Lea & Flood 2014).
"""
from __future__ import annotations

import math

import numpy as np

M64 = (1 << 64) - 1
P = 0x100000001B3
GOLDEN = 0x9E3779B97F4A7C15
ORIENT = ("FR", "RF", "FF", "RR")
_COMP = bytes.maketrans(b"ACGTN", b"TGCAN")
_CODE = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3, ord("N"): 4}


def mix(z: int) -> int:
    """SplitMix64 finaliser (the output function of Steele, Lea & Flood's
    SplitMix64 generator)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def clean(seq: bytes) -> bytes:
    up = bytes(seq).upper()
    return bytes(b if b in b"ACGT" else ord("N") for b in up)


def amplicon_sequence(genome: bytes, start: int, end: int, orient: int) -> bytes:
    s = clean(genome[start:end])
    return s[::-1].translate(_COMP) if orient == 1 else s


def seq_hash(s: bytes) -> int:
    h, pk = 0, 1
    for b in s:
        h = (h + (_CODE[b] + 1) * pk) & M64
        pk = (pk * P) & M64
    return mix(h ^ len(s))


def fmt_tm(v: float) -> str:
    if math.isnan(v):
        return "nan"
    r = round(v * 100)
    a = abs(r)
    return ("-" if r < 0 else "") + f"{a // 100}.{a % 100:02d}"


def records(genomes, hits: np.ndarray, amps: np.ndarray):
    """[(header, sequence, hash)] for every amplicon, in order."""
    out = []
    for a in amps:
        g, st, en, o = int(a["genome"]), int(a["start"]), int(a["end"]), int(a["orient"])
        s = amplicon_sequence(genomes[g], st, en, o)
        head = (f">g{g}:{st}-{en} pair={int(a['pair'])} orient={ORIENT[o]} "
                f"tm={fmt_tm(float(hits['tm'][a['plus_hit']]))},"
                f"{fmt_tm(float(hits['tm'][a['minus_hit']]))}")
        out.append((head, s, seq_hash(s)))
    return out


def fasta_text(recs) -> bytes:
    return b"".join(h.encode() + b"\n" + s + b"\n" for h, s, _ in recs)


def amplitypes(amps: np.ndarray, recs, n_pairs: int, n_genomes: int):
    """(multiset hash, count) per (pair, genome), index pair * n_genomes + genome."""
    hsum = [0] * (n_pairs * n_genomes)
    cnt = [0] * (n_pairs * n_genomes)
    for a, (_, _, h) in zip(amps, recs):
        if int(a["orient"]) in (0, 1):
            q = int(a["pair"]) * n_genomes + int(a["genome"])
            hsum[q] = (hsum[q] + mix(h + GOLDEN)) & M64
            cnt[q] += 1
    return hsum, cnt
