"""Binding sites of degenerate primers with at most k mismatches on both strands
(Section 2.1, "Primer matching").

The paper turns each degenerate primer into a regular expression covering all
of its oligos and up to k mismatches, and removes, after matching, sites with a
mismatch in the 3'-most ``clamp`` bases of the primer.  Because the positions
of a window are independent, "some oligo of the mixture is within Hamming
distance k of the window" is the same as "at most k window positions hold a
base outside that position's IUPAC set"; that plain definition is what
``scan_sequence`` computes.  ``brute_scan`` instead enumerates every oligo.

Readings (where the paper is silent):
  R1  a mismatch is a substitution; no insertions or deletions.
  R2  a degenerate position matches every base of its set.
  R3  every qualifying start is reported, one record per (genome, pos, strand,
      primer), with its mismatch count.
  R4  bytes other than A/C/G/T (after upper-casing) match no primer position.
  R5  each sequence is linear; windows never wrap or cross sequences.
  R6  the clamp covers the primer's 3' end: the right end of the window on
      the + strand, the left end on the - strand.
  R13 positions are 0-based; ``pos`` is the leftmost top-strand base of the
      window for both strands.
  R14 identical windows hit by the fwd and rev primer are separate records.

Patterns per pair: fwd on + (the primer as written), fwd on - (its reverse
complement), rev on +, rev on -.  Records are ordered by (pair, genome, pos,
strand, primer) with + = 0 before - = 1 and fwd = 0 before rev = 1.
"""
from __future__ import annotations

from typing import Iterable, List, Sequence, Tuple

import numpy as np

from . import iupac

HIT_DTYPE = np.dtype([("pair", np.int32), ("genome", np.int32), ("pos", np.int64),
                      ("strand", np.int8), ("primer", np.int8), ("mm", np.int16),
                      ("tm", np.float64)])

_CODE = np.full(256, 4, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _CODE[_c] = _i
    _CODE[_c + 32] = _i  # lower case

# MATCH[m, c] = 1 iff base code c (0..3) is in 4-bit set m; code 4 never matches.
MATCH = np.zeros((16, 5), dtype=np.uint8)
for _m in range(16):
    for _c in range(4):
        MATCH[_m, _c] = (_m >> _c) & 1


def codes(seq) -> np.ndarray:
    if isinstance(seq, str):
        seq = seq.encode()
    if isinstance(seq, (bytes, bytearray)):
        seq = np.frombuffer(seq, dtype=np.uint8)
    return _CODE[np.asarray(seq, dtype=np.uint8)]


def patterns(fwd: str, rev: str) -> List[Tuple[int, int, str]]:
    """(primer index, strand, pattern string in top-strand orientation)."""
    return [(0, 0, iupac.normalise(fwd)), (0, 1, iupac.revcomp(fwd)),
            (1, 0, iupac.normalise(rev)), (1, 1, iupac.revcomp(rev))]


def clamp_positions(length: int, strand: int, clamp: int) -> np.ndarray:
    c = min(clamp, length)
    return np.arange(length - c, length) if strand == 0 else np.arange(0, c)


def window_mismatches(c: np.ndarray, pattern: str) -> Tuple[np.ndarray, np.ndarray]:
    """Mismatch count and per-position match table for every window start."""
    m = iupac.masks(pattern)
    n_win = c.size - m.size + 1
    if n_win <= 0:
        return np.zeros(0, np.int64), np.zeros((m.size, 0), bool)
    match = np.empty((m.size, n_win), dtype=bool)
    for j in range(m.size):
        match[j] = MATCH[m[j], c[j:j + n_win]] != 0
    mm = m.size - match.sum(axis=0, dtype=np.int64)
    return mm, match


def scan_sequence(seq, fwd: str, rev: str, k: int, clamp: int = 0) -> np.ndarray:
    """Hits of one primer pair in one sequence (genome and pair fields 0)."""
    c = codes(seq)
    out = []
    for primer, strand, pat in patterns(fwd, rev):
        mm, match = window_mismatches(c, pat)
        if mm.size == 0:
            continue
        ok = mm <= k
        cp = clamp_positions(len(pat), strand, clamp)
        if cp.size:
            ok &= match[cp].all(axis=0)
        pos = np.flatnonzero(ok)
        rec = np.zeros(pos.size, dtype=HIT_DTYPE)
        rec["pos"] = pos
        rec["strand"] = strand
        rec["primer"] = primer
        rec["mm"] = mm[pos]
        rec["tm"] = np.nan
        out.append(rec)
    if not out:
        return np.zeros(0, dtype=HIT_DTYPE)
    return sort_hits(np.concatenate(out))


def sort_hits(h: np.ndarray) -> np.ndarray:
    order = np.lexsort((h["primer"], h["strand"], h["pos"], h["genome"], h["pair"]))
    return h[order]


def scan_collection(seqs: Sequence, pairs: Iterable) -> np.ndarray:
    """All hits of every pair (fwd, rev, k, clamp) over every sequence."""
    out = []
    for q, pr in enumerate(pairs):
        for g, s in enumerate(seqs):
            h = scan_sequence(s, pr.fwd, pr.rev, pr.k, pr.clamp)
            h["pair"] = q
            h["genome"] = g
            out.append(h)
    if not out:
        return np.zeros(0, dtype=HIT_DTYPE)
    return sort_hits(np.concatenate(out))


def brute_scan(seq, fwd: str, rev: str, k: int, clamp: int = 0) -> np.ndarray:
    """Every oligo of each primer's expansion, on both strands, compared with
    every window by plain Hamming distance; a site is kept iff some oligo is
    within k and equal to the window on the clamp positions.  Reports the
    smallest such distance.  For tiny inputs only."""
    text = bytes(np.asarray(codes(seq), dtype=np.uint8))
    n = len(text)
    best = {}
    for primer, p in enumerate((fwd, rev)):
        L = len(p)
        if n < L:
            continue
        wins = np.lib.stride_tricks.sliding_window_view(np.frombuffer(text, np.uint8), L)
        for o in iupac.expand(p):
            for strand in (0, 1):
                s = o if strand == 0 else iupac.revcomp_plain(o)
                oc = codes(s)
                diff = wins != oc[None, :]
                dist = diff.sum(axis=1)
                cp = clamp_positions(L, strand, clamp)
                clean = ~diff[:, cp].any(axis=1) if cp.size else np.ones(dist.size, bool)
                for i in np.flatnonzero((dist <= k) & clean):
                    key = (int(i), strand, primer)
                    d = int(dist[i])
                    if key not in best or d < best[key]:
                        best[key] = d
    rec = np.zeros(len(best), dtype=HIT_DTYPE)
    for r, ((i, strand, primer), d) in enumerate(sorted(best.items())):
        rec[r] = (0, 0, i, strand, primer, d, np.nan)
    return sort_hits(rec)
