"""Decoy estimate of off-target amplification (Section 2.1, "Amplicon
analysis": amplicons called on decoys made by reversing the genome sequences).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The decoy run is the whole analysis -- sites, melting temperatures, amplicons
-- on every genome reversed (not reverse-complemented), written here exactly
so: the genomes are reversed and the plain oracle runs on them.  Records come
out in the reversed genomes' own coordinates.  ``to_forward_frame`` restates
them in the coordinates of the genomes as given, which is how a run that
scans the decoy in the same pass as the real primers reports them:

* a site at pos p on strand s of a reversed genome of n bases covers
  [n - p - L, n - p) of the genome as given, and is reported there on strand
  1 - s (its window, read forwards, is the primer's position-wise complement
  on strand 0 and the primer reversed on strand 1);
* an amplicon [a, b) becomes [n - b, n - a); its + and - sites exchange roles
  (the reversed genome's - site is now the left end), so FR and RF exchange
  labels while FF and RR stay.

Readings: the paper gives no further detail of the decoy run; it is taken to
use the same primers, k, clamp, melting-temperature conditions, filter and
window as the real run (R22).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import pair as opair
from . import scan as oscan
from . import tm as otm


def reversed_genomes(seqs: Sequence) -> list:
    return [bytes(s)[::-1] for s in seqs]


def run(seqs: Sequence, pairs, p: otm.TmParams = otm.TmParams(), filter_tm: bool = False,
        min_tm: float = 50.0):
    """Hits (with Tm) and amplicons of every pair on the reversed genomes, in
    their own coordinates and canonical order."""
    rs = reversed_genomes(seqs)
    h = oscan.scan_collection(rs, pairs)
    h = otm.fill_tm(h, rs, pairs, p)
    return h, opair.call_amplicons(h, pairs, filter_tm, min_tm)


_SWAP = np.array([opair.RF, opair.FR, opair.FF, opair.RR], dtype=np.int8)


def to_forward_frame(h: np.ndarray, a: np.ndarray, lengths, pairs):
    """The records of ``run`` in the coordinates of the genomes as given,
    re-sorted into canonical order (hit indices of the amplicons follow)."""
    n = np.asarray(lengths, dtype=np.int64)[h["genome"]]
    plen = np.array([[len(pr.fwd), len(pr.rev)] for pr in pairs], dtype=np.int64)
    L = plen[h["pair"], h["primer"]]
    f = h.copy()
    f["pos"] = n - h["pos"].astype(np.int64) - L
    f["strand"] = 1 - h["strand"]
    order = np.lexsort((f["primer"], f["strand"], f["pos"], f["genome"], f["pair"]))
    f = f[order]
    where = np.empty(order.size, dtype=np.int64)
    where[order] = np.arange(order.size)
    g = a.copy()
    na = np.asarray(lengths, dtype=np.int64)[a["genome"]]
    g["start"] = na - a["end"]
    g["end"] = na - a["start"]
    g["orient"] = _SWAP[a["orient"]]
    g["plus_hit"] = where[a["minus_hit"]]
    g["minus_hit"] = where[a["plus_hit"]]
    g = g[np.lexsort((g["orient"], g["end"], g["start"], g["genome"], g["pair"]))]
    return f, g
