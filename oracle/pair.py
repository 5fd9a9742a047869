"""Amplicon calling (Section 2.1, "Amplicon calling"; "Amplicon analysis" item 1).

Sites that passed the clamp and melting-temperature filters are paired when
they lie on opposite strands and the region between them is within the
user's amplicon-length range; every such region is reported, and each
amplicon is labelled by the primers at its two ends: FR (fwd on +, rev on -),
RF (rev on +, fwd on -), FF or RR (the same primer at both ends, off-target).

Readings:
  R10 with the filter on, a site is kept iff its maximum Tm >= min_tm.
  R11 all (+, -) site pairs in the window are reported, FF and RR included.
  R12 an amplicon spans [start, end) with start = pos of the + site and
      end = pos of the - site + that primer's length; its length end - start
      must lie in [min_len, max_len] (bounds inclusive).
Amplicons are ordered by (pair, genome, start, end, orient) with the orient
codes FR = 0, RF = 1, FF = 2, RR = 3.
"""
from __future__ import annotations

import numpy as np

AMP_DTYPE = np.dtype([("pair", np.int32), ("genome", np.int32), ("start", np.int64),
                      ("end", np.int64), ("orient", np.int8), ("plus_hit", np.int64),
                      ("minus_hit", np.int64)])

FR, RF, FF, RR = 0, 1, 2, 3
_ORIENT = {(0, 1): FR, (1, 0): RF, (0, 0): FF, (1, 1): RR}
ORIENT_NAMES = ("FR", "RF", "FF", "RR")


def call_amplicons(hits: np.ndarray, pairs, filter_tm: bool = False,
                   min_tm: float = 50.0) -> np.ndarray:
    """All amplicons from a canonically ordered hit table.  ``plus_hit`` and
    ``minus_hit`` index into ``hits``."""
    out = []
    keep = np.ones(hits.size, bool)
    if filter_tm:
        keep = hits["tm"] >= min_tm
    idx = np.flatnonzero(keep)
    h = hits[idx]
    for q, pr in enumerate(pairs):
        plen = (len(pr.fwd), len(pr.rev))
        sel_q = h["pair"] == q
        for g in np.unique(h["genome"][sel_q]):
            sel = sel_q & (h["genome"] == g)
            plus = np.flatnonzero(sel & (h["strand"] == 0))
            minus = np.flatnonzero(sel & (h["strand"] == 1))
            bpos = h["pos"][minus].astype(np.int64)
            bend = bpos + np.where(h["primer"][minus] == 0, plen[0], plen[1])
            for a in plus:
                start = int(h["pos"][a])
                length = bend - start
                ok = np.flatnonzero((length >= pr.min_len) & (length <= pr.max_len))
                ap = int(h["primer"][a])
                for j in ok:
                    b = minus[j]
                    out.append((q, int(g), start, int(bend[j]),
                                _ORIENT[(ap, int(h["primer"][b]))], int(idx[a]), int(idx[b])))
    amp = np.array(out, dtype=AMP_DTYPE) if out else np.zeros(0, AMP_DTYPE)
    order = np.lexsort((amp["orient"], amp["end"], amp["start"], amp["genome"], amp["pair"]))
    return amp[order]
