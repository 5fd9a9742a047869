"""Pins for the oracle's decoy run (Section 2.1, "Amplicon analysis": decoys
made by reversing the genome sequences): reversal is an involution that
turns a real run into a decoy run, the forward-frame records are the sites
of the primers' position-wise complements on the genomes as given (the
identity a same-pass decoy scan rests on), and a perfect decoy site of a
plain primer has the closed-form Tm."""
import dataclasses

import numpy as np

from oracle import decoy, iupac, pair, scan, tm
from synth import fill, plan


def _real(seqs, pairs):
    h = scan.scan_collection(seqs, pairs)
    h = tm.fill_tm(h, seqs, pairs)
    return h, pair.call_amplicons(h, pairs)


def _collection(seed):
    p = plan.tiny(seed, n_genomes=3, len_lo=2000, len_hi=6000, n_copies=(1, 3))
    return p, [fill.genome_bytes(p, g) for g in range(p.n)]


def _same(x, y, fields):
    assert x.size == y.size
    for f in fields:
        if x[f].dtype.kind == "f":
            assert np.array_equal(x[f], y[f], equal_nan=True), f
        else:
            assert np.array_equal(x[f].astype(np.int64), y[f].astype(np.int64)), f


def test_decoy_of_reversed_genomes_is_the_real_run():
    p, seqs = _collection(41)
    h0, a0 = _real(seqs, p.pairs)
    assert a0.size > 0
    h1, a1 = decoy.run(decoy.reversed_genomes(seqs), p.pairs)
    _same(h1, h0, ("pair", "genome", "pos", "strand", "primer", "mm", "tm"))
    _same(a1, a0, ("pair", "genome", "start", "end", "orient", "plus_hit", "minus_hit"))
    # reversing is not reverse-complementing: the decoy of the genomes as
    # given differs from their real run
    hd, _ = decoy.run(seqs, p.pairs)
    assert not (hd.size == h0.size and np.array_equal(hd["pos"], h0["pos"]))


def test_forward_frame_is_the_scan_of_the_complement_primers():
    p, seqs = _collection(43)
    # the decoy of genomes holding the targets reversed finds them
    rseqs = decoy.reversed_genomes(seqs)
    pairs = p.pairs + [dataclasses.replace(p.pairs[0], k=3, clamp=2)]
    h, a = decoy.run(rseqs, pairs)
    f, g = decoy.to_forward_frame(h, a, p.lengths, pairs)
    assert g.size > 0
    comp = [dataclasses.replace(pr, fwd="".join(iupac.complement_code(c) for c in pr.fwd),
                                rev="".join(iupac.complement_code(c) for c in pr.rev))
            for pr in pairs]
    hc = scan.scan_collection(rseqs, comp)
    _same(f, hc, ("pair", "genome", "pos", "strand", "primer", "mm"))
    ac = pair.call_amplicons(hc, comp)
    # both pairs form amplicons (the second with a clamp and k 3)
    assert set(np.unique(ac["pair"]).tolist()) == {0, 1}
    _same(g, ac, ("pair", "genome", "start", "end", "orient", "plus_hit", "minus_hit"))
    # FR and RF exchange labels, lengths are kept
    assert sorted((a["end"] - a["start"]).tolist()) == sorted((g["end"] - g["start"]).tolist())
    n_fr = int((a["orient"] == pair.FR).sum())
    assert n_fr == int((g["orient"] == pair.RF).sum())


def test_perfect_decoy_site_has_the_closed_form_tm():
    primer = "GATTACAGGCTTACGTACGA"
    rev = "TTGCAGGTACCATGCATAGC"
    pr = plan.PairSpec(primer, rev, k=1, clamp=0, min_len=30, max_len=200)
    rs = np.random.RandomState(5)
    body = "".join(rs.choice(list("ACGT"), size=300))
    # the primer reversed, as it would lie in the genome if the reversed
    # genome held the primer itself
    seq = (body[:100] + primer[::-1] + body[100:]).encode()
    h, _ = decoy.run([seq], [pr])
    sel = (h["mm"] == 0) & (h["primer"] == 0) & (h["strand"] == 0)
    assert sel.sum() == 1
    n = len(seq)
    assert int(h["pos"][sel][0]) == n - 100 - len(primer)
    assert abs(float(h["tm"][sel][0]) - tm.tm_perfect(primer)) < 1e-9
    f, _ = decoy.to_forward_frame(h, np.zeros(0, pair.AMP_DTYPE), [n], [pr])
    k = (f["mm"] == 0) & (f["primer"] == 0)
    assert int(f["pos"][k][0]) == 100 and int(f["strand"][k][0]) == 1
