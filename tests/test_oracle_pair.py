"""Pins for the oracle's amplicon calling: planted amplicons are found with
their exact lengths and FR/RF labels, primer swap relabels, reverse complement
mirrors coordinates, and window bounds are inclusive."""
import numpy as np

from oracle import iupac, pair, scan, tm
from synth import fill, plan


def _amps(seq, pr):
    h = scan.scan_sequence(seq, pr.fwd, pr.rev, pr.k, pr.clamp)
    return h, pair.call_amplicons(h, [pr])


def test_planted_amplicons_have_exact_span_and_orientation():
    p = plan.tiny(31, n_genomes=3, len_lo=3000, len_hi=8000, n_copies=(1, 3))
    pr = p.pairs[0]
    f0, r0, _ = p.template_sites[0]
    tl = len(p.templates[0])
    span = r0 + len(pr.rev) - f0
    seen = 0
    for g in range(p.n):
        seq = fill.genome_bytes(p, g)
        _, a = _amps(seq, pr)
        got = {(int(x["start"]), int(x["end"]), int(x["orient"])) for x in a}
        for c in np.flatnonzero(p.plant_genome == g):
            base = int(p.plant_pos[c])
            if p.plant_strand[c] == 0:
                want = (base + f0, base + f0 + span, pair.FR)
            else:
                want = (base + tl - r0 - len(pr.rev), base + tl - r0 - len(pr.rev) + span, pair.RF)
            # planted sites carry 1% mutations; count only copies whose two
            # sites survived within k
            h = scan.scan_sequence(seq, pr.fwd, pr.rev, pr.k, pr.clamp)
            pos = {(int(r["pos"]), int(r["strand"])) for r in h}
            ends_ok = ((want[0], 0) in pos) and ((want[1] - len(pr.rev if want[2] == pair.FR else pr.fwd), 1) in pos)
            if ends_ok:
                assert want in got
                seen += 1
    assert seen >= 2


def test_primer_swap_relabels_orientations():
    rs = np.random.RandomState(2)
    seq = "".join(rs.choice(list("ACGT"), size=30000))
    fwd, rev = "ACGTAC", "GGTACT"
    P = plan.PairSpec(fwd, rev, k=1, clamp=0, min_len=50, max_len=3000)
    Q = plan.PairSpec(rev, fwd, k=1, clamp=0, min_len=50, max_len=3000)
    _, a = _amps(seq, P)
    _, b = _amps(seq, Q)
    swap = {pair.FR: pair.RF, pair.RF: pair.FR, pair.FF: pair.RR, pair.RR: pair.FF}
    ta = sorted((int(x["start"]), int(x["end"]), swap[int(x["orient"])]) for x in a)
    tb = sorted((int(x["start"]), int(x["end"]), int(x["orient"])) for x in b)
    assert ta == tb and len(ta) > 20
    assert {int(x["orient"]) for x in a} == {0, 1, 2, 3}


def test_reverse_complement_mirrors_amplicons():
    rs = np.random.RandomState(7)
    seq = "".join(rs.choice(list("ACGT"), size=20000))
    P = plan.PairSpec("ACGTAC", "GGTACA", k=1, clamp=1, min_len=40, max_len=2500)
    _, a = _amps(seq, P)
    _, b = _amps(iupac.revcomp_plain(seq), P)
    n = len(seq)
    flip = {pair.FR: pair.RF, pair.RF: pair.FR, pair.FF: pair.FF, pair.RR: pair.RR}
    ta = sorted((n - int(x["end"]), n - int(x["start"]), flip[int(x["orient"])]) for x in a)
    tb = sorted((int(x["start"]), int(x["end"]), int(x["orient"])) for x in b)
    assert ta == tb and len(ta) > 10


def test_window_bounds_are_inclusive_and_all_pairs_reported():
    fwd, rev = "AACCGGT", "TTGGCCA"  # rev's reverse complement is TGGCCAA
    mid = "G" * 30
    seq = "C" * 5 + fwd + mid + iupac.revcomp_plain(rev) + mid + iupac.revcomp_plain(rev) + "C" * 5
    h = scan.scan_sequence(seq, fwd, rev, 0, 0)
    L = len(fwd)
    first = L + 30 + L
    second = first + 30 + L
    for lo, hi, want in ((first, second, 2), (first + 1, second, 1), (first, second - 1, 1),
                         (first, first, 1)):
        a = pair.call_amplicons(h, [plan.PairSpec(fwd, rev, 0, 0, lo, hi)])
        assert sum(int(x["orient"]) == pair.FR for x in a) == want


def test_tm_filter_drops_sites_below_threshold():
    p = plan.tiny(41, n_genomes=2, len_lo=3000, len_hi=5000, n_copies=(2, 3))
    pr = p.pairs[0]
    seqs = [fill.genome_bytes(p, g) for g in range(p.n)]
    h = scan.scan_collection(seqs, [pr])
    h = tm.fill_tm(h, seqs, [pr])
    a_all = pair.call_amplicons(h, [pr])
    thr = float(np.median(h["tm"]))
    a_f = pair.call_amplicons(h, [pr], filter_tm=True, min_tm=thr)
    for x in a_f:
        assert h["tm"][x["plus_hit"]] >= thr and h["tm"][x["minus_hit"]] >= thr
    n_want = sum(1 for x in a_all if h["tm"][x["plus_hit"]] >= thr and h["tm"][x["minus_hit"]] >= thr)
    assert a_f.size == n_want
