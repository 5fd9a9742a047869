"""Pins for the oracle's nearest-neighbour melting temperature: hand-derived
perfect-duplex sums and temperatures, the mismatch-zero reading on hand-worked
duplexes, strand symmetry, monotonicity, the unit of the salt term, and the
maximum over compatible oligos against brute force."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import iupac, scan, tm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rows(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        out.append(line.rstrip("\n").split("\t"))
    return out


@pytest.mark.parametrize("row", rows("nn_perfect_duplex.tsv"), ids=lambda r: r[0])
def test_perfect_duplex_sums_and_tm_match_hand_derivation(row):
    oligo, selfcomp, dh10, ds10, salt, tm_c = row
    o = scan.codes(oligo)
    dh, ds = tm.duplex_terms(o, np.ones((1, o.size), bool))
    sym = tm.SYM_DS if selfcomp == "1" else 0.0
    assert round(float(dh[0]) * 10) == int(dh10)
    assert round((float(ds[0]) + sym) * 10) == int(ds10)
    p = tm.TmParams(selfcomp=selfcomp == "1")
    assert tm.salt_entropy(p, len(oligo)) == pytest.approx(float(salt), abs=2e-5)
    assert tm.tm_perfect(oligo, p) == pytest.approx(float(tm_c), abs=5e-4)


@pytest.mark.parametrize("row", rows("nn_mismatch_mm0.tsv"), ids=lambda r: r[1])
def test_mismatch_zero_reading_matches_hand_derivation(row):
    oligo, opp, dh10, ds10 = row
    o, t = scan.codes(oligo), scan.codes(opp)
    paired = (o == 3 - t)[None, :]
    dh, ds = tm.duplex_terms(o, paired)
    assert round(float(dh[0]) * 10) == int(dh10)
    assert round(float(ds[0]) * 10) == int(ds10)


def test_every_stack_value_is_reached_through_a_duplex():
    # 2-mers: one stack + two initiations; checks the table and its indexing
    for a, b in itertools.product("ACGT", repeat=2):
        dh, ds = tm.duplex_terms(scan.codes(a + b), np.ones((1, 2), bool))
        h, s = tm.NN_UNIFIED[a + b]
        ih = sum(tm.INIT_GC[0] if x in "GC" else tm.INIT_AT[0] for x in (a, b))
        i_s = sum(tm.INIT_GC[1] if x in "GC" else tm.INIT_AT[1] for x in (a, b))
        assert float(dh[0]) == pytest.approx(h + ih)
        assert float(ds[0]) == pytest.approx(s + i_s)


def test_perfect_duplex_tm_is_strand_symmetric():
    rs = np.random.RandomState(1)
    for _ in range(200):
        o = "".join(rs.choice(list("ACGT"), size=rs.randint(5, 33)))
        assert tm.tm_perfect(o) == pytest.approx(tm.tm_perfect(iupac.revcomp_plain(o)), abs=1e-9)


def test_salt_term_vanishes_at_one_molar_and_tm_is_monotone():
    o = "AGCTTGCAAGGCTTACCGTA"
    p1 = tm.TmParams(Na=1000.0, Mg=0.0)
    assert tm.salt_entropy(p1, len(o)) == pytest.approx(0.0, abs=1e-12)
    assert tm.tm_perfect(o, p1) == pytest.approx(tm.tm_perfect(o, tm.TmParams(Na=1000, Mg=0, saltcorr=0)))
    prev = -1e9
    for na in (10, 20, 50, 100, 200, 500):
        t = tm.tm_perfect(o, tm.TmParams(Na=na, Mg=0.0))
        assert t > prev
        prev = t
    prev = -1e9
    for c in (10, 50, 250, 1000, 5000):
        t = tm.tm_perfect(o, tm.TmParams(dnac1=c))
        assert t > prev
        prev = t
    # Mg at or below dNTPs contributes nothing to the sodium equivalent
    assert tm.sodium_equivalent(tm.TmParams(Na=50, Mg=1.0, dNTPs=1.5)) == 50.0
    assert tm.sodium_equivalent(tm.TmParams(Na=50, K=10, Tris=20, Mg=0)) == 70.0


def test_concentration_term():
    assert tm.concentration(tm.TmParams(dnac1=250, dnac2=0)) == pytest.approx(250e-9)
    assert tm.concentration(tm.TmParams(dnac1=250, dnac2=100)) == pytest.approx(200e-9)
    assert tm.concentration(tm.TmParams(dnac1=100, dnac2=250)) == pytest.approx(200e-9)
    assert tm.concentration(tm.TmParams(dnac1=250, dnac2=100, selfcomp=True)) == pytest.approx(250e-9)


def test_site_tm_of_nondegenerate_exact_site_is_the_perfect_duplex():
    rs = np.random.RandomState(4)
    for _ in range(30):
        o = "".join(rs.choice(list("ACGT"), size=rs.randint(8, 30)))
        g = "GATTACA" + o + "CCGG"
        c = scan.codes(g)
        assert tm.site_tm(c, 7, o, 0, 0, 0) == pytest.approx(tm.tm_perfect(o), abs=1e-9)
        g2 = "TT" + iupac.revcomp_plain(o) + "A"
        c2 = scan.codes(g2)
        assert tm.site_tm(c2, 2, o, 1, 0, 0) == pytest.approx(tm.tm_perfect(o), abs=1e-9)


def test_terminal_mismatch_equals_shorter_duplex_with_full_length_salt():
    o = "GCGTACGATCCAGTAGCATC"
    opp = "".join(iupac.BASE_COMP[b] for b in o)
    bad = opp[:-1] + ("A" if opp[-1] != "A" else "C")
    p = tm.TmParams()
    got = tm.tm_duplex(o, bad, p)
    s = scan.codes(o[:-1])
    dh, ds = tm.duplex_terms(s, np.ones((1, s.size), bool))
    want = 1000 * dh[0] / (ds[0] + tm.salt_entropy(p, len(o)) + tm.R_GAS * math.log(250e-9)) - 273.15
    assert got == pytest.approx(want, abs=1e-9)


def brute_site_tm(g, pos, primer, strand, k, clamp, p):
    L = len(primer)
    w = g[pos:pos + L]
    best = float("nan")
    for o in iupac.expand(primer):
        s = o if strand == 0 else iupac.revcomp_plain(o)
        d = sum(1 for a, b in zip(s, w) if a != b)
        c = min(clamp, L)
        cl = range(L - c, L) if strand == 0 else range(0, c)
        if d > k or any(s[j] != w[j] for j in cl):
            continue
        if strand == 0:
            opp = "".join(iupac.BASE_COMP.get(b, "N") for b in w)
        else:
            opp = w[::-1]
        t = tm.tm_duplex(o, opp, p)
        best = t if math.isnan(best) else max(best, t)
    return best


@pytest.mark.parametrize("seed", range(10))
def test_site_tm_is_the_maximum_over_compatible_oligos(seed):
    rs = np.random.RandomState(100 + seed)
    L = rs.randint(8, 16)
    primer = list("".join(rs.choice(list("ACGT"), size=L)))
    for j in rs.choice(L, size=3, replace=False):
        primer[j] = rs.choice(list("RYNDW"))
    primer = "".join(primer)
    k = rs.randint(0, 4)
    clamp = rs.randint(0, 4)
    g = "".join(rs.choice(list("ACGT"), size=400))
    o = iupac.expand(primer)[rs.randint(iupac.degeneracy(primer))]
    g = g[:100] + o + g[100 + L:200] + iupac.revcomp_plain(o) + g[200 + L:]
    c = scan.codes(g)
    h = scan.scan_sequence(g, primer, primer, k, clamp)
    p = tm.TmParams()
    assert h.size >= 2
    for r in h:
        got = tm.site_tm(c, int(r["pos"]), primer, int(r["strand"]), k, clamp, p)
        want = brute_site_tm(g, int(r["pos"]), primer, int(r["strand"]), k, clamp, p)
        assert got == pytest.approx(want, abs=1e-9)
