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


# the default conditions (method 5), every other salt method, and method 7 in
# each of its regimes (R = sqrt[Mg] / [Mon]
# in the middle, >= 6, < 0.22, with dNTPs, without monovalent ions)
SALT_CASES = [dict()] + [dict(saltcorr=m) for m in (0, 1, 2, 3, 4, 6, 7)] + [
    dict(saltcorr=7, Na=10.0, Mg=10.0), dict(saltcorr=7, Na=200.0, Mg=0.5),
    dict(saltcorr=7, Na=50.0, Mg=3.0, dNTPs=0.8), dict(saltcorr=7, Na=0.0, Mg=2.0)]


# ten seeds under the default conditions, three under every other salt case
MAX_CASES = [(seed, 0) for seed in range(10)] + [
    (seed, case) for case in range(1, len(SALT_CASES)) for seed in range(3)]


@pytest.mark.parametrize("seed,case", MAX_CASES)
def test_site_tm_is_the_maximum_over_compatible_oligos(seed, case):
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
    p = tm.TmParams(**SALT_CASES[case])
    assert h.size >= 2
    for r in h:
        got = tm.site_tm(c, int(r["pos"]), primer, int(r["strand"]), k, clamp, p)
        want = brute_site_tm(g, int(r["pos"]), primer, int(r["strand"]), k, clamp, p)
        assert got == pytest.approx(want, abs=1e-9)


OLIGOS = ["AGCTTGCAAGGCTTACCGTA", "GGGCCCGCGGCCGC", "ATATTAATTATAAATTA", "CAGTCAGTCAGT"]


def test_salt_methods_reduce_to_the_one_molar_reference():
    # 1 M monovalent ions and no magnesium is the reference state the methods
    # correct from: methods 1, 3, 4, 5, 6 and 7 leave Tm unchanged there
    for o in OLIGOS:
        t0 = tm.tm_perfect(o, tm.TmParams(Na=1000.0, Mg=0.0, saltcorr=0))
        for m in (1, 3, 4, 5, 6, 7):
            t = tm.tm_perfect(o, tm.TmParams(Na=1000.0, Mg=0.0, saltcorr=m))
            assert t == pytest.approx(t0, abs=1e-9), m
        # Wetmur's form keeps a term at 1 M but tends to Schildkraut-Lifson
        # at low salt
        a = tm.tm_perfect(o, tm.TmParams(Na=1000.0, Mg=0.0, saltcorr=2))
        assert abs(a - t0) > 1.0
        lo1 = tm.tm_perfect(o, tm.TmParams(Na=1e-3, Mg=0.0, saltcorr=1))
        lo2 = tm.tm_perfect(o, tm.TmParams(Na=1e-3, Mg=0.0, saltcorr=2))
        assert abs(lo1 - lo2) < 1e-4


def test_methods_1_to_4_shift_every_oligo_alike():
    shifts = []
    for m in (1, 2, 3, 4):
        p = tm.TmParams(Na=30.0, K=5.0, Mg=1.0, saltcorr=m)
        p0 = tm.TmParams(Na=30.0, K=5.0, Mg=1.0, saltcorr=0)
        d = [tm.tm_perfect(o, p) - tm.tm_perfect(o, p0) for o in OLIGOS]
        assert max(d) - min(d) < 1e-9 and d[0] < 0  # below 1 M: lower Tm
        shifts.append(d[0])
    # four different published corrections
    assert min(abs(a - b) for i, a in enumerate(shifts) for b in shifts[i + 1:]) > 0.1


def test_owczarzy_corrections_add_to_the_reciprocal_kelvin_temperature():
    # methods 6 and 7 add a + b fGC to 1/T (T in kelvin): the same amount for
    # duplexes of equal length and G+C whatever their 1 M stability
    o1, o2 = "AGCTTGCAAGGCTTACCGTA", "ATGCGTCAAGCATGTCAGCA"
    assert len(o1) == len(o2) and tm.gc_count(tm.codes(o1))[0] == tm.gc_count(tm.codes(o2))[0]
    p1 = tm.TmParams(Na=1000.0, Mg=0.0, saltcorr=0)
    assert abs(tm.tm_perfect(o1, p1) - tm.tm_perfect(o2, p1)) > 1.0
    for kw in (dict(saltcorr=6), dict(saltcorr=7), dict(saltcorr=7, Na=10.0, Mg=10.0)):
        d = [1.0 / (tm.tm_perfect(o, tm.TmParams(**kw)) + 273.15) -
             1.0 / (tm.tm_perfect(o, tm.TmParams(Na=1000.0, Mg=0.0, saltcorr=0, dnac1=250.0))
                    + 273.15) for o in (o1, o2)]
        assert abs(d[0] - d[1]) < 1e-12 and abs(d[0]) > 1e-6, kw


def test_method_7_without_magnesium_is_method_6_on_the_monovalent_ions():
    for kw in (dict(Na=50.0, K=10.0, Tris=20.0), dict(Na=150.0), dict(Na=5.0, K=1.0)):
        for o in OLIGOS:
            t7 = tm.tm_perfect(o, tm.TmParams(Mg=0.0, saltcorr=7, **kw))
            t6 = tm.tm_perfect(o, tm.TmParams(Mg=0.0, saltcorr=6, **kw))
            assert t7 == pytest.approx(t6, abs=1e-9)
    # and at R < 0.22 the magnesium is ignored
    o = OLIGOS[0]
    a = tm.tm_perfect(o, tm.TmParams(Na=200.0, Mg=0.5, saltcorr=7))
    b = tm.tm_perfect(o, tm.TmParams(Na=200.0, Mg=0.0, saltcorr=7))
    assert a == pytest.approx(b, abs=1e-9)
    # from sqrt[Mg] / [Mon] = 0.22 on, the magnesium counts (0.32 and 0.77 here)
    for na, mg in ((100.0, 1.0), (50.0, 1.5)):
        c = tm.tm_perfect(o, tm.TmParams(Na=na, Mg=mg, saltcorr=7))
        d = tm.tm_perfect(o, tm.TmParams(Na=na, Mg=0.0, saltcorr=7))
        assert abs(c - d) > 0.1, (na, mg)


def test_free_magnesium_satisfies_mass_action():
    for mg, dn in [(1.5, 0.8), (3.0, 3.0), (2.0, 10.0), (0.5, 0.1), (10.0, 0.2)]:
        x = tm.free_magnesium(tm.TmParams(Mg=mg, dNTPs=dn)) * 1e-3
        M, D = mg * 1e-3, dn * 1e-3
        bound = M - x
        assert 0 < x <= M and D - bound >= 0
        # 1:1 complexes: [MgdNTP] = Ka [Mg][dNTP], Ka = 3e4 per M
        assert bound == pytest.approx(3e4 * x * (D - bound), rel=1e-9)
    assert tm.free_magnesium(tm.TmParams(Mg=1.5, dNTPs=0.0)) == 1.5
    assert tm.free_magnesium(tm.TmParams(Mg=0.0, dNTPs=0.8)) == 0.0


def test_gc_dependent_methods_favour_gc_at_unpaired_positions():
    # two oligos that pair the template alike and differ only at a mismatched
    # position (G against A): equal under methods 0-5; under 6 and 7 below
    # 1 M the G+C-richer duplex is the more stable
    opp = "".join(iupac.BASE_COMP[b] for b in "AGCTTGCAAGGCTTACCGTA")
    o_g = "AGCTTGCAAGGCTGACCGTA"
    o_a = "AGCTTGCAAGGCTAACCGTA"
    assert opp[13] == "A"  # opposite the T of the exact complement
    for m in range(6):
        p = tm.TmParams(saltcorr=m)
        assert tm.tm_duplex(o_g, opp, p) == pytest.approx(tm.tm_duplex(o_a, opp, p), abs=1e-9)
    for m in (6, 7):
        p = tm.TmParams(saltcorr=m)
        assert tm.tm_duplex(o_g, opp, p) > tm.tm_duplex(o_a, opp, p) + 1e-3


def test_salt_method_arguments_are_checked():
    with pytest.raises(ValueError):
        tm.tm_perfect("ACGTACGT", tm.TmParams(saltcorr=8))
    with pytest.raises(ValueError):
        tm.tm_perfect("ACGTACGT", tm.TmParams(Na=0.0, Mg=0.0, saltcorr=6))
    with pytest.raises(ValueError):
        tm.tm_perfect("ACGTACGT", tm.TmParams(Na=0.0, Mg=0.0, saltcorr=7))


# salt methods whose Tm depends on the pairing alone (all but 6 and 7)
PAIRING_CASES = [c for c in SALT_CASES if c.get("saltcorr", 5) not in (6, 7)]


@pytest.mark.parametrize("seed", range(12))
def test_site_tm_by_pairing_equals_the_oligo_maximum(seed):
    """The maximum over sets of paired positions equals the maximum over the
    oligos themselves (site_tm, pinned on brute force above) at every
    position and strand of a genome with planted sites and non-ACGT bases,
    for primers with many degenerate positions, k up to 6 and a clamp."""
    rs = np.random.RandomState(700 + seed)
    L = rs.randint(8, 15)
    primer = list(rs.choice(list("ACGT"), size=L))
    for j in rs.choice(L, size=rs.randint(3, 7), replace=False):
        primer[j] = rs.choice(list("RYSWKMBDHVN"))
    primer = "".join(primer)
    k = int(rs.randint(0, 7))
    clamp = int(rs.randint(0, 3))
    g = list("".join(rs.choice(list("ACGT"), size=300)))
    o = iupac.expand(primer)[rs.randint(iupac.degeneracy(primer))]
    g[40:40 + L] = o
    g[150:150 + L] = iupac.revcomp_plain(o)
    g[230:230 + L] = iupac.revcomp_plain(o)
    g[230 + rs.randint(L)] = "N"
    g = "".join(g)
    c = scan.codes(g)
    p = tm.TmParams(**PAIRING_CASES[seed % len(PAIRING_CASES)])
    finite = 0
    for pos in range(0, len(g) - L + 1):
        for strand in (0, 1):
            got = tm.site_tm_by_pairing(c, pos, primer, strand, k, clamp, p)
            want = tm.site_tm(c, pos, primer, strand, k, clamp, p)
            if math.isnan(want):
                assert math.isnan(got)
            else:
                finite += 1
                assert got == pytest.approx(want, abs=1e-9)
    assert finite >= 2


def test_site_tm_by_pairing_small_cases_against_brute_force():
    g = "TTGACGTAGCCATGNAGCTAGGCATTACGGATCCAT"
    c = scan.codes(g)
    for primer, k, clamp in (("ACGTAGCCATG", 3, 1), ("RCGYAGSCWTG", 4, 0), ("NNGTAGCCAKG", 5, 2)):
        for case in PAIRING_CASES[:4]:
            p = tm.TmParams(**case)
            for pos in range(len(g) - len(primer) + 1):
                for strand in (0, 1):
                    got = tm.site_tm_by_pairing(c, pos, primer, strand, k, clamp, p)
                    want = brute_site_tm(g, pos, primer, strand, k, clamp, p)
                    assert (math.isnan(got) and math.isnan(want)) or \
                        got == pytest.approx(want, abs=1e-9)


def test_site_tm_by_pairing_refuses_the_gc_dependent_methods():
    c = scan.codes("ACGTACGTAC")
    for m in (6, 7):
        with pytest.raises(ValueError):
            tm.site_tm_by_pairing(c, 0, "ACGTACGTAC", 0, 1, 0, tm.TmParams(saltcorr=m))
