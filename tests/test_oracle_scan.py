"""Pins for the oracle's site scan: brute force over every oligo expansion,
textbook special cases, reverse-complement and primer-swap symmetry, and the
planted ground truth of the generator."""
import numpy as np
import pytest

from oracle import iupac, scan
from synth import fill, plan

ACGT = "ACGT"


def rand_seq(rs, n, alphabet=ACGT):
    return "".join(rs.choice(list(alphabet), size=n))


def rand_primer(rs, n, n_deg, codes="RYSWKMBDHVN"):
    s = list(rand_seq(rs, n))
    for j in rs.choice(n, size=min(n_deg, n), replace=False):
        s[j] = rs.choice(list(codes))
    return "".join(s)


def as_tuples(h):
    return [(int(r["pos"]), int(r["strand"]), int(r["primer"]), int(r["mm"])) for r in h]


@pytest.mark.parametrize("seed", range(24))
def test_mask_scan_equals_brute_force_over_every_oligo(seed):
    rs = np.random.RandomState(seed)
    L1, L2 = rs.randint(5, 13), rs.randint(5, 13)
    fwd = rand_primer(rs, L1, rs.randint(0, 4))
    rev = rand_primer(rs, L2, rs.randint(0, 4))
    while iupac.degeneracy(fwd) > 64:
        fwd = rand_primer(rs, L1, 2)
    while iupac.degeneracy(rev) > 64:
        rev = rand_primer(rs, L2, 2)
    k = rs.randint(0, 4)
    clamp = [0, 1, 5, max(L1, L2)][seed % 4]
    n = rs.randint(1, 700)
    # low-complexity text with a planted near-site so hits exist
    seq = list(rand_seq(rs, n, "ACGT" if seed % 3 else "AACGTN"))
    o = iupac.expand(fwd)[0]
    if n > L1 + 10:
        p0 = rs.randint(0, n - L1)
        seq[p0:p0 + L1] = list(o)
    seq = "".join(seq)
    a = scan.scan_sequence(seq, fwd, rev, k, clamp)
    b = scan.brute_scan(seq, fwd, rev, k, clamp)
    assert as_tuples(a) == as_tuples(b)


def test_nondegenerate_k0_equals_exact_substring_occurrences():
    rs = np.random.RandomState(5)
    seq = rand_seq(rs, 20000, "AC")  # low complexity: many occurrences
    fwd, rev = "ACCA", "CAAC"
    fwd, rev = "ACCAC", "CAACA"
    h = scan.scan_sequence(seq, fwd, rev, 0, 0)
    want = set()
    for primer, p in enumerate((fwd, rev)):
        for strand, pat in enumerate((p, iupac.revcomp_plain(p))):
            i = seq.find(pat)
            while i >= 0:
                want.add((i, strand, primer, 0))
                i = seq.find(pat, i + 1)
    assert set(as_tuples(h)) == want and len(want) > 100


def test_full_clamp_equals_k0_and_zero_clamp_equals_no_clamp():
    rs = np.random.RandomState(11)
    seq = rand_seq(rs, 5000)
    fwd, rev = rand_primer(rs, 8, 2), rand_primer(rs, 7, 2)
    full = scan.scan_sequence(seq, fwd, rev, 3, clamp=max(len(fwd), len(rev)))
    exact = scan.scan_sequence(seq, fwd, rev, 0, 0)
    assert as_tuples(full) == as_tuples(exact)
    a = scan.scan_sequence(seq, fwd, rev, 2, clamp=0)
    b = scan.brute_scan(seq, fwd, rev, 2, 0)
    assert as_tuples(a) == as_tuples(b)


def test_hits_grow_with_k_and_with_superset_codes():
    rs = np.random.RandomState(3)
    seq = rand_seq(rs, 8000)
    fwd, rev = rand_primer(rs, 9, 1), rand_primer(rs, 10, 1)
    prev = None
    for k in range(5):
        h = {t[:3]: t[3] for t in as_tuples(scan.scan_sequence(seq, fwd, rev, k, 2))}
        if prev is not None:
            assert set(prev) <= set(h)
            assert all(h[key] == prev[key] for key in prev)
        prev = h
    # replacing a code by a superset (here N) only adds sites and lowers mm
    j = 4
    fwd_n = fwd[:j] + "N" + fwd[j + 1:]
    base = {t[:3]: t[3] for t in as_tuples(scan.scan_sequence(seq, fwd, rev, 2, 0))}
    sup = {t[:3]: t[3] for t in as_tuples(scan.scan_sequence(seq, fwd_n, rev, 2, 0))}
    assert set(base) <= set(sup)
    assert all(sup[key] <= base[key] for key in base)


def test_reverse_complement_symmetry():
    rs = np.random.RandomState(8)
    seq = rand_seq(rs, 6000)
    fwd, rev = rand_primer(rs, 11, 3), rand_primer(rs, 9, 2)
    n = len(seq)
    for clamp in (0, 3):
        a = scan.scan_sequence(seq, fwd, rev, 3, clamp)
        b = scan.scan_sequence(iupac.revcomp_plain(seq), fwd, rev, 3, clamp)
        L = (len(fwd), len(rev))
        mapped = sorted((n - L[p] - i, 1 - s, p, mm) for i, s, p, mm in as_tuples(a))
        assert mapped == as_tuples(b)


def test_non_acgt_bytes_match_nothing_and_case_is_folded():
    seq = "ACGTNACGTRACGT"
    h = scan.scan_sequence(seq, "ACGT", "NNNNN", 0, 0)
    got = set(as_tuples(h))
    assert (0, 0, 0, 0) in got and (5, 0, 0, 0) in got and (10, 0, 0, 0) in got
    # every 5-window of NNNNN touching the N or the R is a mismatch
    assert not any(t[2] == 1 and t[0] <= 4 <= t[0] + 4 for t in got)
    assert as_tuples(scan.scan_sequence(seq.lower(), "ACGT", "NNNNN", 0, 0)) == as_tuples(h)


def test_short_and_empty_sequences():
    assert scan.scan_sequence("", "ACGTA", "ACGTA", 1, 0).size == 0
    assert scan.scan_sequence("ACGT", "ACGTA", "ACGTA", 1, 0).size == 0
    h = scan.scan_sequence("ACGTA", "ACGTA", "ACGTA", 0, 0)
    assert as_tuples(h) == [(0, 0, 0, 0), (0, 0, 1, 0)]


def _planted_truth(p, g, seq_codes):
    """Expected (pos, strand, primer) of every planted primer site of genome g
    and its mismatch count by set membership."""
    out = []
    for c in np.flatnonzero(p.plant_genome == g):
        tid = int(p.plant_template[c])
        f0, r0, q = p.template_sites[tid]
        pr = p.pairs[q]
        tl = len(p.templates[tid])
        lf, lr = len(pr.fwd), len(pr.rev)
        base = int(p.plant_pos[c])
        if p.plant_strand[c] == 0:
            sites = [(base + f0, 0, 0, pr.fwd), (base + r0, 1, 1, iupac.revcomp(pr.rev))]
        else:
            sites = [(base + tl - f0 - lf, 1, 0, iupac.revcomp(pr.fwd)),
                     (base + tl - r0 - lr, 0, 1, pr.rev)]
        for pos, strand, primer, pat in sites:
            m = iupac.masks(pat)
            w = seq_codes[pos:pos + len(pat)]
            mm = int(sum(1 for j in range(len(pat)) if not (w[j] < 4 and (m[j] >> w[j]) & 1)))
            out.append((pos, strand, primer, mm, pat))
    return out


def test_planted_sites_are_found_with_their_mismatch_counts():
    p = plan.tiny(21, n_genomes=4, len_lo=2000, len_hi=6000, n_copies=(1, 3))
    pr = p.pairs[0]
    found = 0
    for g in range(p.n):
        seq = fill.genome_bytes(p, g)
        c = scan.codes(seq)
        h = {t[:3]: t[3] for t in as_tuples(scan.scan_sequence(seq, pr.fwd, pr.rev, pr.k, pr.clamp))}
        for pos, strand, primer, mm, pat in _planted_truth(p, g, c):
            if mm <= pr.k:
                assert h[(pos, strand, primer)] == mm
                found += 1
    assert found >= 2


def test_plain_workload_planted_sites():
    p = plan.plain()
    seq = fill.genome_bytes(p, 0)
    pr = p.pairs[0]
    h = {t[:3]: t[3] for t in as_tuples(scan.scan_sequence(seq, pr.fwd, pr.rev, pr.k, pr.clamp))}
    c = scan.codes(seq)
    truth = _planted_truth(p, 0, c)
    assert len(truth) == 10
    for pos, strand, primer, mm, pat in truth:
        cp = scan.clamp_positions(len(pat), strand, pr.clamp)
        m = iupac.masks(pat)
        clean = all((m[j] >> c[pos + j]) & 1 for j in cp)
        if mm <= pr.k and clean:
            assert h[(pos, strand, primer)] == mm


@pytest.mark.parametrize("seed", range(4))
def test_planted_sites_of_primers_using_every_code(seed):
    """Sites realised by the generator (its own member table) from primers that
    contain every IUPAC code are found exactly (k = 0 after removing mutated
    copies is too strict, so mismatch counts are checked instead)."""
    codes = "RYSWKMBDHVN"
    fwd = plan.random_primer(900 + seed, 0, 24, codes[: 6 + seed])
    rev = plan.random_primer(900 + seed, 1, 22, codes[::-1][: 5 + seed])
    pr = plan.PairSpec(fwd, rev, k=3, clamp=2, min_len=60, max_len=900)
    p = plan.tiny(700 + seed, n_genomes=3, len_lo=3000, len_hi=5000, pair=pr,
                  n_copies=(2, 3))
    found = 0
    for g in range(p.n):
        seq = fill.genome_bytes(p, g)
        c = scan.codes(seq)
        h = {t[:3]: t[3] for t in as_tuples(scan.scan_sequence(seq, fwd, rev, pr.k, 0))}
        for pos, strand, primer, mm, pat in _planted_truth(p, g, c):
            # the generator realises sites from its own member table; an
            # unmutated planted site therefore has mismatch count 0
            if mm <= pr.k:
                assert h[(pos, strand, primer)] == mm
                found += 1
    assert found >= 4
