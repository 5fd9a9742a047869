"""CPU-side checks of libah: the library loads and exports every symbol its
headers declare, host-side layout and validation behave as documented, and
the per-primer-set scan programs compile for gfx950 (no GPU needed)."""
import glob
import os
import re

import numpy as np
import pytest

from paper_2509_13300_amd import _lib as L
from synth import plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"\b(ah_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert {"ah_pack_genomes", "ah_scan_primers", "ah_pair_amplicons", "ah_tm"} <= names
    lib = L.lib()
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.EXPORTS) == names


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="not built"):
        L.lib()


def test_pack_layout():
    lens = np.array([0, 1, 31, 32, 33, 5_000_000], dtype=np.uint64)
    off = L.ah_pack_layout(lens)
    S = (lens + 31) // 32
    want = np.concatenate([[0], np.cumsum((S + 32) // 2 * 2)])
    assert off.tolist() == want.tolist()


@pytest.mark.parametrize("fwd,rev,k,clamp,status", [
    ("ACGTACGTAC", "GGGGCCCCAA", 2, 0, L.AH_OK),
    ("acgtnnRYKM", "BDHVSWacgt", 15, 10, L.AH_OK),
    ("ACGU", "ACGTACGT", 1, 0, L.AH_ERR_LIMIT),          # too short first
    ("ACGUACGTAC", "ACGTACGT", 1, 0, L.AH_ERR_INVALID_PRIMER),
    ("ACGTA-GTAC", "ACGTACGT", 1, 0, L.AH_ERR_INVALID_PRIMER),
    ("A" * 33, "ACGTACGT", 1, 0, L.AH_ERR_LIMIT),
    ("A" * 32, "ACGTACGT", 1, 0, L.AH_OK),
    ("ACGTACGTAC", "ACGTACGT", 16, 0, L.AH_ERR_LIMIT),
    ("ACGTACGTAC", "ACGTACGT", 2, 9, L.AH_ERR_LIMIT),
    ("ACGTACGTAC", "ACGTACGT", 2, 8, L.AH_OK),
])
def test_primer_validation(fwd, rev, k, clamp, status):
    assert L.ah_validate_pairs([(fwd, rev, k, clamp)]) == status
    if status != L.AH_OK:
        assert L.ah_last_error()


def _functions(src, i):
    body = src.split("---- generated pattern program follows ----")[1]
    pf = body.split(f"u32 ah_pf_{i}(")[1].split("\n}\n")[0]
    ex = body.split(f"u32 ah_ex_{i}(")[1].split("\n}\n")[0]
    return pf, ex


def _positions(text):
    return {int(m) for m in re.findall(r"\bp[acgthlx]\[(\d+)\]", text)}


def test_generated_program_tests_every_non_n_position():
    src = L.ah_scan_program_source([("ACGTNRYSWKMBDHV", "NNNNNAAAAC", 1, 2)])
    pf, ex = _functions(src, 0)
    # the exact count tests every position but the N, the clamp ones into cf
    assert ex.count("ah_valid(c, t, 15u)") == 1
    assert ex.count("x = ") == 15 - 1
    assert ex.count("cf |= x") == 2
    # the filter reads every non-N position, the two clamp ones (13, 14) into
    # the clamp chain
    assert _positions(pf) == set(range(15)) - {4}
    clamp = {int(m) for ln in pf.splitlines() if ln.strip().startswith(("u32 cl", "cl ="))
             for m in re.findall(r"\[(\d+)\]", ln)}
    assert clamp == {13, 14}
    # a specific primer gets pigeonhole blocks over exactly its free positions
    src = L.ah_scan_program_source([("ACGTACCGATNGCATTGGCAKT", "GGATCCAAGTTCGACGT", 2, 3)])
    body = src.split("---- generated pattern program follows ----")[1]
    assert re.search(r"pattern 0: .*prefilter: [123] of [345] blocks", body)
    pf, _ = _functions(src, 0)
    blocks = {int(m) for ln in pf.splitlines() if re.match(r"\s+(u32 )?k\d+ =", ln)
              for m in re.findall(r"\[(\d+)\]", ln)}
    assert blocks == set(range(19)) - {10}
    clamp = {int(m) for ln in pf.splitlines() if ln.strip().startswith(("u32 cl", "cl ="))
             for m in re.findall(r"\[(\d+)\]", ln)}
    assert clamp == {19, 20, 21}


def test_prefilter_can_be_switched_off(monkeypatch):
    monkeypatch.setenv("AH_SCAN_PREFILTER", "0")
    src = L.ah_scan_program_source([("ACGTACGTACGTAC", "GGTTCCAAGGTTC", 2, 0)])
    assert "pattern 0: pair 0 primer 0 strand 0, L 14, k 2, exact count" in src
    monkeypatch.setenv("AH_SCAN_PREFILTER", "1")
    src = L.ah_scan_program_source([("ACGTACGTACGTAC", "GGTTCCAAGGTTC", 2, 0)])
    assert re.search(r"pattern 0: .*prefilter: [23] of [45] blocks", src)


def test_tile_mode_count_inside_the_filter_only_for_small_programs(monkeypatch):
    """Wave mode (primers up to U + 1 bases) counts in the filter anyway; in
    tile mode the filter takes the exact count for up to 16 patterns (4
    pairs) and leaves it to a launch of its own for more."""
    def macro(src, name):
        return int(re.search(r"#define %s (\d+)" % name, src).group(1))

    short = ("ACGTACGTACGTAC", "GGTTCCAAGGTTC", 2, 0)
    long_ = ("GCCGCWATGCGGCTWAGCCGCWTAGCGCWT", "GCGGCWTGCCGCWAGCGGCWTGCGCWAGCG", 3, 0)
    src = L.ah_scan_program_source([short])
    assert (macro(src, "AH_WAVE"), macro(src, "AH_TILE_COUNT")) == (1, 0)
    src = L.ah_scan_program_source([long_])
    assert (macro(src, "AH_WAVE"), macro(src, "AH_TILE_COUNT")) == (0, 1)
    src = L.ah_scan_program_source([long_] * 4)
    assert (macro(src, "AH_WAVE"), macro(src, "AH_TILE_COUNT")) == (0, 1)
    src = L.ah_scan_program_source([long_] * 5)
    assert (macro(src, "AH_WAVE"), macro(src, "AH_TILE_COUNT")) == (0, 0)
    monkeypatch.setenv("AH_SCAN_WAVE", "0")
    src = L.ah_scan_program_source([short])
    assert (macro(src, "AH_WAVE"), macro(src, "AH_TILE_COUNT")) == (0, 1)


@pytest.mark.parametrize("n_pairs", [1, 5])
def test_tile_mode_programs_compile_with_and_without_the_count(n_pairs):
    long_ = ("GCCGCWATGCGGCTWAGCCGCWTAGCGCWT", "GCGGCWTGCCGCWAGCGGCWTGCGCWAGCG", 3, 0)
    assert L.ah_scan_program_compile([long_] * n_pairs, has_nmask=n_pairs > 1) > 1000


@pytest.mark.parametrize("seed", range(6))
def test_generated_programs_compile_for_gfx950(seed):
    rs = np.random.RandomState(seed)
    pairs = plan.law_pairs(1000 + seed, 2)
    for p in pairs:
        p.clamp = int(rs.randint(0, 6))
    size = L.ah_scan_program_compile(pairs, has_nmask=bool(seed % 2))
    assert size > 1000


@pytest.mark.parametrize("n_genomes", [1, 1000, 100_000])
@pytest.mark.parametrize("capacity", [0, 1, 5000, 1 << 20, 10_000_000])
def test_workspace_of_a_size_holds_the_list_it_was_sized_for(n_genomes, capacity):
    """A scan run with `capacity` needs at least max(capacity, 2^16) candidate
    records (an overflow's `required` is sized so that a rerun with it as the
    capacity keeps every workgroup's candidates); the minimum workspace for
    that capacity must hold them, whatever its alignment, and the
    recommended one at least as many."""
    g = L.ah_genomes()
    g.n = n_genomes
    g.max_len = 4_000_000
    need = max(capacity, 1 << 16)
    minimum = L.ah_scan_workspace_bytes(g, 1, capacity)
    recommended = L.ah_scan_workspace_bytes(
        g, [("GCMCCTGGYAAACTGTTGG", "AAAGACGTATGACGATCWNA", 2, 0)], capacity)
    assert recommended >= minimum
    for off in (0, 8, 128, 255):
        assert L.ah_scan_candidate_capacity(minimum, n_genomes, capacity, off) >= need
        assert L.ah_scan_candidate_capacity(recommended, n_genomes, capacity, off) >= need
    # and a little less than the minimum holds fewer (the size is tight)
    assert L.ah_scan_candidate_capacity(minimum - 600, n_genomes, capacity) < need


def test_decoy_pair_scans_the_complement_primers():
    """A decoy pair's scan program is that of the position-wise complement
    primers as an ordinary pair (reverse(G) read for P is G read for the
    complement of P); unknown flags are rejected."""
    from oracle import iupac

    fwd, rev = "GCMCCTGGYAAACTGTTGG", "AAAGACGTATGACGATCWNA"
    comp = lambda s: "".join(iupac.complement_code(c) for c in s)  # noqa: E731
    for k, clamp in ((2, 0), (3, 4)):
        dec = L.ah_scan_program_source([(fwd, rev, k, clamp, L.AH_PAIR_DECOY)])
        plain = L.ah_scan_program_source([(comp(fwd), comp(rev), k, clamp)])
        assert dec == plain
        assert dec != L.ah_scan_program_source([(fwd, rev, k, clamp)])
    assert L.ah_validate_pairs([(fwd, rev, 2, 0, 2)]) == L.AH_ERR_INVALID_ARG
    assert L.ah_validate_pairs([(fwd, rev, 2, 0, L.AH_PAIR_DECOY)]) == L.AH_OK


def test_tm_salt_method_arguments_are_checked_before_any_device_work():
    """ah_tm rejects unknown salt methods and ion sets a method cannot use
    (no genomes, no device memory: the checks come first)."""
    import ctypes

    g = L.ah_genomes(None, None, None, None, 0, 1)
    pp = L.primer_pairs([("ACGTACGTAC", "GGCCAATTGG", 1, 0)])
    nres = ctypes.create_string_buffer(32)  # never read on these paths
    bad = [dict(saltcorr=8), dict(saltcorr=-1), dict(Na=0.0, Mg=0.0, saltcorr=6),
           dict(Na=0.0, Mg=0.0, saltcorr=1), dict(Na=0.0, Mg=0.0, saltcorr=7),
           dict(Na=0.0, Mg=1.0, dNTPs=2.0, saltcorr=5)]
    for kw in bad:
        tp = L.tm_params(**kw)
        st = L.lib().ah_tm(ctypes.byref(g), pp, len(pp), ctypes.byref(tp), None,
                           ctypes.addressof(nres), 0, None)
        assert st == L.AH_ERR_INVALID_ARG, kw
        assert "salt" in L.lib().ah_last_error().decode()


def test_pack_layout_takes_genomes_up_to_two_to_the_32_bases():
    top = (1 << 32) - 1  # positions and lengths are 32-bit
    off = L.ah_pack_layout([top, 5])
    words = (top + 31) // 32
    assert int(off[1]) == (words + 31 + 1) // 2 * 2 and int(off[1]) % 2 == 0
    with pytest.raises(L.AhError, match="2\\^32 - 1"):
        L.ah_pack_layout([10, 1 << 32])


def _golden_rows(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    with open(path) as f:
        return [ln.rstrip("\n").split("\t") for ln in f if ln.strip() and not ln.startswith("#")]


_SALT_CONDITIONS = [
    dict(saltcorr=0), dict(saltcorr=1), dict(saltcorr=2), dict(saltcorr=3), dict(saltcorr=4),
    dict(saltcorr=5), dict(saltcorr=6), dict(saltcorr=7),
    dict(saltcorr=7, Na=20.0, K=30.0, Tris=10.0, Mg=3.0, dNTPs=0.8),
    dict(saltcorr=5, dnac1=500.0, dnac2=200.0, K=5.0, Tris=2.0, dNTPs=2.0),
    dict(saltcorr=6, Na=1000.0, Mg=0.0),
]


def test_tm_duplex_matches_the_golden_perfect_duplexes():
    from oracle import tm as otm
    for oligo, selfcomp, _dh, _ds, _salt, tm_c in _golden_rows("nn_perfect_duplex.tsv"):
        opp = "".join("TGCA"["ACGT".index(b)] for b in oligo)
        got = L.ah_tm_duplex(oligo, opp, L.tm_params(selfcomp=selfcomp == "1"))
        assert abs(got - float(tm_c)) < 5e-5, (oligo, got, tm_c)
        want = otm.tm_duplex(oligo, opp, otm.TmParams(selfcomp=selfcomp == "1"))
        assert abs(got - want) < 1e-9


def test_tm_duplex_mismatch_rows_follow_the_hand_derived_sums():
    # Tm from the golden (Delta-H, Delta-S) tenths under the default
    # conditions, written out here from the published closed form
    import math
    for oligo, opp, dh_t, ds_t in _golden_rows("nn_mismatch_mm0.tsv"):
        na = (50.0 + 120.0 * math.sqrt(1.5)) / 1000.0
        ds = int(ds_t) / 10.0 + 0.368 * (len(oligo) - 1) * math.log(na)
        want = 1000.0 * (int(dh_t) / 10.0) / (ds + 1.987 * math.log(250e-9)) - 273.15
        got = L.ah_tm_duplex(oligo, opp, L.tm_params())
        assert abs(got - want) < 1e-9, (oligo, opp, got, want)


@pytest.mark.parametrize("cond", range(len(_SALT_CONDITIONS)))
def test_tm_duplex_matches_the_oracle_on_random_duplexes(cond):
    from oracle import tm as otm
    kw = _SALT_CONDITIONS[cond]
    rng = np.random.default_rng(1000 + cond)
    params = L.tm_params(**kw)
    op = otm.TmParams(**{k: v for k, v in kw.items()})
    comp = {"A": "T", "C": "G", "G": "C", "T": "A"}
    worst = 0.0
    for trial in range(300):
        n = int(rng.integers(2, 41))
        oligo = "".join(rng.choice(list("ACGT"), n))
        opp = [comp[b] for b in oligo]
        for j in rng.choice(n, int(rng.integers(0, min(n, 6) + 1)), replace=False):
            opp[j] = str(rng.choice(list("ACGTN")))  # a mismatch, an N or the same pair
        opp = "".join(opp)
        if trial % 7 == 0:
            oligo = oligo.lower()
        got = L.ah_tm_duplex(oligo, opp, params)
        want = otm.tm_duplex(oligo.upper(), opp, op)
        worst = max(worst, abs(got - want))
    assert worst <= 1e-9, worst


def test_tm_duplex_checks_its_arguments():
    p = L.tm_params()
    with pytest.raises(L.AhError) as e:
        L.ah_tm_duplex("ACGT", "TGC", p)
    assert e.value.status == L.AH_ERR_INVALID_ARG
    with pytest.raises(L.AhError) as e:
        L.ah_tm_duplex("ACNT", "TGCA", p)
    assert e.value.status == L.AH_ERR_INVALID_PRIMER
    with pytest.raises(L.AhError) as e:
        L.ah_tm_duplex("A", "T", p)
    assert e.value.status == L.AH_ERR_LIMIT
    with pytest.raises(L.AhError) as e:
        L.ah_tm_duplex("ACGT", "TGCA", L.tm_params(saltcorr=8))
    assert e.value.status == L.AH_ERR_INVALID_ARG
    with pytest.raises(L.AhError) as e:
        L.ah_tm_duplex("ACGT", "TGCA", L.tm_params(Na=0.0, Mg=0.0))
    assert e.value.status == L.AH_ERR_INVALID_ARG


def _distinct_pairings_brute_force(primer: str, k: int, clamp: int) -> int:
    """Distinct sets of paired positions over the compatible oligos of a
    site whose template base lies in every position's set (the worst case):
    every oligo of the expansion, paired where it carries the template base."""
    import itertools
    from oracle import iupac
    sets = [iupac.members(c) for c in primer]
    site = [s[0] for s in sets]  # template base in every set
    L_ = len(primer)
    seen = set()
    for oligo in itertools.product(*sets):
        paired = tuple(o == t for o, t in zip(oligo, site))
        if L_ - sum(paired) <= k and all(paired[L_ - clamp:]):
            seen.add(paired)
    return len(seen)


@pytest.mark.parametrize("primer,k,clamp", [
    ("ACGRYTACGNACSW", 2, 0), ("ACGRYTACGNACSW", 3, 2), ("RYKMSWACGT", 10, 0),
    ("NNNNACGTAC", 1, 0), ("ACGTACGTAR", 2, 1), ("ACGTACGTAC", 3, 0),
])
def test_tm_pairing_bound_counts_the_distinct_pairings(primer, k, clamp):
    """The bound ah_tm enforces is the number of distinct paired-position
    sets, counted here by brute force over the oligo expansion."""
    import math
    nd = sum(1 for j, c in enumerate(primer) if c not in "ACGT" and j < len(primer) - clamp)
    formula = sum(math.comb(nd, e) for e in range(min(k, nd) + 1))
    assert _distinct_pairings_brute_force(primer, k, clamp) == formula


def test_tm_requests_above_the_pairing_bound_take_the_exact_route_or_are_refused():
    tp = L.tm_params()
    fwd20 = "RYKMSWRYKMSWRYKMSWRY"  # 20 two-fold codes: degeneracy 2^20
    rev = "ACGTACGTACGTACGTACGT"
    # sum_{e <= 6} C(20, e) = 60,460 pairings: enumerated; e <= 7: 137,980,
    # above the bound: the exact route under methods 0-5
    assert L.ah_validate_tm([(fwd20, rev, 6, 0)], tp) == L.AH_OK
    for m in (0, 1, 2, 3, 4, 5):
        assert L.ah_validate_tm([(fwd20, rev, 7, 0)], L.tm_params(saltcorr=m)) == L.AH_OK
    # methods 6 and 7 depend on the G+C count as well: refused above the bound
    for m in (6, 7):
        assert L.ah_validate_tm([(fwd20, rev, 6, 0)], L.tm_params(saltcorr=m)) == L.AH_OK
        assert L.ah_validate_tm([(fwd20, rev, 7, 0)], L.tm_params(saltcorr=m)) == L.AH_ERR_LIMIT
        assert "pairings" in L.ah_last_error() and "G+C" in L.ah_last_error()
    # a clamp over degenerate positions removes them from the count
    assert L.ah_validate_tm([(fwd20, rev, 7, 4)], L.tm_params(saltcorr=6)) == L.AH_OK
    # the exact route needs every pairing's denominator negative: R ln C
    # + salt entropy below -8.2 (two A.T initiations); C = 0.1 M is above
    hot = L.tm_params(saltcorr=0, dnac1=1e8)
    assert L.ah_validate_tm([(fwd20, rev, 6, 0)], hot) == L.AH_OK
    assert L.ah_validate_tm([(fwd20, rev, 7, 0)], hot) == L.AH_ERR_LIMIT
    assert "exact route" in L.ah_last_error()
    # degeneracy alone is no limit: 4^11 oligos, one pairing per site at k = 0
    assert L.ah_validate_tm([("N" * 11, rev, 0, 0)], tp) == L.AH_OK
    assert L.ah_validate_tm([("N" * 32, rev, 15, 0)], tp) == L.AH_OK
    assert L.ah_validate_tm([("ACGTACGTAC", rev, 2, 0)], L.tm_params(saltcorr=9)) == \
        L.AH_ERR_INVALID_ARG
