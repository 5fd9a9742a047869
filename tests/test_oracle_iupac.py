"""Pins for the IUPAC primer model of the oracle (degeneracy counts printed in
the paper, complement algebra, expansion order)."""
import itertools
import os

import pytest

from oracle import iupac

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def paper_primers():
    rows = []
    for line in open(os.path.join(GOLDEN, "paper_primers.tsv")):
        if line.startswith("#") or not line.strip():
            continue
        name, fwd, rev, amp = line.rstrip("\n").split("\t")
        rows.append((name, fwd, rev, int(amp)))
    return rows


def test_titan_total_is_960_as_stated_in_the_paper():
    rows = {r[0]: r for r in paper_primers()}
    _, fwd, rev, _ = rows["Titan"]
    assert iupac.degeneracy(fwd) + iupac.degeneracy(rev) == 960
    assert (iupac.degeneracy(fwd), iupac.degeneracy(rev)) == (576, 384)
    assert len(iupac.expand(fwd)) == 576 and len(set(iupac.expand(fwd))) == 576


@pytest.mark.parametrize("name,fwd_deg,rev_deg", [("V3V4", 16, 16), ("V1V9", 16, 4),
                                                   ("Titan", 576, 384), ("mecA", 1, 1)])
def test_paper_pair_degeneracies(name, fwd_deg, rev_deg):
    rows = {r[0]: r for r in paper_primers()}
    _, fwd, rev, _ = rows[name]
    assert iupac.degeneracy(fwd) == fwd_deg
    assert iupac.degeneracy(rev) == rev_deg


def test_complement_is_an_involution_and_maps_sets():
    for c, s in iupac.SETS.items():
        cc = iupac.complement_code(c)
        assert iupac.complement_code(cc) == c
        assert sorted(iupac.SETS[cc]) == sorted(iupac.BASE_COMP[b] for b in s)
    assert [iupac.complement_code(c) for c in "RYKMBVDHSWN"] == list("YRMKVBHDSWN")


def test_revcomp_expands_to_reverse_complements():
    for p in ("AGRRTTYGATYHTDGYTYAG", "YCNTTCCYTYDYRGTACT", "ACGTN", "BDHV"):
        a = sorted(iupac.revcomp_plain(o) for o in iupac.expand(p))
        b = sorted(iupac.expand(iupac.revcomp(p)))
        assert a == b
        assert iupac.revcomp(iupac.revcomp(p)) == p


def test_expansion_order_is_mixed_radix_5prime_slowest():
    assert iupac.expand("RY") == ["AC", "AT", "GC", "GT"]
    assert iupac.expand("NA")[:4] == ["AA", "CA", "GA", "TA"]
    p = "ANGRT"
    want = ["".join(t) for t in itertools.product("A", "ACGT", "G", "AG", "T")]
    assert iupac.expand(p) == want


def test_invalid_codes_are_rejected_and_case_is_folded():
    with pytest.raises(iupac.PrimerError):
        iupac.normalise("ACGU")
    with pytest.raises(iupac.PrimerError):
        iupac.normalise("AC-G")
    assert iupac.normalise("acgtn") == "ACGTN"


def test_code_sets_follow_the_nomenclature_table():
    for line in open(os.path.join(GOLDEN, "iupac_codes.tsv")):
        if line.startswith("#") or not line.strip():
            continue
        code, bases = line.split()
        assert sorted(iupac.members(code)) == sorted(bases)
        assert iupac.mask(code) == sum(1 << "ACGT".index(b) for b in bases)
    assert set(iupac.members("N")) == set("ACGT")
    assert set(iupac.members("R")) == set("AG")
