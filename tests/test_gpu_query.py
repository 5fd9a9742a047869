"""ah_query (scan, Tm and pairing in one call) gives the same bytes as the
three separate calls, on both of its tails: per segment (pair, genome) --
sorted in registers, in LDS, or through global memory for a segment longer
than LDS holds -- and, past the segment limit, for pairs expected to give
long segments, or when asked (AH_QUERY_SEGMENTED=0), the radix sort with the
Tm computed inside its first pass and the pairing's chunk counts inside its
last."""
import numpy as np
import pytest

from gpu_util import say
from synth import gpu, plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def _both(p, pairs, dev, hit_cap=1 << 16, amp_cap=1 << 16, nmask=None, **kw):
    import torch

    from paper_2509_13300_amd import path

    if nmask is None:
        nmask = p.nrun_genome.size > 0
    ascii, off = gpu.fill_cuda(p, dev)
    coll, _ = path.pack(ascii, off, p.lengths, with_nmask=nmask)
    out = []
    for fused in (False, True):
        buf = path.alloc(coll, pairs, hit_cap, amp_cap, dev)
        buf.hits.fill_(0x5A)  # different stale contents for the two runs
        buf.amps.fill_(0xA5 if fused else 0x3C)
        path.run(coll, pairs, buf, fused=fused, **kw)
        torch.cuda.synchronize()
        rh, ra = path.result(buf.hit_res), path.result(buf.amp_res)
        out.append((rh, ra, path.hits_numpy(buf).tobytes() if rh["status"] == 0 else b"",
                    path.amps_numpy(buf).tobytes() if ra["status"] == 0 else b""))
    return out


@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_query_equals_the_three_calls(dev, seed):
    from paper_2509_13300_amd import _lib as L

    p = plan.tiny(9100 + seed, n_genomes=12, len_lo=2000, len_hi=80000, n_copies=(1, 3),
                  nruns=2 if seed % 2 else 0)
    pairs = [p.pairs[0]] + plan.law_pairs(9200 + seed, 3)
    if seed == 13:
        import dataclasses
        pairs.append(dataclasses.replace(p.pairs[0], decoy=True))
    kw = {}
    if seed == 12:
        kw = dict(filter_tm=True, min_tm=45.0)
    if seed == 14:
        kw = dict(tm=L.tm_params(saltcorr=7, Mg=3.0, dNTPs=0.8))
    sep, fus = _both(p, pairs, dev, **kw)
    say("query", seed, "sites", sep[0]["count"], "amplicons", sep[1]["count"])
    assert sep[0]["status"] == 0 and sep[1]["status"] == 0 and sep[0]["count"] > 0
    assert fus == sep


def test_query_with_a_one_pass_sort(dev):
    """Keys of at most one digit (one pair, one short genome): the sort has a
    single pass, so ah_query runs the Tm and the pairing's first step as the
    separate calls do."""
    pr = plan.PairSpec("ACGTRYACGTAC", "TTGCANNGCA", k=3, clamp=0, min_len=20, max_len=120)
    p = plan.tiny(9300, n_genomes=1, len_lo=100, len_hi=120, pair=pr, n_copies=(1, 1))
    sep, fus = _both(p, [pr], dev)
    assert sep[0]["status"] == 0
    assert fus == sep


@pytest.mark.parametrize("segmented", ["1", "0"])
def test_query_overflow_reports_like_the_three_calls(dev, monkeypatch, segmented):
    """The sites' result as the scan's; the pairing, which needs every site,
    reports an overflow with nothing counted until the sites fit."""
    monkeypatch.setenv("AH_QUERY_SEGMENTED", segmented)
    pr = plan.PairSpec("ACGTACGTAC", "GGCCAATTGG", k=3, clamp=0, min_len=20, max_len=2000)
    p = plan.tiny(9301, n_genomes=4, len_lo=20000, len_hi=40000, pair=pr)
    sep, fus = _both(p, [pr], dev, hit_cap=64, amp_cap=64)
    assert sep[0]["status"] == -4
    assert fus[0] == sep[0]
    assert (fus[1]["status"], fus[1]["count"], fus[1]["required"]) == (-4, 0, 0)
    sep, fus = _both(p, [pr], dev, hit_cap=sep[0]["required"], amp_cap=64)
    assert sep[0]["status"] == 0 and sep[1]["status"] == -4
    assert fus == sep
    sep, fus = _both(p, [pr], dev, hit_cap=sep[0]["required"], amp_cap=sep[1]["required"])
    assert sep[0]["status"] == 0 and sep[1]["status"] == 0 and fus == sep


def test_query_on_the_collection_workload(dev):
    p = plan.collection(60, seed=13302)
    sep, fus = _both(p, p.pairs, dev, hit_cap=1 << 20, amp_cap=1 << 20)
    say("collection-60", sep[0], sep[1])
    assert sep[0]["status"] == 0 and fus == sep


@pytest.mark.parametrize("segmented", ["1", None])
def test_query_segments_longer_than_lds(dev, monkeypatch, segmented):
    """A short primer at k = 3 on genomes of ~300 kbp: thousands of sites per
    (pair, genome), past the 1,024 the segment sort keeps in LDS, so those
    segments are sorted and paired through global memory (forced: left to
    itself, ah_query expects segments this long and takes the radix tail)."""
    if segmented is None:
        monkeypatch.delenv("AH_QUERY_SEGMENTED", raising=False)
    else:
        monkeypatch.setenv("AH_QUERY_SEGMENTED", segmented)
    pr = plan.PairSpec("ACGTACGTAC", "GGCCAATTGG", k=3, clamp=0, min_len=20, max_len=3000)
    p = plan.tiny(9302, n_genomes=3, len_lo=250000, len_hi=350000, pair=pr)
    sep, fus = _both(p, [pr], dev, hit_cap=1 << 16, amp_cap=1 << 21)
    per_genome = np.bincount(np.frombuffer(sep[2], dtype=np.uint32).reshape(-1, 4)[:, 0],
                             minlength=p.n)
    say("long segments: sites per genome", per_genome.tolist(), "amplicons", sep[1]["count"])
    assert per_genome.max() > 2048 and sep[1]["status"] == 0
    assert fus == sep


def test_query_filters_tm_on_long_segments(dev, monkeypatch):
    monkeypatch.setenv("AH_QUERY_SEGMENTED", "1")
    pr = plan.PairSpec("ACGTRCGTAC", "GGCCAATYGG", k=3, clamp=1, min_len=20, max_len=3000)
    p = plan.tiny(9303, n_genomes=2, len_lo=250000, len_hi=300000, pair=pr)
    sep, fus = _both(p, [pr], dev, hit_cap=1 << 16, amp_cap=1 << 21, filter_tm=True, min_tm=30.0)
    assert sep[0]["status"] == 0 and sep[1]["status"] == 0
    assert fus == sep


@pytest.mark.parametrize("n_genomes", [1024, 1025])
def test_query_at_the_segment_limit(dev, n_genomes):
    """Four pairs over 1,024 genomes are 4,096 segments, the most the
    segmented tail takes; 1,025 genomes go to the radix-sort tail."""
    p = plan.tiny(9304, n_genomes=n_genomes, len_lo=200, len_hi=3000, n_copies=(0, 2))
    pairs = [p.pairs[0]] + plan.law_pairs(9305, 3)
    sep, fus = _both(p, pairs, dev, hit_cap=1 << 18, amp_cap=1 << 18)
    say("segment limit", n_genomes, "sites", sep[0]["count"], "amplicons", sep[1]["count"])
    assert sep[0]["status"] == 0 and sep[1]["status"] == 0 and sep[0]["count"] > 0
    assert fus == sep


def test_query_radix_tail_when_asked(dev, monkeypatch):
    monkeypatch.setenv("AH_QUERY_SEGMENTED", "0")
    p = plan.tiny(9306, n_genomes=12, len_lo=2000, len_hi=80000, n_copies=(1, 3), nruns=2)
    pairs = [p.pairs[0]] + plan.law_pairs(9307, 2)
    sep, fus = _both(p, pairs, dev)
    assert sep[0]["status"] == 0 and sep[1]["status"] == 0 and sep[0]["count"] > 0
    assert fus == sep


@pytest.mark.parametrize("group", ["3", "6"])
def test_query_with_records_across_pairs(dev, monkeypatch, group):
    """Pattern groups of 3 or 6 put patterns of two pairs in one candidate
    record: the segmented emit then takes each pattern's places itself
    instead of the verify pass reserving them per record."""
    monkeypatch.setenv("AH_SCAN_GROUP", group)
    p = plan.tiny(9308, n_genomes=12, len_lo=2000, len_hi=80000, n_copies=(1, 3), nruns=2)
    pairs = [p.pairs[0]] + plan.law_pairs(9309, 3)
    sep, fus = _both(p, pairs, dev)
    assert sep[0]["status"] == 0 and sep[1]["status"] == 0 and sep[0]["count"] > 0
    assert fus == sep
