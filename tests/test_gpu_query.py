"""ah_query (scan, Tm and pairing in one call, with the Tm computed inside
the sort's first pass and the pairing's chunk counts inside its last) gives
the same bytes as the three separate calls."""
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


def test_query_overflow_reports_like_the_three_calls(dev):
    pr = plan.PairSpec("ACGTACGTAC", "GGCCAATTGG", k=3, clamp=0, min_len=20, max_len=2000)
    p = plan.tiny(9301, n_genomes=4, len_lo=20000, len_hi=40000, pair=pr)
    sep, fus = _both(p, [pr], dev, hit_cap=64, amp_cap=64)
    assert sep[0]["status"] == -4
    assert fus[0] == sep[0] and fus[1]["status"] == sep[1]["status"]
    sep, fus = _both(p, [pr], dev, hit_cap=sep[0]["required"], amp_cap=1 << 18)
    assert sep[0]["status"] == 0 and fus == sep


def test_query_on_the_collection_workload(dev):
    p = plan.collection(60, seed=13302)
    sep, fus = _both(p, p.pairs, dev, hit_cap=1 << 20, amp_cap=1 << 20)
    say("collection-60", sep[0], sep[1])
    assert sep[0]["status"] == 0 and fus == sep
