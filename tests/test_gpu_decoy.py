"""GPU parity of decoy pairs (the decoy off-target estimate: the analysis on
every genome reversed): a decoy pair scanned in the same pass as real pairs
gives the oracle's run on the reversed genomes, stated in the genomes' own
coordinates -- sites, mismatches, Tm within 0.01 C, the Tm filter's
decisions and amplicons -- and the same records as the decoy alone."""
import dataclasses

import numpy as np
import pytest

from gpu_util import amp_tuples, hit_tuples_gpu, hit_tuples_oracle, run_gpu, run_oracle, say
from synth import plan

pytestmark = pytest.mark.gpu

TM_TOL = 0.01
RICH = plan.PairSpec("ACGTACGTAC", "GGATCCTTGA", k=3, clamp=0, min_len=40, max_len=400)


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def decoy(pr, **kw):
    return dataclasses.replace(pr, decoy=True, **kw)


def check(p, pairs, dev, **kw):
    from paper_2509_13300_amd import path

    coll, buf = run_gpu(p, pairs, dev, hit_cap=1 << 20, amp_cap=1 << 20, **kw)
    res = path.result(buf.hit_res)
    assert res["status"] == 0, res
    gh, ga = path.hits_numpy(buf), path.amps_numpy(buf)
    oh, oa = run_oracle(p, pairs, filter_tm=kw.get("filter_tm", False),
                        min_tm=kw.get("min_tm", 50.0))
    assert hit_tuples_gpu(gh) == hit_tuples_oracle(oh)
    if gh.size:
        err = np.abs(gh["tm"].astype(np.float64) - oh["tm"])
        fin = np.isfinite(oh["tm"])
        assert np.array_equal(np.isfinite(gh["tm"]), fin)
        assert float(err[fin].max(initial=0.0)) <= TM_TOL, float(err[fin].max())
    assert amp_tuples(ga) == amp_tuples(oa)
    return gh, ga


@pytest.mark.parametrize("seed", [501, 502, 503])
def test_decoy_pairs_match_the_oracle_on_reversed_genomes(seed, dev):
    p = plan.tiny(seed, n_genomes=6, len_lo=300, len_hi=60000, n_copies=(0, 2),
                  nruns=2 if seed % 2 else 0)
    law = plan.law_pairs(seed, 1)[0]
    pairs = [p.pairs[0], decoy(p.pairs[0]), RICH, decoy(RICH), decoy(RICH, k=2, clamp=3),
             decoy(law)]
    gh, ga = check(p, pairs, dev)
    dec = np.isin(gh["pair"], [1, 3, 4, 5])
    say("decoy case", seed, "hits", gh.size, "decoy hits", int(dec.sum()), "amplicons", ga.size,
        "decoy amplicons", int(np.isin(ga["pair"], [1, 3, 4, 5]).sum()))
    assert dec.sum() > 100 and np.isin(ga["pair"], [3, 4]).sum() > 0


def test_decoy_tm_filter_matches_the_oracle(dev):
    """The Tm of a decoy site is the primer's against the reversed genome: the
    filter keeps and drops the same sites as the oracle's decoy run."""
    p = plan.tiny(511, n_genomes=4, len_lo=20000, len_hi=60000)
    pairs = [RICH, decoy(RICH), decoy(RICH, clamp=2)]
    gh, _ = check(p, pairs, dev)
    tms = np.sort(gh["tm"][np.isfinite(gh["tm"])].astype(np.float64))
    # a threshold near the median but at least 0.02 C from every site's Tm
    # (within the Tm tolerance of the threshold either decision is right)
    mid = tms.size // 2
    gaps = np.diff(tms[mid - 200: mid + 200])
    i = int(np.argmax(gaps))
    assert gaps[i] > 0.04
    cut = float(tms[mid - 200 + i] + gaps[i] / 2)
    say("decoy Tm filter at", cut)
    gh2, ga2 = check(p, pairs, dev, filter_tm=True, min_tm=cut)
    assert ga2.size > 0


def test_decoy_in_a_batch_equals_the_decoy_alone(dev):
    from paper_2509_13300_amd import path

    p = plan.tiny(521, n_genomes=5, len_lo=5000, len_hi=80000, nruns=1)
    pairs = [RICH, decoy(RICH), p.pairs[0], decoy(p.pairs[0], k=1)]
    _, buf = run_gpu(p, pairs, dev, hit_cap=1 << 20, amp_cap=1 << 20)
    gh, ga = path.hits_numpy(buf), path.amps_numpy(buf)
    for q in (1, 3):
        _, one = run_gpu(p, [pairs[q]], dev, hit_cap=1 << 20, amp_cap=1 << 20)
        h1, a1 = path.hits_numpy(one), path.amps_numpy(one)
        sel = np.flatnonzero(gh["pair"] == q)
        hq = gh[sel].copy()
        hq["pair"] = 0
        assert np.array_equal(hq, h1)
        aq = ga[ga["pair"] == q].copy()
        aq["pair"] = 0
        base = np.uint32(sel[0] if sel.size else 0)
        aq["plus_hit"] -= base
        aq["minus_hit"] -= base
        assert np.array_equal(aq, a1)


def test_decoy_ratio_on_sampled_genomes_of_the_collection(dev):
    """The benchmark collection's V4-like pair with its decoy in one pass, on
    three of its genomes: every record against the oracle."""
    p = plan.collection(1000, seed=13302).subset([0, 417, 998])
    pr = p.pairs[0]
    pairs = [pr, decoy(pr)]
    gh, ga = check(p, pairs, dev)
    n_real = int((ga["pair"] == 0).sum())
    n_dec = int((ga["pair"] == 1).sum())
    say("collection sample: real amplicons", n_real, "decoy amplicons", n_dec,
        "decoy hits", int((gh["pair"] == 1).sum()))
    assert n_real > 0
