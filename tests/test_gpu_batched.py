"""GPU tests of the batched form: many primer pairs in one pass give exactly
the per-pair results, for every kernel shape; the autotuner's choice changes
nothing; a hipGraph replay equals the eager pass."""
import numpy as np
import pytest

from gpu_util import amp_tuples, hit_tuples_gpu, hit_tuples_oracle, random_rate, run_oracle, say
from synth import gpu, plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def batch(dev):
    from paper_2509_13300_amd import path

    pairs = sorted(plan.law_pairs(4401, 64), key=random_rate, reverse=True)[:8]
    for q in pairs:  # windows that fit the small genomes
        q.min_len, q.max_len = 40, 1500
    pairs[3].clamp = 2
    p = plan.tiny(4402, n_genomes=6, len_lo=100000, len_hi=400000, pair=pairs[0], n_copies=(1, 3),
                  span=300)
    ascii, off = gpu.fill_cuda(p, dev)
    coll, _ = path.pack(ascii, off, p.lengths)
    return p, pairs, coll


def run_all(coll, pairs, dev):
    import torch

    from paper_2509_13300_amd import path

    buf = path.alloc(coll, pairs, 1 << 20, 1 << 20, dev)
    path.run(coll, pairs, buf)
    torch.cuda.synchronize()
    assert path.result(buf.hit_res)["status"] == 0
    return path.hits_numpy(buf), path.amps_numpy(buf)


def test_batched_equals_each_pair_alone(batch, dev):
    p, pairs, coll = batch
    hb, ab = run_all(coll, pairs, dev)
    say("batched hits", hb.size, "amplicons", ab.size)
    assert hb.size > 500 and len(set(hb["pair"].tolist())) == len(pairs)
    for q, pr in enumerate(pairs):
        h1, a1 = run_all(coll, [pr], dev)
        sel = hb[hb["pair"] == q].copy()
        sel["pair"] = 0
        assert np.array_equal(sel, h1)  # integer fields and Tm, bit for bit
        base = np.flatnonzero(hb["pair"] == q)[0] if sel.size else 0
        asel = ab[ab["pair"] == q].copy()
        asel["pair"] = 0
        asel["plus_hit"] = asel["plus_hit"] - np.uint32(base)
        asel["minus_hit"] = asel["minus_hit"] - np.uint32(base)
        assert np.array_equal(asel, a1)


def test_batched_matches_oracle_on_two_pairs(batch, dev):
    p, pairs, coll = batch
    sub = [pairs[1], pairs[3]]
    hb, ab = run_all(coll, sub, dev)
    oh, oa = run_oracle(p, sub)
    assert hit_tuples_gpu(hb) == hit_tuples_oracle(oh)
    assert np.abs(hb["tm"].astype(np.float64) - oh["tm"]).max(initial=0.0) <= 0.01
    assert amp_tuples(ab) == amp_tuples(oa)


@pytest.mark.parametrize("shape", [(3, 1), (7, 3), (9, 16), (15, 32), (5, 5), (31, 4)])
def test_every_kernel_shape_gives_the_same_result(batch, dev, shape):
    from paper_2509_13300_amd import _lib as L

    p, pairs, coll = batch
    ref = run_all(coll, pairs, dev)
    L.ah_set_scan_tuning(pairs, shape)
    try:
        assert L.ah_get_scan_tuning(pairs) == shape
        got = run_all(coll, pairs, dev)
    finally:
        L.ah_set_scan_tuning(pairs, None)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_autotuner_choice_changes_nothing(batch, dev):
    import torch

    from paper_2509_13300_amd import _lib as L
    from paper_2509_13300_amd import path

    p, pairs, coll = batch
    ref = run_all(coll, pairs, dev)
    buf = path.alloc(coll, pairs, 1 << 20, 1 << 20, dev)
    shape, ms = L.ah_autotune_scan(path.subset_view(coll, 3), L.primer_pairs(pairs), buf.hits,
                                   buf.hit_cap, buf.hit_res, buf.scan_work, repeats=2)
    torch.cuda.synchronize()
    say("autotuned", shape, ms)
    assert shape[0] in (9, 15) and 1 <= shape[1] <= 16 and ms > 0
    assert L.ah_get_scan_tuning(pairs) == shape
    got = run_all(coll, pairs, dev)
    L.ah_set_scan_tuning(pairs, None)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_graph_replay_equals_eager(batch, dev):
    import torch

    from paper_2509_13300_amd import path

    p, pairs, coll = batch
    buf = path.alloc(coll, pairs, 1 << 20, 1 << 20, dev)
    path.run(coll, pairs, buf)
    torch.cuda.synchronize()
    eager_h, eager_a = path.hits_numpy(buf), path.amps_numpy(buf)
    g = path.capture(coll, pairs, buf)
    for rep in range(3):
        buf.hits.fill_(0xAB)  # eager work between replays
        buf.amps.fill_(0xCD)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(path.hits_numpy(buf), eager_h), rep
        assert np.array_equal(path.amps_numpy(buf), eager_a), rep


def test_full_size_batch_sampled_against_oracle(dev):
    """The batched workload at full size (2,000 genomes, 8.39 Gbp, 64 pairs of
    the law) in one call with the batched benchmark's capacities: the records
    of sampled (pair, genome) cells equal the oracle's, for the pairs planted
    in three genomes, two pairs with hundreds of random sites per genome and
    two pairs with none there."""
    import torch

    from paper_2509_13300_amd import path

    p = plan.batched(2000, n_pairs=64)
    pairs = p.pairs
    ascii, off = gpu.fill_cuda(p, dev)
    coll, _ = path.pack(ascii, off, p.lengths)
    del ascii
    torch.cuda.empty_cache()
    buf = path.alloc(coll, pairs, 1 << 25, 1 << 24, dev)
    say("full batch", coll.n, "genomes", coll.total_bp, "bp", len(pairs), "pairs")
    path.run(coll, pairs, buf)
    torch.cuda.synchronize()
    rh, ra = path.result(buf.hit_res), path.result(buf.amp_res)
    assert rh["status"] == 0 and ra["status"] == 0, (rh, ra)
    h, a = path.hits_numpy(buf), path.amps_numpy(buf)
    say("full batch hits", h.size, "amplicons", a.size)
    checked = 0
    for g in (0, 1000, 1999):
        planted = sorted(set(p.plant_template[p.plant_genome == g].tolist()))  # template t: pair t
        assert planted
        one = p.subset([g])
        for q in planted + [0, 21, 40, 63]:
            oh, oa = run_oracle(one, [pairs[q]])
            cell = (h["pair"] == q) & (h["genome"] == g)
            first = np.flatnonzero(cell)
            sel = h[cell].copy()
            sel["pair"] = 0
            sel["genome"] = 0
            assert hit_tuples_gpu(sel) == hit_tuples_oracle(oh), (g, q)
            assert np.abs(sel["tm"].astype(np.float64) - oh["tm"]).max(initial=0.0) <= 0.01
            acell = (a["pair"] == q) & (a["genome"] == g)
            asel = a[acell].copy()
            asel["pair"] = 0
            asel["genome"] = 0
            if first.size:
                asel["plus_hit"] -= np.uint32(first[0])
                asel["minus_hit"] -= np.uint32(first[0])
            assert amp_tuples(asel) == amp_tuples(oa), (g, q)
            checked += int(oh.size > 0)
            say("genome", g, "pair", q, "hits", sel.size, "amplicons", asel.size, "match the oracle")
    assert checked >= 9
