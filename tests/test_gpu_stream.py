"""GPU tests of the streaming form: a packed collection in pinned host memory,
copied to the GPU chunk by chunk on overlapping streams, gives the same hits,
Tm values and amplicons as the resident collection (bit for bit), for every
slot count, copy-stream count and chunk size; overflow reports the exact
totals."""
import numpy as np
import pytest

from gpu_util import amp_tuples, hit_tuples_gpu, hit_tuples_oracle, run_oracle, say
from synth import gpu, plan

pytestmark = pytest.mark.gpu

PAIR = plan.PairSpec("GTGCCAGCMGCNGCGGTAA", "GGACTACHVGGGTWTCTAAT", k=2, clamp=2, min_len=150,
                     max_len=3000)


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def coll(dev):
    from paper_2509_13300_amd import path

    p = plan.tiny(5501, n_genomes=30, len_lo=20000, len_hi=300000, pair=PAIR, n_copies=(1, 3),
                  nruns=3, span=400)
    ascii, off = gpu.fill_cuda(p, dev)
    c, _ = path.pack(ascii, off, p.lengths, with_nmask=True)
    return p, c, path.to_host(c)


def resident(c, pairs, dev, hit_cap=1 << 18, amp_cap=1 << 18):
    import torch

    from paper_2509_13300_amd import path

    buf = path.alloc(c, pairs, hit_cap, amp_cap, dev)
    path.run(c, pairs, buf)
    torch.cuda.synchronize()
    return path.hits_numpy(buf), path.amps_numpy(buf), path.result(buf.hit_res), \
        path.result(buf.amp_res)


def streamed(hg, pairs, dev, chunk_words, n_slots, n_copy, hit_cap=1 << 18, amp_cap=1 << 18):
    import torch

    from paper_2509_13300_amd import path

    buf = path.stream_alloc(hg, pairs, hit_cap, amp_cap, dev, chunk_words, n_slots)
    copies = [torch.cuda.Stream(dev) for _ in range(n_copy)]
    path.stream_run(hg, pairs, buf, copy_streams=copies)
    torch.cuda.synchronize()
    return path.hits_numpy(buf), path.amps_numpy(buf), path.result(buf.hit_res), \
        path.result(buf.amp_res)


def test_resident_matches_oracle(coll, dev):
    p, c, hg = coll
    h, a, rh, ra = resident(c, [PAIR], dev)
    oh, oa = run_oracle(p, [PAIR])
    say("stream collection", c.n, "genomes", c.total_bp, "bp; hits", h.size, "amplicons", a.size)
    assert h.size > 50 and a.size >= 1
    assert hit_tuples_gpu(h) == hit_tuples_oracle(oh)
    assert np.abs(h["tm"].astype(np.float64) - oh["tm"]).max() <= 0.01
    assert amp_tuples(a) == amp_tuples(oa)


@pytest.mark.parametrize("chunk_words,n_slots,n_copy", [
    (9_600, 2, 0), (40_000, 2, 1), (40_000, 3, 2), (100_000, 4, 2), (1 << 22, 2, 1),
])
def test_streamed_equals_resident(coll, dev, chunk_words, n_slots, n_copy):
    p, c, hg = coll
    h0, a0, _, _ = resident(c, [PAIR], dev)
    h1, a1, rh, ra = streamed(hg, [PAIR], dev, chunk_words, n_slots, n_copy)
    say("chunk", chunk_words, "slots", n_slots, "copy streams", n_copy, "hits", h1.size)
    assert rh["status"] == 0 and ra["status"] == 0
    assert rh["required"] == h0.size and ra["required"] == a0.size
    assert np.array_equal(h1, h0)  # every field, Tm included, bit for bit
    assert np.array_equal(a1, a0)


def test_several_pairs_equal_resident_up_to_pair_order(coll, dev):
    p, c, hg = coll
    pairs = [PAIR, plan.PairSpec("AGAGTTTGATCMTGGCTCAG", "TACGGYTACCTTGTTACGACTT", 3, 0, 100, 6000),
             plan.PairSpec("CCTACGGGNGGCWGCAG", "GACTACHVGGGTATCTAATCC", 2, 1, 100, 2000)]
    h0, a0, _, _ = resident(c, pairs, dev)
    h1, a1, rh, ra = streamed(hg, pairs, dev, 30_000, 3, 2)
    assert rh["status"] == 0 and ra["status"] == 0
    # streamed output is ordered by (chunk, pair, genome, ...): a stable sort
    # by pair gives the resident order
    perm = np.argsort(h1["pair"], kind="stable")
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    assert np.array_equal(h1[perm], h0)
    a1 = a1.copy()
    a1["plus_hit"] = inv[a1["plus_hit"]]
    a1["minus_hit"] = inv[a1["minus_hit"]]
    assert np.array_equal(a1[np.argsort(a1["pair"], kind="stable")], a0)


def test_hit_overflow_reports_exact_total_and_retry_matches(coll, dev):
    p, c, hg = coll
    h0, a0, _, _ = resident(c, [PAIR], dev)
    _, _, rh, ra = streamed(hg, [PAIR], dev, 20_000, 2, 1, hit_cap=h0.size - 7)
    assert rh["status"] != 0 and ra["status"] != 0
    assert rh["required"] == h0.size and rh["count"] == h0.size - 7
    h1, a1, rh, ra = streamed(hg, [PAIR], dev, 20_000, 2, 1, hit_cap=int(rh["required"]))
    assert rh["status"] == 0 and np.array_equal(h1, h0) and np.array_equal(a1, a0)


def test_amplicon_overflow_reports_exact_total(coll, dev):
    p, c, hg = coll
    h0, a0, _, _ = resident(c, [PAIR], dev)
    assert a0.size >= 2
    h1, a1, rh, ra = streamed(hg, [PAIR], dev, 20_000, 2, 1, amp_cap=a0.size - 1)
    assert rh["status"] == 0 and np.array_equal(h1, h0)
    assert ra["status"] != 0 and ra["required"] == a0.size and ra["count"] == a0.size - 1
    assert np.array_equal(a1, a0[: a0.size - 1])  # amplicons are written in order


def test_empty_collection(dev):
    import torch

    from paper_2509_13300_amd import _lib as L
    from paper_2509_13300_amd import path

    hg = L.HostGenomes(torch.zeros(2, dtype=torch.int32, pin_memory=True), np.zeros(1, np.uint64),
                       np.zeros(0, np.uint32))
    buf = path.stream_alloc(hg, [PAIR], 16, 16, dev, 4096, 2)
    buf.hit_res.fill_(0xFF)
    path.stream_run(hg, [PAIR], buf)
    torch.cuda.synchronize()
    assert path.result(buf.hit_res) == {"count": 0, "required": 0, "status": 0}
    assert path.result(buf.amp_res) == {"count": 0, "required": 0, "status": 0}


def test_long_amplicon_pair_streamed_equals_resident(dev):
    """The long-amplicon pair (192 + 768 oligos, k = 3) on the first genomes
    of its collection; one genome also checked against the oracle."""
    from paper_2509_13300_amd import path

    full = plan.stream(10000)
    p = full.subset(np.arange(12))
    pr = p.pairs[0]
    ascii, off = gpu.fill_cuda(p, dev)
    c, _ = path.pack(ascii, off, p.lengths)
    del ascii
    hg = path.to_host(c)
    h0, a0, _, _ = resident(c, [pr], dev, 1 << 20, 1 << 20)
    h1, a1, rh, ra = streamed(hg, [pr], dev, 1 << 20, 3, 2, 1 << 20, 1 << 20)
    say("long pair", c.total_bp, "bp; hits", h0.size, "amplicons", a0.size)
    assert h0.size > 100 and a0.size > 0
    assert np.array_equal(h1, h0) and np.array_equal(a1, a0)
    one = p.subset([3])
    oh, oa = run_oracle(one, [pr])
    g = h0[h0["genome"] == 3].copy()
    g["genome"] = 0
    assert hit_tuples_gpu(g) == hit_tuples_oracle(oh)
    assert np.abs(g["tm"].astype(np.float64) - oh["tm"]).max(initial=0.0) <= 0.01


def test_full_size_collection_sampled_against_oracle(dev):
    """10,000 genomes (~42 Gbp, ~10.5 GB packed) in pinned host memory, in the
    launch configuration that the streaming benchmark times (chunks of 2^26
    words, 3 slots, 2 copy streams): streamed equals resident in full, and
    three sampled genomes equal the oracle."""
    import torch

    from paper_2509_13300_amd import path

    p = plan.stream(10000)
    pr = p.pairs[0]
    hg = path.pack_to_host(lambda ids: gpu.fill_cuda(p.subset(ids), dev), p.lengths, dev)
    say("full stream collection", int(p.lengths.sum()), "bp")
    h1, a1, rh, ra = streamed(hg, [pr], dev, 1 << 26, 3, 2, 1 << 24, 1 << 22)
    assert rh["status"] == 0 and ra["status"] == 0
    say("full stream hits", h1.size, "amplicons", a1.size)
    c = path.to_device(hg, dev)
    h0, a0, _, _ = resident(c, [pr], dev, 1 << 24, 1 << 22)
    del c
    torch.cuda.empty_cache()
    assert np.array_equal(h1, h0) and np.array_equal(a1, a0)
    for g in (0, 4711, 9999):
        one = p.subset([g])
        oh, oa = run_oracle(one, [pr])
        sel = h1[h1["genome"] == g].copy()
        first = np.flatnonzero(h1["genome"] == g)
        sel["genome"] = 0
        assert hit_tuples_gpu(sel) == hit_tuples_oracle(oh), g
        assert np.abs(sel["tm"].astype(np.float64) - oh["tm"]).max(initial=0.0) <= 0.01
        asel = a1[a1["genome"] == g].copy()
        asel["genome"] = 0
        if first.size:
            asel["plus_hit"] -= np.uint32(first[0])
            asel["minus_hit"] -= np.uint32(first[0])
        assert amp_tuples(asel) == amp_tuples(oa), g
        say("genome", g, "hits", sel.size, "amplicons", asel.size, "match the oracle")
