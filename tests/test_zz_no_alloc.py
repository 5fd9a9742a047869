"""The scan entry point that allocates nothing (ah_scan_primers_noalloc)
against ah_scan_primers: same records and result on two calls in a row, the
second on a smaller input (the scratch array keeps the first call's
contents), through the C ABI."""
import ctypes

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


def _collection(p, dev, nmask):
    from paper_2509_13300_amd import path

    ascii, off = gpu.fill_cuda(p, dev)
    coll, _ = path.pack(ascii, off, p.lengths, with_nmask=nmask)
    return coll


def _records(hits, res):
    import torch

    torch.cuda.synchronize()
    r = np.frombuffer(res.cpu().numpy().tobytes(), dtype=np.uint64, count=2)
    st = int(np.frombuffer(res.cpu().numpy().tobytes()[16:20], dtype=np.int32)[0])
    n = int(min(r[0], hits.numel() // 16))
    return hits[: n * 16].cpu().numpy().tobytes(), (int(r[0]), int(r[1]), st)


def _both(coll, pr, cap, dev):
    """(records, result) of ah_scan_primers and of the no-allocation call."""
    import torch

    from paper_2509_13300_amd import _lib as L

    g = coll.view()
    pp = L.primer_pairs([pr])
    work = torch.empty(L.ah_scan_workspace_bytes(g, pp, cap), dtype=torch.uint8, device=dev)
    h1 = torch.empty(cap * 16, dtype=torch.uint8, device=dev)
    r1 = torch.zeros(24, dtype=torch.uint8, device=dev)
    L.ah_scan_primers(g, pp, h1, cap, r1, work)
    want = _records(h1, r1)
    h2 = torch.full((cap * 16,), 0xAB, dtype=torch.uint8, device=dev)
    r2 = torch.full((24,), 0xCD, dtype=torch.uint8, device=dev)
    L.ah_scan_primers_noalloc(g, pp, h2, cap, r2)
    got = _records(h2, r2)
    return want, got


def test_noalloc_scan_equals_the_scan_on_two_calls_in_a_row(dev):
    from paper_2509_13300_amd import _lib as L

    big = plan.tiny(7101, n_genomes=24, len_lo=2000, len_hi=90000, n_copies=(1, 4), nruns=3)
    pr = big.pairs[0]
    small = plan.tiny(7102, n_genomes=3, len_lo=500, len_hi=4000, pair=pr, n_copies=(1, 2))
    cb = _collection(big, dev, True)
    cs = _collection(small, dev, True)
    # kernels compiled (this is the call that may allocate: module load)
    L.ah_scan_prepare([(pr.fwd, pr.rev, pr.k, pr.clamp)], True)
    for label, coll, cap in (("first, 24 genomes", cb, 1 << 15), ("second, 3 genomes", cs, 1 << 12)):
        want, got = _both(coll, pr, cap, dev)
        say("noalloc", label, "sites", want[1][0], "result", got[1])
        assert want[1][2] == 0 and want[1][0] > 0
        assert got == want


def test_noalloc_scan_refuses_what_it_cannot_do_without_allocating(dev):
    import torch

    from paper_2509_13300_amd import _lib as L

    p = plan.tiny(7103, n_genomes=2, len_lo=500, len_hi=2000)
    coll = _collection(p, dev, False)
    g = coll.view()
    res = torch.zeros(24, dtype=torch.uint8, device=dev)
    hits = torch.empty(16 << 10, dtype=torch.uint8, device=dev)
    # a primer set never compiled on this device: nothing is compiled here
    fresh = L.primer_pairs([("ACGTTGCAAGGCTTAGCATC", "TTGACCGATTGCAAGCATGC", 1, 0)])
    st = L.lib().ah_scan_primers_noalloc(ctypes.byref(g), fresh, 1, hits.data_ptr(), 1 << 10,
                                         res.data_ptr(), None)
    assert st == L.AH_ERR_INVALID_ARG and "not loaded" in L.ah_last_error()
    # a capacity whose fixed parts do not fit in the scratch array
    pr = p.pairs[0]
    L.ah_scan_prepare([(pr.fwd, pr.rev, pr.k, pr.clamp)], False)
    pp = L.primer_pairs([pr])
    st = L.lib().ah_scan_primers_noalloc(ctypes.byref(g), pp, 1, hits.data_ptr(), 1 << 24,
                                         res.data_ptr(), None)
    assert st == L.AH_ERR_WORKSPACE and "scratch" in L.ah_last_error()
    torch.cuda.synchronize()
