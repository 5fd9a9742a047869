"""GPU parity of the FASTA records, sequence hashes and amplitypes against
the oracle: records byte-identical but for the Tm digits (within the Tm
tolerance), hashes and amplitypes exact; overflow reports the size and a
rerun at that size gives the same text."""
import dataclasses

import numpy as np
import pytest

from gpu_util import run_gpu, run_oracle, say
from oracle import fasta as ofasta
from synth import fill, plan

pytestmark = pytest.mark.gpu
RICH = plan.PairSpec("ACGTACGTAC", "GGATCCTTGA", k=3, clamp=0, min_len=40, max_len=400)


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def parse(text: bytes):
    lines = text.split(b"\n")
    assert lines[-1] == b""
    return [(lines[i].decode(), lines[i + 1]) for i in range(0, len(lines) - 1, 2)]


def same_header(g: str, o: str):
    gf, of = g.split(" tm="), o.split(" tm=")
    assert gf[0] == of[0], (g, o)
    for x, y in zip(gf[1].split(","), of[1].split(",")):
        if y == "nan":
            assert x == "nan", (g, o)
        else:
            assert abs(float(x) - float(y)) <= 0.0101, (g, o)


def check(p, pairs, dev, text_cap=1 << 24):
    import torch

    from paper_2509_13300_amd import path

    coll, buf = run_gpu(p, pairs, dev, hit_cap=1 << 20, amp_cap=1 << 20)
    fb = path.fasta_alloc(coll, len(pairs), buf.amp_cap, text_cap, dev)
    path.fasta(coll, len(pairs), buf, fb)
    torch.cuda.synchronize()
    r = path.result(fb.text_res)
    oh, oa = run_oracle(p, pairs)
    seqs = [fill.genome_bytes(p, g) for g in range(p.n)]
    recs = ofasta.records(seqs, oh, oa)
    want = ofasta.fasta_text(recs)
    assert r["required"] == len(want)
    if r["status"] != 0:
        return coll, buf, fb, r, want
    got = parse(path.fasta_text(fb))
    assert len(got) == len(recs) == oa.size
    for (gh, gs), (oh_, os_, _) in zip(got, recs):
        same_header(gh, oh_)
        assert gs == os_, gh
    n = oa.size
    gh_hash = fb.seq_hash[:n].cpu().numpy().view(np.uint64)
    assert [int(x) for x in gh_hash] == [h for _, _, h in recs]
    hs, cnt = ofasta.amplitypes(oa, recs, len(pairs), p.n)
    assert [int(x) for x in fb.amplitype.cpu().numpy().view(np.uint64)] == hs
    assert fb.amplitype_n.cpu().numpy().astype(np.int64).tolist() == cnt
    return coll, buf, fb, r, want


@pytest.mark.parametrize("seed", [701, 702])
def test_fasta_records_hashes_and_amplitypes_match_the_oracle(seed, dev):
    p = plan.tiny(seed, n_genomes=6, len_lo=2000, len_hi=40000, n_copies=(1, 3),
                  nruns=2 if seed % 2 else 0)
    pairs = [p.pairs[0], RICH, dataclasses.replace(RICH, decoy=True)]
    _, _, fb, r, want = check(p, pairs, dev)
    say("fasta case", seed, "bytes", r["required"], "records", want.count(b">"))
    assert r["status"] == 0 and want.count(b">") > 100


def test_fasta_of_the_collection_sample(dev):
    p = plan.collection(1000, seed=13302).subset([3, 250, 731])
    _, _, fb, r, want = check(p, p.pairs, dev)
    say("collection fasta bytes", r["required"])
    assert r["status"] == 0 and r["required"] > 0


def test_fasta_overflow_reports_the_size(dev):
    import torch

    from paper_2509_13300_amd import path

    p = plan.tiny(711, n_genomes=3, len_lo=5000, len_hi=20000)
    coll, buf, fb, r, want = check(p, [RICH], dev, text_cap=1000)
    assert r["status"] == -4 and r["required"] == len(want) > 1000
    fb2 = path.fasta_alloc(coll, 1, buf.amp_cap, r["required"], dev)
    path.fasta(coll, 1, buf, fb2)
    torch.cuda.synchronize()
    assert path.result(fb2.text_res)["status"] == 0
    assert len(path.fasta_text(fb2)) == len(want)
