"""Real-FASTA ingest on the GPU: multi-contig genomes written as wrapped,
soft-masked FASTA with IUPAC codes and N runs, read by the library, packed on
the device and scanned; every site, Tm and amplicon against the oracle run on
the oracle reader's records."""
import numpy as np
import pytest

from gpu_util import amp_tuples, hit_tuples_gpu, hit_tuples_oracle, say
from oracle import fastaio
from oracle import pair as opair
from oracle import scan as oscan
from oracle import tm as otm
from synth import fill, plan

pytestmark = pytest.mark.gpu
RICH = plan.PairSpec("ACGTACGTAC", "GGATCCTTGA", k=3, clamp=0, min_len=40, max_len=400)


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def fasta_of(p, rs):
    """The plan's genomes cut into 1-3 contigs each, with lower-case runs,
    IUPAC codes and N runs, wrapped at random widths, CRLF for some."""
    out = []
    for g in range(p.n):
        seq = bytearray(fill.genome_bytes(p, g))
        n = len(seq)
        for _ in range(3):  # soft-masked runs
            a = int(rs.randint(0, n))
            b = min(n, a + int(rs.randint(0, 400)))
            seq[a:b] = bytes(seq[a:b]).lower()
        for _ in range(int(rs.randint(0, 4))):  # IUPAC codes and N runs
            a = int(rs.randint(0, n))
            b = min(n, a + int(rs.randint(1, 30)))
            seq[a:b] = bytes(rs.choice(list(b"NNNRYKMSWBDHV"), size=b - a).astype(np.uint8))
        cuts = sorted(rs.choice(np.arange(1, n), size=min(int(rs.randint(0, 3)), n - 1),
                                replace=False).tolist()) if n > 1 else []
        bounds = [0] + cuts + [n]
        for c in range(len(bounds) - 1):
            part = bytes(seq[bounds[c]:bounds[c + 1]])
            w = int(rs.choice([60, 70, 80, 1000]))
            nl = b"\r\n" if rs.rand() < 0.3 else b"\n"
            body = nl.join(part[i:i + w] for i in range(0, len(part), w))
            out.append(b">genome" + str(g).encode() + b"_contig" + str(c).encode() + b" x" + nl +
                       body + nl)
    return b"".join(out)


@pytest.mark.parametrize("seed", [801, 802])
def test_fasta_text_to_sites_and_amplicons(seed, dev):
    import torch

    from paper_2509_13300_amd import path

    p = plan.tiny(seed, n_genomes=5, len_lo=3000, len_hi=50000, n_copies=(1, 3))
    text = fasta_of(p, np.random.RandomState(seed))
    coll, names, non_acgt = path.read_fasta(text, dev)
    recs = fastaio.read(text)
    assert names == [n for n, _ in recs]
    seqs = [s for _, s in recs]
    assert non_acgt.cpu().numpy()[: len(seqs)].tolist() == [
        sum(1 for b in s.upper() if b not in b"ACGT") for s in seqs]
    pairs = [p.pairs[0], RICH]
    buf = path.alloc(coll, pairs, 1 << 20, 1 << 20, dev)
    path.run(coll, pairs, buf)
    torch.cuda.synchronize()
    gh, ga = path.hits_numpy(buf), path.amps_numpy(buf)
    oh = oscan.scan_collection(seqs, pairs)
    oh = otm.fill_tm(oh, seqs, pairs)
    oa = opair.call_amplicons(oh, pairs)
    assert hit_tuples_gpu(gh) == hit_tuples_oracle(oh)
    fin = np.isfinite(oh["tm"])
    assert np.array_equal(np.isfinite(gh["tm"]), fin)
    assert float(np.abs(gh["tm"].astype(np.float64) - oh["tm"])[fin].max(initial=0)) <= 0.01
    assert amp_tuples(ga) == amp_tuples(oa)
    say("fasta ingest", seed, "records", len(recs), "bytes", len(text), "hits", gh.size,
        "amplicons", ga.size)
    assert gh.size > 100 and ga.size > 0
