"""Pins for the oracle's FASTA records and amplitypes: the SplitMix64
finaliser against the generator's published first outputs, closed-form hash
values, the record layout of a hand-written example, planted copies on
either strand reading alike, and amplitypes that see copy numbers and
variants but not order."""
import numpy as np

from oracle import fasta, pair, scan
from oracle import tm as otm
from synth import fill, plan


def test_mix_is_the_splitmix64_output_function():
    # SplitMix64 seeded with 0 outputs mix(k * golden gamma) for k = 1, 2, ...;
    # the generator's published first outputs
    assert fasta.mix(fasta.GOLDEN) == 0xE220A8397B1DCDAF
    assert fasta.mix(2 * fasta.GOLDEN) == 0x6E789E6AA1B965F4
    assert fasta.mix(0) == 0


def test_sequence_hash_closed_forms():
    # one A: sum = 1, n = 1, so the mixed value is mix(0) = 0
    assert fasta.seq_hash(b"A") == 0
    # sum = (c + 1) for one base: the code enters as c + 1
    assert fasta.seq_hash(b"T") == fasta.mix(4 ^ 1)
    assert fasta.seq_hash(b"") == 0
    # order, length and the N code all matter
    assert fasta.seq_hash(b"AC") != fasta.seq_hash(b"CA")
    assert fasta.seq_hash(b"A") != fasta.seq_hash(b"AA")
    assert fasta.seq_hash(b"ACGN") != fasta.seq_hash(b"ACGT")


def test_record_layout_of_a_worked_example():
    genomes = [b"x" * 10 + b"ACGTTacgtaNNGGC" + b"TTTT"]
    hits = np.zeros(2, dtype=scan.HIT_DTYPE)
    hits["tm"] = [55.125, float("nan")]
    amps = np.zeros(2, dtype=pair.AMP_DTYPE)
    amps[0] = (0, 0, 10, 25, pair.FR, 0, 1)
    amps[1] = (0, 0, 10, 25, pair.RF, 0, 1)
    recs = fasta.records(genomes, hits, amps)
    assert fasta.fasta_text(recs[:1]) == (b">g0:10-25 pair=0 orient=FR tm=55.12,nan\n"
                                          b"ACGTTACGTANNGGC\n")
    # RF: the reverse complement; lower case folded, N kept
    assert recs[1][1] == b"GCCNNTACGTAACGT"
    assert fasta.fmt_tm(-0.004) == "0.00" and fasta.fmt_tm(-1.5) == "-1.50"
    assert fasta.fmt_tm(0.125) == "0.12" and fasta.fmt_tm(0.135) == "0.14"


def test_planted_copies_read_alike_and_amplitypes_count_them():
    p = plan.tiny(61, n_genomes=4, len_lo=6000, len_hi=9000, n_copies=(2, 3))
    pr = p.pairs[0]
    seqs = [fill.genome_bytes(p, g) for g in range(p.n)]
    h = scan.scan_collection(seqs, [pr])
    h = otm.fill_tm(h, seqs, [pr])
    a = pair.call_amplicons(h, [pr])
    recs = fasta.records(seqs, h, a)
    # every FR / RF amplicon of a planted copy has the template's sequence
    # between the two primer sites (up to the 1% mutations), on either strand
    f0, r0, _ = p.template_sites[0]
    tmpl = p.templates[0]
    want = fasta.clean(tmpl[f0:r0 + len(pr.rev)])
    strands = set()
    for x, (head, s, _) in zip(a, recs):
        if int(x["orient"]) in (0, 1) and len(s) == len(want):
            same = sum(u == v for u, v in zip(s, want)) / len(s)
            if same > 0.95:
                strands.add(int(x["orient"]))
    assert strands == {0, 1}
    hs, cnt = fasta.amplitypes(a, recs, 1, p.n)
    fr_rf = np.isin(a["orient"], [0, 1])
    for g in range(p.n):
        assert cnt[g] == int((fr_rf & (a["genome"] == g)).sum())
        assert (hs[g] == 0) == (cnt[g] == 0)


def test_amplitype_sees_copy_numbers_not_order():
    a = np.zeros(5, dtype=pair.AMP_DTYPE)
    a["orient"] = [0, 1, 0, 0, 2]
    a["genome"] = [0, 0, 0, 1, 1]
    seqs = [b"ACGTAC", b"ACGTAC", b"TTGACA", b"TTGACA", b"GGGG"]
    recs = [("", s, fasta.seq_hash(s)) for s in seqs]
    hs, cnt = fasta.amplitypes(a, recs, 1, 3)
    # order-free
    rev = np.ascontiguousarray(a[[2, 1, 0, 3, 4]])
    hs2, _ = fasta.amplitypes(rev, [recs[i] for i in (2, 1, 0, 3, 4)], 1, 3)
    assert hs == hs2
    # genome 0: {ACGTAC x2, TTGACA x1}; genome 1: {TTGACA} (FF not counted)
    assert cnt == [3, 1, 0] and hs[2] == 0
    b = a.copy()
    b["genome"] = [0, 0, 0, 0, 1]
    hs3, cnt3 = fasta.amplitypes(b, recs, 1, 3)
    assert cnt3[0] == 4 and hs3[0] != hs[0]
