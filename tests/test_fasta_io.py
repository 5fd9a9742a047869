"""The library's FASTA reader (host, multi-threaded) against the oracle's
line-by-line reader: wrapped lines of any width, CRLF, blank lines, case,
IUPAC codes, empty records, no final newline, names with blanks, texts large
enough to be read by many threads; sequence bytes before the first record are
an error."""
import numpy as np
import pytest

from oracle import fastaio
from paper_2509_13300_amd import _lib as L


def make_text(rs, n_rec, max_len, crlf=False, final_nl=True):
    alphabet = list(b"ACGTacgtNRYKMSWnBDHV")
    p = np.array([8] * 8 + [1] * 12, dtype=float)
    p /= p.sum()
    nl = b"\r\n" if crlf else b"\n"
    out, recs = [], []
    for r in range(n_rec):
        name = f"rec{r} contig {rs.randint(1000)}".encode()
        n = int(rs.randint(0, max_len + 1)) if r % 7 else 0
        seq = bytes(rs.choice(alphabet, size=n, p=p).astype(np.uint8))
        width = int(rs.choice([10, 60, 61, 80, 1000]))
        lines = [seq[i:i + width] for i in range(0, n, width)]
        if rs.rand() < 0.3:
            lines.insert(int(rs.randint(0, len(lines) + 1)), b"")  # a blank line
        out.append(b">" + name + (b"  " if rs.rand() < 0.2 else b"") + nl + nl.join(lines))
        recs.append((name.decode(), seq))
    text = nl.join(out) + (nl if final_nl else b"")
    if rs.rand() < 0.5:
        text = nl + b"  " + nl + text  # blank lines before the first record
    return text, recs


@pytest.mark.parametrize("case", [(1, 5, 300, False, True), (2, 40, 2000, True, False),
                                  (3, 1, 0, False, True), (4, 300, 50000, False, False),
                                  (5, 120, 90000, True, True)])
def test_reader_matches_the_oracle(case):
    seed, n_rec, max_len, crlf, final_nl = case
    text, recs = make_text(np.random.RandomState(seed), n_rec, max_len, crlf, final_nl)
    want = fastaio.read(text)
    assert [(n, s) for n, s in want] == recs
    seq, off, names = L.fasta_read(text)
    assert names == [n for n, _ in want]
    assert off.size == len(want) + 1 and off[0] == 0
    for r, (_, s) in enumerate(want):
        assert seq[off[r]:off[r + 1]].tobytes() == s, r


def test_empty_text_and_errors():
    seq, off, names = L.fasta_read(b"")
    assert names == [] and off.tolist() == [0]
    seq, off, names = L.fasta_read(b"\n\n>only\n")
    assert names == ["only"] and off.tolist() == [0, 0]
    with pytest.raises(L.AhError) as e:
        L.fasta_read(b"ACGT\n>r\nACGT\n")
    assert e.value.status == L.AH_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        fastaio.read(b"ACGT\n>r\nACGT\n")
