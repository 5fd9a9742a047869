"""FASTA text -> records (Section 2.1: the tool's input is genomes in FASTA).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading R26: a record starts at a line whose first byte is '>'; its name is
the rest of that line without trailing blanks or carriage returns; its
sequence is the bytes of the following lines up to the next record with line
breaks, carriage returns, blanks and tabs removed (case and IUPAC codes kept).
Each record is its own linear sequence (R5): a genome of several contigs is
several records.  Text other than blank lines before the first record is an
error.
"""
from __future__ import annotations

_DROP = b" \t\r"


def read(text: bytes):
    """[(name, sequence bytes)] in file order."""
    recs = []
    for line in bytes(text).split(b"\n"):
        if line.startswith(b">"):
            recs.append([line[1:].rstrip(b" \t\r").decode(errors="replace"), []])
            continue
        body = line.translate(None, _DROP)
        if not body:
            continue
        if not recs:
            raise ValueError("sequence bytes before the first '>' line")
        recs[-1][1].append(body)
    return [(name, b"".join(parts)) for name, parts in recs]
