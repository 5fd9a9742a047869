"""IUPAC degenerate primers (Section 1: a degenerate primer is the mixture of
every oligonucleotide obtained by choosing one compatible base per position;
e.g. N is any base and R is A or G).

Sets follow the standard IUPAC nucleotide nomenclature.  A primer position is
represented as a 4-bit set: bit 0 = A, bit 1 = C, bit 2 = G, bit 3 = T.
"""
from __future__ import annotations

import itertools
from typing import List

import numpy as np

SETS = {
    "A": "A", "C": "C", "G": "G", "T": "T",
    "R": "AG", "Y": "CT", "S": "CG", "W": "AT", "K": "GT", "M": "AC",
    "B": "CGT", "D": "AGT", "H": "ACT", "V": "ACG", "N": "ACGT",
}
BASE_ORDER = "ACGT"
BASE_COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


class PrimerError(ValueError):
    pass


def normalise(primer: str) -> str:
    p = primer.upper()
    bad = [c for c in p if c not in SETS]
    if bad:
        raise PrimerError(f"not an IUPAC nucleotide code: {bad[0]!r}")
    return p


def members(code: str) -> str:
    return SETS[code]


def mask(code: str) -> int:
    return sum(1 << BASE_ORDER.index(b) for b in SETS[code])


def masks(primer: str) -> np.ndarray:
    return np.array([mask(c) for c in normalise(primer)], dtype=np.uint8)


def complement_code(code: str) -> str:
    """Complement of an IUPAC code: the code whose set is the complement of
    every member (A<->T, C<->G, R<->Y, K<->M, B<->V, D<->H; S, W, N fixed)."""
    comp = "".join(sorted(BASE_COMP[b] for b in SETS[code]))
    for c, s in SETS.items():
        if "".join(sorted(s)) == comp:
            return c
    raise AssertionError(code)


def revcomp(primer: str) -> str:
    return "".join(complement_code(c) for c in reversed(normalise(primer)))


def revcomp_plain(seq: str) -> str:
    return "".join(BASE_COMP[b] for b in reversed(seq))


def degeneracy(primer: str) -> int:
    d = 1
    for c in normalise(primer):
        d *= len(SETS[c])
    return d


def expand(primer: str) -> List[str]:
    """Every oligo of the mixture, in mixed-radix order: the 5'-most position
    varies slowest and members go A < C < G < T."""
    p = normalise(primer)
    return ["".join(t) for t in itertools.product(*(SETS[c] for c in p))]
