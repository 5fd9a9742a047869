"""Seeded synthetic inputs (genome collections, primer pairs, job streams).

Shared by the tests, the oracle timing harness and the benchmark.  It holds
no primer-matching, melting-temperature or pairing arithmetic; the CPU filler
(``synth.fill``) and the GPU filler (``synth.gpu``) compute the same bytes from
the same counter-based draws.
"""
from . import plan, rng  # noqa: F401
