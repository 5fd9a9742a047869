"""Counter-based SplitMix64 draws for seeded synthetic inputs.

This module is input-generation infrastructure shared by the tests, the
oracle's timing harness and the benchmark.  It holds none of the scan,
melting-temperature or pairing arithmetic.

Definition (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): SplitMix64 advances a 64-bit state by the odd
constant GAMMA and returns MIX(state), where MIX is the 64-bit finaliser with
multipliers 0xBF58476D1CE4E5B9 / 0x94D049BB133111EB and shifts 30 / 27 / 31.
The i-th output (i = 0, 1, ...) of a generator started at state ``s`` is
therefore MIX(s + (i + 1) * GAMMA), which lets every draw be computed
independently from (stream key, index).  The GPU filler in ``synth/csrc``
implements the same definition; ``tests/test_synth.py`` checks that both agree
bit for bit.

A stream key is ``(seed * GAMMA) XOR (stream * STREAM_MUL)`` (mod 2^64).
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
STREAM_MUL = 0xD1B54A32D192ED03
MASK64 = (1 << 64) - 1

# Stream identifiers (upper bits) for the independent draw families.
S_BASES = 1 << 40          # | genome id : per-base background draws
S_GC = 2 << 40             # per-genome GC fraction
S_LEN = 3 << 40            # per-genome length (two uniforms for Box-Muller)
S_PLANT = 4 << 40          # | genome id : number, slots and strands of copies
S_MUT = 5 << 40            # | global copy id : per-offset mutation draws
S_TEMPLATE = 6 << 40       # | template id : operon template background
S_PRIMER = 7 << 40         # | primer id : primer sequence draws
S_MISC = 8 << 40           # | purpose : everything else (pair laws, jobs)
S_NRUN = 9 << 40           # | genome id : injected non-ACGT runs


def stream_key(seed: int, stream: int) -> int:
    """Key of stream ``stream`` under ``seed`` (Python int, mod 2^64)."""
    return ((seed * GAMMA) & MASK64) ^ ((stream * STREAM_MUL) & MASK64)


def mix64_py(z: int) -> int:
    z &= MASK64
    z ^= z >> 30
    z = (z * MIX1) & MASK64
    z ^= z >> 27
    z = (z * MIX2) & MASK64
    z ^= z >> 31
    return z


def draw_py(key: int, i: int) -> int:
    """The i-th 64-bit output of the stream with key ``key``."""
    return mix64_py(key + (i + 1) * GAMMA)


def draws(key: int, idx: np.ndarray) -> np.ndarray:
    """Vectorised ``draw_py`` over an index array (uint64 result)."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + (idx + np.uint64(1)) * np.uint64(GAMMA)
        z ^= z >> np.uint64(30)
        z *= np.uint64(MIX1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(MIX2)
        z ^= z >> np.uint64(31)
    return z


def uniform01(key: int, idx) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of each draw."""
    return (draws(key, idx) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def uniform_int(key: int, idx, lo: int, hi: int) -> np.ndarray:
    """Integers in [lo, hi] (inclusive) by multiply-shift of the top 32 bits."""
    span = hi - lo + 1
    top = (draws(key, idx) >> np.uint64(32)).astype(np.uint64)
    return (lo + ((top * np.uint64(span)) >> np.uint64(32))).astype(np.int64)
