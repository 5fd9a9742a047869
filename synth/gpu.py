"""GPU realisation of a plan (same bytes as ``synth.fill``), via libsynth.so.

Used to build large synthetic collections directly in HBM; the tests check it
against the numpy filler byte for byte on small plans.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import rng
from .plan import T_MUT, Plan

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libsynth.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run python -m paper_2509_13300_amd.build")
        _LIB = ctypes.CDLL(path)
        vp, u32 = ctypes.c_void_p, ctypes.c_uint32
        _LIB.synth_fill_background.argtypes = [vp, vp, u32, vp, vp, vp]
        _LIB.synth_fill_plants.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp, vp, u32, vp]
        _LIB.synth_fill_nruns.argtypes = [vp, vp, vp, u32, vp]
    return _LIB


def stream_keys(seed: int, base: int, ids: np.ndarray) -> np.ndarray:
    ids = np.asarray(ids, dtype=np.uint64)
    with np.errstate(over="ignore"):
        a = np.uint64((seed * rng.GAMMA) & rng.MASK64)
        b = (np.uint64(base) | ids) * np.uint64(rng.STREAM_MUL)
    return a ^ b


def fill_cuda(plan: Plan, device="cuda:0", stream=None):
    """Return (ascii uint8 tensor, offsets int64 tensor) on ``device``."""
    import torch

    plan.check()  # every write below stays inside its genome
    lib = _lib()
    dev = torch.device(device)
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream)
    off = plan.offsets
    total = int(off[-1])
    out = torch.empty(max(total, 1), dtype=torch.uint8, device=dev)
    d_off = torch.from_numpy(off).to(dev)
    keys = torch.from_numpy(stream_keys(plan.seed, rng.S_BASES, plan.source_ids()).view(np.int64)).to(dev)
    thr = torch.from_numpy(plan.thresholds.astype(np.uint32).reshape(-1).view(np.int32)).to(dev)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    rc = lib.synth_fill_background(ptr(out), ptr(d_off), plan.n, ptr(keys), ptr(thr), st)
    if rc:
        raise RuntimeError(f"synth_fill_background failed: {rc}")
    m = int(plan.plant_genome.size)
    if m:
        tl_all = np.array([len(t) for t in plan.templates], dtype=np.int64)
        tstart_all = np.zeros(len(plan.templates), dtype=np.int64)
        np.cumsum(tl_all[:-1], out=tstart_all[1:])
        tid = plan.plant_template.astype(np.int64)
        tlen = tl_all[tid]
        coff = np.zeros(m + 1, dtype=np.int64)
        np.cumsum(tlen, out=coff[1:])
        dest = off[plan.plant_genome] + plan.plant_pos
        mkeys = stream_keys(plan.seed, rng.S_MUT, plan.copy_ids())
        tb = np.frombuffer(b"".join(plan.templates), dtype=np.uint8)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(dev)  # noqa: E731
        d_coff, d_dest = t(coff, np.int64), t(dest, np.int64)
        d_strand, d_tstart = t(plan.plant_strand, np.uint8), t(tstart_all[tid], np.int64)
        d_tlen, d_tb = t(tlen, np.int32), t(tb, np.uint8)
        d_mk = t(mkeys.view(np.int64), np.int64)
        rc = lib.synth_fill_plants(ptr(out), ptr(d_coff), m, ptr(d_dest), ptr(d_strand), ptr(d_tstart),
                                   ptr(d_tlen), ptr(d_tb), ptr(d_mk), T_MUT, st)
        if rc:
            raise RuntimeError(f"synth_fill_plants failed: {rc}")
    r = int(plan.nrun_genome.size)
    if r:
        pos = torch.from_numpy((off[plan.nrun_genome] + plan.nrun_pos).astype(np.int64)).to(dev)
        ln = torch.from_numpy(plan.nrun_len.astype(np.int32)).to(dev)
        rc = lib.synth_fill_nruns(ptr(out), ptr(pos), ptr(ln), r, st)
        if rc:
            raise RuntimeError(f"synth_fill_nruns failed: {rc}")
    return out, d_off
