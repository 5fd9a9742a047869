"""Helpers for the GPU parity tests: run the libah path on a plan and run the
oracle on the same bytes."""
import sys

import numpy as np

from oracle import decoy as odecoy
from oracle import iupac
from oracle import pair as opair
from oracle import scan as oscan
from oracle import tm as otm
from synth import fill, gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(p, pairs, dev, hit_cap=1 << 16, amp_cap=1 << 16, with_nmask=None, tm=None,
            filter_tm=False, min_tm=50.0):
    import torch

    from paper_2509_13300_amd import path

    if with_nmask is None:
        with_nmask = p.nrun_genome.size > 0
    ascii, off = gpu.fill_cuda(p, dev)
    coll, _ = path.pack(ascii, off, p.lengths, with_nmask=with_nmask)
    buf = path.alloc(coll, pairs, hit_cap, amp_cap, dev)
    path.run(coll, pairs, buf, tm=tm, filter_tm=filter_tm, min_tm=min_tm)
    torch.cuda.synchronize()
    return coll, buf


def run_oracle(p, pairs, tmp=None, filter_tm=False, min_tm=50.0):
    """Hits (with Tm) and amplicons of every pair, in canonical order; a decoy
    pair's records are the oracle's run on the reversed genomes, stated in
    the genomes' own coordinates."""
    seqs = [fill.genome_bytes(p, g) for g in range(p.n)]
    tmp = tmp if tmp is not None else otm.TmParams()
    hs, amps = [], []
    at = 0
    for q, pr in enumerate(pairs):
        if getattr(pr, "decoy", False):
            h, a = odecoy.run(seqs, [pr], tmp, filter_tm, min_tm)
            h, a = odecoy.to_forward_frame(h, a, p.lengths, [pr])
        else:
            h = oscan.scan_collection(seqs, [pr])
            h = otm.fill_tm(h, seqs, [pr], tmp)
            a = opair.call_amplicons(h, [pr], filter_tm, min_tm)
        h["pair"] = q
        a["pair"] = q
        a["plus_hit"] += at
        a["minus_hit"] += at
        at += h.size
        hs.append(h)
        amps.append(a)
    h = np.concatenate(hs) if hs else np.zeros(0, oscan.HIT_DTYPE)
    a = np.concatenate(amps) if amps else np.zeros(0, opair.AMP_DTYPE)
    return h, a


def hit_tuples_gpu(h):
    return [(int(x["pair"]), int(x["genome"]), int(x["pos"]), int(x["strand_primer"]) >> 1,
             int(x["strand_primer"]) & 1, int(x["mm"])) for x in h]


def hit_tuples_oracle(h):
    return [(int(x["pair"]), int(x["genome"]), int(x["pos"]), int(x["strand"]), int(x["primer"]),
             int(x["mm"])) for x in h]


def amp_tuples(a):
    return [(int(x["pair"]), int(x["genome"]), int(x["start"]), int(x["end"]), int(x["orient"]),
             int(x["plus_hit"]), int(x["minus_hit"])) for x in a]


def random_rate(pr):
    """Expected random sites per base (uniform bases), to pick hit-rich pairs."""
    tot = 0.0
    for prim in (pr.fwd, pr.rev):
        d = np.zeros(len(prim) + 1)
        d[0] = 1.0
        for c in prim:
            m = len(iupac.SETS[c]) / 4
            d[1:] = d[1:] * m + d[:-1] * (1 - m)
            d[0] *= m
        tot += 2 * d[: pr.k + 1].sum()
    return tot


# ---- the oracle over a whole collection, one genome per task, in worker
# processes (the plain single-pair path; the genome bytes are regenerated in
# each worker from the plan's seeds).
_POOL_PLAN = None


def _pool_init(p):
    global _POOL_PLAN
    _POOL_PLAN = p


def _oracle_genome(args):
    g, pr = args
    seq = fill.genome_bytes(_POOL_PLAN, g)
    h = oscan.scan_sequence(seq, pr.fwd, pr.rev, pr.k, pr.clamp)
    h["genome"] = 0
    h = otm.fill_tm(h, [seq], [pr])
    a = opair.call_amplicons(h, [pr])
    return g, h, a


def oracle_pool_workers() -> int:
    import os

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return max(1, min(16, cores))  # at most 16: one GPU's share of host cores


def run_oracle_pool(p, pr, ids=None, label="oracle"):
    """Hits (with Tm) and amplicons of pair ``pr`` over genomes ``ids`` of
    plan ``p`` (all by default), in canonical order with genome ids of the
    plan and hit indices into the returned hits."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import time

    ids = list(range(p.n)) if ids is None else [int(g) for g in ids]
    # longest first, so the pool does not end on one long genome
    order = sorted(ids, key=lambda g: -int(p.lengths[g]))
    workers = oracle_pool_workers()
    res = {}
    t0 = time.perf_counter()
    # an executor (not multiprocessing.Pool): a worker that dies raises
    # BrokenProcessPool here instead of leaving the caller waiting
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"),
                                initializer=_pool_init, initargs=(p,)) as ex:
        futs = [ex.submit(_oracle_genome, (g, pr)) for g in order]
        for i, f in enumerate(cf.as_completed(futs)):
            g, h, a = f.result()
            res[g] = (h, a)
            if (i + 1) % 100 == 0 or i + 1 == len(order):
                say(f"{label}: {i + 1}/{len(order)} genomes on {workers} processes, "
                    f"{time.perf_counter() - t0:.1f} s")
    hs, amps, at = [], [], 0
    for g in ids:
        h, a = res[g]
        h = h.copy()
        a = a.copy()
        h["genome"] = g
        a["genome"] = g
        a["plus_hit"] += at
        a["minus_hit"] += at
        at += h.size
        hs.append(h)
        amps.append(a)
    h = np.concatenate(hs) if hs else np.zeros(0, oscan.HIT_DTYPE)
    a = np.concatenate(amps) if amps else np.zeros(0, opair.AMP_DTYPE)
    return h, a
