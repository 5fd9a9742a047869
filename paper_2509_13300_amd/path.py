"""Thin driver of the libah path for Python callers (tests, bench, serving).

It allocates device buffers with torch (the caller side of the C ABI) and
calls the entry points in order: pack, scan, Tm, pair.  No arithmetic of the
method happens here.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import _lib as L


@dataclasses.dataclass
class PackedCollection:
    words: "object"       # torch.int32 [2 * W]
    nmask: "object"       # torch.int32 [W] or None
    word_off: "object"    # torch.int64 [n + 1]
    len: "object"         # torch.int32 [n]
    n: int
    max_len: int
    total_bp: int
    lengths: np.ndarray   # host copy of the lengths

    def view(self) -> L.ah_genomes:
        g = L.ah_genomes()
        g.words = self.words.data_ptr()
        g.nmask = self.nmask.data_ptr() if self.nmask is not None else None
        g.word_off = self.word_off.data_ptr()
        g.len = self.len.data_ptr()
        g.n = self.n
        g.max_len = max(1, self.max_len)
        return g


def pack(ascii, ascii_off, lengths, with_nmask: bool = False, stream=None):
    """Pack ASCII genomes resident on the GPU.  Returns (collection,
    non-ACGT count tensor or None)."""
    import torch

    lengths = np.asarray(lengths, dtype=np.int64)
    dev = ascii.device
    word_off = L.ah_pack_layout(lengths)
    W = int(word_off[-1])
    words = torch.empty(2 * max(W, 1), dtype=torch.int32, device=dev)
    d_word_off = torch.from_numpy(word_off.view(np.int64)).to(dev)
    d_len = torch.empty(max(lengths.size, 1), dtype=torch.int32, device=dev)
    nmask = torch.empty(max(W, 1), dtype=torch.int32, device=dev) if with_nmask else None
    non_acgt = torch.empty(max(lengths.size, 1), dtype=torch.int64, device=dev) if with_nmask else None
    L.ah_pack_genomes(ascii, ascii_off, lengths.size, d_word_off, words, d_len, nmask, non_acgt,
                      stream)
    coll = PackedCollection(words, nmask, d_word_off, d_len, int(lengths.size),
                            int(lengths.max()) if lengths.size else 1, int(lengths.sum()), lengths)
    return coll, non_acgt


@dataclasses.dataclass
class QueryBuffers:
    hits: "object"
    hit_res: "object"
    scan_work: "object"
    amps: "object"
    amp_res: "object"
    pair_work: "object"
    hit_cap: int
    amp_cap: int


def alloc(coll: PackedCollection, n_pairs: int, hit_cap: int, amp_cap: int, device) -> QueryBuffers:
    import torch

    g = coll.view()
    sw = L.ah_scan_workspace_bytes(g, n_pairs, hit_cap)
    pw = L.ah_pair_workspace_bytes(hit_cap, n_pairs)
    return QueryBuffers(
        hits=torch.empty(max(hit_cap, 1) * 16, dtype=torch.uint8, device=device),
        hit_res=torch.zeros(24, dtype=torch.uint8, device=device),
        scan_work=torch.empty(sw, dtype=torch.uint8, device=device),
        amps=torch.empty(max(amp_cap, 1) * 24, dtype=torch.uint8, device=device),
        amp_res=torch.zeros(24, dtype=torch.uint8, device=device),
        pair_work=torch.empty(pw, dtype=torch.uint8, device=device),
        hit_cap=hit_cap, amp_cap=amp_cap)


def run(coll: PackedCollection, pairs: Sequence, buf: QueryBuffers, tm: Optional[L.ah_tm_params] = None,
        filter_tm: bool = False, min_tm: float = 50.0, stream=None, do_tm: bool = True,
        do_pair: bool = True):
    """Enqueue scan (+ Tm, + pairing) for ``pairs`` over the collection."""
    g = coll.view()
    pp = L.primer_pairs(pairs)
    L.ah_scan_primers(g, pp, buf.hits, buf.hit_cap, buf.hit_res, buf.scan_work, stream)
    if do_tm:
        L.ah_tm(g, pp, tm if tm is not None else L.tm_params(), buf.hits, buf.hit_res, buf.hit_cap,
                stream)
    if do_pair:
        L.ah_pair_amplicons(buf.hits, buf.hit_res, buf.hit_cap, pp, L.windows(pairs, filter_tm, min_tm),
                            buf.amps, buf.amp_cap, buf.amp_res, buf.pair_work, stream)


def result(res_tensor) -> dict:
    r = np.frombuffer(res_tensor.cpu().numpy().tobytes(), dtype=np.dtype(
        [("count", "<u8"), ("required", "<u8"), ("status", "<i4"), ("reserved", "<u4")]))[0]
    return {"count": int(r["count"]), "required": int(r["required"]), "status": int(r["status"])}


def hits_numpy(buf: QueryBuffers) -> np.ndarray:
    n = result(buf.hit_res)["count"]
    return np.frombuffer(buf.hits[: n * 16].cpu().numpy().tobytes(), dtype=L.HIT_DTYPE).copy()


def amps_numpy(buf: QueryBuffers) -> np.ndarray:
    n = result(buf.amp_res)["count"]
    return np.frombuffer(buf.amps[: n * 24].cpu().numpy().tobytes(), dtype=L.AMP_DTYPE).copy()


def capture(coll: PackedCollection, pairs: Sequence, buf: QueryBuffers, tm=None, filter_tm=False,
            min_tm: float = 50.0):
    """Record one scan -> Tm -> pairing pass for ``pairs`` into a hipGraph
    (through torch.cuda.CUDAGraph).  Call ``run`` once with the same pairs
    first, so that the specialised kernel and per-set tables exist; the graph
    then replays with no host-side work."""
    import torch

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run(coll, pairs, buf, tm=tm, filter_tm=filter_tm, min_tm=min_tm)
    return g


def subset_view(coll: PackedCollection, n: int) -> L.ah_genomes:
    """View of the first ``n`` genomes of a packed collection (no copy)."""
    g = coll.view()
    g.n = min(n, coll.n)
    return g
