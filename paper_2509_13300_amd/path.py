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


def read_fasta(text: bytes, device, with_nmask: bool = True, stream=None):
    """FASTA text -> a packed collection on the device (one sequence per
    record: a genome of several contigs is several records).  The host reads
    the records (``ah_fasta_read``) straight into pinned memory, the bytes
    cross to the device, the device packs them.  Returns (collection, names,
    non-ACGT count per record or None)."""
    import torch

    seq, off, names = L.fasta_read(text, pinned=True)
    lengths = np.diff(off)
    ascii = seq.to(device, non_blocking=True)
    d_off = torch.from_numpy(off).to(device)
    coll, non_acgt = pack(ascii, d_off, lengths, with_nmask=with_nmask, stream=stream)
    return coll, names, non_acgt


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


def alloc(coll: PackedCollection, pairs, hit_cap: int, amp_cap: int, device) -> QueryBuffers:
    """Buffers for queries of `pairs` (a pair list, sizing the scan's candidate
    list for their filters; or a pair count, for the minimum).  The site and
    amplicon buffers start filled with the byte 0xA5, so that a record a
    result counts but no kernel wrote shows up as such (genome 0xA5A5A5A5)
    instead of as whatever the memory held before."""
    import torch

    g = coll.view()
    n_pairs = pairs if isinstance(pairs, int) else len(pairs)
    sw = L.ah_scan_workspace_bytes(g, pairs, hit_cap)
    pw = L.ah_pair_workspace_bytes(hit_cap, n_pairs)
    return QueryBuffers(
        hits=torch.full((max(hit_cap, 1) * 16,), 0xA5, dtype=torch.uint8, device=device),
        hit_res=torch.zeros(24, dtype=torch.uint8, device=device),
        scan_work=torch.empty(sw, dtype=torch.uint8, device=device),
        amps=torch.full((max(amp_cap, 1) * 24,), 0xA5, dtype=torch.uint8, device=device),
        amp_res=torch.zeros(24, dtype=torch.uint8, device=device),
        pair_work=torch.empty(pw, dtype=torch.uint8, device=device),
        hit_cap=hit_cap, amp_cap=amp_cap)


def run(coll: PackedCollection, pairs: Sequence, buf: QueryBuffers, tm: Optional[L.ah_tm_params] = None,
        filter_tm: bool = False, min_tm: float = 50.0, stream=None, do_tm: bool = True,
        do_pair: bool = True, fused: bool = True):
    """Enqueue scan (+ Tm, + pairing) for ``pairs`` over the collection: the
    whole query in one ah_query call (``fused``), or the separate calls."""
    g = coll.view()
    pp = L.primer_pairs(pairs)
    if fused and do_tm and do_pair:
        L.ah_query(g, pp, L.windows(pairs, filter_tm, min_tm),
                   tm if tm is not None else L.tm_params(), buf.hits, buf.hit_cap, buf.hit_res,
                   buf.amps, buf.amp_cap, buf.amp_res, buf.scan_work, buf.pair_work, stream)
        return
    L.ah_scan_primers(g, pp, buf.hits, buf.hit_cap, buf.hit_res, buf.scan_work, stream)
    if do_tm:
        L.ah_tm(g, pp, tm if tm is not None else L.tm_params(), buf.hits, buf.hit_res, buf.hit_cap,
                stream)
    if do_pair:
        L.ah_pair_amplicons(buf.hits, buf.hit_res, buf.hit_cap, pp, L.windows(pairs, filter_tm, min_tm),
                            buf.amps, buf.amp_cap, buf.amp_res, buf.pair_work, stream)


@dataclasses.dataclass
class FastaBuffers:
    text: "object"         # uint8 [text_cap]
    text_res: "object"     # ah_result
    seq_hash: "object"     # int64 [amp_cap] (uint64 values)
    amplitype: "object"    # int64 [n_pairs * n_genomes] (uint64 values)
    amplitype_n: "object"  # int32 [n_pairs * n_genomes] (uint32 values)
    work: "object"


def fasta_alloc(coll: PackedCollection, n_pairs: int, amp_cap: int, text_cap: int, device) -> FastaBuffers:
    import torch

    groups = max(1, n_pairs * coll.n)
    return FastaBuffers(
        torch.empty(max(1, text_cap), dtype=torch.uint8, device=device),
        torch.zeros(24, dtype=torch.uint8, device=device),
        torch.empty(max(1, amp_cap), dtype=torch.int64, device=device),
        torch.empty(groups, dtype=torch.int64, device=device),
        torch.empty(groups, dtype=torch.int32, device=device),
        torch.empty(L.ah_fasta_workspace_bytes(amp_cap), dtype=torch.uint8, device=device))


def fasta(coll: PackedCollection, n_pairs: int, buf: QueryBuffers, fb: FastaBuffers, stream=None):
    """Enqueue the FASTA records, sequence hashes and amplitypes of the
    amplicons in ``buf`` (after ``run``)."""
    L.ah_amplicon_fasta(coll.view(), buf.hits, buf.amps, buf.amp_res, buf.amp_cap, n_pairs,
                        fb.text, fb.text_res, fb.seq_hash, fb.amplitype, fb.amplitype_n, fb.work,
                        stream)


def fasta_text(fb: FastaBuffers) -> bytes:
    n = result(fb.text_res)["count"]
    return fb.text[:n].cpu().numpy().tobytes()


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
            min_tm: float = 50.0, fused: bool = True):
    """Record one scan -> Tm -> pairing pass for ``pairs`` into a hipGraph
    (through torch.cuda.CUDAGraph).  Call ``run`` once with the same pairs
    first, so that the specialised kernel and per-set tables exist; the graph
    then replays with no host-side work."""
    import torch

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run(coll, pairs, buf, tm=tm, filter_tm=filter_tm, min_tm=min_tm, fused=fused)
    return g


def subset_view(coll: PackedCollection, n: int) -> L.ah_genomes:
    """View of the first ``n`` genomes of a packed collection (no copy)."""
    g = coll.view()
    g.n = min(n, coll.n)
    return g


def to_host(coll: PackedCollection, pin: bool = True) -> L.HostGenomes:
    """Copy a packed collection from HBM into (pinned) host memory, in the
    layout that the streaming calls read."""
    import torch

    words = torch.empty(coll.words.numel(), dtype=torch.int32, pin_memory=pin)
    words.copy_(coll.words)
    nmask = None
    if coll.nmask is not None:
        nmask = torch.empty(coll.nmask.numel(), dtype=torch.int32, pin_memory=pin)
        nmask.copy_(coll.nmask)
    return L.HostGenomes(words, coll.word_off.cpu().numpy().view(np.uint64), coll.lengths, nmask)


@dataclasses.dataclass
class StreamBuffers:
    hits: "object"
    hit_res: "object"
    amps: "object"
    amp_res: "object"
    work: "object"
    hit_cap: int
    amp_cap: int
    cfg: L.ah_stream_config


def stream_alloc(hg: L.HostGenomes, pairs, hit_cap: int, amp_cap: int, device,
                 chunk_words: int, n_slots: int = 3) -> StreamBuffers:
    import torch

    cfg = L.stream_config(chunk_words, n_slots)
    wb = L.ah_stream_workspace_bytes(hg, cfg, pairs, hit_cap)
    return StreamBuffers(
        hits=torch.empty(max(hit_cap, 1) * 16, dtype=torch.uint8, device=device),
        hit_res=torch.zeros(24, dtype=torch.uint8, device=device),
        amps=torch.empty(max(amp_cap, 1) * 24, dtype=torch.uint8, device=device),
        amp_res=torch.zeros(24, dtype=torch.uint8, device=device),
        work=torch.empty(wb, dtype=torch.uint8, device=device),
        hit_cap=hit_cap, amp_cap=amp_cap, cfg=cfg)


def stream_run(hg: L.HostGenomes, pairs: Sequence, buf: StreamBuffers,
               tm: Optional[L.ah_tm_params] = None, filter_tm: bool = False,
               min_tm: float = 50.0, stream=None, copy_streams=()):
    """Scan, Tm and pairing over a host-resident packed collection, copied to
    the GPU chunk by chunk on ``copy_streams``.  Blocks until done."""
    L.ah_stream_query(hg, buf.cfg, L.primer_pairs(pairs), L.windows(pairs, filter_tm, min_tm),
                      tm if tm is not None else L.tm_params(), buf.hits, buf.hit_cap, buf.hit_res,
                      buf.amps, buf.amp_cap, buf.amp_res, buf.work, stream=stream,
                      copy_streams=copy_streams)


def pack_to_host(fill_batch, lengths, device, batch_genomes: int = 500,
                 with_nmask: bool = False, pin: bool = True) -> L.HostGenomes:
    """Build a packed collection in (pinned) host memory without holding it
    all on the GPU: ``fill_batch(ids)`` returns (ascii, ascii_off) device
    tensors for genome ids ``ids``; each batch is packed on the GPU and its
    words copied to their place in the host layout."""
    import torch

    lengths = np.asarray(lengths, dtype=np.int64)
    word_off = L.ah_pack_layout(lengths)
    W = int(word_off[-1])
    words = torch.empty(2 * max(W, 1), dtype=torch.int32, pin_memory=pin)
    nmask = torch.empty(max(W, 1), dtype=torch.int32, pin_memory=pin) if with_nmask else None
    for a in range(0, lengths.size, batch_genomes):
        ids = np.arange(a, min(a + batch_genomes, lengths.size))
        ascii, off = fill_batch(ids)
        c, _ = pack(ascii, off, lengths[ids], with_nmask=with_nmask)
        w0, w1 = int(word_off[ids[0]]), int(word_off[ids[-1] + 1])
        assert int(c.word_off[-1].item()) == w1 - w0  # same per-genome layout
        words[2 * w0: 2 * w1].copy_(c.words[: 2 * (w1 - w0)])
        if with_nmask:
            nmask[w0:w1].copy_(c.nmask[: w1 - w0])
        del ascii, off, c
    torch.cuda.synchronize(device)
    return L.HostGenomes(words, word_off, lengths, nmask)


def to_device(hg: L.HostGenomes, device) -> PackedCollection:
    """Copy a host-resident packed collection into HBM (the resident form)."""
    import torch

    words = hg.words.to(device)
    nmask = hg.nmask.to(device) if hg.nmask is not None else None
    d_off = torch.from_numpy(hg.word_off.view(np.int64)).to(device)
    d_len = torch.from_numpy(np.maximum(hg.len, 0).astype(np.int32)).to(device) if hg.n else \
        torch.zeros(1, dtype=torch.int32, device=device)
    lens = hg.len.astype(np.int64)
    return PackedCollection(words, nmask, d_off, d_len, hg.n, int(lens.max()) if hg.n else 1,
                            int(lens.sum()), lens)


def pack_resident(fill_batch, lengths, device, batch_genomes: int = 500,
                  with_nmask: bool = False) -> PackedCollection:
    """Build a packed collection in HBM batch by batch (only one batch of ASCII
    on the GPU at a time): ``fill_batch(ids)`` returns (ascii, ascii_off)
    device tensors for genome ids ``ids``."""
    import torch

    lengths = np.asarray(lengths, dtype=np.int64)
    word_off = L.ah_pack_layout(lengths)
    W = int(word_off[-1])
    words = torch.empty(2 * max(W, 1), dtype=torch.int32, device=device)
    nmask = torch.empty(max(W, 1), dtype=torch.int32, device=device) if with_nmask else None
    d_len = torch.empty(max(lengths.size, 1), dtype=torch.int32, device=device)
    for a in range(0, lengths.size, batch_genomes):
        ids = np.arange(a, min(a + batch_genomes, lengths.size))
        ascii, off = fill_batch(ids)
        c, _ = pack(ascii, off, lengths[ids], with_nmask=with_nmask)
        w0, w1 = int(word_off[ids[0]]), int(word_off[ids[-1] + 1])
        words[2 * w0: 2 * w1].copy_(c.words[: 2 * (w1 - w0)])
        if with_nmask:
            nmask[w0:w1].copy_(c.nmask[: w1 - w0])
        d_len[ids[0]: ids[-1] + 1].copy_(c.len[: ids.size])
        del ascii, off, c
    d_off = torch.from_numpy(word_off.view(np.int64)).to(device)
    torch.cuda.synchronize(device)
    return PackedCollection(words, nmask, d_off, d_len, int(lengths.size),
                            int(lengths.max()) if lengths.size else 1, int(lengths.sum()), lengths)


class Server:
    """Request loop over a collection resident in HBM (libah's serving
    runtime): jobs are admitted as they arrive, split into parts, and run on
    several device streams at once inside a fixed device pool."""

    def __init__(self, coll: PackedCollection, pool_bytes: int, device, **cfg):
        import torch

        self.coll = coll  # the server borrows its device views
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        self.handle = L.ah_server_create(coll.view(), coll.lengths, L.server_config(**cfg),
                                         self.pool)

    def submit(self, pair, genomes=None, tm=None, filter_tm=False, min_tm=50.0) -> int:
        return L.ah_server_submit(self.handle, pair, genomes, tm, filter_tm, min_tm)

    def wait(self, timeout_s: float = 1.0) -> Optional[dict]:
        return L.ah_server_wait(self.handle, timeout_s)

    def now(self) -> float:
        return L.ah_server_now(self.handle)

    def result(self, status: dict):
        """(hits, amplicons) of a finished job as numpy records: the parts
        concatenated; amplicon hit indices refer to the concatenated hits."""
        import ctypes

        hs, as_, base = [], [], 0
        for i in range(status["n_parts"]):
            pt = L.ah_server_part(self.handle, status["job"], i)
            h = np.frombuffer(ctypes.string_at(pt.hits, pt.n_hits * 16), dtype=L.HIT_DTYPE) \
                if pt.n_hits else np.zeros(0, L.HIT_DTYPE)
            a = np.frombuffer(ctypes.string_at(pt.amplicons, pt.n_amplicons * 24),
                              dtype=L.AMP_DTYPE).copy() if pt.n_amplicons else np.zeros(0, L.AMP_DTYPE)
            a["plus_hit"] += np.uint32(base)
            a["minus_hit"] += np.uint32(base)
            hs.append(h)
            as_.append(a)
            base += h.size
        cat = lambda xs, dt: np.concatenate(xs) if xs else np.zeros(0, dt)  # noqa: E731
        return cat(hs, L.HIT_DTYPE), cat(as_, L.AMP_DTYPE)

    def release(self, job: int):
        L.ah_server_release(self.handle, job)

    def stats(self) -> dict:
        return L.ah_server_stats_get(self.handle)

    def close(self):
        if self.handle:
            L.ah_server_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
