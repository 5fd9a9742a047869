"""Seeded synthetic workload plans (genome collections, primer pairs, jobs).

A *plan* is the small description from which every base of a synthetic genome
collection is computed independently: per-genome lengths and base-composition
thresholds, the operon templates, where mutated copies of them are written,
and optional runs of non-ACGT bytes.  ``synth.fill`` turns a plan into ASCII on
the CPU; ``synth.gpu`` does the same on the GPU.  Neither contains any of the
primer-matching, melting-temperature or pairing arithmetic.

Recipe (one line per workload, sizes as in the stated configurations):

* plain: one 5,000,000 bp genome, GC 0.5, five copies of a 1,500 bp operon
  template mutated at 1% substitutions; fwd 20 nt / rev 19 nt primers with
  three 2-fold degenerate codes each; k = 2, 3' clamp 5, window 200-2000.
* collection(n): n genomes, lengths log-normal (median 4 Mbp, sigma 0.3 in
  ln space) clipped to [1, 12] Mbp, GC uniform in [0.30, 0.70] per genome,
  1-15 copies of a 1,500 bp operon at 1%; a V4-like pair (19 / 20 nt, 2-fold
  and 4-fold codes, degeneracy <= 16 per primer); k = 2; window 200-500.
* stream(n): the collection law with a 5 kbp operon and a long-amplicon pair
  of 192 + 768 oligos (fwd 20 nt with N,N,N,H; rev 18 nt with N,N,N,D,R,W);
  k = 3; window 2000-5500.
* batched(n): lengths clipped to [0.5, 12] Mbp; 64 pairs with primer lengths
  U{15..30}, degeneracy 2^b per primer with b ~ U{0..10} (N counts two bits),
  k ~ U{0..3}, windows from two sorted draws in U[100, 6000] with gap >= 100;
  each genome carries 1-3 copies of targets of 8 of the pairs.
* serving(n): the collection law; a pool of 1,024 pairs from the batched law;
  jobs with Poisson arrivals over genome-id subsets of log-uniform size.

Copies are placed one per equal slot of the genome (uniform inside the slot),
so they never overlap; each copy is on a uniformly drawn strand, and each base
of a copy is independently replaced, with probability 0.01, by one of the three
other bases chosen uniformly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import rng

BASES = b"ACGT"
# Members of each IUPAC code, used only to realise a concrete site from a
# degenerate primer when building operon templates.
_MEMBERS = {
    "A": "A", "C": "C", "G": "G", "T": "T",
    "R": "AG", "Y": "CT", "S": "CG", "W": "AT", "K": "GT", "M": "AC",
    "B": "CGT", "D": "AGT", "H": "ACT", "V": "ACG", "N": "ACGT",
}
_TWO_FOLD = "RYSWKM"
_COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}

T_MUT = round(0.01 * 2**32)  # per-base substitution threshold (p = 0.01)


@dataclasses.dataclass
class PairSpec:
    fwd: str
    rev: str
    k: int = 2
    clamp: int = 0
    min_len: int = 200
    max_len: int = 2000
    decoy: bool = False  # run on the genomes reversed (the decoy estimate)


@dataclasses.dataclass
class Plan:
    """Everything needed to compute the ASCII bytes of a genome collection."""

    seed: int
    lengths: np.ndarray          # int64 [n]
    thresholds: np.ndarray       # uint32 [n, 3]  cumulative A / C / G cut-offs
    templates: List[bytes]       # operon templates (top strand)
    plant_genome: np.ndarray     # int64 [m]
    plant_pos: np.ndarray        # int64 [m]
    plant_strand: np.ndarray     # int8  [m]  0 = as template, 1 = reverse complement
    plant_template: np.ndarray   # int64 [m]
    nrun_genome: np.ndarray      # int64 [r]  runs of 'N' bytes (real-FASTA stand-in)
    nrun_pos: np.ndarray         # int64 [r]
    nrun_len: np.ndarray         # int64 [r]
    pairs: List[PairSpec]
    name: str = "custom"
    # per template: (fwd site offset, rev site offset, pair index) in the
    # template's top strand; the rev site holds the reverse complement.
    template_sites: List[tuple] = dataclasses.field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.lengths.shape[0])

    @property
    def total_bp(self) -> int:
        return int(self.lengths.sum())

    @property
    def offsets(self) -> np.ndarray:
        off = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(self.lengths, out=off[1:])
        return off

    def subset(self, ids) -> "Plan":
        """Plan restricted to genome ids ``ids`` (renumbered 0..len(ids)-1).

        Base draws stay keyed by the *original* genome id, so a genome's bytes
        are identical in the subset and in the full collection."""
        ids = np.asarray(ids, dtype=np.int64)
        remap = -np.ones(self.n, dtype=np.int64)
        remap[ids] = np.arange(ids.size)
        keep = remap[self.plant_genome] >= 0
        keepn = remap[self.nrun_genome] >= 0
        p = dataclasses.replace(
            self,
            lengths=self.lengths[ids].copy(),
            thresholds=self.thresholds[ids].copy(),
            plant_genome=remap[self.plant_genome[keep]],
            plant_pos=self.plant_pos[keep].copy(),
            plant_strand=self.plant_strand[keep].copy(),
            plant_template=self.plant_template[keep].copy(),
            nrun_genome=remap[self.nrun_genome[keepn]],
            nrun_pos=self.nrun_pos[keepn].copy(),
            nrun_len=self.nrun_len[keepn].copy(),
        )
        p._source_ids = ids if not hasattr(self, "_source_ids") else self._source_ids[ids]
        p._copy_ids = (np.flatnonzero(keep) if not hasattr(self, "_copy_ids")
                       else self._copy_ids[keep])
        return p

    def with_lengths(self, lengths) -> "Plan":
        """Same plan with new genome lengths; copies and N runs that no longer
        fit inside their genome are dropped."""
        lengths = np.asarray(lengths, dtype=np.int64).copy()
        tl = np.array([len(t) for t in self.templates], dtype=np.int64)
        keep = self.plant_pos + tl[self.plant_template] <= lengths[self.plant_genome]
        keepn = self.nrun_pos + self.nrun_len <= lengths[self.nrun_genome]
        p = dataclasses.replace(
            self, lengths=lengths,
            plant_genome=self.plant_genome[keep], plant_pos=self.plant_pos[keep],
            plant_strand=self.plant_strand[keep], plant_template=self.plant_template[keep],
            nrun_genome=self.nrun_genome[keepn], nrun_pos=self.nrun_pos[keepn],
            nrun_len=self.nrun_len[keepn])
        if hasattr(self, "_source_ids"):
            p._source_ids = self._source_ids
        p._copy_ids = self.copy_ids()[keep]
        return p

    def check(self) -> None:
        """Raise if a planted copy or N run does not lie inside its genome."""
        tl = np.array([len(t) for t in self.templates], dtype=np.int64)
        if self.plant_genome.size:
            end = self.plant_pos + tl[self.plant_template]
            if np.any(self.plant_pos < 0) or np.any(end > self.lengths[self.plant_genome]):
                raise ValueError("a planted copy lies outside its genome")
        if self.nrun_genome.size:
            end = self.nrun_pos + self.nrun_len
            if np.any(self.nrun_pos < 0) or np.any(end > self.lengths[self.nrun_genome]):
                raise ValueError("an N run lies outside its genome")

    # Identity of genome g / copy c for the per-base draw streams.
    def source_id(self, g: int) -> int:
        return int(self._source_ids[g]) if hasattr(self, "_source_ids") else int(g)

    def source_ids(self) -> np.ndarray:
        return (self._source_ids.copy() if hasattr(self, "_source_ids")
                else np.arange(self.n, dtype=np.int64))

    def copy_ids(self) -> np.ndarray:
        return (self._copy_ids.copy() if hasattr(self, "_copy_ids")
                else np.arange(self.plant_genome.size, dtype=np.int64))


# ---------------------------------------------------------------------------
# primer and template construction

def revcomp_plain(s: str) -> str:
    return "".join(_COMP[c] for c in reversed(s))


def random_primer(seed: int, primer_id: int, length: int, codes: str) -> str:
    """Random ACGT primer of ``length`` with the IUPAC ``codes`` placed at
    distinct random positions."""
    key = rng.stream_key(seed, rng.S_PRIMER | primer_id)
    base_idx = rng.uniform_int(key, np.arange(length), 0, 3)
    s = [chr(BASES[b]) for b in base_idx]
    # distinct positions by a keyed shuffle of 0..length-1
    order = np.argsort(rng.draws(key, np.arange(1000, 1000 + length)), kind="stable")
    for code, pos in zip(codes, order[: len(codes)]):
        s[int(pos)] = code
    return "".join(s)


def realize(seed: int, stream_id: int, primer: str) -> str:
    """One member oligo of a degenerate primer (uniform per position)."""
    key = rng.stream_key(seed, rng.S_PRIMER | (1 << 30) | stream_id)
    out = []
    for j, c in enumerate(primer):
        m = _MEMBERS[c]
        pick = int(rng.uniform_int(key, np.array([j]), 0, len(m) - 1)[0])
        out.append(m[pick])
    return "".join(out)


def template_sites(length: int, span: int, lf: int, lr: int):
    """Offsets of the fwd site and of the reverse-complemented rev site."""
    f0 = max(0, (length - span) // 2)
    return f0, f0 + span - lr


def operon_template(seed: int, template_id: int, length: int, pair: PairSpec,
                    span: int) -> bytes:
    """Random background with realize(fwd) at the left and the reverse
    complement of realize(rev) placed so the amplicon spans ``span`` bp."""
    key = rng.stream_key(seed, rng.S_TEMPLATE | template_id)
    bg = rng.uniform_int(key, np.arange(length), 0, 3)
    t = bytearray(BASES[b] for b in bg)
    f = realize(seed, 2 * template_id, pair.fwd)
    r = revcomp_plain(realize(seed, 2 * template_id + 1, pair.rev))
    f0, r0 = template_sites(length, span, len(pair.fwd), len(pair.rev))
    assert r0 + len(r) <= length and r0 >= f0 + len(f), "template too short for span"
    t[f0:f0 + len(f)] = f.encode()
    t[r0:r0 + len(r)] = r.encode()
    return bytes(t)


# ---------------------------------------------------------------------------
# collections

def _thresholds(gc: np.ndarray) -> np.ndarray:
    p_at = (1.0 - gc) / 2.0
    p_cg = gc / 2.0
    t_a = np.round(p_at * 2**32)
    t_c = t_a + np.round(p_cg * 2**32)
    t_g = t_c + np.round(p_cg * 2**32)
    th = np.stack([t_a, t_c, t_g], axis=1)
    return np.clip(th, 0, 2**32 - 1).astype(np.uint32)


def lognormal_lengths(seed: int, n: int, median: float, sigma: float, lo: float,
                      hi: float) -> np.ndarray:
    key = rng.stream_key(seed, rng.S_LEN)
    u1 = 1.0 - rng.uniform01(key, 2 * np.arange(n))
    u2 = rng.uniform01(key, 2 * np.arange(n) + 1)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    return np.clip(np.round(median * np.exp(sigma * z)), lo, hi).astype(np.int64)


def _plant(seed: int, lengths: np.ndarray, n_templates: int, tlen: List[int],
           copies_lo: int, copies_hi: int, template_choice=None):
    """Copies per genome, one per equal slot, uniform strand."""
    n = lengths.size
    keyp = rng.stream_key(seed, rng.S_PLANT)
    ncop = rng.uniform_int(keyp, np.arange(n), copies_lo, copies_hi)
    g = np.repeat(np.arange(n, dtype=np.int64), ncop)
    m = g.size
    slot = np.arange(m) - np.repeat(np.cumsum(ncop) - ncop, ncop)
    if template_choice is None:
        tid = rng.uniform_int(rng.stream_key(seed, rng.S_PLANT | 1), np.arange(m), 0,
                              n_templates - 1)
    else:
        tid = template_choice(g, slot)
    tl = np.asarray(tlen, dtype=np.int64)[tid]
    slot_len = lengths[g] // ncop[g]
    room = slot_len - tl
    if np.any(room < 0):
        raise ValueError("genome too short for its planted copies")
    u = rng.uniform01(rng.stream_key(seed, rng.S_PLANT | 2), np.arange(m))
    pos = g * 0 + slot * slot_len + np.floor(u * (room + 1)).astype(np.int64)
    strand = rng.uniform_int(rng.stream_key(seed, rng.S_PLANT | 3), np.arange(m), 0, 1)
    return g, pos.astype(np.int64), strand.astype(np.int8), tid.astype(np.int64)


def _empty():
    return np.zeros(0, dtype=np.int64)


def plain(seed: int = 13301) -> Plan:
    """One 5 Mbp genome with five mutated copies of a 1.5 kbp operon."""
    fwd = random_primer(seed, 0, 20, "".join(_TWO_FOLD[i] for i in
                                             rng.uniform_int(rng.stream_key(seed, rng.S_MISC | 1),
                                                             np.arange(3), 0, 5)))
    rev = random_primer(seed, 1, 19, "".join(_TWO_FOLD[i] for i in
                                             rng.uniform_int(rng.stream_key(seed, rng.S_MISC | 2),
                                                             np.arange(3), 0, 5)))
    pair = PairSpec(fwd, rev, k=2, clamp=5, min_len=200, max_len=2000)
    tmpl = operon_template(seed, 0, 1500, pair, 1200)
    lengths = np.array([5_000_000], dtype=np.int64)
    g, pos, strand, tid = _plant(seed, lengths, 1, [len(tmpl)], 5, 5)
    return Plan(seed, lengths, _thresholds(np.array([0.5])), [tmpl], g, pos, strand, tid,
                _empty(), _empty(), _empty(), [pair], name="plain-5Mbp",
                template_sites=[template_sites(1500, 1200, 20, 19) + (0,)])


V4_LIKE_CODES = ("YM", "NW")  # fwd degeneracy 4, rev degeneracy 8


def collection(n: int = 1000, seed: int = 13302, operon: int = 1500, span: int = 290,
               pair: Optional[PairSpec] = None, copies=(1, 15), lo=1e6, hi=12e6,
               median=4e6, name="collection") -> Plan:
    """The multi-genome law: log-normal lengths, per-genome GC, planted operons."""
    if pair is None:
        pair = PairSpec(random_primer(seed, 0, 19, V4_LIKE_CODES[0]),
                        random_primer(seed, 1, 20, V4_LIKE_CODES[1]),
                        k=2, clamp=0, min_len=200, max_len=500)
    lengths = lognormal_lengths(seed, n, median, 0.3, lo, hi)
    gc = 0.30 + 0.40 * rng.uniform01(rng.stream_key(seed, rng.S_GC), np.arange(n))
    tmpl = operon_template(seed, 0, operon, pair, span)
    g, pos, strand, tid = _plant(seed, lengths, 1, [len(tmpl)], copies[0], copies[1])
    return Plan(seed, lengths, _thresholds(gc), [tmpl], g, pos, strand, tid,
                _empty(), _empty(), _empty(), [pair], name=f"{name}-{n}",
                template_sites=[template_sites(operon, span, len(pair.fwd), len(pair.rev)) + (0,)])


def stream(n: int = 10000, seed: int = 13303) -> Plan:
    """Long-amplicon pair (192 + 768 oligos), k = 3, window 2000-5500."""
    pair = PairSpec(random_primer(seed, 0, 20, "NNNH"),
                    random_primer(seed, 1, 18, "NNNDRW"),
                    k=3, clamp=0, min_len=2000, max_len=5500)
    return collection(n, seed, operon=5000, span=2500, pair=pair, name="stream")


def _law_pair(seed: int, pid: int) -> PairSpec:
    key = rng.stream_key(seed, rng.S_MISC | (1 << 20) | pid)
    lf, lr = (int(x) for x in rng.uniform_int(key, np.arange(2), 15, 30))
    bits = [int(x) for x in rng.uniform_int(key, np.arange(2, 4), 0, 10)]
    codes = []
    for side, (b, length) in enumerate(zip(bits, (lf, lr))):
        n_n = int(rng.uniform_int(key, np.array([10 + side]), 0, b // 2)[0])
        n_two = b - 2 * n_n
        while n_n + n_two > length:  # keep codes within the primer length
            n_n += 1
            n_two -= 2
        two = [_TWO_FOLD[int(i)] for i in
               rng.uniform_int(key, np.arange(100 + 40 * side, 100 + 40 * side + n_two), 0, 5)]
        codes.append("N" * n_n + "".join(two))
    k = int(rng.uniform_int(key, np.array([20]), 0, 3)[0])
    a, b = (int(x) for x in rng.uniform_int(key, np.arange(21, 23), 100, 6000))
    lo, hi = min(a, b), max(a, b)
    if hi - lo < 100:
        hi = min(6000, lo + 100)
        lo = hi - 100
    return PairSpec(random_primer(seed, 2 * pid + 2, lf, codes[0]),
                    random_primer(seed, 2 * pid + 3, lr, codes[1]),
                    k=k, clamp=0, min_len=lo, max_len=hi)


def law_pairs(seed: int, count: int) -> List[PairSpec]:
    return [_law_pair(seed, i) for i in range(count)]


def batched(n: int = 2000, seed: int = 13304, n_pairs: int = 64, n_targets: int = 8) -> Plan:
    """Uneven genomes carrying 1-3 copies of targets of ``n_targets`` pairs."""
    pairs = law_pairs(seed, n_pairs)
    templates, sites = [], []
    for t in range(n_targets):
        p = pairs[t]
        span = (p.min_len + p.max_len) // 2
        span = max(span, len(p.fwd) + len(p.rev) + 10)
        templates.append(operon_template(seed, t, span + 200, p, span))
        sites.append(template_sites(span + 200, span, len(p.fwd), len(p.rev)) + (t,))
    lengths = lognormal_lengths(seed, n, 4e6, 0.3, 0.5e6, 12e6)
    gc = 0.30 + 0.40 * rng.uniform01(rng.stream_key(seed, rng.S_GC), np.arange(n))
    g, pos, strand, tid = _plant(seed, lengths, n_targets, [len(t) for t in templates], 1, 3)
    return Plan(seed, lengths, _thresholds(gc), templates, g, pos, strand, tid,
                _empty(), _empty(), _empty(), pairs, name=f"batched-{n}", template_sites=sites)


def serving(n: int = 100000, seed: int = 13305, pool: int = 1024, n_targets: int = 16) -> Plan:
    """Resident collection for the serving loop; ``pairs`` is the job pool."""
    pairs = law_pairs(seed, pool)
    templates, sites = [], []
    for t in range(n_targets):
        p = pairs[t]
        span = max((p.min_len + p.max_len) // 2, len(p.fwd) + len(p.rev) + 10)
        templates.append(operon_template(seed, t, span + 200, p, span))
        sites.append(template_sites(span + 200, span, len(p.fwd), len(p.rev)) + (t,))
    lengths = lognormal_lengths(seed, n, 4e6, 0.3, 1e6, 12e6)
    gc = 0.30 + 0.40 * rng.uniform01(rng.stream_key(seed, rng.S_GC), np.arange(n))
    g, pos, strand, tid = _plant(seed, lengths, n_targets, [len(t) for t in templates], 1, 3)
    return Plan(seed, lengths, _thresholds(gc), templates, g, pos, strand, tid,
                _empty(), _empty(), _empty(), pairs, name=f"serving-{n}", template_sites=sites)


def jobs(seed: int, n_jobs: int, rate: float, n_genomes: int, pool: int,
         lo: int = 10, hi: int = 100000):
    """Poisson arrivals; each job is one pool pair over a random genome subset
    of log-uniform size in [lo, min(hi, n_genomes)].  Returns a list of
    (arrival_s, pair_id, sorted genome ids)."""
    # one draw stream per quantity, so the first n jobs are the same for any
    # n_jobs >= n
    idx = np.arange(n_jobs)
    u = 1.0 - rng.uniform01(rng.stream_key(seed, rng.S_MISC | (2 << 20)), idx)
    arrivals = np.cumsum(-np.log(u) / rate)
    pids = rng.uniform_int(rng.stream_key(seed, rng.S_MISC | (4 << 20)), idx, 0, pool - 1)
    hi = min(hi, n_genomes)
    su = rng.uniform01(rng.stream_key(seed, rng.S_MISC | (5 << 20)), idx)
    sizes = np.round(np.exp(math.log(lo) + su * (math.log(hi) - math.log(lo)))).astype(np.int64)
    out = []
    for j in range(n_jobs):
        kj = rng.stream_key(seed, rng.S_MISC | (3 << 20) | j)
        ids = np.argsort(rng.draws(kj, np.arange(n_genomes)))[: int(sizes[j])]
        out.append((float(arrivals[j]), int(pids[j]), np.sort(ids)))
    return out


def tiny(seed: int, n_genomes: int = 3, len_lo: int = 50, len_hi: int = 4000,
         pair: Optional[PairSpec] = None, n_copies=(0, 3), gc_lo=0.3, gc_hi=0.7,
         nruns: int = 0, span: Optional[int] = None) -> Plan:
    """Small random collection for parity cases (uniform lengths, optional N runs)."""
    key = rng.stream_key(seed, rng.S_LEN)
    lengths = rng.uniform_int(key, np.arange(n_genomes), len_lo, len_hi)
    gc = gc_lo + (gc_hi - gc_lo) * rng.uniform01(rng.stream_key(seed, rng.S_GC),
                                                 np.arange(n_genomes))
    if pair is None:
        pair = PairSpec(random_primer(seed, 0, 20, "RY"), random_primer(seed, 1, 19, "SN"),
                        k=2, clamp=0, min_len=60, max_len=600)
    if span is None:
        span = min(max(pair.min_len + 10, len(pair.fwd) + len(pair.rev) + 5), pair.max_len)
    tl = span + 40
    tmpl = operon_template(seed, 0, tl, pair, span)
    g = pos = strand = tid = _empty()
    if n_copies[1] > 0:
        keyp = rng.stream_key(seed, rng.S_PLANT)
        want = rng.uniform_int(keyp, np.arange(n_genomes), n_copies[0], n_copies[1])
        fits = lengths // np.maximum(want, 1) >= tl
        want = np.where(fits, want, 0)
        gl, pl, sl, tl_ = [], [], [], []
        for gi in range(n_genomes):
            w = int(want[gi])
            if w == 0:
                continue
            slot_len = int(lengths[gi]) // w
            for s in range(w):
                u = rng.uniform01(rng.stream_key(seed, rng.S_PLANT | 2), np.array([gi * 64 + s]))[0]
                gl.append(gi)
                pl.append(s * slot_len + int(u * (slot_len - tl + 1)))
                sl.append(int(rng.uniform_int(rng.stream_key(seed, rng.S_PLANT | 3),
                                              np.array([gi * 64 + s]), 0, 1)[0]))
                tl_.append(0)
        g, pos = np.array(gl, dtype=np.int64), np.array(pl, dtype=np.int64)
        strand, tid = np.array(sl, dtype=np.int8), np.array(tl_, dtype=np.int64)
    ng = np.zeros(0, dtype=np.int64)
    npos = np.zeros(0, dtype=np.int64)
    nlen = np.zeros(0, dtype=np.int64)
    if nruns > 0:
        keyn = rng.stream_key(seed, rng.S_NRUN)
        ng = rng.uniform_int(keyn, np.arange(nruns), 0, n_genomes - 1)
        nlen = rng.uniform_int(keyn, np.arange(nruns, 2 * nruns), 1, 8)
        u = rng.uniform01(keyn, np.arange(2 * nruns, 3 * nruns))
        npos = np.floor(u * np.maximum(lengths[ng] - nlen, 0)).astype(np.int64)
        nlen = np.minimum(nlen, lengths[ng])
    return Plan(seed, lengths.astype(np.int64), _thresholds(gc), [tmpl], g,
                pos.astype(np.int64), strand.astype(np.int8), tid, ng, npos, nlen, [pair],
                name=f"tiny-{seed}",
                template_sites=[template_sites(tl, span, len(pair.fwd), len(pair.rev)) + (0,)])
