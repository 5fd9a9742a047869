"""Nearest-neighbour melting temperature of a primer binding site
(Section 2.1, "Melting temperature filtering").

The paper computes, with a nearest-neighbour (NN) duplex-stability model that
admits mismatches, the melting temperature of every oligonucleotide of the
degenerate primer that is compatible with the site, keeps the site iff the
*maximum* of these is above a user threshold, and reports that maximum.  The
user supplies the primer and template concentrations (dnac1, dnac2), the ion
concentrations (Na, K, Tris, Mg, dNTPs) and the salt-correction method.

Model (float64 throughout):

* Stacks: SantaLucia (1998) unified parameters (identical to Allawi &
  SantaLucia 1997), Delta-H in kcal/mol and Delta-S in cal/(K mol) for the
  stack read 5'->3' on either strand.
* Initiation once per duplex end from that end's terminal pair:
  G.C -> (+0.1, -2.8), A.T -> (+2.3, +4.1).
* Symmetry correction Delta-S -1.4 and total strand concentration C = dnac1
  only when the caller declares the duplex self-complementary (``selfcomp``).
* Salt method 5 (SantaLucia 1998): Delta-S += 0.368 (N - 1) ln([Na+]) with
  [Na+] in mol/L, N the primer length, and the sodium equivalent of von
  Ahsen et al. (2001): Na + K + Tris/2 + 120 sqrt(Mg - dNTPs) mM (the Mg term
  is zero when Mg <= dNTPs).  Method 0: no correction.
* The other methods correct the 1 M temperature Tm1 (no salt term in
  Delta-S), with the same sodium equivalent [Na+] (mol/L) for 1-4 and 6:
    1 Schildkraut & Lifson (1965): Tm1 + 16.6 log10[Na+]
    2 Wetmur (1991):               Tm1 + 16.6 log10([Na+] / (1 + 0.7 [Na+]))
    3 SantaLucia et al. (1996):    Tm1 + 12.5 log10[Na+]
    4 SantaLucia (1998):           Tm1 + 11.7 log10[Na+]
    6 Owczarzy et al. (2004), on 1/T in kelvin:
        1/T = 1/T1 + (4.29 fGC - 3.95) 1e-5 ln[Na+] + 9.40e-6 ln^2[Na+]
    7 Owczarzy et al. (2008), magnesium: with the monovalent ions
      [Mon] = Na + K + Tris/2 and the free magnesium [Mg] left by 1:1 binding
      to dNTPs (association constant 3e4 per M), R = sqrt[Mg] / [Mon]:
      R < 0.22 (or no Mg): method 6 on [Mon];  otherwise
        1/T = 1/T1 + a + b ln[Mg] + fGC (c + d ln[Mg])
              + (e + f ln[Mg] + g ln^2[Mg]) / (2 (N - 1))
      with a 3.92e-5, b -9.11e-6, c 6.26e-5, d 1.42e-5, e -4.82e-4,
      f 5.25e-4, g 8.31e-5; for R < 6, a, d, g are scaled by
      0.843 - 0.352 sqrt[Mon] ln[Mon],
      1.279 - 4.03e-3 ln[Mon] - 8.03e-3 ln^2[Mon] and
      0.486 - 0.258 ln[Mon] + 5.25e-3 ln^3[Mon].
  fGC is the G+C fraction of the oligo over its N positions (R27); methods
  6 and 7 therefore differ between oligos that pair the site alike, and the
  maximum runs over the oligos themselves.  The constants of methods 1-4, 6
  and 7 are the published ones as restated here: parity unpinned against
  the publications (not available here); the tests pin the reductions
  (1 M monovalent, no magnesium) and the oligo-level maximum.
* C = (max(dnac1, dnac2) - min(dnac1, dnac2) / 2) * 1e-9 M otherwise.
* Tm = 1000 Delta-H / (Delta-S + R ln C) - 273.15 with R = 1.987.

Readings:
  R7  a compatible oligo is within k mismatches of the site and matches it on
      every clamp position (the oligos whose own pattern would have matched).
  R8  parameters as above; the configuration's conditions are 50 mM Na+,
      1.5 mM Mg2+, 250 nM primer, template in trace (dnac2 = 0).
  R9  mismatched duplexes ("MM0"): the published mismatch, terminal-mismatch
      and dangling-end tables are not available here, so a stack that contains
      a mismatched pair contributes zero, initiation is taken at the outermost
      paired positions (both ends at the same pair if only one pair is
      formed, none if no pair is formed), and the salt term keeps N - 1.  For a
      perfect duplex this is exactly the closed form above.  Parity against the
      paper's tool for mismatched duplexes: unpinned.
  R20 only the maximum is part of the result.
  R27 for the salt methods that depend on G+C content (6, 7), fGC is the
      G+C fraction of the oligo over all its positions, paired or not.
  R21 every compatible oligo is evaluated, however many there are; for
      methods 0-5 ``site_tm_by_pairing`` takes the same maximum over the sets
      of paired positions, which stays feasible where the oligos are too
      many to list (pinned to ``site_tm`` and to brute force).
Template base opposite oligo position j: the complement of the top-strand base
at pos + j for a + site, the top-strand base at pos + L - 1 - j for a - site.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

from . import iupac
from .scan import codes

R_GAS = 1.987

# SantaLucia (1998) unified / Allawi & SantaLucia (1997): (dH, dS)
NN_UNIFIED = {
    "AA": (-7.9, -22.2), "TT": (-7.9, -22.2),
    "AT": (-7.2, -20.4),
    "TA": (-7.2, -21.3),
    "CA": (-8.5, -22.7), "TG": (-8.5, -22.7),
    "GT": (-8.4, -22.4), "AC": (-8.4, -22.4),
    "CT": (-7.8, -21.0), "AG": (-7.8, -21.0),
    "GA": (-8.2, -22.2), "TC": (-8.2, -22.2),
    "CG": (-10.6, -27.2),
    "GC": (-9.8, -24.4),
    "GG": (-8.0, -19.9), "CC": (-8.0, -19.9),
}
INIT_GC = (0.1, -2.8)
INIT_AT = (2.3, 4.1)
SYM_DS = -1.4

_NH = np.zeros(16)
_NS = np.zeros(16)
for _k, (_h, _s) in NN_UNIFIED.items():
    _i = "ACGT".index(_k[0]) * 4 + "ACGT".index(_k[1])
    _NH[_i], _NS[_i] = _h, _s


@dataclasses.dataclass(frozen=True)
class TmParams:
    dnac1: float = 250.0   # nM, primer
    dnac2: float = 0.0     # nM, template
    Na: float = 50.0       # mM
    K: float = 0.0
    Tris: float = 0.0
    Mg: float = 1.5
    dNTPs: float = 0.0
    saltcorr: int = 5
    selfcomp: bool = False


def sodium_equivalent(p: TmParams) -> float:
    mg = p.Mg - p.dNTPs
    return p.Na + p.K + p.Tris / 2.0 + (120.0 * math.sqrt(mg) if mg > 0 else 0.0)


SALT_METHODS = (0, 1, 2, 3, 4, 5, 6, 7)


def _check_method(p: TmParams) -> None:
    if p.saltcorr not in SALT_METHODS:
        raise ValueError("salt correction method must be one of 0-7")
    if p.saltcorr in (1, 2, 3, 4, 5, 6) and not sodium_equivalent(p) > 0:
        raise ValueError("salt correction needs a positive sodium equivalent")
    if p.saltcorr == 7 and not (monovalent(p) > 0 or free_magnesium(p) > 0):
        raise ValueError("salt correction 7 needs monovalent ions or free magnesium")


def salt_entropy(p: TmParams, length: int) -> float:
    """Method 5's entropy term (zero for every other method)."""
    _check_method(p)
    if p.saltcorr != 5:
        return 0.0
    return 0.368 * (length - 1) * math.log(sodium_equivalent(p) / 1000.0)


def monovalent(p: TmParams) -> float:
    """[Mon] of method 7, mM."""
    return p.Na + p.K + p.Tris / 2.0


def free_magnesium(p: TmParams) -> float:
    """Mg not bound by dNTPs (1:1 complexes, association constant 3e4 / M), mM."""
    mg, d = p.Mg * 1e-3, p.dNTPs * 1e-3
    if mg <= 0:
        return 0.0
    if d <= 0:
        return p.Mg
    ka = 3e4
    b = ka * (d - mg) + 1.0
    return 1e3 * (-b + math.sqrt(b * b + 4.0 * ka * mg)) / (2.0 * ka)


def salt_shift(p: TmParams) -> float:
    """Methods 1-4: the shift of Tm in degrees (zero for the others)."""
    _check_method(p)
    if p.saltcorr not in (1, 2, 3, 4):
        return 0.0
    na = sodium_equivalent(p) / 1000.0
    if p.saltcorr == 1:
        return 16.6 * math.log10(na)
    if p.saltcorr == 2:
        return 16.6 * math.log10(na / (1.0 + 0.7 * na))
    if p.saltcorr == 3:
        return 12.5 * math.log10(na)
    return 11.7 * math.log10(na)


def reciprocal_terms(p: TmParams, length: int):
    """Methods 6 and 7: (A, B) with 1/T = 1/T1 + A + B fGC; None otherwise."""
    _check_method(p)
    if p.saltcorr not in (6, 7):
        return None

    def owczarzy2004(na_molar):
        ln = math.log(na_molar)
        return -3.95e-5 * ln + 9.40e-6 * ln * ln, 4.29e-5 * ln

    if p.saltcorr == 6:
        return owczarzy2004(sodium_equivalent(p) / 1000.0)
    mon = monovalent(p) / 1000.0
    mg = free_magnesium(p) / 1000.0
    if mg <= 0:
        return owczarzy2004(mon)
    ratio = math.sqrt(mg) / mon if mon > 0 else math.inf
    if ratio < 0.22:
        return owczarzy2004(mon)
    a, b, c, d, e, f, g = 3.92e-5, -9.11e-6, 6.26e-5, 1.42e-5, -4.82e-4, 5.25e-4, 8.31e-5
    if ratio < 6.0:
        lm = math.log(mon)
        a *= 0.843 - 0.352 * math.sqrt(mon) * lm
        d *= 1.279 - 4.03e-3 * lm - 8.03e-3 * lm * lm
        g *= 0.486 - 0.258 * lm + 5.25e-3 * lm ** 3
    lg = math.log(mg)
    A = a + b * lg + (e + f * lg + g * lg * lg) / (2.0 * (length - 1))
    return A, c + d * lg


def concentration(p: TmParams) -> float:
    if p.selfcomp:
        return p.dnac1 * 1e-9
    hi, lo = max(p.dnac1, p.dnac2), min(p.dnac1, p.dnac2)
    return (hi - lo / 2.0) * 1e-9


def duplex_terms(oligo: np.ndarray, paired: np.ndarray):
    """Delta-H and Delta-S sums (stacks + initiation) for oligos (rows) with a
    boolean pairing table of the same shape (MM0 for unpaired positions)."""
    oligo = np.atleast_2d(oligo).astype(np.int64)
    paired = np.atleast_2d(paired)
    both = paired[:, :-1] & paired[:, 1:]
    idx = oligo[:, :-1] * 4 + oligo[:, 1:]
    dh = np.where(both, _NH[idx], 0.0).sum(axis=1)
    ds = np.where(both, _NS[idx], 0.0).sum(axis=1)
    any_p = paired.any(axis=1)
    L = oligo.shape[1]
    lo = np.argmax(paired, axis=1)
    hi = L - 1 - np.argmax(paired[:, ::-1], axis=1)
    for end in (lo, hi):
        b = oligo[np.arange(oligo.shape[0]), end]
        gc = (b == 1) | (b == 2)
        dh += np.where(any_p, np.where(gc, INIT_GC[0], INIT_AT[0]), 0.0)
        ds += np.where(any_p, np.where(gc, INIT_GC[1], INIT_AT[1]), 0.0)
    return dh, ds


def tm_from_terms(dh, ds, length: int, p: TmParams, gc=None):
    """Tm in degrees; ``gc``: the oligos' G+C counts (methods 6 and 7)."""
    ds = np.asarray(ds, dtype=np.float64) + salt_entropy(p, length)
    if p.selfcomp:
        ds = ds + SYM_DS
    t = 1000.0 * np.asarray(dh, dtype=np.float64) / (ds + R_GAS * math.log(concentration(p))) - 273.15
    rt = reciprocal_terms(p, length)
    if rt is not None:
        if gc is None:
            raise ValueError("salt methods 6 and 7 need the oligos' G+C counts")
        f_gc = np.asarray(gc, dtype=np.float64) / length
        t = 1.0 / (1.0 / (t + 273.15) + rt[0] + rt[1] * f_gc) - 273.15
    return t + salt_shift(p)


def gc_count(oligo: np.ndarray) -> np.ndarray:
    """G+C bases of each oligo (rows of codes)."""
    o = np.atleast_2d(oligo)
    return ((o == 1) | (o == 2)).sum(axis=1)


def tm_perfect(oligo: str, p: TmParams = TmParams()) -> float:
    """Tm of an ACGT oligo with its exact complement."""
    o = codes(oligo)
    dh, ds = duplex_terms(o, np.ones((1, o.size), bool))
    return float(tm_from_terms(dh, ds, o.size, p, gc_count(o))[0])


def tm_duplex(oligo: str, template_opposite: str, p: TmParams = TmParams()) -> float:
    """Tm of oligo (5'->3') against the template bases written opposite each
    oligo base (template read 3'->5'); a position pairs iff the template base
    is the complement of the oligo base."""
    o = codes(oligo)
    t = codes(template_opposite)
    paired = (t < 4) & (o == (3 - t))
    dh, ds = duplex_terms(o, paired[None, :])
    return float(tm_from_terms(dh, ds, o.size, p, gc_count(o))[0])


def _expansion_codes(primer: str) -> np.ndarray:
    return np.array([codes(o) for o in iupac.expand(primer)], dtype=np.int64)


_EXP_CACHE: dict = {}


def site_tm(genome_codes: np.ndarray, pos: int, primer: str, strand: int, k: int,
            clamp: int, p: TmParams = TmParams()) -> float:
    """Maximum Tm over the oligos of ``primer`` compatible with the site."""
    primer = iupac.normalise(primer)
    L = len(primer)
    if primer not in _EXP_CACHE:
        _EXP_CACHE[primer] = _expansion_codes(primer)
    olig = _EXP_CACHE[primer]
    w = np.asarray(genome_codes[pos:pos + L], dtype=np.int64)
    if strand == 0:
        opp_ok = w  # oligo base j pairs iff it equals the top-strand base
    else:
        r = w[::-1]
        opp_ok = np.where(r < 4, 3 - r, 9)
    paired = olig == opp_ok[None, :]
    mism = L - paired.sum(axis=1)
    c = min(clamp, L)
    ok = mism <= k
    if c > 0:
        ok &= paired[:, L - c:].all(axis=1)
    if not ok.any():
        return float("nan")
    dh, ds = duplex_terms(olig[ok], paired[ok])
    return float(tm_from_terms(dh, ds, L, p, gc_count(olig[ok])).max())


def fill_tm(hits: np.ndarray, seqs, pairs, p: TmParams = TmParams()) -> np.ndarray:
    """Copy of ``hits`` with the ``tm`` field set for every record."""
    h = hits.copy()
    cache = {}
    for r in range(h.size):
        g = int(h["genome"][r])
        if g not in cache:
            cache[g] = codes(seqs[g])
        pr = pairs[int(h["pair"][r])]
        primer = pr.fwd if h["primer"][r] == 0 else pr.rev
        h["tm"][r] = site_tm(cache[g], int(h["pos"][r]), primer, int(h["strand"][r]),
                             pr.k, pr.clamp, p)
    return h


def site_tm_by_pairing(genome_codes: np.ndarray, pos: int, primer: str, strand: int, k: int,
                       clamp: int, p: TmParams = TmParams(), chunk: int = 1 << 16) -> float:
    """``site_tm`` for salt methods 0-5, taken over sets of paired positions
    instead of oligos, for primers whose expansion is too large to list.

    Under R9 a stack or an initiation term involves paired positions only,
    and a paired position carries the base the template fixes there; methods
    0-5 add nothing that depends on the other positions.  So every compatible
    oligo that pairs the site at the same set of positions has the same Tm,
    and the maximum over oligos is the maximum over those sets.  A set is
    formed by some compatible oligo iff it holds every position whose primer
    code admits the template's base and has no other member, holds no
    position whose code excludes it (or faces a non-ACGT base), covers the
    clamp, and leaves at most k positions unpaired."""
    _check_method(p)
    if p.saltcorr in (6, 7):
        raise ValueError("methods 6 and 7 depend on the oligo's G+C count, not only its pairing")
    primer = iupac.normalise(primer)
    L = len(primer)
    w = np.asarray(genome_codes[pos:pos + L], dtype=np.int64)
    if strand == 0:
        need = w  # the oligo base that pairs with the template at each position
    else:
        r = w[::-1]
        need = np.where(r < 4, 3 - r, 9)
    sets = [["ACGT".index(b) for b in iupac.members(ch)] for ch in primer]
    can = np.array([need[j] < 4 and int(need[j]) in sets[j] for j in range(L)])
    c = min(clamp, L)
    if not can[L - c:].all():
        return float("nan")
    budget = k - int((~can).sum())
    if budget < 0:
        return float("nan")
    optional = np.array([j for j in range(L) if can[j] and len(sets[j]) > 1 and j < L - c],
                        dtype=np.int64)
    oligo = np.array([int(need[j]) if can[j] else sets[j][0] for j in range(L)], dtype=np.int64)
    best = -math.inf
    for e in range(min(budget, optional.size) + 1):
        # every e-subset of the optional positions, unpaired
        subsets = list(itertools.combinations(range(optional.size), e))
        combos = np.array(subsets, dtype=np.int64).reshape(len(subsets), e)
        for lo in range(0, combos.shape[0], chunk):
            part = combos[lo:lo + chunk]
            paired = np.tile(can, (part.shape[0], 1))
            if e:
                paired[np.arange(part.shape[0])[:, None], optional[part]] = False
            dh, ds = duplex_terms(np.broadcast_to(oligo, paired.shape), paired)
            best = max(best, float(tm_from_terms(dh, ds, L, p).max()))
    return best
