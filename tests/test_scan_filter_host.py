"""The generated per-pattern filters, run on the CPU: every window with at
most k mismatches and a matching clamp must pass (the filter may pass more;
the exact count decides).  The filter source is interpreted statement by
statement with the bitwise semantics of v_bitop3_b32 (bit i of the table is
the result for operands (i>>2 & 1, i>>1 & 1, i & 1)), over numpy words of 32
windows, for pigeonhole blocks and for the exact-count mode."""
import re

import numpy as np
import pytest

from paper_2509_13300_amd import _lib as L

IUPAC = {"A": "A", "C": "C", "G": "G", "T": "T", "R": "AG", "Y": "CT", "S": "CG", "W": "AT",
         "K": "GT", "M": "AC", "B": "CGT", "D": "AGT", "H": "ACT", "V": "ACG", "N": "ACGT"}
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}
M32 = np.uint32(0xFFFFFFFF)


def bitop3(a, b, c, tt):
    out = np.zeros_like(a)
    for i in range(8):
        if tt >> i & 1:
            out |= ((a if i & 4 else ~a) & (b if i & 2 else ~b) & (c if i & 1 else ~c))
    return out


def run_filter(body, planes):
    """Evaluate a generated filter function body; planes: dict name -> list of
    uint32 arrays indexed by window position."""
    env = {}

    def val(tok):
        tok = tok.strip()
        m = re.fullmatch(r"(p[acgthlx])\[(\d+)\]", tok)
        if m:
            return planes[m.group(1)][int(m.group(2))]
        if tok.endswith("u") and tok[:-1].isdigit():
            return np.full_like(planes["pa"][0], np.uint32(int(tok[:-1])))
        if tok == "0xffffffffu":
            return np.full_like(planes["pa"][0], M32)
        if tok.startswith("~"):
            return ~val(tok[1:])
        return env[tok]

    for line in body.splitlines():
        line = line.strip()
        if not line or line.startswith("//") or line.startswith("__device__"):
            continue
        m = re.fullmatch(r"return (\w+)( & (\w+))?;", line)
        if m:
            r = env[m.group(1)]
            return r & env[m.group(3)] if m.group(3) else r
        m = re.fullmatch(r"(?:const )?(?:u32 )?(\w+) (\|?=) (.+);", line)
        assert m, line
        name, op, expr = m.groups()
        b = re.fullmatch(r"__builtin_amdgcn_bitop3_b32\((.+), (.+), (.+), (0x[0-9a-f]+)\)", expr)
        v = bitop3(val(b.group(1)), val(b.group(2)), val(b.group(3)), int(b.group(4), 16)) if b \
            else val(expr)
        env[name] = env[name] | v if op == "|=" else v
    raise AssertionError("no return")


def window_sets(primer, strand):
    sets = [IUPAC[c] for c in primer.upper()]
    if strand == 0:
        return sets
    return ["".join(sorted(COMP[b] for b in s)) for s in reversed(sets)]


def planned_rate(body, i):
    return float(re.search(rf"// pattern {i}: .*random pass rate ([0-9.e+-]+)", body).group(1))


# bit planes over the windows: the one-hot planes and those of the 2-bit code
# (A=00, C=01, G=10, T=11 in (h, l)), as in the scan kernel
PLANE_SETS = (("pa", "A"), ("pc", "C"), ("pg", "G"), ("pt", "T"), ("ph", "GT"), ("pl", "CT"),
              ("px", "CG"))


def planes_of(win, n_words):
    length = win.shape[1]
    weights = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    planes = {}
    for p, bases in PLANE_SETS:
        bits = np.isin(win, list(bases)).reshape(n_words, 32, length)
        planes[p] = [((bits[:, :, j].astype(np.uint64) * weights).sum(1)).astype(np.uint32)
                     for j in range(length)]
    return planes


def random_pass_rate(fn, length, rs, n_words):
    win = rs.choice(list("ACGT"), size=(n_words * 32, length))
    got = run_filter(fn, planes_of(win, n_words))
    return sum(bin(int(x)).count("1") for x in got) / (n_words * 32)


def check_pair(fwd, rev, k, clamp, rs, n_words=64):
    src = L.ah_scan_program_source([(fwd, rev, k, clamp)])
    body = src.split("---- generated pattern program follows ----")[1]
    for i, (primer, strand) in enumerate([(fwd, 0), (fwd, 1), (rev, 0), (rev, 1)]):
        fn = body.split(f"u32 ah_pf_{i}(")[1].split("\n}\n")[0].split("{", 1)[1]
        # the planner's pass rate matches the filter's on uniform random bases
        # (within sampling error: 20,480 windows)
        planned = planned_rate(body, i)
        measured = random_pass_rate(fn, len(primer), rs, 640)
        assert measured <= 2.0 * planned + 6.0 / 20480, (fwd, rev, i, planned, measured)
        sets = window_sets(primer, strand)
        Lp = len(sets)
        clamp_pos = set(range(Lp - clamp, Lp)) if strand == 0 else set(range(clamp))
        # windows: planted near-matches (0..k+1 mismatches, some in the clamp)
        # and random bases, 32 per word
        W = 32 * n_words
        win = rs.choice(list("ACGT"), size=(W, Lp))
        for w in range(0, W, 2):
            for j in range(Lp):
                win[w, j] = rs.choice(list(sets[j]))
            n_mut = rs.randint(0, k + 2)
            for j in rs.choice(Lp, size=min(n_mut, Lp), replace=False):
                win[w, j] = rs.choice(list("ACGT"))
        mism = np.array([[win[w, j] not in sets[j] for j in range(Lp)] for w in range(W)])
        ok = (mism.sum(1) <= k) & ~mism[:, sorted(clamp_pos)].any(1) if clamp_pos else \
            (mism.sum(1) <= k)
        got = run_filter(fn, planes_of(win, n_words))
        passed = ((got[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(bool).reshape(W)
        missed = np.flatnonzero(ok & ~passed)
        assert missed.size == 0, (fwd, rev, k, clamp, i, missed[:5])
        assert ok.sum() > 0


CASES = [
    ("GCMCCTGGYAAACTGTTGG", "AAAGACGTATGACGATCWNA", 2, 0),
    ("ACGTACCGATNGCATTGGCAKT", "GGATCCAAGTTCGACGT", 2, 3),
    ("ACGTNRYSWKMBDHV", "NNNNNAAAAC", 1, 2),
    ("GTGCCAGCMGCNGCGGTAA", "GGACTACHVGGGTWTCTAAT", 3, 1),
    ("CATCTNGNGGCAAANGCTHT", "TAGNTTARCNTNCDAGTW", 3, 0),
    ("ACGTACGTAC", "GGATCCTTGA", 0, 0),
    ("AGAGTTTGATCMTGGCTCAGRTYGAACGCTGG", "TACGGYTACCTTGTTACGACTT", 3, 5),
]


@pytest.mark.parametrize("case", CASES)
def test_filter_passes_every_site(case):
    check_pair(*case, rs=np.random.RandomState(hash(case) % (1 << 31)))


@pytest.mark.parametrize("case", CASES[:4])
def test_exact_mode_filter_passes_every_site(case, monkeypatch):
    monkeypatch.setenv("AH_SCAN_PREFILTER", "0")
    check_pair(*case, rs=np.random.RandomState(7))


def test_random_pairs():
    rs = np.random.RandomState(11)
    codes = "ACGTACGTACGTRYSWKMBDHVN"
    for _ in range(12):
        fwd = "".join(rs.choice(list(codes), size=rs.randint(10, 31)))
        rev = "".join(rs.choice(list(codes), size=rs.randint(10, 31)))
        check_pair(fwd, rev, int(rs.randint(0, 4)), int(rs.randint(0, 4)), rs, n_words=16)


@pytest.mark.parametrize("case", CASES)
def test_code_plane_literals_pass_every_site(case, monkeypatch):
    """Two-base codes read as one bit plane of the 2-bit code (h, l or h ^ l,
    maybe complemented) instead of the OR of two one-hot planes."""
    monkeypatch.setenv("AH_SCAN_CODE_PLANES", "1")
    src = L.ah_scan_program_source([case[:4]])
    if any(ch in "RYSWKM" for ch in (case[0] + case[1]).upper()):
        assert re.search(r"\bp[hlx]\[\d+\]", src.split("---- generated pattern program follows")[1])
    check_pair(*case, rs=np.random.RandomState(19))
