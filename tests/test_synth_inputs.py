"""The seeded input generator: a byte range of a genome computed on its own
equals the same slice of the whole genome (planted copies and N runs cut at
the range ends included), so long genomes can be checked piecewise."""
import numpy as np

from synth import fill, plan


def test_genome_range_equals_slice_of_the_whole_genome():
    p = plan.tiny(31, n_genomes=3, len_lo=20000, len_hi=40000, n_copies=(2, 3), nruns=3,
                  span=1200)
    rs = np.random.RandomState(7)
    for g in range(p.n):
        whole = fill.genome_bytes(p, g)
        n = whole.size
        cuts = [(0, n), (0, 1), (n - 1, n), (5, 5), (n - 100, n + 50), (-10, 40)]
        for c in np.flatnonzero(p.plant_genome == g):  # ranges that cut a copy
            pos = int(p.plant_pos[c])
            cuts += [(pos - 3, pos + 7), (pos + 100, pos + 5000)]
        for r in np.flatnonzero(p.nrun_genome == g):  # and an N run
            pos = int(p.nrun_pos[r])
            cuts.append((pos + 1, pos + int(p.nrun_len[r]) + 9))
        for _ in range(10):
            a = int(rs.randint(0, n))
            cuts.append((a, a + int(rs.randint(0, 3000))))
        for lo, hi in cuts:
            want = whole[max(lo, 0):min(hi, n)]
            assert np.array_equal(fill.genome_range_bytes(p, g, lo, hi), want), (g, lo, hi)
