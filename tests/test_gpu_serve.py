"""GPU tests of the serving form: jobs over subsets of a resident collection
give the same records as the direct path on the same subset (and the oracle),
and every job's result is the same alone and in a mix of concurrent jobs,
under a tight memory budget and with capacity retries."""
import numpy as np
import pytest

from gpu_util import amp_tuples, hit_tuples_gpu, hit_tuples_oracle, random_rate, run_oracle, say
from synth import gpu, plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def world(dev):
    """80 genomes (5-150 kbp, N runs) and a pool of law pairs ordered from the
    most to the least hit-rich."""
    from paper_2509_13300_amd import path

    p = plan.tiny(6601, n_genomes=80, len_lo=5000, len_hi=150000, n_copies=(0, 2), nruns=2,
                  span=600)
    ascii, off = gpu.fill_cuda(p, dev)
    c, _ = path.pack(ascii, off, p.lengths, with_nmask=True)
    pool = sorted(plan.law_pairs(6602, 24), key=random_rate, reverse=True) + [p.pairs[0]]
    return p, c, pool


def subset_collection(c, ids):
    import torch

    from paper_2509_13300_amd import path

    ids = np.asarray(ids, dtype=np.int64)
    t = torch.from_numpy(ids).to(c.word_off.device)
    off = torch.cat([c.word_off[t], c.word_off[t[-1:] + 1]])
    lens = c.lengths[ids]
    return path.PackedCollection(c.words, c.nmask, off, c.len[t].contiguous(), int(ids.size),
                                 int(lens.max()), int(lens.sum()), lens)


def direct(c, ids, pair, dev):
    """The four entry points on a gathered view of the subset, genome ids
    mapped back to collection ids."""
    import torch

    from paper_2509_13300_amd import path

    sub = subset_collection(c, ids)
    buf = path.alloc(sub, [pair], 1 << 22, 1 << 22, dev)
    path.run(sub, [pair], buf)
    torch.cuda.synchronize()
    h, a = path.hits_numpy(buf), path.amps_numpy(buf)
    ids = np.asarray(ids, dtype=np.uint32)
    h["genome"] = ids[h["genome"]]
    a["genome"] = ids[a["genome"]]
    return h, a


def serve_all(server, jobs, stagger=0.0):
    """Submit every (pair, ids) job (optionally spaced by ``stagger`` s), wait
    for all, return {index: (hits, amplicons, status)}."""
    import time

    ids_of, out = {}, {}
    for i, (pr, ids) in enumerate(jobs):
        ids_of[server.submit(pr, ids)] = i
        if stagger:
            time.sleep(stagger)
    while len(out) < len(jobs):
        st = server.wait(60.0)
        assert st is not None, "a job did not finish within 60 s"
        i = ids_of[st["job"]]
        assert st["status"] == 0, st
        h, a = server.result(st)
        assert h.size == st["hits"] and a.size == st["amplicons"]
        out[i] = (h, a, st)
        server.release(st["job"])
    return out


def job_mix(p, pool, seed, n):
    rs = np.random.RandomState(seed)
    jobs = []
    for j in range(n):
        pr = pool[rs.choice([0, 1, 2, 3, 4, 5, len(pool) - 1])]
        size = int(np.exp(rs.uniform(0, np.log(p.n))))
        ids = np.sort(rs.choice(p.n, size=size, replace=False))
        jobs.append((pr, ids))
    jobs.append((pool[0], None))  # a job over the whole collection
    jobs.append((pool[-1], np.array([p.n - 1])))
    return jobs


def test_job_equals_direct_path_and_oracle(world, dev):
    from paper_2509_13300_amd import path

    p, c, pool = world
    ids = np.array([0, 3, 4, 17, 40, 41, 79])
    srv = path.Server(c, 256 << 20, dev, n_lanes=2, part_bases=200_000)
    try:
        for pr in (pool[0], pool[5], pool[-1]):
            got = serve_all(srv, [(pr, ids)])[0]
            h0, a0 = direct(c, ids, pr, dev)
            assert np.array_equal(got[0], h0) and np.array_equal(got[1], a0)
            assert got[2]["n_parts"] >= 2
            oh, oa = run_oracle(p.subset(ids), [pr])
            h = got[0].copy()
            h["genome"] = np.searchsorted(ids, h["genome"])
            assert hit_tuples_gpu(h) == hit_tuples_oracle(oh)
            assert np.abs(h["tm"].astype(np.float64) - oh["tm"]).max(initial=0.0) <= 0.01
            a = got[1].copy()
            a["genome"] = np.searchsorted(ids, a["genome"])
            assert amp_tuples(a) == amp_tuples(oa)
            say("served", pr.fwd, pr.rev, "k", pr.k, "hits", h.size, "amplicons", a.size)
    finally:
        srv.close()


def test_each_result_is_the_same_alone_and_in_the_mix(world, dev):
    from paper_2509_13300_amd import path

    p, c, pool = world
    jobs = job_mix(p, pool, 6603, 22)
    # a 32 KiB host arena: small parts land in it, larger ones fall back
    cfg = dict(n_lanes=4, part_bases=400_000, host_pool_bytes=32 << 10)
    srv = path.Server(c, 512 << 20, dev, **cfg)
    try:
        alone = {i: serve_all(srv, [job])[0] for i, job in enumerate(jobs)}
        mix = serve_all(srv, jobs)
        staggered = serve_all(srv, jobs, stagger=0.002)
        st = srv.stats()
    finally:
        srv.close()
    say("mix stats", st)
    assert sum(r[0].size for r in alone.values()) > 500
    for i in range(len(jobs)):
        for other in (mix, staggered):
            assert np.array_equal(other[i][0], alone[i][0]), i
            assert np.array_equal(other[i][1], alone[i][1]), i
    for i in (0, len(jobs) - 2, len(jobs) - 1):  # and the same as the direct path
        pr, ids = jobs[i]
        h0, a0 = direct(c, np.arange(p.n) if ids is None else ids, pr, dev)
        assert np.array_equal(alone[i][0], h0) and np.array_equal(alone[i][1], a0)
    assert st["pool_in_use"] == 0 and st["parts_run"] > 3 * len(jobs)
    assert st["host_fallbacks"] > 0 and st["host_pool_high_water"] > 0


def test_tight_pool_admission_changes_nothing(world, dev):
    from paper_2509_13300_amd import path

    p, c, pool = world
    jobs = job_mix(p, pool, 6604, 12)
    srv = path.Server(c, 512 << 20, dev, n_lanes=4, part_bases=400_000)
    try:
        ref = serve_all(srv, jobs)
    finally:
        srv.close()
    # 5 MiB admits two parts (~2.4 MiB each, most of it the candidate list of
    # at least 2^16 records) at a time on four lanes
    srv = path.Server(c, 5 << 20, dev, n_lanes=4, part_bases=400_000)
    try:
        got = serve_all(srv, jobs)
        st = srv.stats()
    finally:
        srv.close()
    say("tight stats", st)
    assert st["admission_waits"] > 0 and st["pool_high_water"] <= 5 << 20
    for i in range(len(jobs)):
        assert np.array_equal(got[i][0], ref[i][0]) and np.array_equal(got[i][1], ref[i][1]), i


def test_capacity_retries_change_nothing(world, dev):
    """capacity_scale 0 leaves every part only the per-genome reserve; parts of
    a hit-rich pair (10-nt primers, k = 3: ~0.014 sites per base) overflow and
    run again with their exact counts."""
    from paper_2509_13300_amd import path

    p, c, pool = world
    rich = plan.PairSpec("ACGTACGTAC", "GGATCCTTGA", k=3, clamp=0, min_len=40, max_len=60)
    jobs = job_mix(p, pool, 6605, 6) + [(rich, np.arange(0, p.n, 3)), (rich, None)]
    srv = path.Server(c, 512 << 20, dev, n_lanes=4, part_bases=400_000)
    try:
        ref = serve_all(srv, jobs)
        assert srv.stats()["retries"] == 0
    finally:
        srv.close()
    srv = path.Server(c, 512 << 20, dev, n_lanes=4, part_bases=400_000, capacity_scale=0.0,
                      host_pool_bytes=256 << 20)
    try:
        got = serve_all(srv, jobs)
        st = srv.stats()
    finally:
        srv.close()
    say("retry stats", st, "rich hits", ref[len(jobs) - 1][0].size)
    assert st["retries"] > 0 and ref[len(jobs) - 1][0].size > 50_000
    for i in range(len(jobs)):
        assert np.array_equal(got[i][0], ref[i][0]) and np.array_equal(got[i][1], ref[i][1]), i
    assert got[len(jobs) - 1][2]["retries"] > 0
    h0, a0 = direct(c, np.arange(p.n), rich, dev)
    assert np.array_equal(ref[len(jobs) - 1][0], h0) and np.array_equal(ref[len(jobs) - 1][1], a0)


def test_errors_and_degenerate_jobs(world, dev):
    from paper_2509_13300_amd import _lib as L
    from paper_2509_13300_amd import path

    p, c, pool = world
    srv = path.Server(c, 1 << 20, dev, n_lanes=1, part_bases=1 << 40)
    try:
        with pytest.raises(L.AhError) as e:
            srv.submit(pool[0], np.array([5, 3]))
        assert e.value.status == L.AH_ERR_INVALID_ARG
        with pytest.raises(L.AhError) as e:
            srv.submit(pool[0], np.array([0, p.n]))
        assert e.value.status == L.AH_ERR_INVALID_ARG
        bad = plan.PairSpec("ACGTXACGTA", "ACGTACGTAC", 1, 0, 10, 100)
        with pytest.raises(L.AhError) as e:
            srv.submit(bad)
        assert e.value.status == L.AH_ERR_INVALID_PRIMER
        # an empty genome list finishes at once with no parts
        j = srv.submit(pool[0], np.array([], dtype=np.uint32))
        st = srv.wait(10.0)
        assert st["job"] == j and st["status"] == 0 and st["n_parts"] == 0 and st["hits"] == 0
        srv.release(j)
        # one part of the whole collection does not fit a 1 MiB pool
        j = srv.submit(pool[0])
        st = srv.wait(30.0)
        assert st["job"] == j and st["status"] == L.AH_ERR_LIMIT
        srv.release(j)
        assert srv.stats()["pool_in_use"] == 0
        assert srv.wait(0.05) is None
    finally:
        srv.close()


def test_full_size_collection_jobs_sampled_against_oracle(dev):
    """The serving workload at full size: the 100,000-genome collection
    (418.7 Gbp, 104.7 GB packed) resident in HBM, a server with the serving
    benchmark's part and capacity settings, the first nine jobs of its Poisson
    job list (one law pair over a log-uniform subset of 11-69,792 genomes
    each) and a job of a planted pair over every 97th genome, submitted
    together.  Every job finishes; in each, the records of its first and last
    genome, of the genome with the most sites, and (planted job) of two
    genomes carrying the target equal the oracle's."""
    import torch

    from paper_2509_13300_amd import path

    p = plan.serving(100000)
    coll = path.pack_resident(lambda ids: gpu.fill_cuda(p.subset(ids), dev), p.lengths, dev)
    say("full serving collection", coll.n, "genomes", coll.total_bp, "bp")
    jobs = [(p.pairs[pid], ids) for _, pid, ids in plan.jobs(13306, 9, 4.0, p.n, len(p.pairs))]
    every = np.arange(0, p.n, 97)
    jobs.append((p.pairs[0], every))  # template 0 belongs to pair 0
    carriers = np.intersect1d(p.plant_genome[p.plant_template == 0], every)
    assert carriers.size >= 2
    cfg = dict(n_lanes=4, n_compilers=8, part_bases=1 << 32, max_part_hits=1 << 25,
               capacity_scale=2.0, host_pool_bytes=8 << 30)
    srv = path.Server(coll, 32 << 30, dev, **cfg)
    try:
        out = serve_all(srv, jobs)
    finally:
        srv.close()
    del coll
    torch.cuda.empty_cache()
    cells = 0
    for j, (pr, ids) in enumerate(jobs):
        h, a, st = out[j]
        say("job", j, "genomes", len(ids), "k", pr.k, "hits", h.size, "amplicons", a.size)
        sample = {int(ids[0]), int(ids[-1])}
        if h.size:  # where this job found the most sites (which genomes to check, not what)
            g_all, cnt = np.unique(h["genome"], return_counts=True)
            sample.add(int(g_all[np.argmax(cnt)]))
        if j == len(jobs) - 1:
            sample.update(int(g) for g in carriers[:2])
        for g in sorted(sample):
            oh, oa = run_oracle(p.subset([g]), [pr])
            cell = h["genome"] == g
            first = np.flatnonzero(cell)
            sel = h[cell].copy()
            sel["genome"] = 0
            assert hit_tuples_gpu(sel) == hit_tuples_oracle(oh), (j, g)
            assert np.abs(sel["tm"].astype(np.float64) - oh["tm"]).max(initial=0.0) <= 0.01
            asel = a[a["genome"] == g].copy()
            asel["genome"] = 0
            if first.size:
                asel["plus_hit"] -= np.uint32(first[0])
                asel["minus_hit"] -= np.uint32(first[0])
            assert amp_tuples(asel) == amp_tuples(oa), (j, g)
            cells += int(oh.size > 0)
    say("sampled genomes with sites", cells)
    assert cells >= 8


def test_a_part_that_fails_after_its_first_launch_frees_its_memory(world, dev, monkeypatch):
    """A part run that fails after queueing device work (forced from the
    host right after its first launch) ends its job with the error, returns
    its pool block only once its stream is idle, and leaves the server able
    to run the same job correctly."""
    from paper_2509_13300_amd import path

    p, c, pool = world
    ids = np.array([1, 2, 5, 9, 30, 31, 60])
    monkeypatch.setenv("AH_SERVER_FAIL_PART", "0")
    srv = path.Server(c, 256 << 20, dev, n_lanes=1, part_bases=200_000)
    monkeypatch.delenv("AH_SERVER_FAIL_PART")
    try:
        job = srv.submit(pool[0], ids)
        st = srv.wait(60.0)
        assert st is not None and st["job"] == job
        assert st["status"] != 0
        srv.release(job)
        assert srv.stats()["pool_in_use"] == 0
        got = serve_all(srv, [(pool[0], ids)])[0]
        h0, a0 = direct(c, ids, pool[0], dev)
        assert np.array_equal(got[0], h0) and np.array_equal(got[1], a0)
        assert srv.stats()["pool_in_use"] == 0
        say("failed part freed its block; rerun equal to the direct path:", h0.size, "hits")
    finally:
        srv.close()
