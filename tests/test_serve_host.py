"""Host-side checks of the serving runtime: configuration errors are reported
before any device work (no GPU needed)."""
import numpy as np
import pytest
import torch

from paper_2509_13300_amd import _lib as L


def genomes_view(n=3):
    g = L.ah_genomes()
    g.words = g.word_off = g.len = 0x1000  # never dereferenced: rejected first
    g.n = n
    g.max_len = 100
    return g


@pytest.mark.parametrize("cfg,match", [
    (dict(n_lanes=0), "n_lanes"), (dict(n_lanes=17), "n_lanes"), (dict(n_compilers=0), "n_compilers"),
    (dict(part_bases=0), "part_bases"), (dict(max_part_hits=0), "part_bases"),
    (dict(capacity_scale=-1.0), "capacity_scale"),
])
def test_bad_server_config_is_rejected(cfg, match):
    pool = torch.empty(1 << 16, dtype=torch.uint8)
    with pytest.raises(L.AhError, match=match) as e:
        L.ah_server_create(genomes_view(), np.ones(3, np.uint32), L.server_config(**cfg), pool)
    assert e.value.status == L.AH_ERR_INVALID_ARG


def test_tiny_pool_is_rejected():
    pool = torch.empty(1000, dtype=torch.uint8)
    with pytest.raises(L.AhError, match="pool") as e:
        L.ah_server_create(genomes_view(), np.ones(3, np.uint32), L.server_config(), pool)
    assert e.value.status == L.AH_ERR_INVALID_ARG


# ---- the serving scheduler's decisions, driven on the host with simulated
# part runs (ah_sched_simulate runs the lanes' own admission, round-robin and
# retry code on a simulated clock).
MB = 1 << 20


def _check_pool(evs, pool):
    """Replays the runs: at no time do the running parts hold more than the
    pool, and no two running parts share pool bytes."""
    for e in evs:
        running = [f for f in evs if f["t_start"] <= e["t_start"] < f["t_end"] or f is e]
        assert sum(f["bytes"] for f in running) <= pool
        spans = sorted((f["block"], f["block"] + f["bytes"]) for f in running)
        assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:])), spans
        assert e["pool_in_use"] <= pool


def test_scheduler_runs_every_part_once_and_respects_the_pool():
    jobs = [(0.0, [(3 * MB, 1.0, 0)] * 5), (0.1, [(2 * MB, 0.5, 0)] * 3), (0.2, [(4 * MB, 0.2, 0)])]
    evs, sts = L.ah_sched_simulate(jobs, n_lanes=4, pool_bytes=8 * MB)
    assert all(s["status"] == 0 for s in sts)
    runs = sorted((e["job"], e["part"]) for e in evs)
    assert runs == sorted((j, q) for j, (_, ps) in enumerate(jobs) for q in range(len(ps)))
    _check_pool(evs, 8 * MB)
    for j, (_, ps) in enumerate(jobs):  # parts of a job start in order
        starts = [e["t_start"] for e in evs if e["job"] == j]
        assert [e["part"] for e in evs if e["job"] == j] == list(range(len(ps)))
        assert starts == sorted(starts)
        assert sts[j]["t_done"] == max(e["t_end"] for e in evs if e["job"] == j)


def test_a_later_job_does_not_wait_behind_a_long_one():
    """Round robin over the running jobs: a one-part job arriving while a
    100-part job runs starts at the next free lane, not after the long job."""
    long_job = (0.0, [(1 * MB, 1.0, 0)] * 100)
    short = (10.5, [(1 * MB, 1.0, 0)])
    evs, sts = L.ah_sched_simulate([long_job, short], n_lanes=2, pool_bytes=64 * MB)
    assert sts[1]["t_start"] == 11.0  # the first lane that frees after its arrival
    assert sts[1]["t_done"] - sts[1]["t_submit"] < 2.0
    assert sts[0]["t_done"] >= 50.0


def test_jobs_take_turns_part_by_part():
    a = (0.0, [(1 * MB, 1.0, 0)] * 4)
    b = (0.0, [(1 * MB, 1.0, 0)] * 4)
    evs, _ = L.ah_sched_simulate([a, b], n_lanes=1, pool_bytes=64 * MB)
    assert [e["job"] for e in evs] == [0, 1, 0, 1, 0, 1, 0, 1]


def test_admission_waits_for_pool_memory_and_never_deadlocks():
    """Parts of 3 MiB on four lanes with a 7 MiB pool: at most two run at a
    time, every part runs, every job ends."""
    jobs = [(0.01 * i, [(3 * MB, 0.3, 0)] * (1 + i % 3)) for i in range(12)]
    evs, sts = L.ah_sched_simulate(jobs, n_lanes=4, pool_bytes=7 * MB)
    assert all(s["status"] == 0 for s in sts)
    _check_pool(evs, 7 * MB)
    for e in evs:
        running = [f for f in evs if f["t_start"] <= e["t_start"] < f["t_end"]]
        assert len(running) <= 2
    assert len(evs) == sum(len(ps) for _, ps in jobs)


def test_a_part_larger_than_the_pool_ends_only_its_job():
    jobs = [(0.0, [(1 * MB, 1.0, 0), (9 * MB, 1.0, 0), (1 * MB, 1.0, 0)]),
            (0.0, [(2 * MB, 1.0, 0)] * 3)]
    evs, sts = L.ah_sched_simulate(jobs, n_lanes=2, pool_bytes=8 * MB)
    assert sts[0]["status"] == L.AH_ERR_LIMIT and sts[1]["status"] == 0
    assert not any(e["job"] == 0 and e["part"] >= 1 for e in evs)  # the rest never starts
    assert sum(e["job"] == 1 for e in evs) == 3


def test_overflowing_parts_run_again_and_their_job_waits_for_them():
    jobs = [(0.0, [(1 * MB, 1.0, 0), (1 * MB, 1.0, 2), (1 * MB, 1.0, 0)])]
    evs, sts = L.ah_sched_simulate(jobs, n_lanes=3, pool_bytes=64 * MB)
    assert sts[0]["status"] == 0 and sts[0]["retries"] == 2
    runs = [e["run"] for e in evs if e["part"] == 1]
    assert runs == [0, 1, 2]
    assert sts[0]["t_done"] == 3.0  # the third run of part 1 ends last


def test_simulation_arguments_are_checked():
    with pytest.raises(L.AhError) as e:
        L.ah_sched_simulate([(0.0, [(1, 1.0, 0)])], n_lanes=0, pool_bytes=MB)
    assert e.value.status == L.AH_ERR_INVALID_ARG
    with pytest.raises(L.AhError) as e:
        L.ah_sched_simulate([(-1.0, [(1, 1.0, 0)])], n_lanes=1, pool_bytes=MB)
    assert e.value.status == L.AH_ERR_INVALID_ARG
