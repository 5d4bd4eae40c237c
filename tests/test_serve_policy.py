"""The serving scheduler's policy on the CPU, with a fake clock and a fake
executor: admission never exceeds the HBM budget or the slot limits, jobs are
admitted in arrival (FIFO) order, every job finishes, a batch takes every job
admitted in its step, and one-launch-per-job mode launches each job alone."""
import numpy as np

import workloads as W
from paper_2605_13864_amd.serve import (SMALL_JOB_BYTES, Pending, Scheduler, SlotPool, job_class,
                                        launch_units)


class FakeExecutor:
    """Completes a batch `cost` seconds (proportional to its bytes) after launch."""

    def __init__(self, clock, gbs=5000.0):
        self.clock, self.gbs = clock, gbs
        self.launched = []

    def launch(self, group, si, batching):
        nbytes = sum(p.nbytes for p in group)
        t_done = self.clock[0] + 5e-6 + nbytes / (self.gbs * 1e9)
        self.launched.append((list(p.idx for p in group), si))
        return t_done, (len({job_class(p.job)[:2] for p in group}) if batching else len(group))


    def done(self, t_done):
        return t_done if self.clock[0] >= t_done else None

    def retire(self, p):
        pass


def simulate(jobs, budget, slots, batching=True, dt=2e-5):
    clock = [0.0]
    ex = FakeExecutor(clock)
    arrivals = [j.arrival_s for j in jobs]
    sch = Scheduler(jobs, arrivals, SlotPool(slots), ex, budget, batching, nstreams=3)
    steps = 0
    budget_ok = True
    while not sch.finished():
        sch.step(clock[0])
        budget_ok &= sch.used <= budget
        clock[0] += dt
        steps += 1
        assert steps < 10_000_000
    return sch, ex, budget_ok


def slots_for(jobs, n=4):
    return {c: n for c in {job_class(j) for j in jobs}}


def test_budget_slots_fifo_and_completion():
    jobs = W.serving_jobs(3000, 5, tpose_k=(5, 10), sum_k=(10, 20))
    budget = 64 << 20
    sch, ex, ok = simulate(jobs, budget, slots_for(jobs, 3))
    assert ok and sch.max_used <= budget
    assert sch.admit_order == sorted(sch.admit_order)        # FIFO
    assert len(sch.admit_order) == len(jobs)
    assert not np.isnan(sch.done_t).any()
    assert np.all(sch.done_t >= np.array([j.arrival_s for j in jobs]))
    assert sum(len(ix) for ix, _ in ex.launched) == len(jobs)   # every job launched once


def test_slot_limit_is_respected():
    jobs = W.serving_jobs(2000, 6, tpose_k=(5, 9), sum_k=(10, 16))
    clock = [0.0]
    ex = FakeExecutor(clock, gbs=50.0)                     # slow device: queues build up
    arrivals = [j.arrival_s for j in jobs]
    limit = 2
    slots = SlotPool(slots_for(jobs, limit))
    sch = Scheduler(jobs, arrivals, slots, ex, 1 << 40, True, 2)
    while not sch.finished():
        sch.step(clock[0])
        counts = {}
        for b in sch.inflight:
            for p in b.jobs:
                counts[p.cls] = counts.get(p.cls, 0) + 1
        assert all(v <= limit for v in counts.values()), counts
        clock[0] += 1e-5
    assert len(sch.admit_order) == len(jobs)


def test_batching_groups_admitted_jobs_and_per_job_mode_does_not():
    jobs = W.serving_jobs(1500, 7, tpose_k=(5, 8), sum_k=(10, 14))
    sch_b, ex_b, _ = simulate(jobs, 1 << 40, slots_for(jobs, 64), batching=True, dt=1e-4)
    sch_p, ex_p, _ = simulate(jobs, 1 << 40, slots_for(jobs, 64), batching=False, dt=1e-4)
    assert sch_b.batches < len(jobs) and sch_b.launches < len(jobs)
    assert sch_p.launches == len(jobs)
    # with a coarse tick, several arrivals share a batch
    assert max(len(ix) for ix, _ in ex_b.launched) > 1


def test_budget_blocks_head_of_line():
    jobs = W.serving_jobs(200, 8, tpose_k=(12, 13), sum_k=(24, 26))
    big = max(j.nbytes for j in jobs)
    sch, ex, ok = simulate(jobs, big, slots_for(jobs, 8))
    assert ok
    # a budget of one largest job admits exactly one job at a time when needed
    assert sch.max_used <= big


def test_launch_units_partition_by_kind_and_size():
    jobs = W.serving_jobs(400, 9, tpose_k=(5, 12), sum_k=(10, 24))
    group = [Pending(i, j, j.nbytes, job_class(j)) for i, j in enumerate(jobs)]
    units = launch_units(group, True)
    assert sorted(p.idx for u in units for p in u) == list(range(len(jobs)))   # a partition
    for u in units:
        assert len({(p.job.kind, p.nbytes < SMALL_JOB_BYTES) for p in u}) == 1
        assert [p.idx for p in u] == sorted(p.idx for p in u)                  # admission order
        assert len(u) == 1 or u[0].nbytes < SMALL_JOB_BYTES                    # large jobs alone
    n_large = sum(1 for p in group if p.nbytes >= SMALL_JOB_BYTES)
    assert 0 < n_large < len(group)
    assert len(units) == n_large + 2
    per = launch_units(group, False)
    assert [[p.idx] for p in group] == [[p.idx for p in u] for u in per]
    # with a backlog the large jobs of a kind share a unit as well
    busy = launch_units(group, True, backlog=True)
    assert sorted(p.idx for u in busy for p in u) == list(range(len(jobs)))
    assert len(busy) == 4
    for u in busy:
        assert len({(p.job.kind, p.nbytes < SMALL_JOB_BYTES) for p in u}) == 1


def test_per_job_units_each_have_their_own_completion():
    jobs = W.serving_jobs(500, 10, tpose_k=(5, 9), sum_k=(10, 16))
    sch, ex, _ = simulate(jobs, 1 << 40, slots_for(jobs, 64), batching=False, dt=1e-4)
    assert all(len(ix) == 1 for ix, _ in ex.launched)
    assert sch.batches == len(jobs) == sch.launches


def test_native_policy_host_check(tmp_path):
    """The native loop's policy (csrc/serve_policy.h) under a fake clock and
    executor (tests/native/serve_policy_check.cpp): budget, FIFO admission,
    completion, the batching rule, failed launches."""
    import os
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        import pytest
        pytest.skip("needs g++")
    here = os.path.dirname(os.path.abspath(__file__))
    exe = os.path.join(tmp_path, "serve_policy_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-o", exe,
                    os.path.join(here, "native", "serve_policy_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "serving policy ok" in r.stdout, r.stdout
