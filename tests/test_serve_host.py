"""Admission logic of the serving loop, with a stand-in executor (no GPU)."""
import threading
import time

import numpy as np
import pytest

from paper_2402_18311_amd import serve


def _jobs(sizes, arrivals):
    return [serve.Job(i, None, 0, a, nbytes=b) for i, (b, a) in enumerate(zip(sizes, arrivals))]


def _runner(log, lock, dt=0.03):
    state = {"used": 0, "active": 0, "max_used": 0}

    def run(job):
        with lock:
            log.append(("start", job.jid))
            state["used"] += job.nbytes
            state["active"] += 1
            state["max_used"] = max(state["max_used"], state["used"])
        time.sleep(dt)
        with lock:
            state["used"] -= job.nbytes
            state["active"] -= 1
            log.append(("end", job.jid))
        job.hpwl_q = 1000 + job.jid
    return run, state


def test_budget_fifo_and_concurrency():
    sizes = [4, 3, 5, 2, 6, 1]
    jobs = _jobs(sizes, [0.0] * 6)
    log, lock = [], threading.Lock()
    run, st = _runner(log, lock)
    sch = serve.Scheduler(8, run)
    sch.serve(jobs)
    starts = [j for e, j in log if e == "start"]
    assert starts == sorted(starts)  # admitted in arrival (then id) order
    assert st["max_used"] <= 8 and sch.peak_bytes <= 8
    assert sch.peak_jobs >= 2  # several jobs on the device at once
    assert all(j.hpwl_q == 1000 + j.jid and j.finish >= j.start >= j.arrival for j in jobs)
    s = serve.stats(jobs)
    assert s["jobs"] == 6 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_oversized_job_runs_alone_and_arrivals_are_respected():
    jobs = _jobs([20, 2, 2], [0.0, 0.0, 0.15])
    log, lock = [], threading.Lock()
    run, st = _runner(log, lock, dt=0.05)
    sch = serve.Scheduler(8, run)
    sch.serve(jobs)
    assert log[:2] == [("start", 0), ("end", 0)]  # bigger than the budget: alone
    assert jobs[2].start >= 0.15 - 1e-3  # not admitted before it arrived
    assert sch.peak_bytes == 20


def test_sequential_baseline_one_at_a_time():
    jobs = _jobs([1, 1, 1], [0.0, 0.0, 0.02])
    log, lock = [], threading.Lock()
    run, st = _runner(log, lock, dt=0.02)
    serve.serve_sequential(jobs, run)
    assert [e for e, _ in log] == ["start", "end"] * 3
    assert all(b.start >= a.finish for a, b in zip(jobs, jobs[1:]))


def test_worker_error_propagates():
    def bad(job):
        raise RuntimeError("boom")
    with pytest.raises(RuntimeError):
        serve.Scheduler(8, bad).serve(_jobs([1], [0.0]))


def test_job_netlists_do_not_depend_on_worker_count():
    from paper_2402_18311_amd import serve
    a = serve.make_jobs(3, 1_000, 4_000, 10, 5, workers=0)
    b = serve.make_jobs(3, 1_000, 4_000, 10, 5, workers=2)
    for ja, jb in zip(a, b):
        assert ja.netlist.n_movable == jb.netlist.n_movable
        assert np.array_equal(ja.netlist.pin_cell, jb.netlist.pin_cell)
        assert np.array_equal(ja.netlist.x0, jb.netlist.x0)
