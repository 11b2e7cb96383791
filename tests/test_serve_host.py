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


class _FakePlacer:
    """Stands in for a Placer on a shared context: counts each slot's iterations; its "HPWL"
    is that count."""

    def __init__(self, ctx, nl):
        self.ctx, self.nl = ctx, nl
        ctx.placers.append(self)

    def new_slot(self):
        s = self.ctx.next_slot
        self.ctx.next_slot += 1
        self.ctx.done[s] = 0
        return s

    def set_positions(self, s, x, y):
        pass

    def set_schedule(self, s, *a):
        pass

    def iterate(self, s, gamma, iters, hpwl=True, graph=False):
        with self.ctx.lock:
            self.ctx.done[s] += iters
            if graph:
                self.ctx.alone.append(iters)

    def hpwl(self, s):
        return [self.ctx.done[s]]

    def close(self):
        self.ctx.closed += 1


class _FakeContext:
    def __init__(self, fail_after=None):
        self.lock = threading.Lock()
        self.done, self.placers, self.calls, self.alone = {}, [], [], []
        self.next_slot, self.closed, self.fail_after = 0, 0, fail_after

    def placer(self, nl):
        return _FakePlacer(self, nl)

    def iterate(self, slots, gammas, iters, hpwl="last", graph=False):
        assert len(slots) == len(gammas) and 1 <= len(slots) <= 32 and iters >= 1
        with self.lock:
            self.calls.append((len(slots), iters))
            if self.fail_after is not None and len(self.calls) > self.fail_after:
                raise RuntimeError("device error")
            for s in slots:
                self.done[s] += iters

    def close(self):
        pass


class _Net:
    def __init__(self, n):
        self.n_movable, self.bin_w = n, 1.0
        self.x0 = self.y0 = None


def test_shared_launch_rounds_give_every_job_its_iterations():
    """Jobs of every size class join and leave the rounds at their own counts: each ends
    with exactly its iteration count, the rounds never pass a job's count, launches take at
    most 32 slots, and every placer is closed."""
    ctxs = []

    def make():
        ctxs.append(_FakeContext())
        return ctxs[-1]
    ex = serve.SharedLaunchExecutor(tick=7, bounds=(100, 1000), make_context=make)
    rng = np.random.default_rng(4)
    jobs = [serve.Job(i, _Net(int(n)), int(it), 0.0, nbytes=1)
            for i, (n, it) in enumerate(zip(rng.integers(10, 5000, 80), rng.integers(1, 40, 80)))]
    try:
        ex.pause()  # let most jobs become resident before the first round
        t = threading.Thread(target=serve.Scheduler(1 << 30, ex.run).serve, args=(jobs,))
        t.start()
        deadline = time.time() + 30
        while ex.waiting() < sum(j.iters > 1 for j in jobs) and time.time() < deadline:
            time.sleep(0.01)
        ex.resume()
        t.join(timeout=30)
        assert not t.is_alive()
    finally:
        ex.resume()
        ex.close()
    assert all(j.hpwl_q == j.iters for j in jobs)
    assert len(ctxs) == 3 and ex.peak_resident > 32
    for c in ctxs:
        assert c.closed == len(c.placers)
        assert all(1 <= n <= 32 and it <= 7 for n, it in c.calls)
        assert all(it <= 7 for it in c.alone)  # a job alone iterates on its own (graph replay)


def test_shared_launch_errors_reach_every_resident_job():
    ex = serve.SharedLaunchExecutor(tick=5, bounds=(), make_context=lambda: _FakeContext(0))
    jobs = [serve.Job(i, _Net(50), 20, 0.0, nbytes=1) for i in range(4)]
    errors = []

    def serve_all():
        try:
            serve.Scheduler(1 << 30, ex.run).serve(jobs)
        except RuntimeError as e:
            errors.append(e)
    try:
        ex.pause()  # all four resident, so the first round is a shared launch, which fails
        t = threading.Thread(target=serve_all)
        t.start()
        deadline = time.time() + 30
        while ex.waiting() < 4 and time.time() < deadline:
            time.sleep(0.01)
        ex.resume()
        t.join(timeout=30)
        assert not t.is_alive()
    finally:
        ex.resume()
        ex.close()
    assert len(errors) == 1 and "device error" in str(errors[0])
    assert all(j.hpwl_q is None for j in jobs)
