"""Serving loop: placement jobs of uneven size, admitted by HBM budget and run concurrently.

A job is one synthetic netlist placed by the plain method: `iters` iterations (objective and
gradient of Eq. 2, Nesterov step) from its initial positions; its result is the exact HPWL of
Eq. 1 after the last one (HPWL_q).  Jobs arrive on a trace.  The server admits them in arrival
order as long as their device buffers (netlist + one slot) fit in the budget — a job larger
than the whole budget is admitted alone — keeps their state resident while they run, and
releases a finished job's memory so the next arrivals are admitted at once.  Two executors:

* per-job streams (`run_on_gpu`): every admitted job runs on its own HIP stream from its own
  host thread (steady-state blocks replayed from a HIP graph), so the kernels of concurrent
  jobs interleave on the device (launches of different streams are not run side by side on
  this stack: two half-machine kernels on two streams take as long as on one);
* shared launches (`SharedLaunchExecutor`): admitted jobs are loaded by their host threads
  onto a shared library context of their size class and, after their first iteration, join
  its resident set; the class's device thread advances every resident job by `tick`
  iterations per round, each pass of an iteration one launch over all of their slots
  (hp_iterate_multi, up to 32 slots a launch, steady blocks replayed from a HIP graph while
  the resident set stays the same), so small jobs no longer cost a launch sequence each;
  classes run on their own streams and interleave.

The baseline is the same trace served sequentially: one job at a time, in arrival order.
Every kernel is deterministic per slot and the shared launches are bit-identical to a slot's
own, so each job's HPWL_q is identical alone and in the mix, under either executor.

    python -m paper_2402_18311_amd.serve --jobs 200 --budget-gb 8

The scheduler is independent of the executor (`run` callable), so its admission logic is
tested on the CPU with a stand-in executor.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import threading
import time

import numpy as np

from . import netgen


@dataclasses.dataclass
class Job:
    jid: int
    netlist: object
    iters: int
    arrival: float            # seconds after the start of the trace
    nbytes: int = 0           # device bytes while resident (netlist buffer + one slot)
    start: float = math.nan   # admission time (trace clock)
    finish: float = math.nan
    hpwl_q: int | None = None

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class Scheduler:
    """Admission by budget in arrival order; one host thread per admitted job.

    `run(job)` executes a job (blocking) and fills job.hpwl_q.  `serve` returns when every job
    has finished; it records the peak resident bytes and the peak number of concurrent jobs."""

    def __init__(self, budget_bytes: int, run):
        self.budget = int(budget_bytes)
        self.run = run
        self.peak_bytes = 0
        self.peak_jobs = 0

    def serve(self, jobs: list[Job]) -> None:
        order = sorted(jobs, key=lambda j: (j.arrival, j.jid))
        cv = threading.Condition()
        used = 0
        active = 0
        errors: list[BaseException] = []
        threads = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731

        def worker(job: Job):
            nonlocal used, active
            try:
                self.run(job)
            except BaseException as e:  # surfaced after the loop
                errors.append(e)
            finally:
                with cv:
                    job.finish = now()
                    used -= job.nbytes
                    active -= 1
                    cv.notify_all()

        i = 0
        with cv:
            while i < len(order):
                job = order[i]
                wait = job.arrival - now()
                if wait > 0:
                    cv.wait(timeout=wait)
                    continue
                fits = used + job.nbytes <= self.budget or active == 0
                if not fits:
                    cv.wait()
                    continue
                used += job.nbytes
                active += 1
                self.peak_bytes = max(self.peak_bytes, used)
                self.peak_jobs = max(self.peak_jobs, active)
                job.start = now()
                t = threading.Thread(target=worker, args=(job,), daemon=True)
                threads.append(t)
                t.start()
                i += 1
        for t in threads:
            t.join()
        if errors:
            raise errors[0]


def serve_sequential(jobs: list[Job], run) -> None:
    """The baseline: one job at a time in arrival order, each started at max(arrival, the
    previous finish)."""
    t0 = time.perf_counter()
    for job in sorted(jobs, key=lambda j: (j.arrival, j.jid)):
        wait = job.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        job.start = time.perf_counter() - t0
        run(job)
        job.finish = time.perf_counter() - t0


def stats(jobs: list[Job]) -> dict:
    lat = np.array([j.latency for j in jobs])
    span = max(j.finish for j in jobs) - min(j.arrival for j in jobs)
    return {"jobs": len(jobs), "jobs_per_s": round(len(jobs) / span, 4),
            "makespan_s": round(span, 4), "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "mean_latency_s": round(float(lat.mean()), 4)}


# ---- jobs on the GPU -------------------------------------------------------------------------
_query = {}


def device_bytes(nl, precision: int = 32) -> int:
    """Device bytes one job holds while resident: its netlist buffer and one slot."""
    from . import hybro as hy
    if precision not in _query:
        _query[precision] = hy.hp_create(0, None, precision)
    ctx = _query[precision]
    shape = hy.hp_shape(nl.n_cells, nl.n_movable, int(len(nl.net_start) - 1),
                        int(len(nl.pin_cell)))
    die = hy.hp_die(float(nl.W), float(nl.H), int(nl.mx), int(nl.my), 1.0, 1, 0)
    return int(hy.hp_netlist_bytes(ctx, shape, die) + hy.hp_slot_bytes(ctx, shape, die) + 512)


def run_on_gpu(job: Job) -> None:
    """Place one job on its own stream: load, iterate, read the HPWL, release."""
    import torch

    from . import hybro as hy
    # The job's kernels run on a stream of its own (not one of torch's pooled streams, which
    # concurrent jobs could share); its buffers come from torch's pool on the default stream,
    # and are dropped only after hp_destroy has synchronised the job's stream, so the next
    # allocation may reuse them at once.
    stream = hy.OwnStream(torch.cuda.current_device())
    try:
        pl = hy.Placer(job.netlist, precision=32, stream=stream)
    except BaseException:
        stream.close()
        raise
    try:
        s = pl.new_slot()
        nl = job.netlist
        pl.set_positions(s, nl.x0, nl.y0)
        pl.set_schedule(s, 1e-4, 4.0, job.iters)
        # the job's result is the exact HPWL after its last iteration; steady-state blocks are
        # replayed from a captured HIP graph on the job's stream
        pl.iterate(s, 4 * nl.bin_w, job.iters, hpwl="last", graph=True)
        job.hpwl_q = int(pl.hpwl(s)[0])
        pl.free_slot(s)
    finally:
        pl.close()
        del pl
        stream.close()


class _LaunchGroup:
    """One shared context and its device thread: the resident jobs of one size class."""

    def __init__(self, tick: int, make_context):
        self.tick = tick
        self.ctx = make_context()
        self.cv = threading.Condition()
        self.resident: list[dict] = []
        self.rounds = 0
        self.peak_resident = 0
        self.stop = False
        self.paused = False
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def _loop(self) -> None:
        while True:
            with self.cv:
                while (self.paused or not self.resident) and not self.stop:
                    self.cv.wait()
                if self.stop:
                    return
                batch = list(self.resident)
            self.peak_resident = max(self.peak_resident, len(batch))
            step = min(self.tick, min(e["left"] for e in batch))
            try:
                if len(batch) == 1:  # alone: its own launches, steady blocks from a HIP graph
                    e = batch[0]
                    e["pl"].iterate(e["slot"], e["gamma"], step, hpwl=False, graph=True)
                for c in range(0, len(batch) if len(batch) > 1 else 0, 32):
                    part = batch[c:c + 32]
                    self.ctx.iterate([e["slot"] for e in part], [e["gamma"] for e in part], step,
                                     hpwl=False, graph=True)
                self.rounds += 1
                done = []
                for e in batch:
                    e["left"] -= step
                    if e["left"] == 0:
                        e["job"].hpwl_q = int(e["pl"].hpwl(e["slot"])[0])
                        done.append(e)
            except BaseException as err:  # every resident job fails with it
                done = batch
                for e in batch:
                    e["error"] = err
            with self.cv:
                for e in done:
                    self.resident.remove(e)
            for e in done:
                e["done"].set()


class SharedLaunchExecutor:
    """Jobs on shared contexts, advanced together in shared launches.

    Jobs are split into size classes by movable cells (`bounds`: class k holds jobs below
    bounds[k], the last class the rest); each class has its own context, stream and device
    thread, so a small job is not held to the iteration rate of a large one while the classes
    still interleave on the device.  `run(job)` (called from the scheduler's per-job thread)
    loads the job onto its class's context, runs its first iteration alone (lambda_0 and the
    scatter grouping), hands it to the device thread and waits for its result; each device
    thread advances its resident jobs by min(tick, fewest iterations left) per round (a job
    alone in its class with its own launches, several in shared launches of up to 32 slots,
    both replaying steady blocks from a HIP graph; the results are the same) and reads a job's
    HPWL when it is done.  The default tick, 16, is a multiple of the 8-iteration graph block
    of the default scatter policy, so that rounds of an unchanged resident set replay it."""

    def __init__(self, tick: int = 16, precision: int = 32,
                 bounds: tuple = (40_000, 160_000, 640_000), make_context=None):
        """make_context: () -> a context (hybro.Context: placer, iterate, close); by default
        one of the given precision on a stream of its own."""
        self._streams = []  # the streams of the default contexts, closed after them
        if make_context is None:
            def make_context():
                import torch

                from . import hybro as hy
                s = hy.OwnStream(torch.cuda.current_device())
                self._streams.append(s)
                return hy.Context(precision=precision, stream=s)
        self.bounds = tuple(bounds)
        self.groups = [_LaunchGroup(int(tick), make_context) for _ in range(len(self.bounds) + 1)]

    def _group(self, job: Job) -> _LaunchGroup:
        n = job.netlist.n_movable
        return self.groups[sum(n >= b for b in self.bounds)]

    @property
    def rounds(self) -> int:
        return sum(g.rounds for g in self.groups)

    @property
    def peak_resident(self) -> int:
        """The most jobs one round of one class advanced together."""
        return max(g.peak_resident for g in self.groups)

    def reset_stats(self) -> None:
        for g in self.groups:
            g.rounds, g.peak_resident = 0, 0

    def run(self, job: Job) -> None:
        g = self._group(job)
        nl = job.netlist
        pl = g.ctx.placer(nl)
        try:
            s = pl.new_slot()
            pl.set_positions(s, nl.x0, nl.y0)
            pl.set_schedule(s, 1e-4, 4.0, job.iters)
            gamma = 4 * nl.bin_w
            first = min(1, job.iters)
            pl.iterate(s, gamma, first, hpwl=False)
            if job.iters == first:
                job.hpwl_q = int(pl.hpwl(s)[0])
                return
            e = {"pl": pl, "slot": s, "gamma": gamma, "left": job.iters - first, "job": job,
                 "done": threading.Event(), "error": None}
            with g.cv:
                g.resident.append(e)
                g.cv.notify_all()
            e["done"].wait()
            if e["error"] is not None:
                raise e["error"]
        finally:
            pl.close()

    def pause(self) -> None:
        """Hold the device threads after their current rounds (jobs still load and join)."""
        for g in self.groups:
            with g.cv:
                g.paused = True

    def resume(self) -> None:
        for g in self.groups:
            with g.cv:
                g.paused = False
                g.cv.notify_all()

    def waiting(self) -> int:
        """Jobs resident (loaded, first iteration done) and not yet finished."""
        n = 0
        for g in self.groups:
            with g.cv:
                n += len(g.resident)
        return n

    def close(self) -> None:
        for g in self.groups:
            with g.cv:
                g.stop = True
                g.cv.notify_all()
        for g in self.groups:
            g.thread.join()
            g.ctx.close()
        for s in self._streams:
            s.close()
        self._streams = []


def _make_one(args):
    c, s = args
    return netgen.make_netlist(netgen.scaled_config(int(c)), s)


def make_jobs(n: int, lo: int, hi: int, iters: int, seed: int, workers: int = 0) -> list[Job]:
    """n netlists shaped like the mid workload with log-uniform sizes in [lo, hi] cells
    (arrival times are set by `poisson_arrivals`), drawn on `workers` processes (0: in this
    one).  Each netlist has its own seed, so the draws do not depend on the worker count."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n)).round().astype(int)
    args = [(int(c), seed * 1000 + i) for i, c in enumerate(sizes)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            nls = pool.map(_make_one, args, chunksize=1)
    else:
        nls = [_make_one(a) for a in args]
    return [Job(i, nl, iters, 0.0) for i, nl in enumerate(nls)]


def poisson_arrivals(jobs: list[Job], rate: float, seed: int) -> None:
    rng = np.random.default_rng(seed + 7)
    t = np.cumsum(rng.exponential(1.0 / rate, len(jobs)))
    for j, a in zip(jobs, t - t[0]):
        j.arrival = float(a)


def fresh(jobs: list[Job]) -> list[Job]:
    return [Job(j.jid, j.netlist, j.iters, j.arrival, j.nbytes) for j in jobs]


def measure(n_jobs=200, lo=10_000, hi=2_200_000, iters=500, budget_gb=8.0, rate_frac=0.8,
            seed=0, log=print, workers=0, tick=16) -> dict:
    """Config 5: capacity of sequential plain solves (all jobs queued at t = 0), then a Poisson
    trace at rate_frac x that capacity served sequentially and by the server with each
    executor."""
    jobs = make_jobs(n_jobs, lo, hi, iters, seed, workers)
    for j in jobs:
        j.nbytes = device_bytes(j.netlist)
    log(f"[serve] {n_jobs} jobs, {sum(j.netlist.n_movable for j in jobs)} cells in all")
    run_on_gpu(fresh(jobs[:1])[0])  # code objects load lazily: warm every kernel once
    cap = fresh(jobs)
    serve_sequential(cap, run_on_gpu)
    capacity = len(cap) / max(j.finish for j in cap)
    rate = rate_frac * capacity
    poisson_arrivals(jobs, rate, seed)
    log(f"[serve] sequential capacity {capacity:.3f} jobs/s; trace at {rate:.3f} jobs/s")
    seq = fresh(jobs)
    serve_sequential(seq, run_on_gpu)
    srv = fresh(jobs)
    sch = Scheduler(int(budget_gb * 2**30), run_on_gpu)
    sch.serve(srv)
    log(f"[serve] per-job streams: {stats(srv)}")
    ex = SharedLaunchExecutor(tick=tick)
    try:
        warm = fresh(jobs[:2])  # the shared-launch kernels' code objects load lazily too
        Scheduler(int(budget_gb * 2**30), ex.run).serve(warm)
        shr = fresh(jobs)
        sch2 = Scheduler(int(budget_gb * 2**30), ex.run)
        ex.reset_stats()
        sch2.serve(shr)
    finally:
        ex.close()
    log(f"[serve] shared launches: {stats(shr)}")
    by_id = lambda js: sorted(js, key=lambda j: j.jid)  # noqa: E731
    same = all(a.hpwl_q == b.hpwl_q == c.hpwl_q
               for a, b, c in zip(by_id(seq), by_id(srv), by_id(shr)))
    return {"config": {"jobs": n_jobs, "cells": [lo, hi], "iters": iters, "budget_gb": budget_gb,
                       "arrival_rate_jobs_per_s": round(rate, 4), "rate_frac_of_capacity": rate_frac,
                       "seed": seed, "tick_iters": tick},
            "sequential_capacity_jobs_per_s": round(capacity, 4),
            "sequential": stats(seq), "served": stats(srv), "served_shared_launches": stats(shr),
            "peak_resident_gb": round(sch.peak_bytes / 2**30, 3), "peak_concurrent_jobs": sch.peak_jobs,
            "shared_launches": {"peak_resident_gb": round(sch2.peak_bytes / 2**30, 3),
                                "peak_concurrent_jobs": sch2.peak_jobs,
                                "peak_jobs_per_launch": ex.peak_resident, "rounds": ex.rounds},
            "equal_hpwl": same}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--jobs", type=int, default=200)
    ap.add_argument("--lo", type=int, default=10_000)
    ap.add_argument("--hi", type=int, default=2_200_000)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--rate-frac", type=float, default=0.8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=8,
                    help="processes drawing the synthetic netlists")
    ap.add_argument("--tick", type=int, default=16,
                    help="iterations per round of the shared-launch executor")
    a = ap.parse_args()
    print(json.dumps(measure(a.jobs, a.lo, a.hi, a.iters, a.budget_gb, a.rate_frac, a.seed,
                             workers=a.workers, tick=a.tick)))


if __name__ == "__main__":
    main()
