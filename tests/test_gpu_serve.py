"""The serving loop on the GPU: jobs of uneven size admitted by budget and run on concurrent
streams give the same HPWL_q as each job alone."""
import pytest

from paper_2402_18311_amd import serve

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    jobs = serve.make_jobs(6, 10_000, 60_000, 60, seed=5)
    for j in jobs:
        j.nbytes = serve.device_bytes(j.netlist)
    budget = int(2.5 * max(j.nbytes for j in jobs))  # admission binds: at most ~3 at once
    alone = serve.fresh(jobs)
    serve.serve_sequential(alone, serve.run_on_gpu)
    mixed = serve.fresh(jobs)
    sch = serve.Scheduler(budget, serve.run_on_gpu)
    sch.serve(mixed)
    assert sch.peak_bytes <= budget and sch.peak_jobs >= 2
    for a, b in zip(alone, mixed):
        assert a.hpwl_q is not None and a.hpwl_q == b.hpwl_q, a.jid
    s = serve.stats(mixed)
    print("served", s, "sequential", serve.stats(alone))


def test_shared_launch_executor_equals_alone():
    """Jobs joining and leaving the shared launches at different rounds (uneven iteration
    counts, a tick that does not divide them, one-iteration jobs that never join) end with
    their alone HPWL_q.  The executor is held until 36 jobs are resident, so its rounds also
    split over two launches of at most 32 slots."""
    import threading
    import time
    jobs = serve.make_jobs(48, 2_000, 30_000, 23, seed=11)
    for k, j in enumerate(jobs):
        j.iters = (1, 7, 23, 40)[k % 4]
        j.nbytes = serve.device_bytes(j.netlist)
    alone = serve.fresh(jobs)
    serve.serve_sequential(alone, serve.run_on_gpu)
    ex = serve.SharedLaunchExecutor(tick=6)
    try:
        ex.pause()
        mixed = serve.fresh(jobs)
        sch = serve.Scheduler(sum(j.nbytes for j in jobs), ex.run)  # all admitted at once
        t = threading.Thread(target=sch.serve, args=(mixed,))
        t.start()
        t_end = time.time() + 60
        while ex.waiting() < 36 and time.time() < t_end and t.is_alive():
            time.sleep(0.01)
        assert ex.waiting() == 36
        ex.resume()
        t.join(timeout=120)
        assert not t.is_alive()
    finally:
        ex.resume()
        ex.close()
    assert ex.peak_resident == 36
    for a, b in zip(alone, mixed):
        assert a.hpwl_q is not None and a.hpwl_q == b.hpwl_q, a.jid
    print("shared launches", serve.stats(mixed), "rounds", ex.rounds,
          "peak per round", ex.peak_resident)


def test_many_jobs_in_flight_have_streams_of_their_own():
    """Forty placers alive at once, each on a stream of its own, iterating with graph capture
    at the same time.  torch's Stream() repeats its pooled streams after 32, so two of them
    would share one (and one's capture would meet the other's work); OwnStreams are distinct,
    and every job ends with its alone HPWL_q."""
    import threading

    import torch

    from paper_2402_18311_amd import hybro as hy
    n = 40
    assert len({torch.cuda.Stream().cuda_stream for _ in range(n)}) <= 32  # the pool
    jobs = serve.make_jobs(n, 2_000, 20_000, 40, seed=9)
    for j in jobs:
        j.nbytes = serve.device_bytes(j.netlist)
    alone = serve.fresh(jobs)
    serve.serve_sequential(alone, serve.run_on_gpu)
    barrier = threading.Barrier(n, timeout=120)
    handles = []

    def run(job):  # as serve.run_on_gpu, held until every placer exists
        stream = hy.OwnStream()
        try:
            pl = hy.Placer(job.netlist, precision=32, stream=stream)
            try:
                nl = job.netlist
                s = pl.new_slot()
                pl.set_positions(s, nl.x0, nl.y0)
                pl.set_schedule(s, 1e-4, 4.0, job.iters)
                handles.append(stream.cuda_stream)
                barrier.wait()
                pl.iterate(s, 4 * nl.bin_w, job.iters, hpwl="last", graph=True)
                job.hpwl_q = int(pl.hpwl(s)[0])
                pl.free_slot(s)
            finally:
                pl.close()
        finally:
            stream.close()
    mixed = serve.fresh(jobs)
    sch = serve.Scheduler(sum(j.nbytes for j in jobs), run)  # all admitted at once
    sch.serve(mixed)
    assert sch.peak_jobs == n and len(set(handles)) == n and all(handles)
    for a, b in zip(alone, mixed):
        assert a.hpwl_q is not None and a.hpwl_q == b.hpwl_q, a.jid
