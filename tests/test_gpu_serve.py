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
