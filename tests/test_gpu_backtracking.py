"""Nesterov step with ePlace backtracking on the device against the FP64 oracle.

In FP64 the device takes the same accept / redo decision as the oracle at every step (the
decision compares two step lengths that both sides form from the same reductions up to
summation order), so positions follow the oracle to 1e-10 of the die over a placement in which
steps are redone.  FP32 and batched runs are checked for their invariants.
"""
import numpy as np
import pytest

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hy():
    from paper_2402_18311_amd import hybro
    return hybro


_cache = {}


def setup(hy, orc, case, prec):
    key = (case, prec)
    if key not in _cache:
        nl = {"tiny": lambda: netgen.make_netlist("tiny", 0),
              "tiny_mm": lambda: netgen.make_small(1000, 1100, 64, seed=1, n_fixed=6,
                                                   movable_macros=True, macro_frac=0.3),
              "mid": lambda: netgen.make_netlist("mid", 0)}[case]()
        _cache[key] = (nl, hy.Placer(nl, precision=prec), orc.Oracle(nl))
    return _cache[key]


@pytest.mark.parametrize("case", ["tiny", "tiny_mm"])
def test_backtracking_follows_oracle_fp64(hy, orc, case):
    nl, pl, o = setup(hy, orc, case, 64)
    gamma = 4 * nl.bin_w
    n = nl.n_movable
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, 1e-4, 4.0, 200)
    pl.set_backtracking(s, True)
    st = o.new_state(nl.x0, nl.y0)
    ratio = o.lambda_ratio(4.0, 200)
    lam = None
    rejects = 0
    for it in range(80):
        pl.eval(s, gamma, want_host=False)
        r = o.eval(st["v"][:n], st["v"][n:], gamma)
        gw = np.concatenate([r["gwx"], r["gwy"]])
        gd = np.concatenate([r["gdx"], r["gdy"]])
        if lam is None:
            lam = 1e-4 * np.abs(gw).sum() / np.abs(gd).sum()
        pl.step(s)
        redo = o.nesterov_step_bt(lam, gw + lam * gd, st)
        rejects += redo
        if not redo:
            lam *= ratio
        sd = pl.state(s)
        assert sd["rejects"] == rejects, it
        assert sd["k"] == st["k"], it
        x, y = pl.positions(s)
        u = np.concatenate([x, y])
        assert np.max(np.abs(u - st["u"])) < 1e-10 * nl.W, it
        assert sd["lambda_"] == pytest.approx(lam, rel=1e-12), it
    print(f"{case}: {rejects} of 80 steps redone")
    assert rejects > 0  # the redo path ran
    pl.set_backtracking(s, False)
    pl.free_slot(s)


def test_backtracking_iterate_matches_single_calls_and_batches(hy, orc):
    """hp_iterate with backtracking equals the same iterations one call at a time, and a slot in
    a batch of three equals the slot alone (decisions are per slot, on the device)."""
    nl, pl, o = setup(hy, orc, "tiny", 64)
    gamma = 4 * nl.bin_w
    ss = [pl.new_slot() for _ in range(4)]
    for k, s in enumerate(ss):
        pl.set_positions(s, *nl.random_positions(300 + (k % 3)))
        pl.set_schedule(s, 1e-4, 4.0, 200)
        pl.set_backtracking(s, True)
    # slot 3 repeats slot 0's start, one call at a time
    pl.iterate(ss[:3], gamma, 50, hpwl=True)
    for _ in range(50):
        pl.eval(ss[3], gamma, want_host=False)
        pl.step(ss[3])
    a, b = pl.positions(ss[0]), pl.positions(ss[3])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert pl.state(ss[0])["rejects"] == pl.state(ss[3])["rejects"]
    for k in (1, 2):  # alone
        pl.set_positions(ss[3], *nl.random_positions(300 + k))
        pl.set_backtracking(ss[3], True)
        pl.iterate(ss[3], gamma, 50, hpwl=True)
        a, b = pl.positions(ss[k]), pl.positions(ss[3])
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for s in ss:
        pl.free_slot(s)


def test_backtracking_fp32_mid_places(hy, orc):
    """mid in FP32 with backtracking: some steps are redone, the state counts them, and the
    placement reaches an HPWL within a few percent of the plain method's."""
    nl, pl, o = setup(hy, orc, "mid", 32)
    gamma = 4 * nl.bin_w
    res = {}
    for bt in (False, True):
        s = pl.new_slot()
        pl.set_positions(s, nl.x0, nl.y0)
        pl.set_schedule(s, 1e-4, 4.0, 400)
        pl.set_backtracking(s, bt)
        pl.iterate(s, gamma, 400, hpwl=True)
        st = pl.state(s)
        res[bt] = (st["hpwl_q"], st["k"], st["rejects"], st["overflow"])
        pl.free_slot(s)
    print(res)
    assert res[False][2] == 0 and res[False][1] == 400
    assert res[True][2] > 0 and res[True][1] + res[True][2] == 400
    assert res[True][0] < 1.05 * res[False][0]
