"""Parity of the preconditioned Nesterov step (the gradient descent of Sec. 3.1 in ePlace's
accelerated form) in both of its device forms: the fused form (every block of the update
reduces the step's norms itself, up to 1024 cell-gradient partials) and the closing-reduction
form (a one-block reduction forms the step first), which netlists above 262,144 movable cells
take, the large workload included.

The step is isolated from the gradient: the oracle's step is fed the device's own gradient
and lambda, so the only differences are the step's arithmetic and the rounding of positions
to the compute type.  Bar (FP32): the displacement of every step within 1e-5 of its own L2
norm plus two units in the last place of the positions (the FP32 storage of u and v; one ulp
at coordinate 1000 is 6e-5, about 3e-4 of a 0.1-bin step at mid), the BB length within 1e-5
relative.  FP64: 1e-10 on both."""
import numpy as np
import pytest

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hy():
    from paper_2402_18311_amd import hybro
    return hybro


_NETS = {
    "tiny": lambda: netgen.make_netlist("tiny", 0),
    "small": lambda: netgen.make_small(20_011, 21_003, 128, seed=3, n_fixed=40),
    # above 1024 cell-gradient partials (262,144 cells): the closing-reduction form; a small
    # grid keeps the oracle cheap
    "big300k": lambda: netgen.make_small(300_000, 313_500, 128, seed=5, n_fixed=40),
    "mid": lambda: netgen.make_netlist("mid", 0),
    # the full large workload (2.2 M movable cells), in the closing-reduction form it runs in
    "large": lambda: netgen.make_netlist("large", 0),
}
_cache = {}


def setup(hy, orc, case, prec):
    key = (case, prec)
    if key not in _cache:
        nl = _NETS[case]()
        _cache[key] = (nl, hy.Placer(nl, precision=prec), orc.Oracle(nl))
    return _cache[key]


def _ulp(v, prec):
    return np.spacing(np.abs(v).astype(np.float32)).astype(np.float64) if prec == 32 \
        else np.spacing(np.abs(v))


@pytest.mark.parametrize("case,prec,forced", [
    ("small", 32, False), ("small", 32, True), ("small", 64, True), ("tiny", 64, False),
    ("big300k", 32, False), ("big300k", 64, False), ("mid", 32, False), ("large", 32, False)])
def test_step_parity_on_device_gradient(hy, orc, case, prec, forced):
    nl, pl, o = setup(hy, orc, case, prec)
    n = nl.n_movable
    gamma = 4 * nl.bin_w
    parts = (n + 255) // 256
    if forced:
        pl.set_tunable(hy.HP_TUNE_FUSED_STEP_PARTS, 0)
    try:
        assert (parts > pl.tunable(hy.HP_TUNE_FUSED_STEP_PARTS)) == (forced or parts > 1024)
        s = pl.new_slot()
        pl.set_positions(s, nl.x0, nl.y0)
        pl.set_schedule(s, 1e-4, 4.0, 200)
        st = o.new_state(nl.x0, nl.y0)
        worst = 0.0
        for it in range(4):
            _, gx, gy = pl.eval(s, gamma, grads=True)
            g = np.concatenate([gx.cpu().numpy()[0], gy.cpu().numpy()[0]]).astype(np.float64)
            lam = pl.state(s)["lambda_"]
            v0 = st["v"].copy()
            o.nesterov_step(lam, g, st)
            pl.step(s)
            x, y = pl.positions(s)
            u = np.concatenate([x, y]).astype(np.float64)
            d_orc = st["u"] - v0
            err = np.linalg.norm(u - st["u"])
            if prec == 32:
                bar = 1e-5 * np.linalg.norm(d_orc) + 2.0 * np.linalg.norm(_ulp(st["u"], 32))
            else:
                bar = 1e-10 * np.linalg.norm(d_orc) + 1e-10 * nl.W
            worst = max(worst, err / max(np.linalg.norm(d_orc), 1e-300))
            assert err <= bar, (it, err, bar, np.linalg.norm(d_orc))
            sd = pl.state(s)
            assert sd["k"] == st["k"] and sd["a"] == pytest.approx(st["a"], rel=1e-14)
            assert sd["alpha"] == pytest.approx(st["alpha"], rel=1e-5 if prec == 32 else 1e-10)
            # the look-ahead point v too
            vx, vy = pl.eval_positions(s)
            vd = np.concatenate([vx, vy]).astype(np.float64)
            vbar = (1e-5 * np.linalg.norm(st["v"] - v0) + 3.0 * np.linalg.norm(_ulp(st["v"], 32))
                    if prec == 32 else 1e-10 * (np.linalg.norm(st["v"] - v0) + nl.W))
            assert np.linalg.norm(vd - st["v"]) <= vbar, it
        print(f"{case} fp{prec} forced={forced}: worst step error / step norm {worst:.2e}")
        pl.free_slot(s)
    finally:
        pl.set_tunable(hy.HP_TUNE_FUSED_STEP_PARTS, 1024)


@pytest.mark.parametrize("case,prec", [("small", 32), ("tiny", 64)])
def test_closing_reduction_form_is_bit_identical(hy, orc, case, prec):
    """Both forms reduce the same partials in the same order: the same bits, step after step."""
    nl, pl, o = setup(hy, orc, case, prec)
    gamma = 4 * nl.bin_w
    a, b = pl.new_slot(), pl.new_slot()
    for s in (a, b):
        pl.set_positions(s, nl.x0, nl.y0)
        pl.set_schedule(s, 1e-4, 4.0, 200)

    def snap(s):
        st = pl.state(s)
        x, y = pl.positions(s)
        vx, vy = pl.eval_positions(s)
        return (st["k"], st["a"], st["alpha"], st["lambda_"], x.tobytes(), y.tobytes(),
                vx.tobytes(), vy.tobytes())
    try:
        for chunk in (1, 5, 11):
            pl.set_tunable(hy.HP_TUNE_FUSED_STEP_PARTS, 1024)
            pl.iterate(a, gamma, chunk, hpwl=True)
            pl.set_tunable(hy.HP_TUNE_FUSED_STEP_PARTS, 0)
            pl.iterate(b, gamma, chunk, hpwl=True)
            assert snap(a) == snap(b), chunk
            assert pl.hpwl(a)[0] == pl.hpwl(b)[0]
    finally:
        pl.set_tunable(hy.HP_TUNE_FUSED_STEP_PARTS, 1024)
        pl.free_slot(a)
        pl.free_slot(b)


def test_tunables_reject_bad_values(hy, orc):
    nl, pl, o = setup(hy, orc, "tiny", 64)
    L = hy.lib()
    for which, value in ((hy.HP_TUNE_FUSED_STEP_PARTS, -1), (hy.HP_TUNE_FUSED_STEP_PARTS, 1025),
                         (hy.HP_TUNE_SPECTRAL_THREADS, 256), (hy.HP_TUNE_CHARGE_RECORDS, 2),
                         (hy.HP_TUNE_NONTEMPORAL, 2), (hy.HP_TUNE_NONTEMPORAL, -1), (7, 0)):
        assert L.hp_set_tunable(pl.ctx, pl.netlist, which, value) == hy.HP_EINVAL
    assert L.hp_set_tunable(pl.ctx, 99, hy.HP_TUNE_SPECTRAL_THREADS, 0) == hy.HP_ESTATE
    assert pl.tunable(hy.HP_TUNE_FUSED_STEP_PARTS) == 1024
    assert pl.tunable(hy.HP_TUNE_SPECTRAL_THREADS) == 0
    assert pl.tunable(hy.HP_TUNE_CHARGE_RECORDS) == 1
    assert pl.tunable(hy.HP_TUNE_NONTEMPORAL) == 0


@pytest.mark.parametrize("threads", [512, 1024])
def test_spectral_width_changes_no_field(hy, orc, threads):
    nl, pl, o = setup(hy, orc, "small", 32)
    gamma = 4 * nl.bin_w
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    try:
        pl.eval(s, gamma, lam=0.5, keep_maps=True)
        ref = [pl.map(s, m) for m in (hy.HP_MAP_EX, hy.HP_MAP_EY)]
        pl.set_tunable(hy.HP_TUNE_SPECTRAL_THREADS, threads)
        pl.eval(s, gamma, lam=0.5, keep_maps=True)
        got = [pl.map(s, m) for m in (hy.HP_MAP_EX, hy.HP_MAP_EY)]
        for r, g in zip(ref, got):
            assert np.array_equal(r, g)
    finally:
        pl.set_tunable(hy.HP_TUNE_SPECTRAL_THREADS, 0)
        pl.free_slot(s)


def test_mid_fp32_placement_lands_on_the_oracle(hy, orc):
    """End to end (Eq. 1): the device's FP32 plain placement of mid (1000 iterations) ends
    within 0.5% of the FP64 oracle's final exact HPWL (tests/golden/mid_place_fp64.json,
    written by tests/golden/make_mid_place_golden.py from the oracle alone).  The two
    trajectories separate chaotically over a run, so the bar is on the final value."""
    from helpers import load_json
    ref = load_json("mid_place_fp64.json")
    nl, pl, o = setup(hy, orc, "mid", 32)
    gamma = 4 * nl.bin_w
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, ref["lambda0_scale"], ref["lambda_decades"], ref["iterations"])
    trace = []
    for k in range(ref["iterations"] // 100):
        pl.iterate(s, gamma, 100, hpwl=True)
        trace.append(int(pl.hpwl(s)[0]))
    want = ref["final_hpwl_q"]
    print("mid fp32 HPWL every 100:", [t / 65536 for t in trace])
    print("oracle fp64           :", [t / 65536 for t in ref["hpwl_q_every_100"]])
    assert abs(trace[-1] - want) <= 0.005 * want, (trace[-1] / 65536, want / 65536)
    pl.free_slot(s)


@pytest.mark.parametrize("case,prec", [("small", 32), ("tiny", 64)])
def test_interleaved_sweep_order_is_bit_identical(hy, orc, case, prec):
    """The interleaved block order of the net sweep moves no pin's work between lanes: the
    same gradients, steps and exact HPWL, bit for bit."""
    nl, pl, o = setup(hy, orc, case, prec)
    gamma = 4 * nl.bin_w
    a, b = pl.new_slot(), pl.new_slot()
    for s in (a, b):
        pl.set_positions(s, nl.x0, nl.y0)
        pl.set_schedule(s, 1e-4, 4.0, 200)
    try:
        for chunk in (1, 6, 10):
            pl.set_tunable(hy.HP_TUNE_SWEEP_INTERLEAVE, 0)
            _, gxa, gya = pl.eval(a, gamma, grads=True)
            pl.step(a)
            pl.iterate(a, gamma, chunk, hpwl=True)
            pl.set_tunable(hy.HP_TUNE_SWEEP_INTERLEAVE, 1)
            _, gxb, gyb = pl.eval(b, gamma, grads=True)
            pl.step(b)
            pl.iterate(b, gamma, chunk, hpwl=True)
            assert torch_equal(gxa, gxb) and torch_equal(gya, gyb)
            assert pl.hpwl(a)[0] == pl.hpwl(b)[0]
            xa, ya = pl.positions(a)
            xb, yb = pl.positions(b)
            assert np.array_equal(xa, xb) and np.array_equal(ya, yb), chunk
    finally:
        pl.set_tunable(hy.HP_TUNE_SWEEP_INTERLEAVE, 0)
        pl.free_slot(a)
        pl.free_slot(b)


def torch_equal(a, b):
    return bool((a.cpu() == b.cpu()).all())


@pytest.mark.parametrize("case,prec", [("small", 32), ("tiny", 64)])
def test_nontemporal_sweep_is_bit_identical(hy, orc, case, prec):
    """Cache hints on the sweep's pin loads and gradient stores change no value: the same
    gradients, steps and exact HPWL, bit for bit, eagerly and under graph replay (a placer on
    a stream of its own, which graph replay needs)."""
    import torch
    nl = _NETS[case]()
    pl = hy.Placer(nl, precision=prec, stream=torch.cuda.Stream())
    gamma = 4 * nl.bin_w
    a, b = pl.new_slot(), pl.new_slot()
    for s in (a, b):
        pl.set_positions(s, nl.x0, nl.y0)
        pl.set_schedule(s, 1e-4, 4.0, 200)
    try:
        for chunk, graph in ((1, False), (6, False), (24, True)):
            pl.set_tunable(hy.HP_TUNE_NONTEMPORAL, 0)
            _, gxa, gya = pl.eval(a, gamma, grads=True)
            pl.step(a)
            pl.iterate(a, gamma, chunk, hpwl=True, graph=graph)
            pl.set_tunable(hy.HP_TUNE_NONTEMPORAL, 1)
            assert pl.tunable(hy.HP_TUNE_NONTEMPORAL) == 1
            _, gxb, gyb = pl.eval(b, gamma, grads=True)
            pl.step(b)
            pl.iterate(b, gamma, chunk, hpwl=True, graph=graph)
            assert torch_equal(gxa, gxb) and torch_equal(gya, gyb)
            assert pl.hpwl(a)[0] == pl.hpwl(b)[0]
            xa, ya = pl.positions(a)
            xb, yb = pl.positions(b)
            assert np.array_equal(xa, xb) and np.array_equal(ya, yb), chunk
    finally:
        pl.close()


@pytest.mark.parametrize("case,prec", [("small", 32), ("tiny", 64)])
def test_charge_records_are_bit_identical(hy, orc, case, prec):
    """A rebuilt grouping's accumulation reading the counting pass's charge records, or
    gathering each cell's data itself, sums the same integers: the same maps, steps and exact
    HPWL, bit for bit (the grouping rebuilt at every evaluation, so every accumulation takes
    the path under test)."""
    nl, pl, o = setup(hy, orc, case, prec)
    gamma = 4 * nl.bin_w
    saved = pl.scatter_policy()
    pl.set_scatter_policy(1, False)
    a, b = pl.new_slot(), pl.new_slot()
    for s in (a, b):
        pl.set_positions(s, nl.x0, nl.y0)
        pl.set_schedule(s, 1e-4, 4.0, 200)
    try:
        for chunk in (1, 5, 9):
            pl.set_tunable(hy.HP_TUNE_CHARGE_RECORDS, 1)
            pl.eval(a, gamma, lam=0.5, keep_maps=True)
            ra = pl.map(a, hy.HP_MAP_RHO_MOV)
            pl.iterate(a, gamma, chunk, hpwl=True)
            pl.set_tunable(hy.HP_TUNE_CHARGE_RECORDS, 0)
            pl.eval(b, gamma, lam=0.5, keep_maps=True)
            rb = pl.map(b, hy.HP_MAP_RHO_MOV)
            pl.iterate(b, gamma, chunk, hpwl=True)
            assert np.array_equal(ra, rb)
            assert pl.hpwl(a)[0] == pl.hpwl(b)[0]
            xa, ya = pl.positions(a)
            xb, yb = pl.positions(b)
            assert np.array_equal(xa, xb) and np.array_equal(ya, yb), chunk
    finally:
        pl.set_tunable(hy.HP_TUNE_CHARGE_RECORDS, 1)
        pl.set_scatter_policy(*saved)
        pl.free_slot(a)
        pl.free_slot(b)
