"""Pins of the oracle's Nesterov step, perturbation, best-of selection and placer loop."""
import math

import numpy as np
import pytest
import scipy.stats

from helpers import GOLDEN, cells_only
from paper_2402_18311_amd import netgen


def test_splitmix64_published_vector(orc):
    with open(f"{GOLDEN}/splitmix64_seed1234567.txt") as f:
        want = [int(l) for l in f if l.strip() and not l.startswith("#")]
    assert [orc.splitmix(1234567, i) for i in range(5)] == want


def _quad_setup(orc, n=50, seed=0):
    # cells without pins: the preconditioner is max(1, 0 + 0 * area) = 1 at lambda = 0
    rng = np.random.default_rng(seed)
    W = 100.0
    nl = cells_only(np.ones(n), np.ones(n), W, W, 8, rng.uniform(10, 80, n), rng.uniform(10, 80, n))
    return orc.Oracle(nl), nl, np.concatenate([rng.uniform(20, 70, n), rng.uniform(20, 70, n)])


def test_nesterov_first_step_and_bb_exact_on_quadratic(orc):
    # f = c/2 |x - t|^2: g = c (v - t).  Step 0 moves by alpha_0 = 0.1 wb / max|g| with no
    # momentum ((a_0 - 1)/a_1 = 0).  Step 1's Barzilai-Borwein length is |dv| / |dg| = 1/c,
    # so u_2 = v_1 - (1/c) c (v_1 - t) = t exactly (the textbook property of BB on a
    # quadratic with a scalar Hessian).
    o, nl, t = _quad_setup(orc)
    c = 0.37
    st = o.new_state(nl.x0, nl.y0)
    v0 = st["v"].copy()
    g = c * (st["v"] - t)
    o.nesterov_step(0.0, g, st)
    a1 = (1 + math.sqrt(5)) / 2
    alpha0 = 0.1 * nl.bin_w / np.abs(g).max()
    assert st["k"] == 1 and st["a"] == pytest.approx(a1) and st["alpha"] == pytest.approx(alpha0)
    assert np.allclose(st["u"], v0 - alpha0 * g, rtol=1e-15, atol=1e-12)
    assert np.allclose(st["v"], st["u"])  # no momentum on the first step
    assert np.array_equal(st["v_prev"], v0) and np.allclose(st["gp_prev"], g)
    u1 = st["u"].copy()
    g = c * (st["v"] - t)
    o.nesterov_step(0.0, g, st)
    assert st["alpha"] == pytest.approx(1 / c, rel=1e-12)
    assert np.allclose(st["u"], t, atol=1e-10)
    a2 = (1 + math.sqrt(4 * a1 * a1 + 1)) / 2
    assert np.allclose(st["v"], t + (a1 - 1) / a2 * (t - u1), atol=1e-10)


def test_nesterov_preconditioner_and_clamp(orc):
    # a cell with 3 pins and area 2: P = max(1, 3 + lambda * 2); at lambda = 1, P = 5
    nl = cells_only([2.0, 1.0], [1.0, 1.0], 16.0, 16.0, 4, [5.0, 1.0], [5.0, 0.5],
                    nets=[[(0, 0, 0), (1, 0, 0)], [(0, 1, 0), (1, 0, 0)], [(0, 0, 0), (1, 0, 0)]])
    o = orc.Oracle(nl)
    st = o.new_state(nl.x0, nl.y0)
    g = np.array([10.0, 2.0, 5.0, 40.0])  # gx0, gx1, gy0, gy1
    o.nesterov_step(1.0, g, st)
    gt = g / np.array([5.0, 4.0, 5.0, 4.0])  # cell 1: 3 pins + 1 * area 1
    alpha = 0.1 * 4.0 / np.abs(gt).max()
    assert st["alpha"] == pytest.approx(alpha)
    want = np.array([5.0, 1.0, 5.0, 0.5]) - alpha * gt
    want = np.clip(want, 0, [14.0, 15.0, 15.0, 15.0])
    assert np.allclose(st["u"], want)
    # near the walls, the first step (0.1 bin = 0.4 here) is clamped into the die
    st = o.new_state(np.array([13.9, 0.1]), np.array([14.8, 0.2]))
    o.nesterov_step(0.0, np.array([-1.0, 1.0, -1.0, 1.0]), st)
    assert np.array_equal(st["u"], [14.0, 0.0, 15.0, 0.0])
    assert np.array_equal(st["v"], [14.0, 0.0, 15.0, 0.0])


@pytest.fixture(scope="module")
def tiny(orc):
    nl = netgen.make_netlist("tiny", 0)
    return nl, orc.Oracle(nl)


def test_perturb_selection_is_m_smallest_keys(orc, tiny):
    nl, o = tiny
    for frac, seed in [(0.5, 7), (0.05, 123), (0.0, 1), (1.0, 2), (0.3333, 2**63 + 5)]:
        x, y, idx = o.perturb(nl.x0, nl.y0, orc.GAUSS, frac, 8.0, seed)
        m = int(math.floor(frac * nl.n_movable + 0.5))
        keys = np.array([orc.splitmix(seed, i) for i in range(nl.n_movable)], dtype=np.uint64)
        order = np.lexsort((np.arange(nl.n_movable), keys))  # by key, then index
        assert len(idx) == m
        assert np.array_equal(idx, np.sort(order[:m]))
        moved = (x != nl.x0) | (y != nl.y0)
        assert not moved[np.setdiff1d(np.arange(nl.n_movable), idx)].any()
    # deterministic by seed, different across seeds
    a = o.perturb(nl.x0, nl.y0, orc.GAUSS, 0.5, 8.0, 9)
    b = o.perturb(nl.x0, nl.y0, orc.GAUSS, 0.5, 8.0, 9)
    c = o.perturb(nl.x0, nl.y0, orc.GAUSS, 0.5, 8.0, 10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
    assert not np.array_equal(a[2], c[2])


def test_perturb_among_selects_within_the_pool(orc, tiny):
    """Shuffle of Sec. 4.2 selects p% of the macros only: the round(p * |pool|) pool cells with
    the smallest (draw >> 1, id), found here by brute force; nothing outside the pool moves, and
    the pool's order does not matter."""
    nl, o = tiny
    rng = np.random.default_rng(4)
    pool = rng.choice(nl.n_movable, 137, replace=False).astype(np.int32)
    for mode, frac, seed in [(orc.GAUSS, 0.5, 3), (orc.SHUFFLE, 0.5, 8), (orc.GAUSS, 0.1, 2**64 - 1),
                             (orc.SHUFFLE, 1.0, 5)]:
        x, y, idx = o.perturb_among(nl.x0, nl.y0, mode, frac, 8.0, seed, pool)
        m = int(math.floor(frac * len(pool) + 0.5))
        keys = np.array([orc.splitmix(seed, int(c)) >> 1 for c in pool], dtype=np.uint64)
        order = np.lexsort((pool, keys))
        assert np.array_equal(idx, np.sort(pool[order[:m]]))
        moved = (x != nl.x0) | (y != nl.y0)
        assert not moved[np.setdiff1d(np.arange(nl.n_movable), idx)].any()
        x2, y2, idx2 = o.perturb_among(nl.x0, nl.y0, mode, frac, 8.0, seed, pool[::-1].copy())
        assert np.array_equal(idx2, idx) and np.array_equal(x2, x) and np.array_equal(y2, y)
    x, y, idx = o.perturb_among(nl.x0, nl.y0, orc.SHUFFLE, 0.5, 0.0, 1, np.zeros(0, np.int32))
    assert len(idx) == 0 and np.array_equal(x, nl.x0) and np.array_equal(y, nl.y0)


def test_shuffle_among_macros_keeps_their_places(orc):
    """Shuffling equal macros among themselves permutes their places exactly; the standard
    cells stay where they are."""
    n_std, n_mac = 300, 40
    W = 400.0
    rng = np.random.default_rng(6)
    w = np.concatenate([np.full(n_std, 2.0), np.full(n_mac, 24.0)])
    h = np.concatenate([np.ones(n_std), np.full(n_mac, 16.0)])
    x = np.round(rng.uniform(0, W - w) * 256) / 256
    y = np.round(rng.uniform(0, W - h) * 256) / 256
    nl = cells_only(w, h, W, W, 64, x, y)
    o = orc.Oracle(nl)
    macros = np.arange(n_std, n_std + n_mac, dtype=np.int32)
    nx, ny, idx = o.perturb_among(nl.x0, nl.y0, orc.SHUFFLE, 0.5, 0.0, 21, macros)
    assert len(idx) == 20 and np.all(idx >= n_std)
    assert sorted(zip(nx[idx], ny[idx])) == sorted(zip(x[idx], y[idx]))
    assert np.array_equal(nx[:n_std], x[:n_std]) and np.array_equal(ny[:n_std], y[:n_std])


def test_gauss_displacements_are_normal(orc):
    n = 100_000
    W = 1e6
    nl = cells_only(np.ones(n), np.ones(n), W, W, 1024, np.full(n, W / 2), np.full(n, W / 2))
    o = orc.Oracle(nl)
    x, y, idx = o.perturb(nl.x0, nl.y0, orc.GAUSS, 1.0, 8.0, 42)
    sigma = 8.0 * nl.bin_w
    for d in ((x - nl.x0) / sigma, (y - nl.y0) / sigma):
        assert scipy.stats.kstest(d, "norm").pvalue > 0.01
    r = np.corrcoef((x - nl.x0), (y - nl.y0))[0, 1]
    assert abs(r) < 0.02


def test_shuffle_permutes_centres(orc):
    for m in [1, 2, 3, 5, 100, 1000, 4097]:
        p = [orc.shuffle_perm(j, m, 77) for j in range(m)]
        assert sorted(p) == list(range(m))
    n = 2000
    rng = np.random.default_rng(3)
    W = 200.0
    snap = lambda v: np.round(v * 256) / 256  # centre +- w/2 is then exact
    nl = cells_only(np.full(n, 2.0), np.ones(n), W, W, 64, snap(rng.uniform(0, W - 2, n)),
                    snap(rng.uniform(0, W - 1, n)))
    o = orc.Oracle(nl)
    x, y, idx = o.perturb(nl.x0, nl.y0, orc.SHUFFLE, 0.5, 0.0, 11)
    assert len(idx) == 1000
    before = sorted(zip(nl.x0[idx], nl.y0[idx]))
    after = sorted(zip(x[idx], y[idx]))
    assert before == after  # equal widths: the multiset of locations is preserved exactly
    assert np.mean(x[idx] != nl.x0[idx]) > 0.99
    rest = np.setdiff1d(np.arange(n), idx)
    assert np.array_equal(x[rest], nl.x0[rest])


def test_uniform_restart_covers_die(orc, tiny):
    nl, o = tiny
    x, y, idx = o.perturb(nl.x0, nl.y0, orc.UNIFORM, 0.0, 0.0, 5)
    assert len(idx) == nl.n_movable
    w = nl.cell_w[: nl.n_movable]
    assert np.all(x >= 0) and np.all(x <= nl.W - w)
    assert scipy.stats.kstest(x / (nl.W - w), "uniform").pvalue > 0.01


def test_argmin_ties_to_lowest(orc):
    assert orc.argmin_i64([5, 3, 3, 9]) == 1
    assert orc.argmin_i64([2]) == 0
    v = np.random.default_rng(0).integers(0, 5, 100)
    assert orc.argmin_i64(v) == int(np.argmin(v))


def test_placer_reduces_hpwl_and_spreads(orc, tiny):
    nl, o = tiny
    x, y, tr = o.place(nl.x0, nl.y0, 200, 4 * nl.bin_w, 1e-4, 4.0)
    h0 = o.hpwl_q(nl.x0, nl.y0)
    assert tr["hpwl_q"][-1] == o.hpwl_q(x, y)
    assert tr["hpwl_q"][-1] < 0.4 * h0
    assert tr["overflow"][-1] <= 0.10  # the density constraint D(s) <= eps of Eq. 1
    w = nl.cell_w[: nl.n_movable]
    assert np.all(x >= 0) and np.all(x <= nl.W - w)


def _quadratic(n, seed, W=1e6):
    """n pinless cells in the middle of a huge die (no clamping; preconditioner 1 at lambda 0)
    and the gradient of f(x) = 1/2 sum c_i (x_i - t_i)^2 over both axes."""
    rng = np.random.default_rng(seed)
    x = W / 2 + rng.uniform(-50, 50, n)
    y = W / 2 + rng.uniform(-50, 50, n)
    nl = cells_only(np.ones(n), np.ones(n), W, W, 64, x, y)
    t = np.concatenate([x, y]) + rng.uniform(-20, 20, 2 * n)
    return nl, t


def test_backtracking_step_equals_plain_step_without_rejections(orc):
    """On a linear objective (a constant gradient) the gradient difference is zero, the step
    length stays the first one, no step is rejected, and the backtracking method is the plain
    one, bit for bit."""
    nl, _ = _quadratic(40, 1)
    o = orc.Oracle(nl)
    g = np.random.default_rng(5).uniform(-1, 1, 2 * nl.n_movable)
    a = o.new_state(nl.x0, nl.y0)
    b = o.new_state(nl.x0, nl.y0)
    for _ in range(10):
        o.nesterov_step(0.0, g, a)
        assert not o.nesterov_step_bt(0.0, g, b)
        for key in ("u", "v", "v_prev", "gp_prev"):
            assert np.array_equal(a[key], b[key])
        assert (a["k"], a["a"], a["alpha"]) == (b["k"], b["a"], b["alpha"])


def test_backtracking_redoes_the_last_step_shorter(orc):
    """A curvature that jumps after a step makes the prediction at the reached point shorter
    than the step that reached it: the step is redone from its own start along the same
    direction, scaled by the ratio of the two lengths, and nothing else of the state moves."""
    nl, t = _quadratic(30, 2)
    o = orc.Oracle(nl)
    st = o.new_state(nl.x0, nl.y0)
    c = np.random.default_rng(7).uniform(0.02, 0.05, 2 * nl.n_movable)
    rejected = [o.nesterov_step_bt(0.0, c * (st["v"] - t), st) for _ in range(6)]
    while rejected[-1]:  # end on an accepted step with some momentum
        rejected.append(o.nesterov_step_bt(0.0, c * (st["v"] - t), st))
    assert st["k"] >= 4
    before = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    c2 = 8.0 * c  # stiffer: the reached point predicts a much shorter step
    assert o.nesterov_step_bt(0.0, c2 * (st["v"] - t), st)
    assert st["alpha"] < 0.95 * before["alpha"]
    for key in ("v_prev", "gp_prev", "u_prev"):
        assert np.array_equal(st[key], before[key])
    assert (st["k"], st["a"], st["a_prev"]) == (before["k"], before["a"], before["a_prev"])
    # the redo moves from the step's start along the same direction, shorter by alpha'/alpha
    d_old = before["u"] - before["v_prev"]
    d_new = st["u"] - before["v_prev"]
    np.testing.assert_allclose(d_new, d_old * (st["alpha"] / before["alpha"]), rtol=1e-9,
                               atol=1e-9)
    # and the momentum term is the one of that step: v - u is parallel to u - u_prev
    m_old = before["v"] - before["u"]
    m_new = st["v"] - st["u"]
    ratio_u = (st["u"] - before["u_prev"]) / (before["u"] - before["u_prev"])
    np.testing.assert_allclose(m_new, m_old * ratio_u, rtol=1e-6, atol=1e-8)  # 5e5 coordinates


def test_backtracking_first_redo_has_no_momentum(orc):
    """Redoing the very first step (a_prev = 1) leaves no momentum: v = u."""
    nl, t = _quadratic(20, 3)
    o = orc.Oracle(nl)
    st = o.new_state(nl.x0, nl.y0)
    assert not o.nesterov_step_bt(0.0, 0.2 * (st["v"] - t), st)
    u1 = st["u"].copy()
    assert o.nesterov_step_bt(0.0, 50.0 * (st["v"] - t), st)
    assert np.array_equal(st["u"], st["v"]) and st["k"] == 1
    np.testing.assert_allclose(st["u"] - st["v_prev"],
                               (u1 - st["v_prev"]) * st["alpha"] / (0.1 * nl.bin_w / np.max(
                                   np.abs(0.2 * (np.concatenate([nl.x0, nl.y0]) - t)))),
                               rtol=1e-9, atol=1e-9)


@pytest.fixture(scope="module")
def mm(orc):
    nl = netgen.make_small(1000, 1100, 64, seed=1, n_fixed=6, movable_macros=True, macro_frac=0.3)
    return nl, orc.Oracle(nl)


def test_wiremask_single_macro_is_brute_force_hpwl_argmin(orc, mm):
    """One macro alone: its new place is the bin-corner position that minimises the whole
    netlist's exact HPWL (Eq. 1), found by evaluating the HPWL at every candidate, ties to the
    smaller displacement and then the lower index."""
    nl, o = mm
    x0, y0 = nl.random_positions(3)
    for m in nl.macros[:3]:
        x, y, moved = o.wiremask(x0, y0, [m])
        bw, bh = nl.bin_w, nl.bin_h
        w, h = nl.cell_w[m], nl.cell_h[m]
        nci = int((round(nl.W * 65536) - round(w * 65536)) // round(bw * 65536)) + 1
        ncj = int((round(nl.H * 65536) - round(h * 65536)) // round(bh * 65536)) + 1
        best = None
        tx, ty = x0.copy(), y0.copy()
        for j in range(ncj):
            for i in range(nci):
                tx[m], ty[m] = i * bw, j * bh
                key = (o.hpwl_q(tx, ty), abs(round(i * bw * 65536) - round(x0[m] * 65536)) +
                       abs(round(j * bh * 65536) - round(y0[m] * 65536)), j * nci + i)
                best = key if best is None or key < best else best
        idx = best[2]
        assert (x[m], y[m]) == ((idx % nci) * bw, (idx // nci) * bh)
        assert moved == int((x[m], y[m]) != (x0[m], y0[m]))
        others = np.arange(nl.n_movable) != m
        assert np.array_equal(x[others], x0[others]) and np.array_equal(y[others], y0[others])


def test_wiremask_leaves_listed_macros_apart(orc, mm):
    """All six macros in turn: none overlaps another afterwards (free places exist), every new
    place is a bin corner inside the die, and the HPWL changes only through the macros."""
    nl, o = mm
    x0, y0 = nl.random_positions(5)
    x, y, moved = o.wiremask(x0, y0, nl.macros)
    assert moved > 0
    ms = nl.macros
    for a in ms:
        assert x[a] + nl.cell_w[a] <= nl.W and y[a] + nl.cell_h[a] <= nl.H
        assert abs(x[a] / nl.bin_w - round(x[a] / nl.bin_w)) < 1e-12
        for b in ms:
            if a < b:
                assert not (x[a] < x[b] + nl.cell_w[b] and x[b] < x[a] + nl.cell_w[a] and
                            y[a] < y[b] + nl.cell_h[b] and y[b] < y[a] + nl.cell_h[a]), (a, b)
    rest = np.setdiff1d(np.arange(nl.n_movable), ms)
    assert np.array_equal(x[rest], x0[rest])


def test_wiremask_macro_without_room_stays(orc):
    """Two listed 40 x 60 macros on a 64 x 64 die: wherever one goes it overlaps the other, so
    neither has a free candidate and both stay."""
    W = 64.0
    nl = cells_only([40.0, 40.0, 1.0], [60.0, 60.0, 1.0], W, W, 16, [0.0, 20.0, 30.0],
                    [0.0, 2.0, 30.0], nets=[[(0, 1.0, 1.0), (2, 0.5, 0.5)],
                                            [(1, 2.0, 2.0), (2, 0.5, 0.5)]])
    o = orc.Oracle(nl)
    x, y, moved = o.wiremask(nl.x0, nl.y0, [0, 1])
    assert moved == 0 and np.array_equal(x, nl.x0) and np.array_equal(y, nl.y0)
    # with the second macro out of the list it is no obstacle, and the first one moves
    x, y, moved = o.wiremask(nl.x0, nl.y0, [0])
    assert moved == 1 and (x[0], y[0]) != (0.0, 0.0)
