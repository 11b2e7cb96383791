"""Movable macros on the HIP path (mixed-size placement, the setting of Shuffle in Sec. 4.2).

Macros whose charge spans more than nine bins on an axis or covers eight bin areas take their
own scatter and gather (one block per cell: its bins and its pins); the others stay in the
tiled scatter.  Against the FP64 oracle:
charge maps, overflow numerators and HPWL bit for bit; wirelength and energy to 1e-5
relative and gradients to 1e-4 relative L2 in FP32 (1e-10 in FP64); perturbation among the
macros with the oracle's indices bit for bit.
"""
import numpy as np
import pytest

from paper_2402_18311_amd import netgen

from helpers import cells_only

pytestmark = pytest.mark.gpu

TOL = {32: dict(tot=1e-5, l2=1e-4), 64: dict(tot=1e-10, l2=1e-10)}


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _huge():
    """One macro covering 90% x 50% of the die (57 x 32 bins), a second one in the die's
    corner, 300 standard cells and nets touching all of them."""
    rng = np.random.default_rng(12)
    W, M, n_std = 256.0, 64, 300
    w = np.concatenate([np.full(n_std, 2.0), [230.5, 40.0]])
    h = np.concatenate([np.ones(n_std), [128.0, 36.0]])
    x = np.round(np.concatenate([rng.uniform(0, W - 2, n_std), [12.25, 214.0]]) * 256) / 256
    y = np.round(np.concatenate([rng.uniform(0, W - 1, n_std), [100.0, 219.5]]) * 256) / 256
    nets = []
    for e in range(320):
        cs = rng.choice(n_std + 2, rng.integers(2, 7), replace=False)
        nets.append([(int(c), float(np.round(rng.uniform(0, w[c]) * 256) / 256),
                      float(np.round(rng.uniform(0, h[c]) * 256) / 256)) for c in cs])
    nl = cells_only(w, h, W, W, M, x, y, nets)
    nl.macros = np.array([n_std, n_std + 1], np.int32)
    return nl


def _shuffled(nl, seed):
    """The same netlist with its movable cells renumbered at random, so that the macros sit
    among standard cells of neighbouring ids (the generator numbers them last)."""
    import dataclasses
    assert nl.n_fillers == 0
    nm = nl.n_movable
    order = np.random.default_rng(seed).permutation(nm)
    inv = np.empty(nm, np.int64)
    inv[order] = np.arange(nm)
    pc = nl.pin_cell.astype(np.int64)
    mov = pc < nm
    pc[mov] = inv[pc[mov]]
    return dataclasses.replace(
        nl, cell_w=np.concatenate([nl.cell_w[:nm][order], nl.cell_w[nm:]]),
        cell_h=np.concatenate([nl.cell_h[:nm][order], nl.cell_h[nm:]]),
        pin_cell=pc.astype(nl.pin_cell.dtype), x0=nl.x0[order], y0=nl.y0[order],
        macros=np.sort(inv[nl.macros]).astype(np.int32))


_CASES = {
    # 6 movable macros of up to 25 x 18 bins among 1000 standard cells, 64^2 bins
    "tiny_mm": lambda: netgen.make_small(1000, 1100, 64, seed=1, n_fixed=6, movable_macros=True,
                                         macro_frac=0.3),
    # 40 movable macros, 20 k cells, 128^2 bins
    "small_mm": lambda: netgen.make_small(20_011, 21_003, 128, seed=3, n_fixed=40,
                                          movable_macros=True),
    # the same with the cells renumbered: macros between standard cells of one 64-cell group
    "small_mm_shuffled": lambda: _shuffled(netgen.make_small(20_011, 21_003, 128, seed=3,
                                                             n_fixed=40, movable_macros=True), 7),
    "huge": _huge,
    # the 210 k-cell netlist with its 500 macros movable
    "mid_mm": lambda: netgen.make_netlist("mid_mm", 0),
}
_cache = {}


@pytest.fixture(scope="module")
def hy():
    from paper_2402_18311_amd import hybro
    return hybro


def setup(hy, orc, case, prec):
    key = (case, prec)
    if key not in _cache:
        nl = _CASES[case]()
        _cache[key] = (nl, hy.Placer(nl, precision=prec), orc.Oracle(nl))
    return _cache[key]


EVAL = [("tiny_mm", 64), ("tiny_mm", 32), ("small_mm", 32), ("small_mm", 64),
        ("small_mm_shuffled", 32), ("small_mm_shuffled", 64), ("huge", 64), ("huge", 32),
        ("mid_mm", 32)]


@pytest.mark.parametrize("case,prec", EVAL)
def test_macro_eval_parity(hy, orc, case, prec):
    nl, pl, o = setup(hy, orc, case, prec)
    tol = TOL[prec]
    gamma = 4 * nl.bin_w
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    assert pl.hpwl(s)[0] == o.hpwl_q(nl.x0, nl.y0)
    lam = 0.37
    (wl, en, ov), gx, gy = pl.eval(s, gamma, lam=lam, keep_maps=True, grads=True)
    ref = o.eval(nl.x0, nl.y0, gamma, maps=True)
    assert np.array_equal(pl.map(s, hy.HP_MAP_RHO_MOV), ref["rho_mov"])
    assert pl.state(s)["overflow_num"] == ref["overflow_num"]
    assert wl[0] == pytest.approx(ref["wl"], rel=tol["tot"])
    assert en[0] == pytest.approx(ref["energy"], rel=tol["tot"])
    g = np.concatenate([gx.cpu().numpy()[0], gy.cpu().numpy()[0]])
    gref = np.concatenate([ref["gwx"] + lam * ref["gdx"], ref["gwy"] + lam * ref["gdy"]])
    assert rel_l2(g, gref) < tol["l2"]
    # the macros' own density forces (large, and computed by the block-per-cell pass)
    m = nl.macros
    gd = np.concatenate([g[m] - ref["gwx"][m], g[nl.n_movable + m] - ref["gwy"][m]]) / lam
    assert rel_l2(gd, np.concatenate([ref["gdx"][m], ref["gdy"][m]])) < 10 * tol["l2"]
    pl.free_slot(s)


@pytest.mark.parametrize("case,prec", [("tiny_mm", 64), ("tiny_mm", 32), ("small_mm", 32),
                                       ("huge", 64)])
def test_macro_exact_adjoint_parity(hy, orc, case, prec):
    nl, pl, o = setup(hy, orc, case, prec)
    tol = TOL[prec]
    gamma = 4 * nl.bin_w
    s = pl.new_slot()
    x, y = nl.x0.copy(), nl.y0.copy()
    pl.set_positions(s, x, y)
    lam = 0.61
    (wl, en, ov), gx, gy = pl.eval(s, gamma, lam=lam, grads=True, grad_mode=1)
    ref = o.eval(x, y, gamma, grad_mode=1)
    assert en[0] == pytest.approx(ref["energy"], rel=tol["tot"])
    g = np.concatenate([gx.cpu().numpy()[0], gy.cpu().numpy()[0]])
    gref = np.concatenate([ref["gwx"] + lam * ref["gdx"], ref["gwy"] + lam * ref["gdy"]])
    assert rel_l2(g, gref) < tol["l2"]
    pl.free_slot(s)


@pytest.mark.parametrize("case,prec", [("tiny_mm", 64), ("small_mm", 32), ("mid_mm", 32)])
def test_macro_maps_exact_along_a_placement(hy, orc, case, prec):
    """Along a placement from the initial positions (the macros move too), the charge map and
    overflow numerator at every evaluation point stay bit-exact."""
    nl, pl, o = setup(hy, orc, case, prec)
    gamma = 4 * nl.bin_w
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, 1e-4, 4.0, 200)
    for it in range(9):
        keep = it % 3 == 2
        vx, vy = pl.eval_positions(s)
        pl.eval(s, gamma, keep_maps=keep)
        rm, rf = o.density_q(vx, vy)
        _, num = o.overflow(rm, rf)
        assert pl.state(s)["overflow_num"] == num, it
        if keep:
            assert np.array_equal(pl.map(s, hy.HP_MAP_RHO_MOV), rm), it
        pl.step(s)
    x, y = pl.positions(s)
    assert not np.array_equal(x[nl.macros], nl.x0[nl.macros])  # the macros did move
    pl.free_slot(s)


@pytest.mark.parametrize("case,prec", [("tiny_mm", 64), ("tiny_mm", 32)])
def test_macro_nesterov_steps_follow_oracle(hy, orc, case, prec):
    """lambda_0 and three [eval, step] iterations with movable macros follow the oracle."""
    nl, pl, o = setup(hy, orc, case, prec)
    gamma = 4 * nl.bin_w
    n = nl.n_movable
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, 1e-4, 4.0, 200)
    st = o.new_state(nl.x0, nl.y0)
    ratio = o.lambda_ratio(4.0, 200)
    tol = 1e-10 if prec == 64 else 2e-5
    lam = None
    for it in range(3):
        (wl, en, ov), gx, gy = pl.eval(s, gamma, grads=True)
        ref = o.eval(st["v"][:n], st["v"][n:], gamma)
        gw = np.concatenate([ref["gwx"], ref["gwy"]])
        gd = np.concatenate([ref["gdx"], ref["gdy"]])
        lam = 1e-4 * np.abs(gw).sum() / np.abs(gd).sum() if it == 0 else lam * ratio
        assert pl.state(s)["lambda_"] == pytest.approx(lam, rel=1e-12 if prec == 64 else 1e-5)
        g = np.concatenate([gx.cpu().numpy()[0], gy.cpu().numpy()[0]])
        assert rel_l2(g, gw + lam * gd) < TOL[prec]["l2"]
        pl.step(s)
        o.nesterov_step(lam, gw + lam * gd, st)
        x, y = pl.positions(s)
        u = np.concatenate([x, y]).astype(np.float64)
        assert np.max(np.abs(u - st["u"])) < tol * nl.W, it
    pl.free_slot(s)


def test_macro_fp64_placement_matches_oracle(hy, orc):
    """150 iterations of the placer in FP64 with six movable macros."""
    nl, pl, o = setup(hy, orc, "tiny_mm", 64)
    gamma = 4 * nl.bin_w
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, 1e-4, 4.0, 150)
    pl.run(s, 150, gamma)
    hq = pl.hpwl(s)[0]
    x, y, tr = o.place(nl.x0, nl.y0, 150, gamma, 1e-4, 4.0)
    ref = tr["hpwl_q"][-1]
    assert abs(hq - ref) <= 1e-6 * ref
    gx, gy = pl.positions(s)
    assert np.max(np.abs(gx - x)) < 1e-5 * nl.W and np.max(np.abs(gy - y)) < 1e-5 * nl.H
    pl.free_slot(s)


@pytest.mark.parametrize("case,prec", [("tiny_mm", 64), ("small_mm", 32)])
def test_macro_batched_slots_equal_single(hy, orc, case, prec):
    nl, pl, o = setup(hy, orc, case, prec)
    gamma = 4 * nl.bin_w
    K = 3
    ss = [pl.new_slot() for _ in range(K)]
    for k, s in enumerate(ss):
        pl.set_positions(s, *nl.random_positions(200 + k))
    pl.run(ss, 6, gamma)
    batched = [pl.positions(s) for s in ss]
    hb = pl.hpwl(ss)
    for k, s in enumerate(ss):
        pl.set_positions(s, *nl.random_positions(200 + k))
        pl.run(s, 6, gamma)
        x, y = pl.positions(s)
        assert np.array_equal(x, batched[k][0]) and np.array_equal(y, batched[k][1])
        assert pl.hpwl(s)[0] == hb[k]
    for s in ss:
        pl.free_slot(s)


@pytest.mark.parametrize("case,prec", [("tiny_mm", 64), ("small_mm", 32), ("mid_mm", 32)])
@pytest.mark.parametrize("mode,frac", [(1, 0.5), (0, 0.5), (1, 1.0)])
def test_perturb_among_macros_parity(hy, orc, case, prec, mode, frac):
    """Shuffle (Sec. 4.2): p% of the macros exchange places; indices are the oracle's."""
    nl, pl, o = setup(hy, orc, case, prec)
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    seed = 0xABCD_0123_4567_89EF + mode
    pool = nl.macros[::-1].copy()  # any order
    idx = pl.perturb(s, mode, frac, 8.0, seed, cells=pool)
    x, y = pl.positions(s)
    rx, ry, ridx = o.perturb_among(nl.x0, nl.y0, mode, frac, 8.0, seed, pool)
    assert np.array_equal(idx, ridx)
    assert len(idx) == int(np.floor(frac * len(pool) + 0.5))
    tol = 1e-9 * nl.W if prec == 64 else 4e-7 * nl.W
    assert np.max(np.abs(x - rx)) < tol and np.max(np.abs(y - ry)) < tol
    assert pl.state(s)["k"] == 0
    pl.free_slot(s)


def test_perturb_among_a_pool_of_standard_cells(hy, orc):
    nl, pl, o = setup(hy, orc, "small_mm", 32)
    s = pl.new_slot()
    x0, y0 = nl.random_positions(9)
    pl.set_positions(s, x0, y0)
    pool = np.random.default_rng(2).choice(nl.n_movable, 5003, replace=False).astype(np.int32)
    idx = pl.perturb(s, 0, 0.3, 8.0, 77, cells=pool)
    x, y = pl.positions(s)
    rx, ry, ridx = o.perturb_among(x0, y0, 0, 0.3, 8.0, 77, pool)
    assert np.array_equal(idx, ridx) and len(idx) == 1501
    assert np.max(np.abs(x - rx)) < 4e-7 * nl.W and np.max(np.abs(y - ry)) < 4e-7 * nl.W
    pl.free_slot(s)


def test_perturb_among_rejects_bad_pools(hy, orc):
    import ctypes as C
    nl, pl, o = setup(hy, orc, "tiny_mm", 64)
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    L = hy.lib()
    cnt = C.c_int32(-7)

    def call(mode, cells, n=None):
        a = None if cells is None else np.ascontiguousarray(cells, dtype=np.int32)
        n = len(a) if n is None else n
        p = None if a is None else a.ctypes.data
        return L.hp_perturb_among(pl.ctx, s, mode, 0.5, 8.0, C.c_uint64(1), p, n, None,
                                  C.byref(cnt))

    assert call(1, [0, 5, 5]) == hy.HP_EINVAL  # repeated
    assert call(1, [0, nl.n_movable]) == hy.HP_EINVAL  # not a movable cell
    assert call(1, [-1]) == hy.HP_EINVAL
    assert call(2, [0, 1]) == hy.HP_EINVAL  # uniform restart takes no pool
    assert call(1, None, 3) == hy.HP_EINVAL
    assert cnt.value == -7  # nothing was written
    x, y = pl.positions(s)
    assert np.array_equal(x, nl.x0) and np.array_equal(y, nl.y0)
    assert call(1, np.zeros(0, np.int32)) == hy.HP_OK and cnt.value == 0
    assert call(1, None, 0) == hy.HP_OK and cnt.value == 0
    pl.free_slot(s)
