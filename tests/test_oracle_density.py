"""Pins of the oracle's density map, overflow, Poisson solve and density gradient
(the D term of Eqs. 1-2 under the ePlace electrostatic reading)."""
import math

import numpy as np
import pytest
import scipy.fft

from helpers import cells_only, load_json, netlist_from_dict
from paper_2402_18311_amd import netgen

U40 = 2**40  # one unit of area in the integer map


def test_density_hand_cases(orc):
    d = load_json("hand_netlist.json")
    o = orc.Oracle(netlist_from_dict(d), stretch=False)
    rm, rf = o.density_q(np.array(d["x"]), np.array(d["y"]))
    want = np.zeros((4, 4), np.int64)
    for key, v in d["rho_mov_nostretch"].items():
        k, j = map(int, key.split(","))
        want[k, j] = v
    assert np.array_equal(rm, want)
    assert not rf.any()  # the only fixed object is a zero-area pad
    # straddling: c1 at (3, 2.5) covers x [3,5) -> bins 1 and 2, one unit each, y in bin 1
    rm, _ = o.density_q(np.array([1.0, 3.0, 2.0]), np.array([1.0, 2.5, 5.0]))
    assert rm[1, 1] == U40 and rm[1, 2] == U40
    # clipped at the die edge: c2 at (7.5, 7.5) keeps only a 0.5 x 0.5 corner
    rm, _ = o.density_q(np.array([1.0, 4.0, 7.5]), np.array([1.0, 2.0, 7.5]))
    assert rm[3, 3] == U40 // 4


def test_density_stretched_single_cell(orc):
    # a 1x1 cell on 2x2 bins is stretched to 2 sqrt(2) on each side, charge scaled by 1/8
    nl = cells_only([1.0], [1.0], 8.0, 8.0, 4, [1.0], [1.0])
    o = orc.Oracle(nl)
    rm, _ = o.density_q(nl.x0, nl.y0)
    ws = math.sqrt(2) * 2.0
    wq = round(ws * 4096)
    lo = 4096 + round((1.0 - ws) / 2 * 4096)
    o0, o1 = 8192 - lo, lo + wq - 8192
    r = round(65536 / 8)
    assert rm[0, 0] == r * o0 * o0 and rm[0, 1] == r * o1 * o0 and rm[1, 1] == r * o1 * o1
    assert rm.sum() == o.total_charge_q() == r * wq * wq
    assert abs(rm.sum() / U40 - 1.0) < 2**-12  # the charge equals the cell area


def test_density_sum_equals_area_and_permutation_invariance(orc):
    nl = netgen.make_netlist("tiny", 1)
    o = orc.Oracle(nl)
    w, h = nl.cell_w[:1000], nl.cell_h[:1000]
    m = 2 * nl.bin_w  # keep every stretched rectangle inside the die
    rng = np.random.default_rng(5)
    x = rng.uniform(m, nl.W - w - m)
    y = rng.uniform(m, nl.H - h - m)
    rm, _ = o.density_q(x, y)
    assert rm.sum() == o.total_charge_q()
    assert abs(rm.sum() / U40 - np.sum(w * h)) <= 1000 * 2.0**-10
    perm = rng.permutation(1000)
    nl2 = cells_only(w[perm], h[perm], nl.W, nl.H, nl.mx, x[perm], y[perm])
    rm2, _ = orc.Oracle(nl2).density_q(nl2.x0, nl2.y0)
    assert np.array_equal(rm, rm2)


def test_density_matches_continuous_map(orc):
    small = netgen.make_small(3000, 3100, 32, seed=2)
    o = orc.Oracle(small)
    rm, rf = o.density_q(small.x0, small.y0)
    cont = o.density_float(small.x0, small.y0)
    err = np.abs((rm + rf) / U40 - cont)
    # each rectangle edge moves by <= 2^-13, so each cell's charge in a bin moves by a bit more
    # than its perimeter share of 2^-12; a loose per-bin bound:
    assert err.max() < 1e-2 and err.sum() / cont.sum() < 1e-4


def test_fixed_macros_map(orc):
    nl = netgen.make_small(2000, 2100, 32, seed=4, n_fixed=6)
    o = orc.Oracle(nl)
    _, rf = o.density_q(nl.x0, nl.y0)
    area = np.sum(nl.cell_w[nl.n_movable:] * nl.cell_h[nl.n_movable:])
    # macros are placed inside the die on a 2^-8 grid, so their map is exact
    assert rf.sum() == round(area * U40)
    assert rf.max() <= round(nl.bin_w * nl.bin_h * U40)  # no overlap between macros


def test_overflow_hand_case(orc):
    # five 1x1 cells stacked in one 2x2 bin (area 4): one unit of area over capacity
    nl = cells_only([1.0] * 5, [1.0] * 5, 8.0, 8.0, 4, [0.5] * 5, [0.5] * 5)
    o = orc.Oracle(nl, stretch=False)
    rm, rf = o.density_q(nl.x0, nl.y0)
    v, num = o.overflow(rm, rf, 1.0)
    assert num == U40 and v == pytest.approx(0.2, rel=1e-15)
    v, num = o.overflow(rm, rf, 0.5)  # capacity 2: three units over
    assert num == 3 * U40
    # spread out: no overflow
    nl = cells_only([1.0] * 5, [1.0] * 5, 8.0, 8.0, 4, [0.5, 2.5, 4.5, 6.5, 0.5],
                    [0.5, 0.5, 0.5, 0.5, 2.5])
    o = orc.Oracle(nl, stretch=False)
    assert o.overflow(*o.density_q(nl.x0, nl.y0), 1.0)[1] == 0


# ---- spectral Poisson solve ----------------------------------------------------------------

@pytest.mark.parametrize("mx,my", [(4, 4), (8, 8), (16, 8), (8, 16)])
def test_dct_brute_vs_separable(orc, mx, my):
    rho = np.random.default_rng(mx * 10 + my).random((my, mx))
    assert np.allclose(orc.dct2(rho, brute=True), orc.dct2(rho), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("M", [8, 64, 256])
def test_dct_matches_scipy(orc, M):
    rho = np.random.default_rng(M).random((M, M))
    a = orc.dct2(rho)
    ref = scipy.fft.dctn(rho, type=2)  # 4 * sum cos cos per the type-II definition
    c = np.where(np.arange(M) == 0, 1.0, 2.0)
    ref = ref * np.outer(c, c) / (4.0 * M * M)
    assert np.allclose(a, ref, rtol=1e-10, atol=1e-13)


def test_dct_inverts(orc):
    # rho = sum a_uv cos cos with the chosen normalization
    M = 16
    rho = np.random.default_rng(3).random((M, M))
    a = orc.dct2(rho)
    j = np.arange(M)
    C = np.cos(np.pi * np.outer(np.arange(M), j + 0.5) / M)  # C[u, j]
    back = C.T @ a @ C  # back[k, j] = sum_v sum_u C[v,k] a[v,u] C[u,j]
    assert np.allclose(back, rho, atol=1e-12)


def test_single_cosine_mode_closed_form(orc):
    M, W = 32, 64.0
    u0, v0 = 3, 5
    j = np.arange(M) + 0.5
    rho = np.outer(np.cos(np.pi * v0 * j / M), np.cos(np.pi * u0 * j / M))  # [k, j]
    r = orc.poisson(rho, W, W)
    wu, wv = np.pi * u0 / W, np.pi * v0 / W
    den = wu**2 + wv**2
    assert np.allclose(r["psi"], rho / den, atol=1e-12)
    ex = np.outer(np.cos(np.pi * v0 * j / M), np.sin(np.pi * u0 * j / M)) * wu / den
    ey = np.outer(np.sin(np.pi * v0 * j / M), np.cos(np.pi * u0 * j / M)) * wv / den
    assert np.allclose(r["ex"], ex, atol=1e-12) and np.allclose(r["ey"], ey, atol=1e-12)
    wb = W / M
    assert r["energy"] == pytest.approx(0.5 * wb * wb * np.sum(rho * r["psi"]), rel=1e-12)


def test_energy_parseval_and_field_is_minus_grad_psi(orc):
    M, W = 64, 100.0
    rho = np.random.default_rng(9).random((M, M)) * 2
    r = orc.poisson(rho, W, W)
    wb = W / M
    assert r["energy"] == pytest.approx(0.5 * wb * wb * np.sum(rho * r["psi"]), rel=1e-11)
    assert r["energy"] > 0
    assert abs(r["psi"].mean()) < 1e-12 * np.abs(r["psi"]).max()  # DC dropped
    # the field is the exact derivative of the cosine series of psi; compare to the central
    # difference of psi on interior bins (second-order accurate for this smooth sum)
    smooth = np.outer(np.cos(np.pi * 2 * (np.arange(M) + .5) / M),
                      np.cos(np.pi * 1 * (np.arange(M) + .5) / M)) + 1.0
    r = orc.poisson(smooth, W, W)
    dpsi = (r["psi"][:, 2:] - r["psi"][:, :-2]) / (2 * wb)
    assert np.allclose(-dpsi, r["ex"][:, 1:-1], rtol=2e-3, atol=1e-3 * np.abs(r["ex"]).max())


def test_fd5_satisfies_discrete_poisson(orc):
    # with the 5-point eigenvalues, -lap_h psi = rho - mean on the bin grid, Neumann walls
    M, W = 32, 40.0
    rho = np.random.default_rng(4).random((M, M))
    r = orc.poisson(rho, W, W, fd5=True)
    p = np.pad(r["psi"], 1, mode="edge")  # reflecting (Neumann) boundary
    h = W / M
    lap = (p[1:-1, 2:] + p[1:-1, :-2] + p[2:, 1:-1] + p[:-2, 1:-1] - 4 * p[1:-1, 1:-1]) / h**2
    assert np.allclose(-lap, rho - rho.mean(), atol=1e-11)


# ---- density gradient ----------------------------------------------------------------------

def _fd_setup(orc, M, seed=0, n=40):
    W = 32.0
    rng = np.random.default_rng(seed)
    w = np.round(rng.uniform(1, 4, n) * 256) / 256
    h = np.ones(n)
    x = rng.uniform(1.5, W - 5.5, n)
    y = rng.uniform(1.5, W - 2.5, n)
    nl = cells_only(w, h, W, W, M, x, y)
    return orc.Oracle(nl), x, y


@pytest.mark.parametrize("M", [16, 32])
def test_exact_density_gradient_matches_fd(orc, M):
    o, x, y = _fd_setup(orc, M)
    wb = 32.0 / M
    rho = o.density_float(x, y) / (wb * wb)
    psi = orc.poisson(rho, 32.0, 32.0)["psi"]
    gx, gy = o.grad_exact(x, y, psi)
    h = 1e-6
    fdx, fdy = np.zeros_like(gx), np.zeros_like(gy)
    for i in range(len(x)):
        for arr, out in ((x, fdx), (y, fdy)):
            a = arr.copy()
            a[i] += h
            ep = o.energy_float(a, y) if arr is x else o.energy_float(x, a)
            a[i] -= 2 * h
            em = o.energy_float(a, y) if arr is x else o.energy_float(x, a)
            out[i] = (ep - em) / (2 * h)
    g = np.concatenate([gx, gy])
    fd = np.concatenate([fdx, fdy])
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-6


def test_field_gradient_converges_to_exact(orc):
    errs, coss = [], []
    for M in (16, 32, 64, 128):
        o, x, y = _fd_setup(orc, M, seed=0, n=60)
        wb = 32.0 / M
        out = o.eval(x, y, 1.0, maps=True)
        rho = o.density_float(x, y) / (wb * wb)
        psi = orc.poisson(rho, 32.0, 32.0)["psi"]
        ex_, ey_ = o.grad_exact(x, y, psi)
        f = np.concatenate([out["gdx"], out["gdy"]])
        e = np.concatenate([ex_, ey_])
        errs.append(np.linalg.norm(f - e) / np.linalg.norm(e))
        coss.append(f @ e / np.linalg.norm(f) / np.linalg.norm(e))
    # the field force is the exact derivative only in the limit of small bins: the error
    # falls with every halving of the bin and the direction converges
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[0] / errs[3] > 2.5
    assert coss[3] > 0.99


def test_field_gradient_descends_energy(orc):
    nl = netgen.make_small(2000, 2100, 32, seed=6)
    o = orc.Oracle(nl)
    out = o.eval(nl.x0, nl.y0, 4 * nl.bin_w)
    step = 0.2 * nl.bin_w / np.abs(np.concatenate([out["gdx"], out["gdy"]])).max()
    out2 = o.eval(nl.x0 - step * out["gdx"], nl.y0 - step * out["gdy"], 4 * nl.bin_w)
    assert out2["energy"] < out["energy"]


def test_oracle_inputs_of_any_float_dtype(orc):
    """Marshalling: positions given as float32 (values exact in both types) produce the same
    results as float64 ones, i.e. the converted copies outlive the C call."""
    from paper_2402_18311_amd import netgen
    nl = netgen.make_small(3_001, 3_100, 32, seed=5, n_fixed=8)
    o = orc.Oracle(nl)
    x64, y64 = nl.random_positions(2)
    x32, y32 = x64.astype(np.float32), y64.astype(np.float32)
    assert np.array_equal(x32.astype(np.float64), x64)  # generator values are multiples of 2^-8
    for _ in range(3):  # fresh temporaries each time, so freed memory would be reused
        assert o.hpwl_q(x32, y32) == o.hpwl_q(x64, y64)
        r32, f32 = o.density_q(x32, y32)
        r64, f64 = o.density_q(x64, y64)
        assert np.array_equal(r32, r64) and np.array_equal(f32, f64)
        e32 = o.eval(x32, y32, 4 * nl.bin_w)
        e64 = o.eval(x64, y64, 4 * nl.bin_w)
        assert e32["overflow_num"] == e64["overflow_num"] and e32["wl"] == e64["wl"]
