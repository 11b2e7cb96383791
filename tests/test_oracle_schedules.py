"""Pins of the oracle's placer schedules (the "run until convergence" reading of Alg. 1 and the
lambda ramp of Eq. 2) and of its FFT path for the Poisson solve's transforms.

The schedule values are pinned at the anchor points that define the reading, not by retyping
its formulas: the smoothing gamma is 10x its 4-bin base at overflow 1 and 0.1x at overflow
0.1, log-linear in between; the penalty factor mu is 1.05 while the HPWL falls or holds, 1 when
it grows by 0.35% of itself per iteration, 1/1.05 at twice that, and never outside
[0.95, 1.05].  Each check below also runs against planted mistakes (a swapped coefficient, a
flipped sign, an off-by-one) and requires that every one of them is caught."""
import math

import numpy as np
import pytest

from oracle import alg1_oracle as A
from paper_2402_18311_amd import netgen


# ---- gamma, mu, stopping rule ----------------------------------------------------------------
def _check_gamma(gamma):
    for bw in (1.0, 2.5):
        assert gamma(1.0, bw) == pytest.approx(40.0 * bw, rel=1e-12)
        assert gamma(0.1, bw) == pytest.approx(0.4 * bw, rel=1e-12)
        # log-linear between the anchors: the midpoint overflow gives the geometric mean
        assert gamma(0.55, bw) == pytest.approx(4.0 * bw, rel=1e-12)
        # and below the lower anchor it keeps falling along the same line
        assert gamma(0.0, bw) == pytest.approx(0.4 * bw * 10 ** (-0.1 / 0.45), rel=1e-12)


def _check_mu(mu):
    H = 2_000_000.0
    assert mu(H, H) == pytest.approx(1.05, rel=1e-15)             # no change: upper clamp
    assert mu(H - 50_000, H) == pytest.approx(1.05, rel=1e-15)    # falling: upper clamp
    step = 0.0035 * H * 10                                        # 0.35% of H per iteration
    assert mu(H + step, H) == pytest.approx(1.0, rel=1e-14)
    assert mu(H + 2 * step, H) == pytest.approx(1.0 / 1.05, rel=1e-14)
    assert mu(H + 0.5 * step, H) == pytest.approx(math.sqrt(1.05), rel=1e-14)
    assert mu(H + 10 * step, H) == pytest.approx(0.95, rel=1e-15)  # lower clamp
    assert mu(123.0, 0.0) == 1.05                                  # no previous HPWL yet


def _check_stop(plateau, stop):
    assert plateau(999_000, 1_000_000)          # fell by exactly 0.1%: level
    assert not plateau(998_999, 1_000_000)      # fell by a little more: still falling
    assert plateau(1_000_500, 1_000_000)        # rose: level
    assert plateau(1_000_000, 1_000_000)
    assert stop(0.10, True) and stop(0.05, True)
    assert not stop(0.1000001, True)
    assert not stop(0.05, False)


def test_gamma_anchor_points():
    _check_gamma(A._gamma)


def test_mu_anchor_points():
    _check_mu(A._mu)


def test_stopping_rule_hand_values():
    _check_stop(A._plateau, A._stop)


def _scripted(looks):
    """A block function that returns the scripted (HPWL, overflow) looks in turn and records
    the smoothing, ratio and length of every block it is asked to run."""
    calls = []

    def block(g, ratio, n):
        calls.append((g, ratio, n))
        return looks[len(calls) - 1]
    return block, calls


def _check_loop(loop):
    H0 = 1_000_000.0
    looks = [
        (900_000.0, 0.50),   # falling fast, overflow high
        (890_000.0, 0.20),   # still falling by more than 0.1%
        (895_000.0, 0.12),   # rose (level) but overflow above 0.10: continue
        (894_900.0, 0.09),   # fell by ~0.011% (level) and overflow <= 0.10: stop here
        (0.0, 0.0),          # never reached
    ]
    block, calls = _scripted(looks)
    k, h, tau = loop(block, 1.0, H0, 1000, 1.0)
    assert (k, h, tau) == (40, 894_900.0, 0.09)
    assert [n for _, _, n in calls] == [10, 10, 10, 10]
    # the smoothing of each block follows the overflow of the look before it
    want_g = [40.0, 4.0 * 10 ** (-1 / 9), 4.0 * 10 ** (-7 / 9), 4.0 * 10 ** ((2.4 - 11) / 9)]
    assert [g for g, _, _ in calls] == pytest.approx(want_g, rel=1e-12)
    # ratio 1.05 before the first look and while the HPWL falls; after the rise of 5000 on
    # 890000 (500 per iteration, 0.056%: a sixth of the 0.35% that gives 1) it is interior
    r3 = 1.05 ** (1 - (5000 / 10) / (0.0035 * 890_000))
    assert [r for _, r, _ in calls] == pytest.approx([1.05, 1.05, 1.05, r3], rel=1e-12)
    assert 1.0 < r3 < 1.05
    # the cap ends the loop even while the rule says go on; the last block is shorter
    block, calls = _scripted([(900_000.0 - i, 0.5) for i in range(10)])
    k, _, _ = loop(block, 1.0, H0, 25, 1.0)
    assert k == 25 and [n for _, _, n in calls] == [10, 10, 5]
    # already converged at the start (no look yet, so not level): one block runs
    block, calls = _scripted([(H0, 0.05), (H0, 0.05)])
    k, _, _ = loop(block, 0.05, H0, 1000, 1.0)
    assert k == 10 and len(calls) == 1


def test_schedule_loop_on_a_scripted_trace():
    _check_loop(A.schedule_loop)


def _fails(check, *fns):
    try:
        check(*fns)
    except AssertionError:
        return True
    return False


def test_planted_schedule_mistakes_are_caught():
    """Each plausible slip in the schedule functions fails one of the pins above."""
    g_swapped = lambda tau, bw: 4.0 * bw * 10.0 ** ((9.0 / 20.0) * tau - 11.0 / 9.0)
    g_sign = lambda tau, bw: 4.0 * bw * 10.0 ** ((20.0 / 9.0) * tau + 11.0 / 9.0)
    g_base = lambda tau, bw: 8.0 * bw * 10.0 ** ((20.0 / 9.0) * tau - 11.0 / 9.0)
    for g in (g_swapped, g_sign, g_base):
        assert _fails(_check_gamma, g)

    def mu_sign(h, hp):
        return min(1.05, max(0.95, 1.05 ** (1.0 + ((h - hp) / 10) / (0.0035 * hp))))

    def mu_per_block(h, hp):  # the change over 10 iterations, not per iteration
        return min(1.05, max(0.95, 1.05 ** (1.0 - (h - hp) / (0.0035 * hp))))

    def mu_unclamped(h, hp):
        return 1.05 ** (1.0 - ((h - hp) / 10) / (0.0035 * hp)) if hp > 0 else 1.05
    for m in (mu_sign, mu_per_block, mu_unclamped):
        assert _fails(_check_mu, m)

    plateau_sign = lambda h, hp: hp - h >= -0.001 * hp
    plateau_strict = lambda h, hp: h - hp > -0.001 * hp
    stop_or = lambda tau, level: tau <= 0.10 or level
    assert _fails(_check_stop, plateau_sign, A._stop)
    assert _fails(_check_stop, plateau_strict, A._stop)
    assert _fails(_check_stop, A._plateau, stop_or)

    def loop_stale_gamma(block, tau0, h0, max_iters, bw):  # gamma from the first overflow
        tau, hp, ratio, k, level = tau0, h0, 1.05, 0, False
        g = A._gamma(tau0, bw)
        while k < max_iters and not A._stop(tau, level):
            n = min(10, max_iters - k)
            h, tau = block(g, ratio, n)
            k += n
            level, ratio, hp = A._plateau(h, hp), A._mu(h, hp), h
        return k, hp, tau

    def loop_no_cap(block, tau0, h0, max_iters, bw):  # blocks of 10 past the cap
        tau, hp, ratio, k, level = tau0, h0, 1.05, 0, False
        while k < max_iters and not A._stop(tau, level):
            h, tau = block(A._gamma(tau, bw), ratio, 10)
            k += 10
            level, ratio, hp = A._plateau(h, hp), A._mu(h, hp), h
        return k, hp, tau
    assert _fails(_check_loop, loop_stale_gamma)
    assert _fails(_check_loop, loop_no_cap)


# ---- lambda ramp of the plain placer (Eq. 2: lambda starts small and grows) -------------------
def test_place_lambda_ramp(orc):
    nl = netgen.make_netlist("tiny", 0)
    o = orc.Oracle(nl)
    g = 4 * nl.bin_w
    T = 12
    _, _, tr = o.place(nl.x0, nl.y0, T, g, 1e-4, 4.0)
    lam = tr["lam"]
    # lambda_0 = 1e-4 |grad WL|_1 / |grad N|_1 at the initial placement (one evaluation there)
    r = o.eval(nl.x0, nl.y0, g)
    l0 = 1e-4 * (np.abs(r["gwx"]).sum() + np.abs(r["gwy"]).sum()) / \
        (np.abs(r["gdx"]).sum() + np.abs(r["gdy"]).sum())
    assert lam[0] == pytest.approx(l0, rel=1e-12)
    # four decades over the run: step k uses lambda_0 10^(4 k / T), the last one 10^(4 (T-1)/T)
    k = np.arange(T)
    assert lam / lam[0] == pytest.approx(10.0 ** (4.0 * k / T), rel=1e-12)
    assert lam[-1] / lam[0] < 1e4 and lam[-1] / lam[0] > 10 ** (4.0 * (T - 1) / T) * (1 - 1e-12)


# ---- FFT path of the transforms --------------------------------------------------------------
@pytest.mark.parametrize("mx,my", [(4, 4), (8, 4), (4, 16), (16, 16)])
def test_dct_fft_matches_brute(orc, mx, my):
    rho = np.random.default_rng(mx * 31 + my).random((my, mx))
    want = orc.dct2(rho, brute=True)
    got = orc.dct2(rho, fft=True)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("mx,my", [(64, 32), (32, 128)])
def test_dct_fft_matches_sums(orc, mx, my):
    rho = np.random.default_rng(mx + my).random((my, mx))
    want = orc.dct2(rho)
    got = orc.dct2(rho, fft=True)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_single_mode_through_fft(orc):
    """A single cosine mode has exactly one coefficient (closed form), through the FFT path."""
    mx, my, u, v = 32, 16, 5, 3
    j, k = np.arange(mx) + 0.5, np.arange(my) + 0.5
    rho = np.outer(np.cos(np.pi * v * k / my), np.cos(np.pi * u * j / mx))
    a = orc.dct2(rho, fft=True)
    want = np.zeros((my, mx))
    want[v, u] = 1.0
    assert np.max(np.abs(a - want)) <= 1e-13


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_synthesis_fft_matches_definition(orc, mode):
    mx, my = 8, 4
    A = np.random.default_rng(mode).standard_normal((my, mx))
    fx = np.sin if mode == 1 else np.cos
    fy = np.sin if mode == 2 else np.cos
    want = np.zeros((my, mx))
    for k in range(my):
        for j in range(mx):
            for v in range(my):
                for u in range(mx):
                    want[k, j] += A[v, u] * fx(np.pi * u * (j + 0.5) / mx) * \
                        fy(np.pi * v * (k + 0.5) / my)
    for fft in (False, True):
        got = orc.synth2(A, mode, fft=fft)
        assert np.max(np.abs(got - want)) <= 1e-12


def test_synthesis_fft_inverts_dct(orc):
    rho = np.random.default_rng(7).random((64, 128))
    a = orc.dct2(rho, fft=True)
    back = orc.synth2(a, 0, fft=True)
    assert np.max(np.abs(back - rho)) <= 1e-12


@pytest.mark.parametrize("fd5", [False, True])
def test_poisson_fft_equals_sums(orc, fd5):
    rho = np.random.default_rng(3).random((32, 64))
    r0 = orc.poisson(rho, 96.0, 48.0, fd5=fd5)
    r1 = orc.poisson(rho, 96.0, 48.0, fd5=fd5, fft=True)
    assert r1["energy"] == pytest.approx(r0["energy"], rel=1e-12)
    for key in ("a", "psi", "ex", "ey"):
        assert np.max(np.abs(r1[key] - r0[key])) <= 1e-12 * np.max(np.abs(r0[key]))


def test_eval_fft_equals_eval(orc):
    nl = netgen.make_netlist("tiny", 1)
    o = orc.Oracle(nl)
    g = 4 * nl.bin_w
    r0 = o.eval(nl.x0, nl.y0, g)
    r1 = o.eval(nl.x0, nl.y0, g, fft=True)
    assert r1["energy"] == pytest.approx(r0["energy"], rel=1e-12)
    assert r1["overflow_num"] == r0["overflow_num"] and r1["wl"] == r0["wl"]
    gd0 = np.concatenate([r0["gdx"], r0["gdy"]])
    gd1 = np.concatenate([r1["gdx"], r1["gdy"]])
    assert np.linalg.norm(gd1 - gd0) <= 1e-12 * np.linalg.norm(gd0)
