"""Hybro's outer loop (Alg. 1) on the FP64 oracle.

TEST INFRASTRUCTURE ONLY: used by the tests to pin the device driver.  Written from the
algorithm, not from the device driver (they share no code): place from the initial positions;
then each round perturbs the best solution (Sec. 4.2), places again and keeps the smaller exact
HPWL (Eq. 1).  The placer's schedules and stopping rule are the ePlace-style reading recorded
in the design notes:
  * stop when the overflow (the D(s) <= eps measure of Eq. 1) is at most 0.10 and the HPWL
    fell by at most 0.1% of itself over the last 10 iterations (or rose), or after max_iters
    iterations; overflow and HPWL are looked at every 10 iterations (a look happens before
    the first stop);
  * smoothing gamma = 4 bins x 10^((20/9) tau - 11/9) for the next 10 iterations, from the
    overflow tau at the last look;
  * the penalty weight lambda starts at 1e-4 |grad WL|_1 / |grad N|_1 (first evaluation) and is
    multiplied after every step by mu = min(1.05, max(0.95, 1.05^(1 - dH / (0.0035 H)))), where
    dH is the HPWL change per iteration over the last 10 and H the HPWL before them (mu = 1.05
    until the first look).
"""
from __future__ import annotations

import numpy as np


def _gamma(tau, bin_w):
    return 4.0 * bin_w * 10.0 ** ((20.0 / 9.0) * tau - 11.0 / 9.0)


def _mu(h, h_prev):
    if h_prev <= 0:
        return 1.05
    m = 1.05 ** (1.0 - ((h - h_prev) / 10) / (0.0035 * h_prev))
    return min(1.05, max(0.95, m))


def _plateau(h, h_prev):
    """The HPWL has stopped falling: it fell by at most 0.1% of its previous value, or rose."""
    return h - h_prev >= -0.001 * h_prev


def _stop(tau, level):
    """Stop once the overflow is at most 0.10 and the HPWL has stopped falling."""
    return tau <= 0.10 and level


def schedule_loop(block, tau0, h0, max_iters, bin_w):
    """The placer's control loop.  block(gamma, ratio, n) runs n placer iterations with
    smoothing gamma, multiplying lambda by ratio after every step, and returns the exact HPWL
    of the major solution and the overflow after them.  Looks happen every 10 iterations (the
    last block may be shorter, at the cap); returns (iterations, last HPWL, last overflow)."""
    tau, h_prev, ratio, k, level = tau0, h0, 1.05, 0, False
    while k < max_iters and not _stop(tau, level):
        n = min(10, max_iters - k)
        h, tau = block(_gamma(tau, bin_w), ratio, n)
        k += n
        level = _plateau(h, h_prev)
        ratio = _mu(h, h_prev)
        h_prev = h
    return k, h_prev, tau


def place_to_convergence(o, nl, x, y, max_iters, real=None):
    """Returns the final (x, y) of the major solution, iterations run, HPWL_q and overflow.
    With `real` = (oracle of the netlist without its filler cells, target density), the
    overflow the rules read is that of the real cells (the first movable cells) alone."""
    n = nl.n_movable
    st = o.new_state(x, y)

    def real_tau(r):
        if real is None:
            return r["overflow"]
        o_real, rho_t = real
        k = o_real.nl.n_movable
        rm, rf = o_real.density_q(st["v"][:k], st["v"][n:n + k])
        return o_real.overflow(rm, rf, rho_t)[0]

    lam = [None]

    def block(g, ratio, steps):
        tau = None
        for _ in range(steps):
            r = o.eval(st["v"][:n], st["v"][n:], g)
            gw = np.concatenate([r["gwx"], r["gwy"]])
            gd = np.concatenate([r["gdx"], r["gdy"]])
            if lam[0] is None:
                lam[0] = 1e-4 * np.abs(gw).sum() / np.abs(gd).sum()
            o.nesterov_step(lam[0], gw + lam[0] * gd, st)
            lam[0] *= ratio
            if real is None:
                tau = r["overflow"]
        if real is not None:  # the real cells' overflow at v, where the next evaluation is taken
            tau = real_tau(None)
        return o.hpwl_q(st["u"][:n], st["u"][n:]), tau

    tau0 = real_tau(o.eval(st["v"][:n], st["v"][n:], _gamma(1.0, nl.bin_w)))
    h0 = o.hpwl_q(st["u"][:n], st["u"][n:])
    k, h, tau = schedule_loop(block, tau0, h0, max_iters, nl.bin_w)
    return st["u"][:n].copy(), st["u"][n:].copy(), k, h, tau


def hybro(o, nl, rounds, mode, fraction, sigma_bins, seed, max_iters, pool=None, real=None):
    """Per-round trace: iterations, HPWL_q of the round's placement, best HPWL_q so far.  With
    `pool` (e.g. the movable macros, or the real cells beside fillers) the perturbation selects
    among those cells only; `real` as in place_to_convergence."""
    bx, by, k, best, tau = place_to_convergence(o, nl, nl.x0, nl.y0, max_iters, real)
    trace = [(k, best, best)]
    for r in range(rounds):
        if pool is None:
            px, py, _ = o.perturb(bx, by, mode, fraction, sigma_bins, seed + r)
        else:
            px, py, _ = o.perturb_among(bx, by, mode, fraction, sigma_bins, seed + r, pool)
        x, y, k, h, tau = place_to_convergence(o, nl, px, py, max_iters, real)
        if h < best:
            bx, by, best = x, y, h
        trace.append((k, h, best))
    return trace
