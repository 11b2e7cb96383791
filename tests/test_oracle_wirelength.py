"""Pins of the oracle's HPWL (Eq. 1) and weighted-average wirelength (Eq. 3)."""
import math

import numpy as np
import pytest

from helpers import load_json, netlist_from_dict
from paper_2402_18311_amd import netgen


@pytest.fixture(scope="module")
def hand(orc):
    d = load_json("hand_netlist.json")
    return d, orc.Oracle(netlist_from_dict(d), stretch=False)


def test_hpwl_hand_example(hand):
    d, o = hand
    x, y = np.array(d["x"]), np.array(d["y"])
    assert o.hpwl(x, y) == d["hpwl"]
    tot, per = o.hpwl_q(x, y, per_net=True)
    assert tot == int(d["hpwl"] * 65536)
    assert list(per) == [int(v * 65536) for v in d["hpwl_per_net"]]


def test_hpwl_q_translation_invariant_and_bounded(orc):
    nl = netgen.make_netlist("tiny", 3)
    o = orc.Oracle(nl)
    x, y = nl.x0, nl.y0
    h0 = o.hpwl_q(x, y)
    # pads are fixed, so translate a netlist without fixed pins: drop nets touching pads
    keep = [e for e in range(nl.n_nets)
            if np.all(nl.pin_cell[nl.net_start[e]:nl.net_start[e + 1]] < nl.n_movable)]
    pins = np.concatenate([np.arange(nl.net_start[e], nl.net_start[e + 1]) for e in keep])
    ns = np.concatenate([[0], np.cumsum([nl.net_start[e + 1] - nl.net_start[e] for e in keep])])
    sub = netgen.Netlist(**{**nl.__dict__, "net_start": ns.astype(np.int32),
                           "pin_cell": nl.pin_cell[pins], "pin_ox": nl.pin_ox[pins],
                           "pin_oy": nl.pin_oy[pins]})
    os_ = orc.Oracle(sub)
    a = os_.hpwl_q(x, y)
    assert a == os_.hpwl_q(x + 0.25, y - 3.0)  # exact shifts by multiples of 2^-16
    # quantized vs float HPWL: each pin coordinate carries <= 2^-16 of rounding error
    hf = o.hpwl(x, y)
    assert abs(h0 / 65536 - hf) <= 4 * 2.0**-16 * nl.n_nets + 1e-9 * hf


def test_wa_two_pin_closed_form(orc):
    # Eq. 3 for two pins a distance D apart is D * tanh(D / (2 gamma)).
    for D, g in [(4.0, 1.0), (0.3, 2.0), (100.0, 7.5), (1e-3, 4.0)]:
        v = orc.wa_net_axis([10.0, 10.0 + D], g, grad=False)
        assert v == pytest.approx(D * math.tanh(D / (2 * g)), rel=1e-13, abs=1e-13)  # abs: a few ulps of the coordinate 10


def test_wa_shifted_equals_literal_eq3(orc):
    rng = np.random.default_rng(0)
    for d in [2, 3, 7, 20]:
        px = rng.uniform(-3, 3, d)
        for g in [0.5, 1.0, 3.0]:
            assert orc.wa_net_axis(px, g, grad=False) == pytest.approx(
                orc.wa_literal(px, g), rel=1e-12)


def test_wa_bounds_and_limit(orc):
    # 0 <= WL <= HPWL, and HPWL - WL <= 2 (n-1) gamma / e per axis; WL -> HPWL as gamma -> 0
    rng = np.random.default_rng(1)
    for d in [2, 5, 50, 500]:
        px = rng.uniform(0, 100, d)
        hp = px.max() - px.min()
        for g in [10.0, 1.0, 0.1, 0.01]:
            v = orc.wa_net_axis(px, g, grad=False)
            assert -1e-12 <= v <= hp + 1e-12
            assert hp - v <= 2 * (d - 1) * g / math.e + 1e-9
        assert orc.wa_net_axis(px, 1e-4, grad=False) == pytest.approx(hp, rel=1e-5)


def test_wa_gradient_properties(orc):
    rng = np.random.default_rng(2)
    px = rng.uniform(0, 20, 9)
    g = 2.0
    v, dp = orc.wa_net_axis(px, g)
    assert abs(dp.sum()) < 1e-13  # translation invariance
    h = 1e-6
    for i in range(len(px)):
        e = np.zeros_like(px)
        e[i] = h
        fd = (orc.wa_net_axis(px + e, g, grad=False) - orc.wa_net_axis(px - e, g, grad=False)) / (2 * h)
        assert dp[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    # homogeneity: WL(c x; c gamma) = c WL(x; gamma)
    assert orc.wa_net_axis(3 * px, 3 * g, grad=False) == pytest.approx(3 * v, rel=1e-13)


def test_wa_total_gradient_fd_and_hpwl_limit(orc):
    nl = netgen.make_netlist("tiny", 0)
    o = orc.Oracle(nl)
    x, y = nl.x0.copy(), nl.y0.copy()
    gamma = 4 * nl.bin_w
    wl, gx, gy = o.wa(x, y, gamma)
    assert 0 < wl <= o.hpwl(x, y)
    h = 1e-5
    for i in [0, 17, 333, 999]:
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (o.wa(xp, y, gamma)[0] - o.wa(xm, y, gamma)[0]) / (2 * h)
        assert gx[i] == pytest.approx(fd, rel=1e-5, abs=1e-7)
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        fd = (o.wa(x, yp, gamma)[0] - o.wa(x, ym, gamma)[0]) / (2 * h)
        assert gy[i] == pytest.approx(fd, rel=1e-5, abs=1e-7)
    # gamma -> 0: WA tends to HPWL (bound 4 (n_e - 1) gamma / e summed over nets)
    d = nl.degrees()
    for g in [1.0, 0.1, 0.01]:
        v = o.wa(x, y, g)[0]
        assert 0 <= o.hpwl(x, y) - v <= 4 * np.sum(np.maximum(d - 1, 0)) * g / math.e + 1e-6


def test_zero_offsets_reduce_to_cell_coordinates(orc, hand):
    d, _ = hand
    d2 = dict(d, pin_ox=[0.0] * 6, pin_oy=[0.0] * 6)
    o = orc.Oracle(netlist_from_dict(d2), stretch=False)
    # Eq. 1 with cell coordinates: net0 c0(1,1), c1(4,2): 3 + 1; net1 c0, c2(2,5), pad(8,4): 7 + 4
    assert o.hpwl(np.array(d["x"]), np.array(d["y"])) == 15.0
