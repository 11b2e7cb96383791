"""Degenerate inputs through the C ABI, against the FP64 oracle: no net with two pins, the
smallest bin grid (8 x 8), nets among fixed objects only, one net over every movable cell
(the block-per-net path), one cell on some fifty nets (its pin gradients over many
batches), and pin offsets too fine for the sweep's compact offsets.  An empty placement (no movable cell) is refused at load.  Bars as in test_gpu_parity: integer outputs bit for bit; FP32 totals
to 1e-5 relative and gradients / fields to 1e-4 relative L2; FP64 to 1e-10."""
import dataclasses

import numpy as np
import pytest

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu

TOL = {32: dict(tot=1e-5, l2=1e-4), 64: dict(tot=1e-10, l2=1e-10)}


def _single_pin_nets(nl):
    """Every pin its own net: the sweep has no net to visit."""
    return dataclasses.replace(nl, net_start=np.arange(len(nl.pin_cell) + 1, dtype=np.int32))


def _with_nets(nl, nets, seed):
    """nl plus the given nets (lists of cell ids), pins at random offsets inside their cells."""
    rng = np.random.default_rng(seed)
    starts = [int(nl.net_start[-1])]
    cells, ox, oy = [], [], []
    for net in nets:
        for c in net:
            cells.append(c)
            ox.append(np.round(rng.random() * nl.cell_w[c] * 256) / 256)
            oy.append(np.round(rng.random() * nl.cell_h[c] * 256) / 256)
        starts.append(starts[-1] + len(net))
    return dataclasses.replace(
        nl, net_start=np.concatenate([nl.net_start, np.array(starts[1:], np.int32)]),
        pin_cell=np.concatenate([nl.pin_cell, np.array(cells, np.int32)]),
        pin_ox=np.concatenate([nl.pin_ox, np.array(ox)]),
        pin_oy=np.concatenate([nl.pin_oy, np.array(oy)]))


def _fixed_only_nets(nl):
    f = np.arange(nl.n_movable, nl.n_cells)
    return _with_nets(nl, [f[:2], f[2:5], f[5:13], f[::3]], seed=11)


def _one_net_over_all(nl):
    return _with_nets(nl, [np.arange(nl.n_movable)], seed=12)


def _fine_offsets(nl):
    """Pin offsets at 2^-17 steps: too fine for the sweep's compact (int16) offsets, so the
    full-width ones are read."""
    fx = np.minimum(nl.pin_ox + 2.0 ** -17, nl.cell_w[nl.pin_cell])
    return dataclasses.replace(nl, pin_ox=fx)


def _hub_cell(nl):
    """Cell 0 on 37 more two-pin nets and 4 wider ones: its pin gradients are gathered over
    many batches with a ragged last one."""
    rng = np.random.default_rng(13)
    others = rng.choice(np.arange(1, nl.n_movable), size=37 + 4 * 5, replace=False)
    nets = [[0, int(c)] for c in others[:37]]
    nets += [[0] + [int(c) for c in others[37 + 5 * k:37 + 5 * k + 5]] for k in range(4)]
    return _with_nets(nl, nets, seed=14)


CASES = {
    "single_pin_nets": lambda: _single_pin_nets(netgen.make_netlist("tiny", 0)),
    "grid_8x8": lambda: netgen.make_small(300, 320, 8, seed=5, n_fixed=4),
    "fixed_only_nets": lambda: _fixed_only_nets(netgen.make_netlist("tiny", 0)),
    "one_net_over_all": lambda: _one_net_over_all(netgen.make_netlist("tiny", 0)),
    "hub_cell": lambda: _hub_cell(netgen.make_netlist("tiny", 0)),
    "fine_offsets": lambda: _fine_offsets(netgen.make_small(3_000, 3_150, 64, seed=15, n_fixed=8)),
}


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def close(a, b, rel):
    return abs(a - b) <= rel * max(1.0, abs(b))


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("case", list(CASES))
def test_degenerate_netlists_match_oracle(orc, case, prec):
    from paper_2402_18311_amd import hybro as hy
    nl = CASES[case]()
    o = orc.Oracle(nl)
    pl = hy.Placer(nl, precision=prec)
    tol = TOL[prec]
    gamma = 4 * nl.bin_w
    s = pl.new_slot()
    try:
        pl.set_positions(s, nl.x0, nl.y0)
        assert pl.hpwl(s)[0] == o.hpwl_q(nl.x0, nl.y0)
        lam = 0.37
        (wl, en, ov), gx, gy = pl.eval(s, gamma, lam=lam, keep_maps=True, grads=True)
        ref = o.eval(nl.x0, nl.y0, gamma, maps=True)
        assert np.array_equal(pl.map(s, hy.HP_MAP_RHO_MOV), ref["rho_mov"])
        assert np.array_equal(pl.map(s, hy.HP_MAP_RHO_FIXED), ref["rho_fixed"])
        assert pl.state(s)["overflow_num"] == ref["overflow_num"]
        assert close(wl[0], ref["wl"], tol["tot"])
        assert close(en[0], ref["energy"], tol["tot"])
        for which, key in ((hy.HP_MAP_PSI, "psi"), (hy.HP_MAP_EX, "ex"), (hy.HP_MAP_EY, "ey")):
            assert rel_l2(pl.map(s, which), ref[key]) < tol["l2"], key
        g = np.concatenate([gx.cpu().numpy()[0], gy.cpu().numpy()[0]])
        gref = np.concatenate([ref["gwx"] + lam * ref["gdx"], ref["gwy"] + lam * ref["gdy"]])
        assert rel_l2(g, gref) < tol["l2"]
        if case == "hub_cell":  # the cell with the most pins, on its own
            n = nl.n_movable
            for k in (0, n):
                assert abs(g[k] - gref[k]) <= tol["l2"] * max(1.0, abs(gref[k])), (k, g[k], gref[k])
        # a few placer iterations, then the exact HPWL of the device's placement
        pl.set_schedule(s, 1e-4, 4.0, 50)
        pl.iterate(s, gamma, 7, hpwl=True)
        x, y = pl.positions(s)
        assert pl.state(s)["hpwl_q"] == o.hpwl_q(x.astype(np.float64), y.astype(np.float64))
        assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
    finally:
        pl.free_slot(s)
        pl.close()


def _bad(kind):
    nl = netgen.make_netlist("tiny", 0)
    if kind == "net_start_decreasing":
        ns = nl.net_start.copy()
        ns[5], ns[6] = ns[6], ns[5]
        return dataclasses.replace(nl, net_start=ns)
    if kind == "pin_cell_out_of_range":
        pc = nl.pin_cell.copy()
        pc[17] = nl.n_cells
        return dataclasses.replace(nl, pin_cell=pc)
    if kind == "offset_not_finite":
        ox = nl.pin_ox.copy()
        ox[3] = np.nan
        return dataclasses.replace(nl, pin_ox=ox)
    if kind == "bins_not_power_of_two":
        return dataclasses.replace(nl, mx=48)
    if kind == "die_too_large":
        return dataclasses.replace(nl, W=20000.0, H=20000.0)
    if kind == "no_movable_cells":  # every cell fixed where it starts: nothing to place
        n = nl.n_movable
        return dataclasses.replace(nl, n_movable=0, fixed_x=np.concatenate([nl.x0, nl.fixed_x]),
                                   fixed_y=np.concatenate([nl.y0, nl.fixed_y]),
                                   x0=np.zeros(0), y0=np.zeros(0)) if n else nl
    if kind == "cell_wider_than_die":
        w = nl.cell_w.copy()
        w[0] = nl.W * 2
        return dataclasses.replace(nl, cell_w=w)
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["net_start_decreasing", "pin_cell_out_of_range",
                                  "offset_not_finite", "bins_not_power_of_two", "die_too_large",
                                  "cell_wider_than_die", "no_movable_cells"])
def test_invalid_netlists_are_rejected(kind):
    """Load-time validation on the host: a bad netlist or die is refused with HP_EINVAL and a
    message, before any device work."""
    from paper_2402_18311_amd import hybro as hy
    with pytest.raises(hy.HybroError) as e:
        hy.Placer(_bad(kind), precision=32)
    assert e.value.code == hy.HP_EINVAL
    assert str(e.value)
