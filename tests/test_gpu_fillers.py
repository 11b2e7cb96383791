"""Filler cells for a target density below 1 (ePlace): the overflow of the real cells.

Fillers are pinless movable cells after the real ones; they take part in the charge map and
its field like any cell, and the overflow of Eq. 1's density constraint counts the real cells
only (hp_overflow_of_cells).  Against the FP64 oracle on the netlist without the fillers: the
numerator bit for bit.
"""
import numpy as np
import pytest

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu

RHO_T = 0.9


@pytest.fixture(scope="module")
def hy():
    from paper_2402_18311_amd import hybro
    return hybro


_cache = {}


def setup(hy, orc, case, prec):
    key = (case, prec)
    if key not in _cache:
        real = {"small": lambda: netgen.make_small(20_011, 21_003, 128, seed=3, n_fixed=40),
                "tiny_mm": lambda: netgen.make_small(1000, 1100, 64, seed=1, n_fixed=6,
                                                     movable_macros=True, macro_frac=0.3)}[case]()
        nl = netgen.with_fillers(real, RHO_T, seed=4)
        _cache[key] = (real, nl, hy.Placer(nl, precision=prec, target_density=RHO_T),
                       orc.Oracle(real))
    return _cache[key]


@pytest.mark.parametrize("case,prec", [("small", 32), ("small", 64), ("tiny_mm", 64)])
def test_overflow_of_real_cells_parity(hy, orc, case, prec):
    real, nl, pl, o = setup(hy, orc, case, prec)
    n_real = real.n_movable
    assert nl.n_fillers > 0
    s = pl.new_slot()
    for it, (x, y) in enumerate([(nl.x0, nl.y0), nl.random_positions(8)]):
        pl.set_positions(s, x, y)
        pl.eval(s, 4 * nl.bin_w, lam=1.0, want_host=False)
        num_all, _ = pl.overflow_of_cells(s, nl.n_movable)
        assert num_all == pl.state(s)["overflow_num"], it  # the evaluation's own
        num, ov = pl.overflow_of_cells(s)
        rm, rf = o.density_q(np.asarray(x)[:n_real], np.asarray(y)[:n_real])
        ref, ref_num = o.overflow(rm, rf, RHO_T)
        assert num == ref_num, it
        assert ov == pytest.approx(ref, rel=1e-15)
        assert pl.overflow_of_cells(s, 0) == (0, 0.0)
    pl.free_slot(s)


def test_overflow_of_cells_drops_kept_maps_and_checks_range(hy, orc):
    real, nl, pl, o = setup(hy, orc, "small", 32)
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.eval(s, 4 * nl.bin_w, lam=1.0, keep_maps=True)
    pl.map(s, hy.HP_MAP_RHO_MOV)
    a = pl.overflow_of_cells(s)
    with pytest.raises(hy.HybroError):
        pl.map(s, hy.HP_MAP_RHO_MOV)
    assert pl.overflow_of_cells(s) == a  # the map was cleared before the pass, and after it
    L = hy.lib()
    for bad in (-1, nl.n_movable + 1):
        assert L.hp_overflow_of_cells(pl.ctx, s, bad, None, None) == hy.HP_EINVAL
    # the next evaluation still sees a clean map
    pl.eval(s, 4 * nl.bin_w, lam=1.0, keep_maps=True)
    rm, _ = orc.Oracle(nl).density_q(nl.x0, nl.y0)
    assert np.array_equal(pl.map(s, hy.HP_MAP_RHO_MOV), rm)
    pl.free_slot(s)


def test_fillers_let_real_cells_cluster(hy, orc):
    """600 iterations of the plain method at target density 0.9 on the 20 k-cell netlist: with
    fillers the real cells' HPWL ends lower than without (they no longer spread over the whole
    die), at a real-cell overflow below 0.2."""
    real, nl, pl, o = setup(hy, orc, "small", 32)
    out = {}
    for name, net, placer in (("fillers", nl, pl),
                              ("plain", real, hy.Placer(real, precision=32, target_density=RHO_T))):
        s = placer.new_slot()
        placer.set_positions(s, net.x0, net.y0)
        placer.set_schedule(s, 1e-4, 4.0, 600)
        placer.iterate(s, 4 * net.bin_w, 600, hpwl=True)
        out[name] = (placer.state(s)["hpwl_q"], placer.overflow_of_cells(s, real.n_movable)[1])
        placer.free_slot(s)
    print(out)
    assert out["fillers"][0] < out["plain"][0]
    assert out["fillers"][1] < 0.2
