"""The allocation-free exact HPWL (hp_hpwl_noalloc, for callers that cannot allocate device
memory) against the slot-based hp_hpwl, bit for bit (an integer result), through the C ABI: two
calls in a row on one GPU, the second on a smaller netlist, so the shared static scratch holds
the first call's partials when the second starts."""
import numpy as np
import pytest

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu


def _pairs(torch, nl, x, y, dtype):
    xy = np.empty((nl.n_cells, 2), np.float64)
    xy[:nl.n_movable, 0], xy[:nl.n_movable, 1] = x, y
    xy[nl.n_movable:, 0], xy[nl.n_movable:, 1] = nl.fixed_x, nl.fixed_y
    return torch.tensor(xy, dtype=dtype, device="cuda")


@pytest.mark.parametrize("prec", [32, 64])
def test_noalloc_hpwl_equals_slot_hpwl(prec):
    import torch
    from paper_2402_18311_amd import hybro as hy
    nets = [netgen.make_small(20_011, 21_003, 128, seed=3, n_fixed=40),  # larger first
            netgen.make_netlist("tiny", 0)]
    dtype = torch.float32 if prec == 32 else torch.float64
    for nl in nets:
        pl = hy.Placer(nl, precision=prec)
        s = pl.new_slot()
        x, y = nl.random_positions(11)
        pl.set_positions(s, x, y)
        want = int(pl.hpwl(s)[0])
        # positions exactly as the slot holds them (rounded to the compute type)
        ux, uy = pl.positions(s)
        xy = _pairs(torch, nl, ux, uy, dtype)
        out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        hy.hp_hpwl_noalloc(pl.ctx, pl.netlist, xy, out)
        torch.cuda.synchronize()
        assert int(out.item()) == want, (nl.name, int(out.item()), want)
        # a second call on the same positions after other work gives the same value
        pl.iterate(s, 4 * nl.bin_w, 3, hpwl=True)
        hy.hp_hpwl_noalloc(pl.ctx, pl.netlist, xy, out)
        torch.cuda.synchronize()
        assert int(out.item()) == want
        pl.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    from paper_2402_18311_amd import hybro as hy
    nl = netgen.make_netlist("tiny", 0)
    pl = hy.Placer(nl, precision=32)
    L = hy.lib()
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    xy = torch.zeros((nl.n_cells, 2), dtype=torch.float32, device="cuda")
    assert L.hp_hpwl_noalloc(pl.ctx, pl.netlist, None, out.data_ptr()) == hy.HP_EINVAL
    assert L.hp_hpwl_noalloc(pl.ctx, pl.netlist, xy.data_ptr() + 4, out.data_ptr()) == hy.HP_EINVAL
    assert L.hp_hpwl_noalloc(pl.ctx, 77, xy.data_ptr(), out.data_ptr()) == hy.HP_ESTATE
    pl.close()
