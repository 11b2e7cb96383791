"""Hybro's outer loop (Alg. 1) on the device against the oracle's, and its invariants."""
import numpy as np
import pytest

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,frac", [("gauss", 0.05), ("shuffle", 0.5)])
def test_alg1_matches_oracle_fp64(orc, mode, frac):
    """Tiny netlist in FP64: every round runs the same number of placer iterations and reaches
    the same HPWL as the oracle's driver (the decisions read exact integers; the float path
    differs from the oracle's only in summation order).  The placements are capped at 120
    iterations: with lambda growing 5% a step, rounding differences grow with the horizon
    (about 6e-7 in HPWL after 400 iterations), so longer runs are checked for invariants."""
    from oracle import alg1_oracle
    from paper_2402_18311_amd import alg1, hybro
    nl = netgen.make_netlist("tiny", 0)
    pl = hybro.Placer(nl, precision=64)
    res = alg1.hybro(pl, 2, mode, frac, 8.0, seed=11, max_iters=120)
    o = orc.Oracle(nl)
    ref = alg1_oracle.hybro(o, nl, 2, alg1.MODES[mode], frac, 8.0, 11, 120)
    for t, (k, h, best) in zip(res["trace"], ref):
        print(mode, t["iters"], k, t["hpwl_q"], h)
        assert t["iters"] == k
        assert abs(t["hpwl_q"] - h) <= 1e-6 * h
        assert abs(t["best_hpwl_q"] - best) <= 1e-6 * best
    pl.close()


def test_alg1_shuffle_macros_matches_oracle_fp64(orc):
    """Hybro-Shuffle (Sec. 4.2): half of the movable macros exchange places each round; the
    device driver follows the oracle's round by round (tiny netlist with six macros, FP64)."""
    from oracle import alg1_oracle
    from paper_2402_18311_amd import alg1, hybro
    nl = netgen.make_small(1000, 1100, 64, seed=1, n_fixed=6, movable_macros=True,
                           macro_frac=0.3)
    pl = hybro.Placer(nl, precision=64)
    res = alg1.hybro(pl, 2, "shuffle-macros", 0.5, 0.0, seed=5, max_iters=120)
    o = orc.Oracle(nl)
    ref = alg1_oracle.hybro(o, nl, 2, hybro.HP_PERTURB_SHUFFLE, 0.5, 0.0, 5, 120, pool=nl.macros)
    for t, (k, h, best) in zip(res["trace"], ref):
        print(t["iters"], k, t["hpwl_q"], h)
        assert t["iters"] == k
        assert abs(t["hpwl_q"] - h) <= 1e-6 * h
        assert abs(t["best_hpwl_q"] - best) <= 1e-6 * best
    pl.close()


@pytest.mark.parametrize("mode,frac", [("shuffle", 0.5), ("gauss", 0.05)])
def test_alg1_with_fillers_matches_oracle_fp64(orc, mode, frac):
    """Filler cells at target density 0.9 on the tiny netlist in FP64: the device driver reads
    the real cells' overflow and perturbs real cells only; the oracle driver, given the
    filler-free netlist for that overflow and the real cells as the pool, takes the same
    iterations and reaches the same HPWL round by round."""
    import numpy as np
    from oracle import alg1_oracle
    from paper_2402_18311_amd import alg1, hybro
    real = netgen.make_netlist("tiny", 0)
    nl = netgen.with_fillers(real, 0.9, seed=2)
    pl = hybro.Placer(nl, precision=64, target_density=0.9)
    res = alg1.hybro(pl, 2, mode, frac, 8.0, seed=13, max_iters=200)
    o = orc.Oracle(nl)
    pool = np.arange(real.n_movable, dtype=np.int32)
    ref = alg1_oracle.hybro(o, nl, 2, alg1.MODES[mode], frac, 8.0, 13, 200, pool=pool,
                            real=(orc.Oracle(real), 0.9))
    for t, (k, h, best) in zip(res["trace"], ref):
        print(mode, t["iters"], k, t["hpwl_q"], h, round(t["overflow"], 4))
        assert t["iters"] == k
        assert abs(t["hpwl_q"] - h) <= 1e-6 * h
        assert abs(t["best_hpwl_q"] - best) <= 1e-6 * best
    pl.close()


def test_alg1_wiremask_rounds_keep_invariants():
    """Hybro-WireMask on the 20 k-cell netlist with 40 movable macros: every round starts from
    the WireMask pass over the incumbent, the best HPWL never rises and is the smallest round
    result."""
    from paper_2402_18311_amd import alg1, hybro
    nl = netgen.make_small(20_011, 21_003, 128, seed=3, n_fixed=40, movable_macros=True)
    pl = hybro.Placer(nl, precision=32)
    res = alg1.hybro(pl, 2, "wiremask", 1.0, 0.0, seed=0, max_iters=400)
    tr = res["trace"]
    bests = [t["best_hpwl_q"] for t in tr]
    assert all(b1 <= b0 for b0, b1 in zip(bests, bests[1:]))
    assert bests[-1] == min(t["hpwl_q"] for t in tr)
    print([(t["iters"], t["hpwl_q"] / 65536, t.get("kept")) for t in tr])
    pl.close()


def test_alg1_invariants_mid():
    """mid in FP32: the best HPWL never rises, equals the smallest round result, and every
    placement stops at the overflow target or the iteration cap."""
    from paper_2402_18311_amd import alg1, hybro
    nl = netgen.make_netlist("mid", 0)
    pl = hybro.Placer(nl, precision=32)
    res = alg1.hybro(pl, 2, "gauss", 0.05, 8.0, seed=3, max_iters=600)
    tr = res["trace"]
    bests = [t["best_hpwl_q"] for t in tr]
    assert all(b1 <= b0 for b0, b1 in zip(bests, bests[1:]))
    assert bests[-1] == min(t["hpwl_q"] for t in tr) == res["best_hpwl_q"]
    for t in tr:
        assert t["overflow"] <= alg1.TAU_STOP or t["iters"] == 600
    print([(t["iters"], t["hpwl_q"] / 65536, round(t["overflow"], 4)) for t in tr])
    pl.close()
