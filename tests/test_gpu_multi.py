"""Shared launches over slots of different netlists (hp_iterate_multi): each pass of an
iteration is one launch over every slot, each block reading its slot's netlist from the
descriptor at the head of the slot buffer.  The bar is bit identity with each slot iterated
alone by hp_iterate on a context of its own (positions u and v, the optimiser state, lambda
and the exact HPWL of Eq. 1), over netlists that differ in every size the launches depend on:
bin grids (square and not), cell and net counts, movable macros (big-cell blocks), nets wide
enough for a block each, and scatter rebuild intervals."""
import dataclasses

import numpy as np
import pytest

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hy():
    from paper_2402_18311_amd import hybro
    return hybro


def _rect(nl, my):
    """The same netlist on a grid of my rows (mx columns unchanged)."""
    return dataclasses.replace(nl, my=my)


_NETS32 = {
    "small": (lambda: netgen.make_small(20_011, 21_003, 128, seed=3, n_fixed=40), 1),
    "mm": (lambda: netgen.make_small(6_000, 6_300, 64, seed=4, n_fixed=12, movable_macros=True), 4),
    "tiny": (lambda: netgen.make_netlist("tiny", 0), 2),
    "rect": (lambda: _rect(netgen.make_small(9_000, 9_400, 128, seed=6, n_fixed=20), 32), 3),
    "scaled": (lambda: netgen.make_netlist(netgen.scaled_config(70_000, bins=256), 2), 1),
}
_NETS64 = {
    "tiny": (lambda: netgen.make_netlist("tiny", 0), 2),
    "tiny_mm": (lambda: netgen.make_small(1000, 1100, 64, seed=1, n_fixed=6, movable_macros=True), 1),
    "rect": (lambda: _rect(netgen.make_small(3_000, 3_150, 64, seed=8, n_fixed=10), 16), 4),
}


def _snap(pl, s):
    st = pl.state(s)
    x, y = pl.positions(s)
    vx, vy = pl.eval_positions(s)
    return {"k": st["k"], "a": st["a"], "alpha": st["alpha"], "lambda": st["lambda_"],
            "u": (x.tobytes(), y.tobytes()), "v": (vx.tobytes(), vy.tobytes()),
            "hpwl": int(pl.hpwl(s)[0])}


def _start(pl, s, nl, seed):
    rng = np.random.default_rng(seed)
    n = nl.n_movable
    x = np.clip(nl.x0 + rng.normal(0, 2 * nl.bin_w, n), 0, nl.W - nl.cell_w[:n])
    y = np.clip(nl.y0 + rng.normal(0, 2 * nl.bin_h, n), 0, nl.H - nl.cell_h[:n])
    pl.set_positions(s, x, y)
    pl.set_schedule(s, 1e-4, 4.0, 300)


@pytest.mark.parametrize("prec,closing,graph", [(32, False, False), (32, True, False),
                                                (64, False, False), (32, False, True),
                                                (64, False, True)])
def test_shared_launches_match_each_slot_alone(hy, prec, closing, graph):
    """closing: one netlist takes the closing-reduction step form (as above 262,144 movable
    cells), which puts the whole shared launch in that form; else every slot takes the fused
    step.  graph: the shared launches replay steady blocks from a captured HIP graph (the
    slots' rebuild intervals make a 24-iteration block), in calls long enough to replay.
    The 'small' netlist iterated alone takes the non-temporal sweep, which launches that mix
    netlists leave out: the same values either way."""
    nets = _NETS32 if prec == 32 else _NETS64
    built = {k: (make(), every) for k, (make, every) in nets.items()}
    stream = hy.OwnStream() if graph else None
    ctx = hy.Context(precision=prec, stream=stream)
    alone, shared = {}, {}
    try:
        for k, (nl, every) in built.items():
            for where in ("alone", "shared"):
                pl = hy.Placer(nl, precision=prec) if where == "alone" else ctx.placer(nl)
                pl.set_scatter_policy(every, every % 2 == 0)
                if closing and k == "tiny" and where == "shared":
                    pl.set_tunable(hy.HP_TUNE_FUSED_STEP_PARTS, 0)
                if k == "small" and where == "alone":  # hinted sweep alone, plain when shared
                    pl.set_tunable(hy.HP_TUNE_NONTEMPORAL, 1)
                # two slots of the first netlist, one of every other
                ss = [pl.new_slot() for _ in range(2 if k == "small" or k == "tiny" else 1)]
                for j, s in enumerate(ss):
                    _start(pl, s, nl, 17 * j + len(k))
                    pl.iterate(s, 4 * nl.bin_w, 1, hpwl=False)  # steady state
                (alone if where == "alone" else shared)[k] = (pl, ss)
        slots = [s for pl, ss in shared.values() for s in ss]
        gammas = [4 * pl.nl.bin_w for pl, ss in shared.values() for s in ss]
        chunks = ((3, "last"), (5, True), (9, "last"))
        if graph:
            chunks = ((3, "last"), (60, "last"), (5, True), (50, True), (9, "last"))
        for chunk, hpwl in chunks:
            ctx.iterate(slots, gammas, chunk, hpwl=hpwl, graph=graph)
            for k, (pl, ss) in alone.items():
                for s in ss:
                    pl.iterate(s, 4 * pl.nl.bin_w, chunk, hpwl=hpwl)
            for k in built:
                (pa, sa_), (pb, sb) = alone[k], shared[k]
                for a, b in zip(sa_, sb):
                    ra, rb = _snap(pa, a), _snap(pb, b)
                    for f in ra:
                        assert ra[f] == rb[f], (k, chunk, f)
            print(f"fp{prec} after +{chunk}: HPWL " + ", ".join(
                f"{k} {_snap(shared[k][0], shared[k][1][0])['hpwl'] / 65536:.1f}" for k in built))
        if graph:
            captures, replays = hy.hp_graph_stats(ctx.ctx)
            print(f"graph blocks captured {captures}, replayed {replays}")
            assert captures >= 1 and replays >= 2
    finally:
        for pl, _ in alone.values():
            pl.close()
        for pl, _ in shared.values():
            pl.close()
        ctx.close()
        if stream is not None:
            stream.close()


def test_shared_launch_errors(hy):
    L = hy.lib()
    ctx = hy.Context(precision=32)
    a = ctx.placer(netgen.make_netlist("tiny", 0))
    b = ctx.placer(netgen.make_small(300, 320, 16, seed=9, n_fixed=6))
    try:
        sa, sb = a.new_slot(), b.new_slot()
        for pl, s in ((a, sa), (b, sb)):
            pl.set_positions(s, pl.nl.x0, pl.nl.y0)

        def call(slots, gammas, flags=0, iters=2):
            sl = np.asarray(slots, np.int32)
            g = np.asarray(gammas, np.float64)
            return L.hp_iterate_multi(ctx.ctx, sl.ctypes.data, len(sl), g.ctypes.data, flags, iters)
        # not yet in steady state (no lambda, no grouping)
        assert call([sa, sb], [1.0, 1.0]) == hy.HP_ESTATE
        a.iterate(sa, 4 * a.nl.bin_w, 1, hpwl=False)
        assert call([sa, sb], [1.0, 1.0]) == hy.HP_ESTATE  # b still fresh
        b.iterate(sb, 4 * b.nl.bin_w, 1, hpwl=False)
        assert call([sa, sb], [1.0, 1.0]) == hy.HP_OK
        assert call([sa, sa], [1.0, 1.0]) == hy.HP_EINVAL  # listed twice
        assert call([sa, sb], [1.0, 0.0]) == hy.HP_EINVAL  # gamma
        assert call([sa, sb], [1.0, float("nan")]) == hy.HP_EINVAL
        # graph replay needs a stream other than the null stream; unknown flags
        assert call([sa, sb], [1.0, 1.0], flags=hy.HP_ITER_GRAPH) == hy.HP_EINVAL
        assert call([sa, sb], [1.0, 1.0], flags=1 << 9) == hy.HP_EINVAL
        assert call([sa, sb], [1.0, 1.0], iters=-1) == hy.HP_EINVAL
        assert call([sa, 999], [1.0, 1.0]) == hy.HP_ESTATE
        assert call(list(range(33)), [1.0] * 33) == hy.HP_EINVAL
        # a kept map leaves the slot out of steady state until its next iteration
        a.eval(sa, 4 * a.nl.bin_w, lam=0.5, keep_maps=True)
        assert call([sa, sb], [1.0, 1.0]) == hy.HP_ESTATE
        a.iterate(sa, 4 * a.nl.bin_w, 1, hpwl=False)
        assert call([sa, sb], [1.0, 1.0]) == hy.HP_OK
        # a netlist with a live slot cannot be released
        assert L.hp_netlist_free(ctx.ctx, b.netlist) == hy.HP_ESTATE
        assert L.hp_netlist_free(ctx.ctx, 77) == hy.HP_ESTATE
    finally:
        a.close()
        b.close()
        ctx.close()
