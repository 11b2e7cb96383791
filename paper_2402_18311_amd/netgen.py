"""Seeded synthetic netlists shaped like the placement benchmarks the paper evaluates on.

The paper measures on ISPD 2005 and ICCAD 2015 designs (Sec. 5.1, Table 1); those suites are
not available here, so this module builds random netlists with the same kind of structure:
unit-height standard cells, fixed I/O pads or fixed macros, a skewed net-degree mix and
Rent-like locality.  It is the ONE module shared by the GPU path and the CPU oracle, and it
holds none of the placement method's arithmetic: it only draws sizes, positions and
connectivity.  Every float it emits is a multiple of 2**-8 and exactly representable in
FP32, so the FP32 device path and the FP64 oracle see identical inputs.

Netlist conventions (problem statement of Sec. 3, Eq. 1):
  * cells [0, n_movable) are movable, [n_movable, n_cells) are fixed (pads or macros);
  * positions are lower-left corners on the die [0, W] x [0, H];
  * nets are a CSR over pins: pins of net e are net_start[e] .. net_start[e+1]-1;
    pin p sits on cell pin_cell[p] at offset (pin_ox[p], pin_oy[p]) from its lower-left.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_Q = 256.0  # every generated length is a multiple of 1/_Q


def _snap(v):
    return np.round(np.asarray(v, dtype=np.float64) * _Q) / _Q


@dataclasses.dataclass
class Netlist:
    name: str
    n_movable: int
    n_cells: int
    cell_w: np.ndarray  # float64 [n_cells]
    cell_h: np.ndarray  # float64 [n_cells]
    fixed_x: np.ndarray  # float64 [n_cells - n_movable], lower-left
    fixed_y: np.ndarray
    net_start: np.ndarray  # int32 [n_nets + 1]
    pin_cell: np.ndarray  # int32 [n_pins]
    pin_ox: np.ndarray  # float64 [n_pins]
    pin_oy: np.ndarray
    W: float
    H: float
    mx: int
    my: int
    x0: np.ndarray  # float64 [n_movable] initial lower-left x
    y0: np.ndarray
    seed: int = 0
    macros: np.ndarray | None = None  # int32 ids of the movable macros, when there are any
    n_fillers: int = 0  # the last n_fillers movable cells are fillers (charge, no pins)

    @property
    def n_nets(self) -> int:
        return int(self.net_start.shape[0] - 1)

    @property
    def n_pins(self) -> int:
        return int(self.pin_cell.shape[0])

    @property
    def n_fixed(self) -> int:
        return self.n_cells - self.n_movable

    @property
    def bin_w(self) -> float:
        return self.W / self.mx

    @property
    def bin_h(self) -> float:
        return self.H / self.my

    def degrees(self) -> np.ndarray:
        return np.diff(self.net_start)

    def random_positions(self, seed: int):
        """Uniform random lower-left positions inside the die for the movable cells."""
        rng = np.random.default_rng(seed)
        w = self.cell_w[: self.n_movable]
        h = self.cell_h[: self.n_movable]
        x = rng.random(self.n_movable) * (self.W - w)
        y = rng.random(self.n_movable) * (self.H - h)
        return (x.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64))


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_movable: int
    n_nets: int
    bins: int
    fixed: str  # "pads" | "macros" | "none"
    n_fixed: int
    degrees: str  # "mix" | "mix_big" | "powerlaw"
    utilisation: float = 0.70
    macro_frac: float = 0.0
    locality: bool = True
    max_degree: int = 5000
    movable_macros: bool = False  # the macros are movable cells [n_movable, n_movable + n_fixed)


# The five workload shapes; sizes mirror Table 1 (adaptec1 for "mid", the largest
# superblue designs for "large").
TINY = Config("tiny", 1_000, 1_100, 64, "pads", 40, "mix")
MID = Config("mid", 210_000, 220_000, 512, "macros", 500, "mix_big", macro_frac=0.20)
LARGE = Config("large", 2_200_000, 2_300_000, 1024, "macros", 8_000, "powerlaw",
               macro_frac=0.20)
# "mid" with its 500 macros movable (the mixed-size case of Hybro-Shuffle, Sec. 4.2): the same
# draws as "mid", the macros starting at their legal, non-overlapping places.
MID_MM = dataclasses.replace(MID, name="mid_mm", movable_macros=True)
CONFIGS = {c.name: c for c in (TINY, MID, LARGE, MID_MM)}


def scaled_config(n_movable: int, name: str | None = None, bins: int | None = None) -> Config:
    """A netlist shaped like 'mid' at another size: nets ~1.045x cells, macros pro rata
    covering 20% of the die, bins = next power of two >= sqrt(cells)/2 (serving jobs)."""
    if bins is None:
        bins = 1 << max(3, math.ceil(math.log2(max(8.0, math.sqrt(n_movable) / 2))))
    n_mac = max(4, round(500 * n_movable / 210_000))
    return Config(name or f"scaled{n_movable}", n_movable, round(1.045 * n_movable), bins,
                  "macros", n_mac, "mix_big", macro_frac=0.20)


def _draw_degrees(rng, cfg: Config, n: int) -> np.ndarray:
    if cfg.degrees in ("mix", "mix_big"):
        u = rng.random(n)
        d = np.empty(n, dtype=np.int64)
        big = 0.001 if cfg.degrees == "mix_big" else 0.0
        s = 1.0 - big
        c2, c3, c10 = 0.60 * s, 0.80 * s, 0.97 * s
        d[u < c2] = 2
        d[(u >= c2) & (u < c3)] = 3
        m = (u >= c3) & (u < c10)
        d[m] = rng.integers(4, 11, size=int(m.sum()))
        m = (u >= c10) & (u < s)
        d[m] = rng.integers(11, 51, size=int(m.sum()))
        m = u >= s
        d[m] = rng.integers(200, 2001, size=int(m.sum()))
        return d
    if cfg.degrees == "powerlaw":
        ks = np.arange(2, cfg.max_degree + 1, dtype=np.float64)
        p = ks ** -2.5
        p /= p.sum()
        return rng.choice(ks.astype(np.int64), size=n, p=p)
    raise ValueError(cfg.degrees)


def _place_macros(rng, n_mac: int, side: float, frac: float):
    aspect = rng.uniform(0.5, 2.0, n_mac)
    area = np.exp(rng.uniform(0.0, math.log(16.0), n_mac))
    area *= frac * side * side / area.sum()
    w = _snap(np.maximum(np.sqrt(area * aspect), 1.0 / _Q))
    h = _snap(np.maximum(np.sqrt(area / aspect), 1.0 / _Q))
    order = np.argsort(-(w * h), kind="stable")
    xs = np.zeros(n_mac)
    ys = np.zeros(n_mac)
    px = np.empty(0)
    py = np.empty(0)
    pw = np.empty(0)
    ph = np.empty(0)
    for i in order:
        for _ in range(10_000):
            x = _snap(rng.uniform(0.0, side - w[i]))
            y = _snap(rng.uniform(0.0, side - h[i]))
            if px.size == 0 or not np.any((x < px + pw) & (px < x + w[i]) &
                                          (y < py + ph) & (py < y + h[i])):
                break
        else:  # pragma: no cover - only with absurd densities
            raise RuntimeError("macro placement failed")
        xs[i], ys[i] = x, y
        px = np.append(px, x)
        py = np.append(py, y)
        pw = np.append(pw, w[i])
        ph = np.append(ph, h[i])
    return w, h, xs, ys


def make_netlist(cfg: Config | str, seed: int = 0) -> Netlist:
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    rng = np.random.default_rng([seed, cfg.n_movable, cfg.n_nets, cfg.bins])
    n = cfg.n_movable
    w_mov = _snap(rng.uniform(1.0, 4.0, n))
    h_mov = np.ones(n)
    mov_area = float((w_mov * h_mov).sum())
    f_mac = cfg.macro_frac if cfg.fixed == "macros" else 0.0
    side_raw = math.sqrt(mov_area / (cfg.utilisation * (1.0 - f_mac)))
    M = cfg.bins
    bin_w = math.ceil(side_raw / M * _Q) / _Q  # bin width is a multiple of 2**-8
    side = M * bin_w

    if cfg.fixed == "pads":
        t = np.arange(cfg.n_fixed) * (4.0 * side / cfg.n_fixed)
        fx = np.where(t < side, t, np.where(t < 2 * side, side, np.where(t < 3 * side,
                                                                       3 * side - t, 0.0)))
        fy = np.where(t < side, 0.0, np.where(t < 2 * side, t - side,
                                              np.where(t < 3 * side, side, 4 * side - t)))
        fw = np.zeros(cfg.n_fixed)
        fh = np.zeros(cfg.n_fixed)
        fx, fy = _snap(fx), _snap(fy)
    elif cfg.fixed == "macros":
        fw, fh, fx, fy = _place_macros(rng, cfg.n_fixed, side, f_mac)
    else:
        fw = fh = fx = fy = np.zeros(0)
    n_fixed = fx.shape[0]
    n_cells = n + n_fixed
    cell_w = np.concatenate([w_mov, fw])
    cell_h = np.concatenate([h_mov, fh])

    deg = _draw_degrees(rng, cfg, cfg.n_nets)
    deg = np.minimum(deg, n)
    net_start = np.zeros(cfg.n_nets + 1, dtype=np.int64)
    np.cumsum(deg, out=net_start[1:])
    P = int(net_start[-1])
    pin_cell = np.empty(P, dtype=np.int64)
    for d in np.unique(deg):
        nets = np.nonzero(deg == d)[0]
        k = nets.shape[0]
        if cfg.locality and d < 200:
            win = min(n, max(64, 16 * int(d)))
            anchor = rng.integers(0, n - win + 1, size=k)
        else:
            win = n
            anchor = np.zeros(k, dtype=np.int64)
        r = rng.integers(0, win - d + 1, size=(k, int(d)))
        r.sort(axis=1)
        r += np.arange(d)  # strictly increasing => distinct cells within a net
        cells = anchor[:, None] + r
        pos = net_start[nets][:, None] + np.arange(d)
        pin_cell[pos.ravel()] = cells.ravel()
    if n_fixed:
        hit = rng.random(P) < 0.02
        pin_cell[hit] = n + rng.integers(0, n_fixed, size=int(hit.sum()))
    pw = cell_w[pin_cell]
    ph = cell_h[pin_cell]
    pin_ox = _snap(rng.random(P) * pw)
    pin_oy = _snap(rng.random(P) * ph)

    x0 = rng.random(n) * (side - w_mov)
    y0 = rng.random(n) * (side - h_mov)
    x0 = x0.astype(np.float32).astype(np.float64)
    y0 = y0.astype(np.float32).astype(np.float64)
    macros = None
    if cfg.movable_macros and cfg.fixed == "macros":
        # fixed ids already follow the movable ones, so pins keep their cells
        macros = np.arange(n, n_cells, dtype=np.int32)
        x0 = np.concatenate([x0, fx])
        y0 = np.concatenate([y0, fy])
        n, fx, fy = n_cells, np.zeros(0), np.zeros(0)
    nl = Netlist(
        name=cfg.name, n_movable=n, n_cells=n_cells,
        cell_w=cell_w.astype(np.float64), cell_h=cell_h.astype(np.float64),
        fixed_x=fx.astype(np.float64), fixed_y=fy.astype(np.float64),
        net_start=net_start.astype(np.int32), pin_cell=pin_cell.astype(np.int32),
        pin_ox=pin_ox, pin_oy=pin_oy, W=float(side), H=float(side), mx=M, my=M,
        x0=x0, y0=y0, seed=seed, macros=macros)
    return nl


def with_fillers(nl: Netlist, target_density: float, seed: int = 0) -> Netlist:
    """The netlist with ePlace filler cells for a target density below 1: pinless movable cells
    of the standard cells' mean width and unit height, appended after the movable cells (fixed
    ids shift up, pins follow), as many as fill target_density x (die - fixed area) minus the
    movable area, at uniform random starting places."""
    n = nl.n_movable
    fixed_area = float((nl.cell_w[n:] * nl.cell_h[n:]).sum())
    mov_area = float((nl.cell_w[:n] * nl.cell_h[:n]).sum())
    std = np.ones(n, bool)
    if nl.macros is not None:
        std[nl.macros] = False
    fw = float(_snap(nl.cell_w[:n][std].mean()))
    room = target_density * (nl.W * nl.H - fixed_area) - mov_area
    k = max(0, int(room // fw))
    rng = np.random.default_rng([seed, n, k])
    fx = _snap(rng.random(k) * (nl.W - fw)).astype(np.float32).astype(np.float64)
    fy = _snap(rng.random(k) * (nl.H - 1.0)).astype(np.float32).astype(np.float64)
    pin_cell = nl.pin_cell.astype(np.int64)
    pin_cell = np.where(pin_cell >= n, pin_cell + k, pin_cell).astype(np.int32)
    return dataclasses.replace(
        nl, name=f"{nl.name}+fill", n_movable=n + k, n_cells=nl.n_cells + k,
        cell_w=np.concatenate([nl.cell_w[:n], np.full(k, fw), nl.cell_w[n:]]),
        cell_h=np.concatenate([nl.cell_h[:n], np.ones(k), nl.cell_h[n:]]),
        pin_cell=pin_cell, x0=np.concatenate([nl.x0, fx]), y0=np.concatenate([nl.y0, fy]),
        n_fillers=k)


def make_small(n_movable: int, n_nets: int, bins: int, seed: int = 0, fixed: str = "macros",
               n_fixed: int = 8, degrees: str = "mix_big", movable_macros: bool = False,
               macro_frac: float = 0.20) -> Netlist:
    """A reduced netlist for parity tests (spans several tiles and ragged tails).  With
    movable_macros the n_fixed macros become movable cells after the standard cells."""
    cfg = Config(f"small{n_movable}", n_movable, n_nets, bins, fixed, n_fixed, degrees,
                 macro_frac=macro_frac if fixed == "macros" else 0.0,
                 max_degree=min(5000, n_movable), movable_macros=movable_macros)
    return make_netlist(cfg, seed)
