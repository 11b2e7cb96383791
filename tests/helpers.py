"""Small input builders shared by the tests (no method arithmetic here)."""
import json
import os

import numpy as np

from paper_2402_18311_amd.netgen import Netlist

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_json(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def netlist_from_dict(d) -> Netlist:
    n_mov = d["n_movable"]
    return Netlist(
        name="hand", n_movable=n_mov, n_cells=len(d["cell_w"]),
        cell_w=np.array(d["cell_w"], float), cell_h=np.array(d["cell_h"], float),
        fixed_x=np.array(d["fixed_x"], float), fixed_y=np.array(d["fixed_y"], float),
        net_start=np.array(d["net_start"], np.int32), pin_cell=np.array(d["pin_cell"], np.int32),
        pin_ox=np.array(d["pin_ox"], float), pin_oy=np.array(d["pin_oy"], float),
        W=float(d["W"]), H=float(d["H"]), mx=int(d["mx"]), my=int(d["my"]),
        x0=np.array(d["x"], float), y0=np.array(d["y"], float))


def cells_only(w, h, W, H, M, x, y, nets=None):
    """Movable cells with optional nets given as lists of (cell, ox, oy)."""
    nets = nets or []
    starts = [0]
    pc, ox, oy = [], [], []
    for net in nets:
        for c, a, b in net:
            pc.append(c)
            ox.append(a)
            oy.append(b)
        starts.append(len(pc))
    n = len(w)
    return Netlist(
        name="cells", n_movable=n, n_cells=n, cell_w=np.asarray(w, float),
        cell_h=np.asarray(h, float), fixed_x=np.zeros(0), fixed_y=np.zeros(0),
        net_start=np.array(starts, np.int32), pin_cell=np.array(pc, np.int32),
        pin_ox=np.array(ox, float), pin_oy=np.array(oy, float), W=float(W), H=float(H),
        mx=M, my=M, x0=np.asarray(x, float), y0=np.asarray(y, float))
