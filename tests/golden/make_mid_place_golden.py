"""Writes mid_place_fp64.json: the FP64 oracle's plain placement of the mid synthetic netlist
(seed 0), the end-to-end reference for the device's FP32 placement of the same netlist.

Calls only the oracle (and the seeded input generator).  The run: 1000 iterations of the
placer of Sec. 3.1 (objective of Eq. 2 with the WA wirelength of Eq. 3 and the electrostatic
density, preconditioned Nesterov step) from the generator's initial positions, smoothing
gamma = 4 bin widths, lambda_0 = 1e-4 |grad WL|_1 / |grad N|_1 growing four decades over the
run; the Poisson transforms through the oracle's FFT path (equal to its cosine sums to
rounding, pinned in tests/test_oracle_schedules.py).  Records the exact HPWL of Eq. 1 (2^-16
units) after every 100th step and the overflow of the last evaluation.

    python tests/golden/make_mid_place_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2402_18311_amd import netgen  # noqa: E402

ITERS = 1000


def main():
    nl = netgen.make_netlist("mid", 0)
    o = O.Oracle(nl)
    gamma = 4 * nl.bin_w
    t0 = time.time()
    _, _, tr = o.place(nl.x0, nl.y0, ITERS, gamma, 1e-4, 4.0, fft=True)
    rec = {
        "netlist": "mid, seed 0",
        "iterations": ITERS,
        "gamma_bins": 4.0,
        "lambda0_scale": 1e-4,
        "lambda_decades": 4.0,
        "hpwl_q_every_100": [int(tr["hpwl_q"][k]) for k in range(99, ITERS, 100)],
        "final_hpwl_q": int(tr["hpwl_q"][-1]),
        "final_overflow": float(tr["overflow"][-1]),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "mid_place_fp64.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
