"""Benchmark of the placer hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large] [--no-cpu-baseline]

Headline workload: the "large" synthetic netlist (2.2 M movable unit-height cells, 8,000 fixed
macros on 20% of the die, 2.3 M nets with a power-law degree mix up to 5,000 pins, 1024 x 1024
bins, FP32 with the int64 charge map), the largest configuration that fits one GPU.  One step
is one iteration of the plain placer (Sec. 3.1): the objective and gradient of Eq. 2 (WA
wirelength of Eq. 3, charge scatter, Poisson solve, field gather, overflow) and the
preconditioned Nesterov step, with the exact HPWL of Eq. 1 taken every 10 iterations (the
cadence at which the Alg. 1 driver reads it; the rate with the HPWL after every iteration is
reported beside it).  W untimed iterations from the initial positions, then K timed ones of
the same placement (its lambda schedule spans the configuration's 2,000 iterations).

Prints one JSON line: iterations/s, per-step milliseconds, the roofline of the dominant kernel
(its share of the compulsory bytes per iteration / its average duration from HIP events on its
launches in the timed region) and the CPU oracle's rate on a bounded sample of the same
workload; secondary lines: a Hybro round on "mid" (adaptec1-sized), the batched round of 32
restarts, mid with movable macros, and the serving mix.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CONFIG_ITERS = {"large": 2000, "mid": 1000, "tiny": 200}
HPWL_EVERY = 10  # the Alg. 1 driver reads the exact HPWL and the overflow every 10 iterations
# Sources that define the first launch of an evaluation (the dominant kernel); a stored HBM
# traffic record is used only while their hash matches the one it was measured with.
FRONT_SOURCES = ["paper_2402_18311_amd/csrc/k_sweep.hip", "paper_2402_18311_amd/csrc/hp_binning.h",
                 "paper_2402_18311_amd/csrc/hp_device.h", "paper_2402_18311_amd/csrc/hp_internal.h"]
CALIB_BYTES = 256 << 20  # the calibration copy: 256 MiB read and 256 MiB written
METRIC = ("placer iters/sec + HBM GB/s; batched-vs-plain restarts/sec, p50/p99 at equal HPWL")


def traffic_file(kernel, workload):
    return os.path.join("profiles", f"{kernel}_{workload}_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def compulsory_bytes(nl, rs=4):
    """Compulsory HBM bytes of one iteration, one slot: each static or state array read once,
    each output written once, intermediates (pin gradients, charge maps, field maps, spectral
    work arrays, partial sums) not counted.  Returns the evaluation's and the step's totals
    and each kernel's share:
      B_eval = 4 (E + 1) + 12 P + 8 N_all + 16 N_mov + 8 N_mov + 8 M^2
        (net offsets; pin cell ids and two FP32 offsets; every position; the movable cells'
        static charge geometry; the gradient out; the fixed cells' int64 charge map),
      B_step = 64 N_mov
        (v, u, g, v_prev, g~_prev read, 8 bytes of preconditioner inputs, u and v written).
    Shares: the first launch of an evaluation (net sweep and charge scatter) reads the
    topology, the positions and the charge geometry; the row pass of the Poisson solve reads
    the fixed map; the gradient pass writes the gradient; the update does the step."""
    E, P = nl.n_nets, nl.n_pins
    N, Nall = nl.n_movable, nl.n_cells
    M2 = nl.mx * nl.my
    share = {
        "eval_front_kernel": 4 * (E + 1) + 12 * P + 8 * Nall + 16 * N,
        "spec_rows_fwd": 8 * M2,
        "cell_grad_kernel": 8 * N,
        "step_update_kernel": 64 * N,
    }
    b_eval = 4 * (E + 1) + 12 * P + 8 * Nall + 24 * N + 8 * M2
    return b_eval, 64 * N, share


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_iterations(o, nl, gamma, iters, ratio):
    """Seconds of each of `iters` oracle placer iterations from the initial positions:
    objective and gradient (FFT path of the Poisson transforms), Nesterov step, exact HPWL."""
    n = nl.n_movable
    st = o.new_state(nl.x0, nl.y0)
    lam = None
    times = []
    for _ in range(iters):
        t0 = time.perf_counter()
        r = o.eval(st["v"][:n], st["v"][n:], gamma, fft=True)
        gw = np.concatenate([r["gwx"], r["gwy"]])
        gd = np.concatenate([r["gdx"], r["gdy"]])
        lam = 1e-4 * np.abs(gw).sum() / np.abs(gd).sum() if lam is None else lam * ratio
        o.nesterov_step(lam, gw + lam * gd, st)
        o.hpwl_q(st["u"][:n], st["u"][n:])
        times.append(time.perf_counter() - t0)
    return times


def cpu_extra(netgen, seed):
    """The oracle on the other workloads (reported beside the headline's baseline, not part of
    it): tiny, its full 200 iterations; mid, the median of 20 iterations, extrapolated to 1000;
    the batched round, 32 mid slots advanced 2 iterations each with one slot per host thread at
    a time, extrapolated to 1000 iterations per restart.  One thread and all threads each."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    all_threads = O.num_threads()
    out = {"cpu_model": _cpu_model(), "threads_all": all_threads}
    tiny = netgen.make_netlist("tiny", seed)
    o = O.Oracle(tiny)
    g = 4 * tiny.bin_w
    row = {}
    for th in (1, all_threads):
        O.set_threads(th)
        ts = _oracle_iterations(o, tiny, g, 200, o.lambda_ratio(4.0, 200))
        row[f"{th}_threads"] = {"run_s": round(sum(ts), 3), "iter_per_s": round(200 / sum(ts), 2)}
    out["tiny"] = dict(row, sample="the full 200-iteration placement from the initial positions")
    mid = netgen.make_netlist("mid", seed)
    o = O.Oracle(mid)
    g = 4 * mid.bin_w
    ratio = o.lambda_ratio(4.0, 1000)
    row = {}
    for th in (1, all_threads):
        O.set_threads(th)
        tm = float(np.median(_oracle_iterations(o, mid, g, 20, ratio)))
        row[f"{th}_threads"] = {"iter_per_s": round(1 / tm, 3),
                                "extrapolated_1000_iter_s": round(1000 * tm, 1)}
    out["mid"] = dict(row, sample="median of 20 iterations from the initial positions; 1000 "
                                  "iterations extrapolated, not run")
    K, it = 32, 2

    def slot(_):
        O.set_threads(1)  # this worker's parallel loops on one thread
        return sum(_oracle_iterations(o, mid, g, it, ratio))
    with ThreadPoolExecutor(max_workers=all_threads) as ex:
        t0 = time.perf_counter()
        list(ex.map(slot, range(K)))
        wall = time.perf_counter() - t0
    O.set_threads(all_threads)
    rate = K * it / wall
    out["batched"] = {"slot_iter_per_s": round(rate, 3),
                      "restarts_per_s_1000_iter": round(rate / 1000, 5),
                      "sample": f"{K} mid slots x {it} iterations from the initial positions, "
                                f"one slot per thread at a time on {all_threads} threads; 1000 "
                                f"iterations per restart extrapolated, not run"}
    return out


def cpu_baseline(nl, gamma, iters=5, label="large"):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload: `iters` whole
    placer iterations (objective + gradient with the FFT path of the Poisson transforms,
    Nesterov step, exact HPWL) from the initial positions, once on one thread and once on all
    the threads OpenMP is given; the rate is from the median iteration."""
    from oracle import oracle as O
    o = O.Oracle(nl)
    n = nl.n_movable
    all_threads = O.num_threads()
    nproc = os.cpu_count()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    ratio = o.lambda_ratio(4.0, CONFIG_ITERS.get(label, 1000))

    def run(threads):
        O.set_threads(threads)
        return float(np.median(_oracle_iterations(o, nl, gamma, iters, ratio)))

    t1 = run(1)
    tn = run(all_threads)
    O.set_threads(all_threads)
    total = CONFIG_ITERS.get(label, 1000)
    return {"value": round(1.0 / tn, 4), "unit": "iter/s", "cores": all_threads,
            "kind": "oracle",
            "sample": f"median of {iters} placer iterations (objective + gradient with the FFT "
                      f"path of the Poisson transforms, Nesterov step, exact HPWL) of the "
                      f"{label} workload from its initial placement, FP64, on {all_threads} "
                      f"threads; a {total}-iteration run extrapolates to {total * tn:.0f} s "
                      f"(extrapolated, not run)",
            "cpu_model": _cpu_model(), "nproc": nproc, "cpus_available": avail,
            "threads_all": all_threads,
            "iter_per_s_1_thread": round(1.0 / t1, 4),
            "iter_per_s_all_threads": round(1.0 / tn, 4),
            "extrapolated_run_s": {"1_thread": round(total * t1, 1),
                                   "all_threads": round(total * tn, 1), "iterations": total}}


def sources_hash(files=FRONT_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_summary(fetch_dir, write_dir, kernel="eval_front_kernel", last=None, workload="large"):
    """Per-launch HBM traffic of `kernel` from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for the 256 MiB
    calibration copy of the same run (--copy-calibration).  With `last`, the average is over
    the kernel's last `last` dispatches (the timed round of the profiled run) and the average
    over all of them is recorded beside it.  Writes traffic_file(kernel, workload)."""
    import csv
    import glob

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        vals, calib = [], []
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if kernel in r["Kernel_Name"]:
                vals.append((int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0), v))
            elif "copyBuffer" in r["Kernel_Name"]:
                calib.append(v)
        vals = [v for _, v in sorted(vals)]
        tail = vals[-last:] if last else vals
        return sum(tail) / len(tail), max(calib), len(tail), sum(vals) / len(vals)

    fe, fc, n1, fe_all = load(fetch_dir, "FETCH_SIZE")
    wr, wc, n2, wr_all = load(write_dir, "WRITE_SIZE")
    kib = CALIB_BYTES / 1024
    ff, wf = kib / fc, kib / wc
    traffic = (fe * ff + wr * wf) * 1024
    rec = {"kernel": kernel, "workload": workload, "fetch_kib_per_launch": round(fe, 1),
           "write_kib_per_launch": round(wr, 1), "launches": [n1, n2],
           "all_launches_fetch_write_kib": [round(fe_all, 1), round(wr_all, 1)],
           "calibration_copy_kib": [round(fc, 1), round(wc, 1)],
           "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
           "traffic_bytes_per_launch": int(traffic), "sources_hash": sources_hash()}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, traffic_file(kernel, workload)), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def trace_summary(trace_dir, last):
    """Per-kernel launch counts and average durations from a rocprofv3 --kernel-trace CSV:
    over all launches and over each kernel's last `last` launches (the timed region of a
    bench run whose timed iterations come last)."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)[0]
    rows = []
    for r in csv.DictReader(open(f)):
        name = r["Kernel_Name"].split("(")[0]
        rows.append((int(r["Start_Timestamp"]), name,
                     (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3))
    rows.sort()
    per = {}
    for _, name, us in rows:
        per.setdefault(name, []).append(us)
    out = {}
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        tail = v[-last:] if last else v
        out[name] = {"launches": len(v), "avg_us": round(sum(v) / len(v), 2),
                     "last_launches": len(tail), "last_avg_us": round(sum(tail) / len(tail), 2)}
    print(json.dumps(out, indent=1))
    return out


def stored_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` measured by counters, or None if absent
    or stale (the kernel's sources changed since)."""
    path = os.path.join(ROOT, traffic_file(kernel, workload))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel") != kernel or rec.get("sources_hash") != sources_hash():
        return None
    return rec["traffic_bytes_per_launch"]


def batched_round(pl, hy, nl, gamma, inc, K, T, seed0):
    """One batched Hybro round (K perturbed restarts of the incumbent, each Gaussian 5%,
    sigma 8 bins, then T iterations and the exact HPWL of the result): the K restarts one slot
    at a time, as one K-slot launch sequence, and as K slots with steady-state blocks replayed
    from a captured HIP graph.  Returns restarts/s of each and whether every restart's final
    HPWL_q agrees bit for bit across the three."""
    import torch
    ix = torch.empty(nl.n_movable, dtype=torch.float32, device="cuda")
    iy = torch.empty_like(ix)
    hy.hp_get_positions(pl.ctx, inc, ix, iy, True)
    res = {}
    c0, r0 = hy.hp_graph_stats(pl.ctx)
    for mode in ("plain", "batched", "graph"):
        slots = [pl.new_slot() for _ in range(K)]
        for s in slots:
            pl.set_positions(s, ix, iy)
            pl.set_schedule(s, 1e-4, 4.0, T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, s in enumerate(slots):
            pl.perturb(s, hy.HP_PERTURB_GAUSS, 0.05, 8.0, seed0 + k, want_idx=False)
            if mode == "plain":
                pl.iterate(s, gamma, T, hpwl="last")
        if mode != "plain":
            pl.iterate(slots, gamma, T, hpwl="last", graph=mode == "graph")
        q = pl.hpwl(slots)  # reduces the last sweeps (synchronises)
        dt = time.perf_counter() - t0
        res[mode] = (K / dt, dt, [int(v) for v in q])
        for s in slots:
            pl.free_slot(s)
    c1, r1 = hy.hp_graph_stats(pl.ctx)
    # the kernel split of a batched iteration: the same restarts, 20 iterations with events on
    # every launch after 5 untimed ones (a separate pass; the timed modes above carry none)
    slots = [pl.new_slot() for _ in range(K)]
    for k, s in enumerate(slots):
        pl.set_positions(s, ix, iy)
        pl.set_schedule(s, 1e-4, 4.0, T)
        pl.perturb(s, hy.HP_PERTURB_GAUSS, 0.05, 8.0, seed0 + k, want_idx=False)
    pl.iterate(slots, gamma, 5, hpwl=False)
    hy.hp_profile_enable(pl.ctx, True)
    hy.hp_profile_read(pl.ctx, reset=True)
    pl.iterate(slots, gamma, 20, hpwl=False)
    prof = hy.hp_profile_read(pl.ctx, reset=True)
    hy.hp_profile_enable(pl.ctx, False)
    for s in slots:
        pl.free_slot(s)
    split = {k: {"launches": c, "avg_us": round(1e3 * ms / max(c, 1), 2),
                 "us_per_iteration": round(1e3 * ms / 20, 2)}
             for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    return {"restarts": K, "iterations": T,
            "batched_restarts_per_s": round(res["batched"][0], 3),
            "graph_restarts_per_s": round(res["graph"][0], 3),
            "plain_restarts_per_s": round(res["plain"][0], 3),
            "speedup": round(max(res["batched"][0], res["graph"][0]) / res["plain"][0], 3),
            "batched_round_s": round(res["batched"][1], 4),
            "graph_round_s": round(res["graph"][1], 4),
            "plain_rounds_s": round(res["plain"][1], 4),
            "graph_blocks": {"captured": c1 - c0, "replayed": r1 - r0},
            "equal_hpwl": res["batched"][2] == res["plain"][2] == res["graph"][2],
            "best_hpwl": min(res["batched"][2]) / 65536,
            "kernels_per_batched_iteration": split,
            "hpwl": "exact HPWL of each restart after its last iteration (Alg. 1)"}


def mid_lines(hy, netgen, args):
    """Secondary lines on the "mid" netlist (adaptec1-sized, 512 x 512 bins, FP32): the
    incumbent from a full placement (untimed), then one timed Hybro round (Gaussian-perturb 5%
    of the cells by 8 bins, mid_steps placer iterations, keep the better), and the batched
    round of `batch` restarts against the same restarts one slot at a time."""
    import torch
    nl = netgen.make_netlist("mid", args.seed)
    gamma = 4 * nl.bin_w
    K, W = args.mid_steps, args.mid_warmup
    pl = hy.Placer(nl, precision=32, stream=torch.cuda.Stream())  # capturable stream
    work, inc = pl.new_slot(), pl.new_slot()
    pl.set_positions(work, nl.x0, nl.y0)
    pl.set_schedule(work, 1e-4, 4.0, max(W, 1))
    pl.iterate(work, gamma, W, hpwl="last")
    pl.hpwl(work)
    pl.select_best([work], inc)
    ix = torch.empty(nl.n_movable, dtype=torch.float32, device="cuda")
    iy = torch.empty_like(ix)
    hy.hp_get_positions(pl.ctx, inc, ix, iy, True)

    def restart(iters):
        pl.set_positions(work, ix, iy)
        pl.set_schedule(work, 1e-4, 4.0, iters)

    from paper_2402_18311_amd import autotune
    restart(K)
    pl.perturb(work, hy.HP_PERTURB_GAUSS, 0.05, 8.0, 0x7E57, want_idx=False)
    policy, _ = autotune.tune_scatter(pl, [work], gamma)
    restart(K)
    b_eval, b_step, share = compulsory_bytes(nl)
    hy.hp_profile_enable(pl.ctx, True, "eval_front_kernel")
    hy.hp_profile_read(pl.ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.perturb(work, hy.HP_PERTURB_GAUSS, 0.05, 8.0, 0xC0FFEE, want_idx=False)
    pl.iterate(work, gamma, K, hpwl="last", graph=True)
    pl.select_best([work], inc, want_host=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c, ms = hy.hp_profile_read(pl.ctx, reset=True).get("eval_front_kernel", (0, 0.0))
    hy.hp_profile_enable(pl.ctx, False)
    avg = ms * 1e-3 / max(c, 1)
    out = {"mid": {
        "workload": f"mid: {nl.n_movable} movable cells, {nl.n_fixed} fixed macros, "
                    f"{nl.n_nets} nets / {nl.n_pins} pins, {nl.mx}x{nl.my} bins, FP32; one Hybro "
                    f"round (Gaussian perturb 5%, sigma 8 bins) of {K} iterations (HIP-graph "
                    f"replay of steady-state blocks) and the exact HPWL after them, after a "
                    f"{W}-iteration placement",
        "iter_per_s": round(K / dt, 2), "ms_per_step": round(1e3 * dt / K, 5), "steps": K,
        "warmup": W, "final_hpwl": pl.state(inc)["hpwl_q"] / 65536,
        "scatter_policy": {"regroup_every": policy[0], "deferred": policy[1]},
        "compulsory_bytes_per_iter": b_eval + b_step,
        "compulsory_gbs": round((b_eval + b_step) / (dt / K) / 1e9, 1),
        "front_kernel_avg_us": round(avg * 1e6, 3) if c else None,
        "front_kernel_frac": round(share["eval_front_kernel"] / avg / 1e9 / HBM_PEAK_GBS, 4)
        if c else None,
        "note": "the mid working set fits the 256 MB Infinity Cache: reported, not the "
                "HBM roofline case"}}
    if args.batch > 0:
        log(f"[bench] batched round: {args.batch} restarts x {args.batch_iters} iterations")
        out["batched"] = batched_round(pl, hy, nl, gamma, inc, args.batch, args.batch_iters, 0xB00)
    pl.close()
    return out


def macros_run(hy, netgen, seed, warm, steps):
    """The mid netlist with its 500 macros movable (mixed-size placement; the macros take the
    block-per-cell charge path): iterations/s over `steps` plain-method iterations after
    `warm`, then one Hybro-Shuffle round (half of the macros exchange places, Sec. 4.2, and
    `steps` iterations follow) and one WireMask pass over all macros, each timed on its own."""
    import torch
    nl = netgen.make_netlist("mid_mm", seed)
    pl = hy.Placer(nl, precision=32)
    g = 4 * nl.bin_w
    s = pl.new_slot()
    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, 1e-4, 4.0, warm + steps)
    pl.iterate(s, g, warm, hpwl=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.iterate(s, g, steps, hpwl=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h0 = pl.hpwl(s)[0]
    w = pl.new_slot()
    ix = torch.empty(nl.n_movable, dtype=torch.float32, device="cuda")
    iy = torch.empty_like(ix)
    hy.hp_get_positions(pl.ctx, s, ix, iy, True)
    pl.set_positions(w, ix, iy)
    pl.set_schedule(w, 1e-4, 4.0, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    moved = pl.perturb(w, hy.HP_PERTURB_SHUFFLE, 0.5, 0.0, 0x5EED, want_idx=False,
                       cells=nl.macros)
    pl.iterate(w, g, steps, hpwl=True)
    h1 = pl.hpwl(w)[0]  # synchronises
    dr = time.perf_counter() - t1
    # one WireMask pass (Sec. 4.2) over every macro of the same placement, largest first
    pl.set_positions(w, ix, iy)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    wm_moved = pl.wiremask(w)  # synchronises
    dw = time.perf_counter() - t2
    h2 = pl.hpwl(w)[0]
    out = {"workload": f"mid_mm: {nl.n_movable} movable cells of which {len(nl.macros)} macros, "
                       f"{nl.n_nets} nets / {nl.n_pins} pins, {nl.mx}x{nl.my} bins, FP32",
           "iter_per_s": round(steps / dt, 2), "ms_per_step": round(1e3 * dt / steps, 4),
           "steps": steps, "warmup": warm, "hpwl": h0 / 65536,
           "shuffle_round": {"macros_moved": int(moved), "iterations": steps,
                             "seconds": round(dr, 4), "hpwl": h1 / 65536},
           "wiremask_pass": {"macros": len(nl.macros), "macros_moved": int(wm_moved),
                             "seconds": round(dw, 4), "hpwl_before": h0 / 65536,
                             "hpwl_after": h2 / 65536}}
    pl.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed placer iterations")
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed iterations of the same placement before the timed ones")
    ap.add_argument("--workload", default="large")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--locality", choices=("rent", "none"), default="rent",
                    help="none: every net draws its cells from the whole index range (a "
                         "sensitivity check of the synthetic netlists' index locality)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-extra", action="store_true",
                    help="also time the oracle on tiny, mid and the batched round")
    ap.add_argument("--cpu-iters", type=int, default=5,
                    help="oracle iterations per thread setting of the CPU baseline")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without the per-launch events (no roofline)")
    ap.add_argument("--mid-steps", type=int, default=1000,
                    help="timed iterations of the Hybro round on mid (0 skips the mid lines)")
    ap.add_argument("--mid-warmup", type=int, default=1000)
    ap.add_argument("--macro-steps", type=int, default=1000,
                    help="timed iterations on mid with movable macros (0 skips it)")
    ap.add_argument("--serve-jobs", type=int, default=16,
                    help="jobs of the serving-mix trace (0 skips it)")
    ap.add_argument("--batch", type=int, default=32,
                    help="restarts of the batched-round measurement (0 skips it)")
    ap.add_argument("--batch-iters", type=int, default=1000)
    ap.add_argument("--pmc-last", type=int, default=None,
                    help="with --pmc-summary: average the kernel's last N dispatches only")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="reduce two rocprofv3 --pmc output folders to the stored traffic "
                         "record and exit")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="reduce a rocprofv3 --kernel-trace output folder to per-kernel "
                         "averages (all launches and the last --pmc-last of each) and exit")
    ap.add_argument("--scatter-policy", metavar="EVERY,DEFERRED",
                    help="use this charge-scatter policy (e.g. 8,1) instead of timing the "
                         "candidates before the round")
    ap.add_argument("--launch-shape",
                    metavar="INTERLEAVE,SPECTRAL_THREADS[,CHARGE_RECORDS[,NONTEMPORAL]]",
                    help="use these launch shapes (e.g. 1,0,1,0) instead of timing the "
                         "candidates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, copy 256 MiB device-to-device once: the "
                         "reference dispatch for scaling hardware byte counters")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, last=args.pmc_last, workload=args.workload)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.pmc_last)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the placer runs on a single MI355X; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2402_18311_amd import hybro as hy
    from paper_2402_18311_amd import netgen
    if not os.path.exists(hy.LIB_PATH):
        from paper_2402_18311_amd import build as b
        b.build()

    cfg = netgen.CONFIGS[args.workload]
    if args.locality == "none":
        cfg = dataclasses.replace(cfg, locality=False, name=f"{cfg.name}_nolocality")
    nl = netgen.make_netlist(cfg, args.seed)
    gamma = 4 * nl.bin_w
    K, W = args.steps, args.warmup
    total = CONFIG_ITERS.get(args.workload, W + K)
    pl = hy.Placer(nl, precision=32)
    s = pl.new_slot()
    log(f"[bench] {nl.name}: {nl.n_movable} movable, {nl.n_fixed} fixed, {nl.n_nets} nets, "
        f"{nl.n_pins} pins, {nl.mx}x{nl.my} bins; warmup {W}, steps {K}")
    def run(slot, iters):
        """iters placer iterations with the exact HPWL (Eq. 1) and overflow read every
        HPWL_EVERY iterations, the cadence at which the Alg. 1 driver looks at them."""
        done = 0
        while done < iters:
            c = min(HPWL_EVERY, iters - done)
            pl.iterate(slot, gamma, c, hpwl="last")
            done += c

    pl.set_positions(s, nl.x0, nl.y0)
    pl.set_schedule(s, 1e-4, 4.0, total)
    run(s, W)
    pl.hpwl(s)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    # untimed: the scatter's grouping policy, timed on scratch slots from the current positions
    if args.scatter_policy:
        e, d = (int(v) for v in args.scatter_policy.split(","))
        pl.set_scatter_policy(e, bool(d))
        policy, tune_ms = pl.scatter_policy(), {}
    else:
        from paper_2402_18311_amd import autotune
        policy, tune_ms = autotune.tune_scatter(pl, [s], gamma)
    log(f"[bench] scatter policy {policy} ({tune_ms})")
    launch = {}
    if args.launch_shape:
        v = [int(x) for x in args.launch_shape.split(",")]
        i, sp = v[0], v[1]
        rec, nt = (v[2] if len(v) > 2 else 1), (v[3] if len(v) > 3 else 0)
        pl.set_tunable(hy.HP_TUNE_SWEEP_INTERLEAVE, i)
        pl.set_tunable(hy.HP_TUNE_SPECTRAL_THREADS, sp)
        pl.set_tunable(hy.HP_TUNE_CHARGE_RECORDS, rec)
        pl.set_tunable(hy.HP_TUNE_NONTEMPORAL, nt)
        launch = {"interleave": i, "spectral_threads": sp, "charge_records": rec,
                  "nontemporal": nt}
    elif not args.scatter_policy:
        launch, _ = autotune.tune_launch(pl, [s], gamma)
    log(f"[bench] launch shape {launch}")

    # untimed: the kernel table, a scratch slot from the current positions with events on
    # every launch
    prof = {}
    every_iter_ms = None
    eval_us = None
    if not args.no_profile:
        P = min(K, 100)
        x, y = pl.positions(s)
        t = pl.new_slot()
        pl.set_positions(t, x, y)
        pl.set_schedule(t, 1e-4, 4.0, total)
        run(t, 2)
        hy.hp_profile_enable(pl.ctx, True)
        hy.hp_profile_read(pl.ctx, reset=True)
        run(t, P)
        pl.hpwl(t)
        prof = hy.hp_profile_read(pl.ctx, reset=True)
        hy.hp_profile_enable(pl.ctx, False)
        # the same iterations with the exact HPWL after every one (for comparison)
        pl.set_positions(t, x, y)
        pl.set_schedule(t, 1e-4, 4.0, total)
        pl.iterate(t, gamma, 2, hpwl=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pl.iterate(t, gamma, P, hpwl=True)
        pl.hpwl(t)
        every_iter_ms = 1e3 * (time.perf_counter() - t1) / P
        # the evaluation alone (objective and gradient at the slot's lambda, no step): events
        # around 30 evaluations after 10 untimed ones
        lam = pl.state(t)["lambda_"]
        ev = []
        for i in range(40):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pl.eval(t, gamma, lam=lam, want_host=False)
            e1.record()
            if i >= 10:
                ev.append((e0, e1))
        torch.cuda.synchronize()
        eval_us = [1e3 * a.elapsed_time(b) for a, b in ev]
        pl.free_slot(t)
    b_eval, b_step, share = compulsory_bytes(nl)
    kernels = {k: {"launches": c, "avg_us": 1e3 * ms / max(c, 1), "total_ms": ms}
               for k, (c, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    dom = next((k for k in kernels if share.get(k, 0) > 0), None)

    # the timed region: K iterations of the placement; only the dominant kernel's launches
    # carry events
    if dom:
        hy.hp_profile_enable(pl.ctx, True, dom)
        hy.hp_profile_read(pl.ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(s, K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    live = {}
    if dom:
        live = hy.hp_profile_read(pl.ctx, reset=True)
        hy.hp_profile_enable(pl.ctx, False)
    final = pl.state(s)
    log(f"[bench] timed {K} iterations in {dt:.3f} s; HPWL {final['hpwl_q'] / 65536:.1f}")
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    roof = None
    if dom and dom in live:
        c, ms = live[dom]
        avg_s = ms * 1e-3 / max(c, 1)
        achieved = share[dom] / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic(dom, args.workload if args.locality == "rent" else nl.name),
                "kernel": dom, "compulsory_bytes_per_launch": int(share[dom]), "launches": c,
                "avg_us": round(avg_s * 1e6, 3)}
    for k, v in kernels.items():
        if share.get(k, 0) > 0:
            v["compulsory_gbs"] = round(share[k] / (v["avg_us"] * 1e-6) / 1e9, 1)
    ms_step = 1e3 * dt / K
    out = {
        "metric": METRIC, "value": round(K / dt, 2), "unit": "iter/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{nl.name}: {nl.n_movable} movable cells, {nl.n_fixed} fixed "
                               f"macros (20% of die), {nl.n_nets} nets / {nl.n_pins} pins, "
                               f"{nl.mx}x{nl.my} bins, FP32 with the int64 charge map, "
                               f"gamma = 4 bins; plain placer iterations {W}..{W + K} of a "
                               f"{total}-iteration schedule from the initial positions, the "
                               f"exact HPWL and overflow read every {HPWL_EVERY} iterations"
                               + ("; nets draw their cells from the whole index range (no "
                                  "index locality)" if args.locality == "none" else ""),
                   "global_batch": 1, "parallelism": "single-gpu"},
        "compulsory_bytes_per_iter": {"eval": b_eval, "step": b_step},
        "hbm_gbps_compulsory": round((b_eval + b_step) / (ms_step * 1e-3) / 1e9, 1),
        "hbm_frac_compulsory": round((b_eval + b_step) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "timing": ("value: wall clock of the timed iterations, GPU synchronised on both sides; "
                   "roofline: HIP events around every launch of the dominant kernel in that "
                   "region; kernels: a separate run on a scratch slot from the same positions "
                   "with events on every launch"),
        "final_hpwl": final["hpwl_q"] / 65536,
        "ms_per_step_hpwl_every_iteration": round(every_iter_ms, 5) if every_iter_ms else None,
        "eval_us": ({"mean": round(float(np.mean(eval_us)), 2),
                     "p50": round(float(np.median(eval_us)), 2), "evals": len(eval_us),
                     "warmup": 10, "note": "objective and gradient at a fixed lambda, no step; "
                                           "HIP events around each evaluation"}
                    if eval_us else None),
        "tuning": {"scatter_policy": {"regroup_every": policy[0], "deferred": policy[1]},
                   "ms_per_iter": {k: round(v, 4) for k, v in tune_ms.items()},
                   "launch_shape": {k: (v if not isinstance(v, dict) else
                                        {kk: round(vv, 4) for kk, vv in v.items()})
                                    for k, v in launch.items()}},
        "roofline": roof,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in kernels.items()},
    }
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(nl, gamma, iters=args.cpu_iters, label=args.workload)
    pl.close()
    del pl
    if args.mid_steps > 0:
        log(f"[bench] mid: {args.mid_warmup} + {args.mid_steps} iterations (Hybro round)")
        out.update(mid_lines(hy, netgen, args))
    if args.macro_steps > 0:
        log(f"[bench] movable macros: 600 + {args.macro_steps} iterations, one shuffle round")
        out["movable_macros"] = macros_run(hy, netgen, args.seed, 600, args.macro_steps)
    if args.serve_jobs > 0:
        from paper_2402_18311_amd import serve
        log(f"[bench] serving mix: {args.serve_jobs} jobs, 10 k - 2.2 M cells, 500 iterations")
        out["serving"] = serve.measure(args.serve_jobs, 10_000, 2_200_000, 500, 8.0, 0.8,
                                       args.seed, log=log)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if args.cpu_extra:
        log("[bench] timing the CPU oracle on tiny, mid and the batched round ...")
        out["cpu_extra"] = cpu_extra(netgen, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
