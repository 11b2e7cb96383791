"""ctypes front-end of the FP64 CPU oracle (hybro_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg of
the benchmark.  The device library and its Python binding never import this module.  This
file only marshals numpy arrays; every step of the arithmetic is in hybro_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hybro_oracle.c")
_LIB = os.path.join(_HERE, "liborc_hybro.so")

GAUSS, SHUFFLE, UNIFORM = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Net(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32), ("n_movable", C.c_int32), ("n_nets", C.c_int32),
        ("n_pins", C.c_int32), ("mx", C.c_int32), ("my", C.c_int32),
        ("W", C.c_double), ("H", C.c_double),
        ("cell_w", C.c_void_p), ("cell_h", C.c_void_p),
        ("fixed_x", C.c_void_p), ("fixed_y", C.c_void_p),
        ("net_start", C.c_void_p), ("pin_cell", C.c_void_p),
        ("pin_ox", C.c_void_p), ("pin_oy", C.c_void_p),
        ("net_weight", C.c_void_p), ("stretch", C.c_int32),
    ]


class _EvalParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("target_density", C.c_double),
                ("grad_mode", C.c_int32), ("fd5", C.c_int32), ("fft", C.c_int32)]


class _NestScalars(C.Structure):
    _fields_ = [("k", C.c_int32), ("a", C.c_double), ("alpha", C.c_double)]


class _NestBtScalars(C.Structure):
    _fields_ = [("k", C.c_int32), ("a", C.c_double), ("a_prev", C.c_double),
                ("alpha", C.c_double), ("rejected", C.c_int32)]


class _PlaceParams(C.Structure):
    _fields_ = [("ev", _EvalParams), ("iters", C.c_int32), ("lambda0_scale", C.c_double),
                ("lambda_decades", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P, d, i32, i64, u64 = C.c_void_p, C.c_double, C.c_int32, C.c_int64, C.c_uint64
        sig = {
            "orc_hpwl": (d, [P, P, P]),
            "orc_hpwl_q": (i64, [P, P, P, P]),
            "orc_wa_literal": (d, [P, C.c_int, d]),
            "orc_wa_net_axis": (d, [P, C.c_int, d, P]),
            "orc_wa": (d, [P, P, P, d, P, P, P]),
            "orc_density_q": (None, [P, P, P, P, P]),
            "orc_total_charge_q": (i64, [P]),
            "orc_overflow": (d, [P, P, P, d, P]),
            "orc_density_float": (None, [P, P, P, P]),
            "orc_dct2_brute": (None, [C.c_int, C.c_int, P, P]),
            "orc_dct2": (None, [C.c_int, C.c_int, P, P]),
            "orc_dct2_fft": (None, [C.c_int, C.c_int, P, P]),
            "orc_synth2": (None, [C.c_int, C.c_int, P, C.c_int, C.c_int, P]),
            "orc_poisson": (d, [C.c_int, C.c_int, d, d, P, C.c_int, C.c_int, P, P, P, P]),
            "orc_density_grad_field": (None, [P, P, P, P, P, P, P]),
            "orc_density_grad_exact": (None, [P, P, P, P, P, P]),
            "orc_density_energy_float": (d, [P, P, P, C.c_int]),
            "orc_eval": (None, [P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]),
            "orc_nesterov_step": (None, [P, d, P, P, P, P, P, P]),
            "orc_nesterov_step_bt": (None, [P, d, P, P, P, P, P, P, P]),
            "orc_lambda_ratio": (d, [d, C.c_int]),
            "orc_place": (None, [P, P, P, P, P, P, P, P]),
            "orc_splitmix": (u64, [u64, u64]),
            "orc_shuffle_perm": (u64, [u64, u64, u64]),
            "orc_perturb": (i32, [P, P, P, C.c_int, d, d, u64, P]),
            "orc_perturb_among": (i32, [P, P, P, C.c_int, d, d, u64, P, i32, P]),
            "orc_wiremask": (i32, [P, P, P, P, i32]),
            "orc_argmin_i64": (i32, [P, i32]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """The oracle bound to one netlist (a paper_2402_18311_amd.netgen.Netlist or lookalike)."""

    def __init__(self, nl, stretch: bool = True, net_weight=None):
        self.nl = nl
        self._keep = [
            _f64(nl.cell_w), _f64(nl.cell_h), _f64(nl.fixed_x), _f64(nl.fixed_y),
            np.ascontiguousarray(nl.net_start, dtype=np.int32),
            np.ascontiguousarray(nl.pin_cell, dtype=np.int32),
            _f64(nl.pin_ox), _f64(nl.pin_oy),
            None if net_weight is None else _f64(net_weight),
        ]
        k = self._keep
        self.net = _Net(nl.n_cells, nl.n_movable, len(k[4]) - 1, len(k[5]), nl.mx, nl.my,
                        float(nl.W), float(nl.H), _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]),
                        _p(k[4]), _p(k[5]), _p(k[6]), _p(k[7]), _p(k[8]), int(stretch))
        self.nb = nl.mx * nl.my
        self.L = lib()

    @property
    def ref(self):
        return C.byref(self.net)

    # -- Eq. 1 --------------------------------------------------------------------------
    def hpwl(self, x, y) -> float:
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y = _f64(x), _f64(y)
        return self.L.orc_hpwl(self.ref, _p(x), _p(y))

    def hpwl_q(self, x, y, per_net=False):
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y = _f64(x), _f64(y)
        pn = np.zeros(self.net.n_nets, dtype=np.int64) if per_net else None
        t = self.L.orc_hpwl_q(self.ref, _p(x), _p(y), _p(pn))
        return (t, pn) if per_net else t

    # -- Eq. 3 --------------------------------------------------------------------------
    def wa(self, x, y, gamma, per_net=False):
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y = _f64(x), _f64(y)
        N = self.nl.n_movable
        gx, gy = np.zeros(N), np.zeros(N)
        pn = np.zeros(self.net.n_nets) if per_net else None
        wl = self.L.orc_wa(self.ref, _p(x), _p(y), float(gamma), _p(gx), _p(gy),
                           _p(pn))
        return (wl, gx, gy, pn) if per_net else (wl, gx, gy)

    # -- density ------------------------------------------------------------------------
    def density_q(self, x, y):
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y = _f64(x), _f64(y)
        rm = np.zeros(self.nb, dtype=np.int64)
        rf = np.zeros(self.nb, dtype=np.int64)
        self.L.orc_density_q(self.ref, _p(x), _p(y), _p(rm), _p(rf))
        return rm.reshape(self.nl.my, self.nl.mx), rf.reshape(self.nl.my, self.nl.mx)

    def total_charge_q(self) -> int:
        return int(self.L.orc_total_charge_q(self.ref))

    def overflow(self, rho_mov, rho_fixed, target_density=1.0):
        num = C.c_int64(0)
        rm = np.ascontiguousarray(rho_mov, dtype=np.int64)
        rf = np.ascontiguousarray(rho_fixed, dtype=np.int64)
        v = self.L.orc_overflow(self.ref, _p(rm), _p(rf), float(target_density), C.byref(num))
        return v, num.value

    def density_float(self, x, y):
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y = _f64(x), _f64(y)
        rho = np.zeros(self.nb)
        self.L.orc_density_float(self.ref, _p(x), _p(y), _p(rho))
        return rho.reshape(self.nl.my, self.nl.mx)

    def grad_field(self, x, y, ex, ey):
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y, ex, ey = _f64(x), _f64(y), _f64(ex), _f64(ey)
        N = self.nl.n_movable
        gx, gy = np.zeros(N), np.zeros(N)
        self.L.orc_density_grad_field(self.ref, _p(x), _p(y), _p(ex),
                                      _p(ey), _p(gx), _p(gy))
        return gx, gy

    def grad_exact(self, x, y, psi):
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y, psi = _f64(x), _f64(y), _f64(psi)
        N = self.nl.n_movable
        gx, gy = np.zeros(N), np.zeros(N)
        self.L.orc_density_grad_exact(self.ref, _p(x), _p(y), _p(psi),
                                      _p(gx), _p(gy))
        return gx, gy

    def energy_float(self, x, y, fd5=False):
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y = _f64(x), _f64(y)
        return self.L.orc_density_energy_float(self.ref, _p(x), _p(y), int(fd5))

    # -- objective ----------------------------------------------------------------------
    def eval(self, x, y, gamma, target_density=1.0, grad_mode=0, fd5=False, maps=False,
             fft=False):
        """fft: the Poisson solve's transforms through the FFT path (same values to rounding;
        used for timing) instead of the plain cosine sums."""
        # float64 copies held for the duration of the call (ctypes keeps only addresses)
        x, y = _f64(x), _f64(y)
        N = self.nl.n_movable
        nb = self.nb
        pr = _EvalParams(float(gamma), float(target_density), int(grad_mode), int(fd5),
                         int(fft))
        wl, en, ov, on = C.c_double(), C.c_double(), C.c_double(), C.c_int64()
        gwx, gwy, gdx, gdy = (np.zeros(N) for _ in range(4))
        rm = np.zeros(nb, dtype=np.int64) if maps else None
        rf = np.zeros(nb, dtype=np.int64) if maps else None
        psi, ex, ey = ((np.zeros(nb) for _ in range(3)) if maps else (None, None, None))
        self.L.orc_eval(self.ref, _p(x), _p(y), C.byref(pr), C.byref(wl),
                        C.byref(en), C.byref(ov), C.byref(on), _p(gwx), _p(gwy), _p(gdx),
                        _p(gdy), _p(rm), _p(rf), _p(psi), _p(ex), _p(ey))
        out = dict(wl=wl.value, energy=en.value, overflow=ov.value, overflow_num=on.value,
                   gwx=gwx, gwy=gwy, gdx=gdx, gdy=gdy)
        if maps:
            sh = (self.nl.my, self.nl.mx)
            out.update(rho_mov=rm.reshape(sh), rho_fixed=rf.reshape(sh), psi=psi.reshape(sh),
                       ex=ex.reshape(sh), ey=ey.reshape(sh))
        return out

    def nesterov_step(self, lam, g, state):
        """state: dict u, v, v_prev, gp_prev ([2N] float64 each), k, a, alpha (mutated)."""
        s = _NestScalars(int(state["k"]), float(state["a"]), float(state["alpha"]))
        g = _f64(g)
        self.L.orc_nesterov_step(self.ref, float(lam), _p(g), _p(state["u"]), _p(state["v"]),
                                 _p(state["v_prev"]), _p(state["gp_prev"]), C.byref(s))
        state.update(k=s.k, a=s.a, alpha=s.alpha)
        return state

    def nesterov_step_bt(self, lam, g, state):
        """The step with backtracking; state as new_state(..., backtracking=True) (mutated);
        returns whether the step was rejected and redone."""
        s = _NestBtScalars(int(state["k"]), float(state["a"]), float(state["a_prev"]),
                           float(state["alpha"]), 0)
        g = _f64(g)
        self.L.orc_nesterov_step_bt(self.ref, float(lam), _p(g), _p(state["u"]), _p(state["v"]),
                                    _p(state["v_prev"]), _p(state["gp_prev"]),
                                    _p(state["u_prev"]), C.byref(s))
        state.update(k=s.k, a=s.a, a_prev=s.a_prev, alpha=s.alpha)
        return bool(s.rejected)

    @staticmethod
    def new_state(x, y):
        u = np.concatenate([_f64(x), _f64(y)])
        return dict(u=u.copy(), v=u.copy(), v_prev=u.copy(), gp_prev=np.zeros_like(u), k=0,
                    a=1.0, alpha=0.0, u_prev=u.copy(), a_prev=1.0)

    def lambda_ratio(self, decades, iters):
        return self.L.orc_lambda_ratio(float(decades), int(iters))

    def place(self, x, y, iters, gamma, lambda0_scale, lambda_decades, target_density=1.0,
              grad_mode=0, fd5=False, fft=False):
        x = _f64(x).copy()
        y = _f64(y).copy()
        pp = _PlaceParams(_EvalParams(float(gamma), float(target_density), int(grad_mode),
                                      int(fd5), int(fft)), int(iters), float(lambda0_scale),
                          float(lambda_decades))
        hp = np.zeros(iters, dtype=np.int64)
        wl = np.zeros(iters)
        ov = np.zeros(iters)
        lam = np.zeros(iters)
        self.L.orc_place(self.ref, C.byref(pp), _p(x), _p(y), _p(hp), _p(wl), _p(ov), _p(lam))
        return x, y, dict(hpwl_q=hp, wl=wl, overflow=ov, lam=lam)

    # -- perturbation -------------------------------------------------------------------
    def perturb(self, x, y, mode, fraction, sigma_bins, seed):
        x = _f64(x).copy()
        y = _f64(y).copy()
        idx = np.zeros(max(1, self.nl.n_movable), dtype=np.int32)
        m = self.L.orc_perturb(self.ref, _p(x), _p(y), int(mode), float(fraction),
                               float(sigma_bins), C.c_uint64(seed & (2**64 - 1)).value, _p(idx))
        return x, y, idx[:m].copy()

    def wiremask(self, x, y, macros):
        """WireMask perturbation of the listed macros, in order; returns (x, y, moved)."""
        x = _f64(x).copy()
        y = _f64(y).copy()
        macros = np.ascontiguousarray(macros, dtype=np.int32)
        moved = self.L.orc_wiremask(self.ref, _p(x), _p(y), _p(macros), len(macros))
        return x, y, moved

    def perturb_among(self, x, y, mode, fraction, sigma_bins, seed, cells):
        """Perturbation restricted to the distinct movable cells `cells` (e.g. the macros)."""
        x = _f64(x).copy()
        y = _f64(y).copy()
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        idx = np.zeros(max(1, self.nl.n_movable), dtype=np.int32)
        m = self.L.orc_perturb_among(self.ref, _p(x), _p(y), int(mode), float(fraction),
                                     float(sigma_bins), C.c_uint64(seed & (2**64 - 1)).value,
                                     _p(cells), len(cells), _p(idx))
        return x, y, idx[:m].copy()


# -- grid-level functions (no netlist) ----------------------------------------------------
def dct2(rho, brute=False, fft=False):
    """Cosine coefficients a_uv: the O(M^4) double sum (brute), the FFT path (fft), or the
    two 1-D cosine sums (default)."""
    rho = _f64(rho)
    my, mx = rho.shape
    a = np.zeros_like(rho)
    f = lib().orc_dct2_brute if brute else (lib().orc_dct2_fft if fft else lib().orc_dct2)
    f(mx, my, _p(rho), _p(a))
    return a


def synth2(A, mode=0, fft=False):
    """sum_uv A_vu Bx(u, j) By(v, k); mode 0 cos-cos, 1 sin-cos, 2 cos-sin (x-y)."""
    A = _f64(A)
    my, mx = A.shape
    out = np.zeros_like(A)
    lib().orc_synth2(mx, my, _p(A), int(mode), int(fft), _p(out))
    return out


def poisson(rho_bar, W, H, fd5=False, fft=False):
    rho_bar = _f64(rho_bar)
    my, mx = rho_bar.shape
    a, psi, ex, ey = (np.zeros_like(rho_bar) for _ in range(4))
    e = lib().orc_poisson(mx, my, float(W), float(H), _p(rho_bar), int(fd5), int(fft), _p(a),
                          _p(psi), _p(ex), _p(ey))
    return dict(energy=e, a=a, psi=psi, ex=ex, ey=ey)


def wa_net_axis(px, gamma, grad=True):
    px = _f64(px)
    g = np.zeros_like(px) if grad else None
    v = lib().orc_wa_net_axis(_p(px), len(px), float(gamma), _p(g))
    return (v, g) if grad else v


def wa_literal(px, gamma):
    px = _f64(px)
    return lib().orc_wa_literal(_p(px), len(px), float(gamma))


def splitmix(seed, i):
    return int(lib().orc_splitmix(seed & (2**64 - 1), i))


def shuffle_perm(j, m, seed):
    return int(lib().orc_shuffle_perm(j, m, seed & (2**64 - 1)))


def num_threads():
    return int(lib().orc_num_threads())


def set_threads(n):
    """Thread count of the oracle's later parallel loops (timing only)."""
    lib().orc_set_threads(int(n))


def argmin_i64(v):
    v = np.ascontiguousarray(v, dtype=np.int64)
    return int(lib().orc_argmin_i64(_p(v), len(v)))
