"""Python binding of libhybro (the C ABI of include/hybro.h).

The hp_* functions below have the C names and only marshal arguments; every step of the
placer runs in the library's HIP kernels.  PyTorch provides the device memory (uint8 tensors
lent to the library) and the stream.  There is no fallback: if libhybro.so is missing or no
GPU is present, these calls raise.

`Placer` is a convenience owner of one netlist and its slots.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhybro.so")

HP_OK, HP_EINVAL, HP_ENOMEM, HP_EDEVICE, HP_ESTATE, HP_ENOTIMPL = 0, -1, -2, -3, -4, -5
HP_PERTURB_GAUSS, HP_PERTURB_SHUFFLE, HP_PERTURB_UNIFORM = 0, 1, 2
HP_MAP_RHO_MOV, HP_MAP_RHO_FIXED, HP_MAP_PSI, HP_MAP_EX, HP_MAP_EY = 0, 1, 2, 3, 4
HP_ITER_HPWL, HP_ITER_GRAPH, HP_ITER_HPWL_LAST = 1, 2, 4
HP_GRAD_FIELD, HP_GRAD_EXACT, HP_GRAD_DENSITY_ONLY = 0, 1, 2
HP_TUNE_FUSED_STEP_PARTS, HP_TUNE_SPECTRAL_THREADS, HP_TUNE_SWEEP_INTERLEAVE = 0, 1, 2
HP_TUNE_CHARGE_RECORDS, HP_TUNE_NONTEMPORAL = 3, 4


class hp_die(C.Structure):
    _fields_ = [("W", C.c_double), ("H", C.c_double), ("mx", C.c_int32), ("my", C.c_int32),
                ("target_density", C.c_double), ("stretch", C.c_int32), ("fd5", C.c_int32)]


class hp_shape(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_movable", C.c_int32), ("n_nets", C.c_int32),
                ("n_pins", C.c_int32)]


class hp_eval_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("lambda_", C.c_double), ("grad_mode", C.c_int32),
                ("keep_maps", C.c_int32)]


class hp_iter_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("flags", C.c_int32)]


class hp_slot_state(C.Structure):
    _fields_ = [("k", C.c_int64), ("hpwl_q", C.c_int64), ("overflow_num", C.c_int64),
                ("a", C.c_double), ("alpha", C.c_double), ("lambda_", C.c_double),
                ("wl", C.c_double), ("energy", C.c_double), ("overflow", C.c_double),
                ("rejects", C.c_int64)]


class HybroError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhybro error {code}: {msg}")
        self.code = code


_lib = None
_P = C.c_void_p
_SIGS = {
    "hp_create": [C.POINTER(_P), C.c_int, _P, C.c_int],
    "hp_destroy": [_P],
    "hp_last_error": [],
    "hp_netlist_bytes": [_P, C.POINTER(hp_shape), C.POINTER(hp_die)],
    "hp_slot_bytes": [_P, C.POINTER(hp_shape), C.POINTER(hp_die)],
    "hp_load_netlist_csr": [_P, C.POINTER(hp_shape), C.POINTER(hp_die), _P, _P, _P, _P, _P, _P,
                            _P, _P, _P, _P, C.c_size_t, C.POINTER(C.c_int32)],
    "hp_slot_alloc": [_P, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_int32)],
    "hp_slot_free": [_P, C.c_int32],
    "hp_netlist_free": [_P, C.c_int32],
    "hp_set_positions": [_P, C.c_int32, _P, _P, C.c_int],
    "hp_get_positions": [_P, C.c_int32, _P, _P, C.c_int],
    "hp_get_eval_positions": [_P, C.c_int32, _P, _P, C.c_int],
    "hp_set_schedule": [_P, C.c_int32, C.c_double, C.c_double, C.c_int32],
    "hp_set_lambda_ratio": [_P, C.c_int32, C.c_double],
    "hp_set_backtracking": [_P, C.c_int32, C.c_int32],
    "hp_overflow_of_cells": [_P, C.c_int32, C.c_int32, _P, _P],
    "hp_perturb_wiremask": [_P, C.c_int32, _P, C.c_int32, _P],
    "hp_set_scatter_policy": [_P, C.c_int32, C.c_int32, C.c_int32],
    "hp_get_scatter_policy": [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
    "hp_set_tunable": [_P, C.c_int32, C.c_int32, C.c_int32],
    "hp_get_tunable": [_P, C.c_int32, C.c_int32, C.POINTER(C.c_int32)],
    "hp_eval_objective_grad": [_P, _P, C.c_int32, C.POINTER(hp_eval_params), _P, _P, _P, _P, _P],
    "hp_nesterov_step": [_P, _P, C.c_int32],
    "hp_iterate": [_P, _P, C.c_int32, C.POINTER(hp_iter_params), C.c_int32],
    "hp_graph_stats": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "hp_iterate_multi": [_P, _P, C.c_int32, _P, C.c_int32, C.c_int32],
    "hp_perturb": [_P, C.c_int32, C.c_int, C.c_double, C.c_double, C.c_uint64, _P, _P],
    "hp_perturb_among": [_P, C.c_int32, C.c_int, C.c_double, C.c_double, C.c_uint64, _P,
                         C.c_int32, _P, _P],
    "hp_hpwl": [_P, _P, C.c_int32, _P, _P],
    "hp_hpwl_noalloc": [_P, C.c_int32, _P, _P],
    "hp_select_best": [_P, _P, C.c_int32, C.c_int32, _P],
    "hp_get_map": [_P, C.c_int32, C.c_int, _P],
    "hp_get_state": [_P, C.c_int32, C.POINTER(hp_slot_state)],
    "hp_profile_enable": [_P, C.c_int, C.c_char_p],
    "hp_profile_read": [_P, _P, C.c_int32, C.POINTER(C.c_int32), C.c_int],
}


class hp_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("count", C.c_int64), ("total_ms", C.c_double)]


def hp_profile_enable(ctx, on, only_kernel=None):
    _chk(lib().hp_profile_enable(ctx, int(on), None if only_kernel is None else only_kernel.encode()))


def hp_profile_read(ctx, reset=True):
    """{kernel name: (launches, total ms)} accumulated since the last read."""
    n = C.c_int32()
    _chk(lib().hp_profile_read(ctx, None, 0, C.byref(n), 0))
    arr = (hp_kernel_time * max(1, n.value))()
    _chk(lib().hp_profile_read(ctx, arr, n.value, C.byref(n), int(reset)))
    return {arr[i].name.decode(): (arr[i].count, arr[i].total_ms) for i in range(n.value)}


def lib():
    """Load libhybro.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2402_18311_amd.build`")
        # torch first: it brings its own HIP runtime (soname libamdhip64.so.7), and the library
        # must bind to that same runtime rather than load a second one from the ROCm install
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.hp_last_error.restype = C.c_char_p
        L.hp_netlist_bytes.restype = C.c_size_t
        L.hp_slot_bytes.restype = C.c_size_t
        # the HIP runtime the library binds to, for OwnStream
        L.hipStreamCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
        L.hipStreamSynchronize.argtypes = [C.c_void_p]
        L.hipStreamDestroy.argtypes = [C.c_void_p]
        for f in (L.hipStreamCreateWithFlags, L.hipStreamSynchronize, L.hipStreamDestroy):
            f.restype = C.c_int
        _lib = L
    return _lib


class OwnStream:
    """A HIP stream created for one placer or context and destroyed by close().

    torch.cuda.Stream() hands out streams round-robin from a fixed pool per device, so placers
    created far enough apart (a serving loop with many jobs in flight) can be given the same
    stream, and one placer's graph capture then meets the other's work on it.  This stream
    belongs to its user alone: default priority, non-blocking with respect to the null stream
    as torch's are, created through the HIP runtime that the library itself calls.  The owner
    closes it after the placer or context that uses it."""

    def __init__(self, device=0):
        import torch
        h = C.c_void_p()
        with torch.cuda.device(device):
            rc = lib().hipStreamCreateWithFlags(C.byref(h), 1)  # hipStreamNonBlocking
        if rc != 0 or not h.value:
            raise HybroError(HP_EDEVICE, f"hipStreamCreateWithFlags returned {rc}")
        self.device = device
        self.cuda_stream = h.value

    def close(self):
        if self.cuda_stream:
            h, self.cuda_stream = C.c_void_p(self.cuda_stream), 0
            rc = lib().hipStreamSynchronize(h)
            rc2 = lib().hipStreamDestroy(h)
            if rc or rc2:
                raise HybroError(HP_EDEVICE, f"stream sync/destroy returned {rc}/{rc2}")


def _chk(rc):
    if rc != HP_OK:
        raise HybroError(rc, lib().hp_last_error().decode())
    return rc


def _ptr(a):
    """Address of a numpy array, a torch tensor, or None."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


# ---- C-ABI functions (same names) -----------------------------------------------------------
def hp_create(device=0, stream=None, precision=32):
    ctx = _P()
    _chk(lib().hp_create(C.byref(ctx), device, stream, precision))
    return ctx


def hp_destroy(ctx):
    _chk(lib().hp_destroy(ctx))


def hp_last_error():
    return lib().hp_last_error().decode()


def hp_netlist_bytes(ctx, shape, die):
    return lib().hp_netlist_bytes(ctx, C.byref(shape), C.byref(die))


def hp_slot_bytes(ctx, shape, die):
    return lib().hp_slot_bytes(ctx, C.byref(shape), C.byref(die))


def hp_load_netlist_csr(ctx, shape, die, cell_w, cell_h, fixed_x, fixed_y, net_start, pin_cell,
                        pin_ox, pin_oy, net_weight, dev_buf, dev_bytes):
    out = C.c_int32()
    _chk(lib().hp_load_netlist_csr(ctx, C.byref(shape), C.byref(die), _ptr(cell_w), _ptr(cell_h),
                                   _ptr(fixed_x), _ptr(fixed_y), _ptr(net_start), _ptr(pin_cell),
                                   _ptr(pin_ox), _ptr(pin_oy), _ptr(net_weight), dev_buf,
                                   dev_bytes, C.byref(out)))
    return out.value


def hp_slot_alloc(ctx, netlist, dev_buf, dev_bytes):
    out = C.c_int32()
    _chk(lib().hp_slot_alloc(ctx, netlist, dev_buf, dev_bytes, C.byref(out)))
    return out.value


def hp_slot_free(ctx, slot):
    _chk(lib().hp_slot_free(ctx, slot))


def hp_netlist_free(ctx, netlist):
    _chk(lib().hp_netlist_free(ctx, netlist))


def hp_set_positions(ctx, slot, x, y, on_device):
    _chk(lib().hp_set_positions(ctx, slot, _ptr(x), _ptr(y), int(on_device)))


def hp_get_positions(ctx, slot, x, y, on_device):
    _chk(lib().hp_get_positions(ctx, slot, _ptr(x), _ptr(y), int(on_device)))


def hp_get_eval_positions(ctx, slot, x, y, on_device):
    _chk(lib().hp_get_eval_positions(ctx, slot, _ptr(x), _ptr(y), int(on_device)))


def hp_set_lambda_ratio(ctx, slot, ratio):
    _chk(lib().hp_set_lambda_ratio(ctx, slot, float(ratio)))


def hp_set_backtracking(ctx, slot, on):
    _chk(lib().hp_set_backtracking(ctx, slot, int(bool(on))))


def wiremask_order(nl):
    """The movable macros by decreasing area, ties by id (the order of the WireMask pass)."""
    m = np.asarray(nl.macros if nl.macros is not None else [], dtype=np.int64)
    area = nl.cell_w[m] * nl.cell_h[m]
    return m[np.lexsort((m, -area))].astype(np.int32)


def hp_perturb_wiremask(ctx, slot, macros):
    """WireMask pass over `macros` (distinct movable ids, in pass order); returns the number
    of macros that moved."""
    macros = np.ascontiguousarray(macros, dtype=np.int32)
    moved = C.c_int32()
    _chk(lib().hp_perturb_wiremask(ctx, slot, _ptr(macros) if len(macros) else None, len(macros),
                                   C.byref(moved)))
    return moved.value


def hp_overflow_of_cells(ctx, slot, n_counted):
    """(numerator, overflow) of the charge of movable cells [0, n_counted) at v."""
    num = C.c_int64()
    ov = C.c_double()
    _chk(lib().hp_overflow_of_cells(ctx, slot, int(n_counted), C.byref(num), C.byref(ov)))
    return num.value, ov.value


def hp_set_scatter_policy(ctx, netlist, regroup_every, deferred):
    _chk(lib().hp_set_scatter_policy(ctx, netlist, int(regroup_every), int(bool(deferred))))


def hp_get_scatter_policy(ctx, netlist):
    r, d = C.c_int32(), C.c_int32()
    _chk(lib().hp_get_scatter_policy(ctx, netlist, C.byref(r), C.byref(d)))
    return int(r.value), bool(d.value)


def hp_set_tunable(ctx, netlist, which, value):
    _chk(lib().hp_set_tunable(ctx, netlist, int(which), int(value)))


def hp_get_tunable(ctx, netlist, which):
    v = C.c_int32()
    _chk(lib().hp_get_tunable(ctx, netlist, int(which), C.byref(v)))
    return int(v.value)


def hp_set_schedule(ctx, slot, lambda0_scale, decades, total_iters):
    _chk(lib().hp_set_schedule(ctx, slot, lambda0_scale, decades, total_iters))


def _slots(slots):
    a = np.ascontiguousarray(np.atleast_1d(slots), dtype=np.int32)
    return a, a.ctypes.data, len(a)


def hp_eval_objective_grad(ctx, slots, gamma, lam=-1.0, grad_mode=0, keep_maps=False,
                           want_host=True, grad_x=None, grad_y=None):
    a, p, n = _slots(slots)
    prm = hp_eval_params(float(gamma), float(lam), int(grad_mode), int(keep_maps))
    wl = np.zeros(n) if want_host else None
    en = np.zeros(n) if want_host else None
    ov = np.zeros(n) if want_host else None
    _chk(lib().hp_eval_objective_grad(ctx, p, n, C.byref(prm), _ptr(wl), _ptr(en), _ptr(ov),
                                      _ptr(grad_x), _ptr(grad_y)))
    return (wl, en, ov) if want_host else None


def hp_nesterov_step(ctx, slots):
    a, p, n = _slots(slots)
    _chk(lib().hp_nesterov_step(ctx, p, n))


def hp_iterate(ctx, slots, gamma, iters, flags):
    a, p, n = _slots(slots)
    prm = hp_iter_params(float(gamma), int(flags))
    _chk(lib().hp_iterate(ctx, p, n, C.byref(prm), int(iters)))


def hp_iterate_multi(ctx, slots, gammas, iters, flags):
    a, p, n = _slots(slots)
    g = np.ascontiguousarray(np.broadcast_to(np.asarray(gammas, dtype=np.float64), (n,)))
    _chk(lib().hp_iterate_multi(ctx, p, n, g.ctypes.data, int(flags), int(iters)))


def hp_graph_stats(ctx):
    """(captured blocks, replayed blocks) of hp_iterate's graph mode on this context."""
    c, r = C.c_int64(), C.c_int64()
    _chk(lib().hp_graph_stats(ctx, C.byref(c), C.byref(r)))
    return int(c.value), int(r.value)


def hp_perturb(ctx, slot, mode, fraction, sigma_bins, seed, n_movable, want_idx=True):
    """Returns the moved cells' indices (ascending), or their count if want_idx is False."""
    cnt = C.c_int32()
    buf = np.zeros(max(1, n_movable), dtype=np.int32) if want_idx else None
    _chk(lib().hp_perturb(ctx, slot, int(mode), float(fraction), float(sigma_bins),
                          C.c_uint64(int(seed) & (2**64 - 1)), _ptr(buf), C.byref(cnt)))
    return buf[: cnt.value].copy() if want_idx else cnt.value


def hp_perturb_among(ctx, slot, mode, fraction, sigma_bins, seed, cells, n_movable,
                     want_idx=True):
    """hp_perturb over the pool `cells` (distinct movable ids, e.g. the macros)."""
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    cnt = C.c_int32()
    buf = np.zeros(max(1, n_movable), dtype=np.int32) if want_idx else None
    _chk(lib().hp_perturb_among(ctx, slot, int(mode), float(fraction), float(sigma_bins),
                                C.c_uint64(int(seed) & (2**64 - 1)), _ptr(cells), len(cells),
                                _ptr(buf), C.byref(cnt)))
    return buf[: cnt.value].copy() if want_idx else cnt.value


def hp_hpwl(ctx, slots, want_host=True):
    a, p, n = _slots(slots)
    q = np.zeros(n, dtype=np.int64) if want_host else None
    _chk(lib().hp_hpwl(ctx, p, n, _ptr(q), None))
    return q


def hp_hpwl_noalloc(ctx, netlist, xy, out_q):
    """Exact HPWL of device pairs xy [n_cells, 2] into device int64 out_q [1] (no slot, no
    allocation; the library's static scratch holds the partial sums)."""
    _chk(lib().hp_hpwl_noalloc(ctx, int(netlist), _ptr(xy), _ptr(out_q)))


def hp_select_best(ctx, slots, incumbent, want_host=True):
    a, p, n = _slots(slots)
    out = C.c_int32(-2)
    _chk(lib().hp_select_best(ctx, p, n, incumbent, C.byref(out) if want_host else None))
    return out.value if want_host else None


def hp_get_map(ctx, slot, which, shape, dtype):
    dst = np.zeros(shape, dtype=dtype)
    _chk(lib().hp_get_map(ctx, slot, int(which), dst.ctypes.data))
    return dst


def hp_get_state(ctx, slot):
    s = hp_slot_state()
    _chk(lib().hp_get_state(ctx, slot, C.byref(s)))
    return {f: getattr(s, f) for f, _ in hp_slot_state._fields_}


# ---- convenience owner -----------------------------------------------------------------------
class Placer:
    """One netlist on the GPU with any number of slots (placement instances).

    Buffers are torch uint8 tensors on `device`; the library runs on `stream` (any object with
    a `cuda_stream` handle), by default torch's current stream of that device at construction
    time.  Placers in use at the same time from different threads each need a stream no other
    placer uses: an OwnStream, not torch.cuda.Stream(), whose pooled streams repeat."""

    def __init__(self, nl, precision=32, device=0, stretch=True, fd5=False,
                 target_density=1.0, net_weight=None, stream=None, context=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libhybro needs a ROCm GPU; none is visible")
        self.torch = torch
        self.nl = nl
        self.context = context
        if context is not None:  # a netlist of a shared context (its precision, device, stream)
            precision, self.dev, self.stream = context.precision, context.dev, context.stream
        else:
            self.dev = torch.device("cuda", device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.precision = precision
        self.dtype = np.float32 if precision == 32 else np.float64
        self.tdtype = torch.float32 if precision == 32 else torch.float64
        self.ctx = (context.ctx if context is not None else
                    hp_create(self.dev.index or 0, C.c_void_p(self.stream.cuda_stream), precision))
        try:
            self._load(nl, target_density, stretch, fd5, net_weight)
        except BaseException:
            if context is None:
                hp_destroy(self.ctx)  # a refused netlist leaves no context behind
            self.ctx = None
            raise

    def _load(self, nl, target_density, stretch, fd5, net_weight):
        self.shape = hp_shape(nl.n_cells, nl.n_movable, int(len(nl.net_start) - 1),
                              int(len(nl.pin_cell)))
        self.die = hp_die(float(nl.W), float(nl.H), int(nl.mx), int(nl.my),
                          float(target_density), int(stretch), int(fd5))
        nb = hp_netlist_bytes(self.ctx, self.shape, self.die)
        if nb == 0:
            raise HybroError(HP_EINVAL, hp_last_error())
        self._netbuf = self._alloc(nb)
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)  # noqa: E731
        self._keep = [f64(nl.cell_w), f64(nl.cell_h), f64(nl.fixed_x), f64(nl.fixed_y),
                      i32(nl.net_start), i32(nl.pin_cell), f64(nl.pin_ox), f64(nl.pin_oy),
                      None if net_weight is None else f64(net_weight)]
        k = self._keep
        self.netlist = hp_load_netlist_csr(self.ctx, self.shape, self.die, *k,
                                           self._netbuf.data_ptr(), nb)
        self.slot_bytes = hp_slot_bytes(self.ctx, self.shape, self.die)
        self._slotbufs = {}

    def _alloc(self, nbytes):
        t = self.torch.empty(int(nbytes) + 256, dtype=self.torch.uint8, device=self.dev)
        off = (-t.data_ptr()) % 256
        return t[off: off + int(nbytes)]

    def new_slot(self):
        buf = self._alloc(self.slot_bytes)
        s = hp_slot_alloc(self.ctx, self.netlist, buf.data_ptr(), self.slot_bytes)
        self._slotbufs[s] = buf
        return s

    def free_slot(self, s):
        hp_slot_free(self.ctx, s)
        self._slotbufs.pop(s, None)

    def set_positions(self, s, x, y):
        if isinstance(x, np.ndarray):
            hp_set_positions(self.ctx, s, np.ascontiguousarray(x, self.dtype),
                             np.ascontiguousarray(y, self.dtype), False)
        else:
            hp_set_positions(self.ctx, s, x.contiguous(), y.contiguous(), True)

    def positions(self, s):
        x = np.zeros(self.nl.n_movable, self.dtype)
        y = np.zeros(self.nl.n_movable, self.dtype)
        hp_get_positions(self.ctx, s, x, y, False)
        return x, y

    def eval_positions(self, s):
        """The look-ahead point v where the next evaluation is taken."""
        x = np.zeros(self.nl.n_movable, self.dtype)
        y = np.zeros(self.nl.n_movable, self.dtype)
        hp_get_eval_positions(self.ctx, s, x, y, False)
        return x, y

    def set_schedule(self, s, lambda0_scale=1e-4, decades=4.0, total_iters=1000):
        hp_set_schedule(self.ctx, s, lambda0_scale, decades, total_iters)

    def wiremask(self, s, macros=None):
        """WireMask perturbation of slot s over `macros` (default: the netlist's movable
        macros, largest area first, ties by id); returns how many moved."""
        if macros is None:
            macros = wiremask_order(self.nl)
        return hp_perturb_wiremask(self.ctx, s, macros)

    def overflow_of_cells(self, s, n_counted=None):
        """Overflow of the first n_counted movable cells (default: all but the fillers)."""
        if n_counted is None:
            n_counted = self.nl.n_movable - getattr(self.nl, "n_fillers", 0)
        return hp_overflow_of_cells(self.ctx, s, n_counted)

    def set_backtracking(self, s, on=True):
        """ePlace backtracking of the Nesterov step for slot s (see hybro.h)."""
        hp_set_backtracking(self.ctx, s, on)

    def eval(self, slots, gamma, lam=-1.0, keep_maps=False, grads=False, want_host=True,
             grad_mode=0):
        slots = list(np.atleast_1d(slots))
        gx = gy = None
        if grads:
            gx = self.torch.empty((len(slots), self.nl.n_movable), dtype=self.tdtype, device=self.dev)
            gy = self.torch.empty_like(gx)
        r = hp_eval_objective_grad(self.ctx, slots, gamma, lam, grad_mode, keep_maps, want_host,
                                   gx, gy)
        if grads:
            return r, gx, gy
        return r

    def step(self, slots):
        hp_nesterov_step(self.ctx, list(np.atleast_1d(slots)))

    def hpwl(self, slots, want_host=True):
        return hp_hpwl(self.ctx, list(np.atleast_1d(slots)), want_host)

    def perturb(self, s, mode, fraction, sigma_bins, seed, want_idx=True, cells=None):
        """Perturb slot s; with `cells`, only among those movable cells (e.g. the macros)."""
        if cells is not None:
            return hp_perturb_among(self.ctx, s, mode, fraction, sigma_bins, seed, cells,
                                    self.nl.n_movable, want_idx)
        return hp_perturb(self.ctx, s, mode, fraction, sigma_bins, seed, self.nl.n_movable,
                          want_idx)

    def select_best(self, slots, incumbent, want_host=True):
        return hp_select_best(self.ctx, list(np.atleast_1d(slots)), incumbent, want_host)

    def map(self, s, which):
        sh = (self.nl.my, self.nl.mx)
        dt = np.int64 if which in (HP_MAP_RHO_MOV, HP_MAP_RHO_FIXED) else self.dtype
        return hp_get_map(self.ctx, s, which, sh, dt)

    def state(self, s):
        return hp_get_state(self.ctx, s)

    def set_scatter_policy(self, regroup_every=4, deferred=True):
        """Grouping policy of the charge scatter for every slot (speed only; see hybro.h)."""
        hp_set_scatter_policy(self.ctx, self.netlist, regroup_every, deferred)

    def scatter_policy(self):
        return hp_get_scatter_policy(self.ctx, self.netlist)

    def set_tunable(self, which, value):
        """A launch-shape setting of the netlist (speed only; see hybro.h)."""
        hp_set_tunable(self.ctx, self.netlist, which, value)

    def tunable(self, which):
        return hp_get_tunable(self.ctx, self.netlist, which)

    def run(self, slots, iters, gamma, hpwl_every=0):
        """iters x [evaluate at v, Nesterov step] on the slots; returns HPWL_q trace if asked."""
        trace = []
        for it in range(iters):
            self.eval(slots, gamma, want_host=False)
            self.step(slots)
            if hpwl_every and (it + 1) % hpwl_every == 0:
                trace.append(self.hpwl(slots))
        return trace

    def iterate(self, slots, gamma, iters, hpwl=True, graph=False):
        """iters x [evaluate at v, Nesterov step] in one call (the loop runs in the library),
        with the exact HPWL after every iteration (hpwl=True), after the last one only
        (hpwl="last") or never; `graph` replays steady-state blocks from a captured HIP graph
        (the placer's stream must not be the null stream)."""
        flags = ((HP_ITER_HPWL_LAST if hpwl == "last" else HP_ITER_HPWL if hpwl else 0) |
                 (HP_ITER_GRAPH if graph else 0))
        hp_iterate(self.ctx, list(np.atleast_1d(slots)), gamma, iters, flags)

    def close(self):
        """Synchronise and destroy the context (on a shared context: free this netlist's slots
        and the netlist), then drop the device buffers."""
        if self.ctx is not None:
            if self.context is None:
                hp_destroy(self.ctx)
            else:
                for s in list(self._slotbufs):
                    hp_slot_free(self.ctx, s)
                hp_netlist_free(self.ctx, self.netlist)
            self.ctx = None
        self._slotbufs = {}
        self._netbuf = None


class Context:
    """A library context holding several netlists (one Placer each, made by `placer`), whose
    slots iterate together in shared launches (`iterate`): the batched iterations of several
    placement jobs.  Placers of one context share its precision, device and stream."""

    def __init__(self, precision=32, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libhybro needs a ROCm GPU; none is visible")
        self.precision = precision
        self.dev = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.ctx = hp_create(device, C.c_void_p(self.stream.cuda_stream), precision)

    def placer(self, nl, **kw):
        return Placer(nl, context=self, **kw)

    def iterate(self, slots, gammas, iters, hpwl="last", graph=False):
        """iters placer iterations of every listed slot (slots of any of this context's
        netlists, each in steady state: one Placer.iterate on it first) with its own gamma,
        each pass of an iteration one launch over all of them; hpwl and graph as for
        Placer.iterate (graph replay needs a stream other than the null stream)."""
        flags = ((HP_ITER_HPWL_LAST if hpwl == "last" else HP_ITER_HPWL if hpwl else 0) |
                 (HP_ITER_GRAPH if graph else 0))
        hp_iterate_multi(self.ctx, list(np.atleast_1d(slots)), gammas, iters, flags)

    def close(self):
        if self.ctx is not None:
            hp_destroy(self.ctx)
            self.ctx = None
