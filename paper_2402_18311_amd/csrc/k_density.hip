// Per-cell kernels: the fixed cells' static charge map, and the fused cell gradient (sum of the
// cell's pin gradients of Eq. 3 plus the electrostatic force on its charge).
//
// Charge model (the density D of Eqs. 1-2, ePlace reading): the die is cut into mx x my bins
// of bq x hq units of 2^-12.  A movable cell's charge rectangle is its own, stretched to at
// least sqrt(2) bins per side around the cell centre, with its charge density scaled by
// r = w h / (w' h').  Its charge in bin (j, k) is r_q * ox_j * oy_k with r_q in 2^-16 and the
// overlaps in 2^-12, i.e. in units of 2^-40 area, exact in int64.  (The movable cells' map
// is built by the binned scatter.)
#include "hp_device.h"

namespace hp {

struct RectQ {
    int l, r, b, t;
};

__device__ __forceinline__ RectQ cell_rect(const NetDev &nd, double x, double y, int4 c) {
    // c = (w'q, h'q, dxq, dyq); left edge q12(x) + dxq, clipped to the die
    const long long L = q12(x) + c.z, B = q12(y) + c.w;
    RectQ q;
    q.l = (int)min(max(L, 0LL), (long long)nd.wq_die);
    q.r = (int)min(max(L + c.x, 0LL), (long long)nd.wq_die);
    q.b = (int)min(max(B, 0LL), (long long)nd.hq_die);
    q.t = (int)min(max(B + c.y, 0LL), (long long)nd.hq_die);
    return q;
}

// The same rectangle in 32-bit arithmetic from a position of the compute type: scaling by 2^12
// is exact and is rounded once (half to even) in either type, and the die validation keeps
// every coordinate below 2^26, so the result equals cell_rect's.
template <typename T> __device__ __forceinline__ int q12i(T v);
template <> __device__ __forceinline__ int q12i<float>(float v) { return __float2int_rn(v * 4096.0f); }
template <> __device__ __forceinline__ int q12i<double>(double v) { return __double2int_rn(v * 4096.0); }
template <typename T>
__device__ __forceinline__ RectQ cell_rect_i(const NetDev &nd, T x, T y, int4 c) {
    const int L = q12i<T>(x) + c.z, B = q12i<T>(y) + c.w;
    RectQ q;
    q.l = min(max(L, 0), nd.wq_die);
    q.r = min(max(L + c.x, 0), nd.wq_die);
    q.b = min(max(B, 0), nd.hq_die);
    q.t = min(max(B + c.y, 0), nd.hq_die);
    return q;
}

__device__ __forceinline__ int overlap(int lo, int hi, int idx, int w) {
    const int a = max(lo, idx * w), b = min(hi, (idx + 1) * w);
    return b > a ? b - a : 0;
}

// Fixed cells: their true rectangle with charge scale 1 (r_q = 2^16), computed once at load.
__global__ __launch_bounds__(kBlock) void fixed_map_kernel(NetDev nd, const double *fxy,
                                                           const double *fwh,
                                                           unsigned long long *rho) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nd.n_fixed) return;
    const double w = fwh[i], h = fwh[nd.n_fixed + i];
    if (!(w > 0.0) || !(h > 0.0)) return;  // pads carry no charge
    int4 c;
    c.x = (int)q12(w);
    c.y = (int)q12(h);
    c.z = 0;
    c.w = 0;
    const RectQ q = cell_rect(nd, fxy[i], fxy[nd.n_fixed + i], c);
    if (q.r <= q.l || q.t <= q.b) return;
    for (int k = q.b / nd.hq; k <= (q.t - 1) / nd.hq; ++k) {
        const long long oy = overlap(q.b, q.t, k, nd.hq);
        for (int j = q.l / nd.bq; j <= (q.r - 1) / nd.bq; ++j) {
            const long long ox = overlap(q.l, q.r, j, nd.bq);
            atomicAdd(&rho[(size_t)k * nd.mx + j], (unsigned long long)(65536LL * ox * oy));
        }
    }
}

// d/dlo of the overlap of [lo, hi] (both moving with the cell, clipped to [0, Wd]) with the
// bin [a, b]: +1 for a moving upper edge inside the bin, -1 for a moving lower edge; an edge
// clipped by the die does not move.  At a touching edge (zero overlap) the derivative of the
// motion that enters the bin is kept.
__device__ __forceinline__ double d_overlap(double lo_raw, double hi_raw, double a, double b,
                                            double Wd) {
    const double lo = fmin(fmax(lo_raw, 0.0), Wd), hi = fmin(fmax(hi_raw, 0.0), Wd);
    const double dlo = (lo_raw >= 0.0 && lo_raw < Wd) ? 1.0 : 0.0;
    const double dhi = (hi_raw >= 0.0 && hi_raw < Wd) ? 1.0 : 0.0;
    const double s = lo >= a ? lo : a, ds = lo >= a ? dlo : 0.0;
    const double t = hi < b ? hi : b, dt = hi < b ? dhi : 0.0;
    const double o = t - s, d = dt - ds;
    if (o > 0.0) return d;
    if (o == 0.0) return d > 0.0 ? d : 0.0;
    return 0.0;
}
__device__ __forceinline__ double overlap_d(double lo, double hi, double a, double b) {
    const double s = lo > a ? lo : a, t = hi < b ? hi : b;
    return t > s ? t - s : 0.0;
}

// Exact adjoint of the density energy for cell i: dN/dx_i = sum_b psi_b d q_ib / dx_i, with
// q_ib = r * overlap_x * overlap_y of the cell's continuous (unquantized) charge rectangle —
// its stretched size and charge scale in FP64 — so the gradient is that of the continuous
// map's energy, with psi from the integer map.  Bins in row-major order over the rectangle and
// the bins touching it.
struct ExactRect {
    double L, B, ws, hs, sc, l, r, b, t;
    int j0, j1, k0, k1;  // the bins touching the rectangle
};
template <typename T>
__device__ __forceinline__ ExactRect exact_rect(const NetDev &nd, int i, double x, double y) {
    const T *wh = reinterpret_cast<const T *>(nd.cell_wh);
    const double w = (double)wh[i], h = (double)wh[nd.n_mov + i];
    ExactRect e;
    e.ws = w;
    e.hs = h;
    e.sc = 1.0;
    if (nd.stretch) {
        e.ws = fmax(w, M_SQRT2 * nd.wb);
        e.hs = fmax(h, M_SQRT2 * nd.hb);
        e.sc = (w * h) / (e.ws * e.hs);
    }
    e.L = x + (w - e.ws) * 0.5;
    e.B = y + (h - e.hs) * 0.5;
    e.l = fmin(fmax(e.L, 0.0), nd.W);
    e.r = fmin(fmax(e.L + e.ws, 0.0), nd.W);
    e.b = fmin(fmax(e.B, 0.0), nd.H);
    e.t = fmin(fmax(e.B + e.hs, 0.0), nd.H);
    e.j0 = max(0, (int)floor(e.l / nd.wb) - 1);
    e.j1 = min(nd.mx - 1, (int)floor(e.r / nd.wb) + 1);
    e.k0 = max(0, (int)floor(e.b / nd.hb) - 1);
    e.k1 = min(nd.my - 1, (int)floor(e.t / nd.hb) + 1);
    return e;
}
// bin (j, k)'s terms psi_b dq/dx and psi_b dq/dy
template <typename T>
__device__ __forceinline__ void exact_term(const NetDev &nd, const ExactRect &e, const T *psi,
                                           int j, int k, double &sx, double &sy) {
    const double oy = overlap_d(e.b, e.t, k * nd.hb, (k + 1) * nd.hb);
    const double doy = d_overlap(e.B, e.B + e.hs, k * nd.hb, (k + 1) * nd.hb, nd.H);
    const double ox = overlap_d(e.l, e.r, j * nd.wb, (j + 1) * nd.wb);
    const double dox = d_overlap(e.L, e.L + e.ws, j * nd.wb, (j + 1) * nd.wb, nd.W);
    const double ps = (double)psi[(size_t)k * nd.mx + j];
    sx += ps * e.sc * dox * oy;
    sy += ps * e.sc * ox * doy;
}
template <typename T>
__device__ void exact_adjoint(const NetDev &nd, const T *psi, int i, double x, double y, T &gdx,
                              T &gdy) {
    const ExactRect e = exact_rect<T>(nd, i, x, y);
    double sx = 0.0, sy = 0.0;
    for (int k = e.k0; k <= e.k1; ++k)
        for (int j = e.j0; j <= e.j1; ++j) exact_term<T>(nd, e, psi, j, k, sx, sy);
    gdx = (T)sx;
    gdy = (T)sy;
}

// ---- big cells (the movable macros): one block per cell and slot --------------------------
// Their footprints span up to the whole grid and they carry many pins, so the per-thread loops
// of the tiled scatter and of the cell gradient would serialise hundreds of loads in one lane.
// Instead the bins and pins of one cell are dealt over a block: the scatter (a block range of
// the first launch of an evaluation) adds each bin's integer charge to rho with global atomics,
// and the gradient pass reduces the cell's pin gradients and its footprint's field (or
// exact-adjoint) terms over the block in FP64 and stores the wirelength part in g and the
// density part in gd, where the cell gradient pass picks them up.
template <typename T, bool RAG>
__global__ __launch_bounds__(kBlock) void big_grad_kernel(NetDev nda, SlotArgs sa, SlotLayout La,
                                                          int grad_mode) {
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    if (RAG && (int)blockIdx.x >= nd.n_big) return;  // past the slot's own big cells
    const int i = nd.big_ids[blockIdx.x];
    const vec2<T> p = reinterpret_cast<const vec2<T> *>(base + L.v)[i];
    double s[4] = {0.0, 0.0, 0.0, 0.0};  // wirelength x, y; density x, y
    const vec2<T> *pg = reinterpret_cast<const vec2<T> *>(base + L.pin_grad);
    const int jend = (grad_mode & GRAD_DENSITY_ONLY) ? 0 : nd.cell_pin_start[i + 1];
    for (int j = nd.cell_pin_start[i] + threadIdx.x; j < jend; j += kBlock) {
        const vec2<T> gp = pg[nd.cell_pins[j]];
        s[0] += (double)gp.x;
        s[1] += (double)gp.y;
    }
    if (grad_mode & GRAD_EXACT) {
        const ExactRect e = exact_rect<T>(nd, i, (double)p.x, (double)p.y);
        const T *psi = reinterpret_cast<const T *>(base + L.psi);
        const int nj = e.j1 - e.j0 + 1, nk = e.k1 - e.k0 + 1;
        for (int b = threadIdx.x; b < nj * nk; b += kBlock)
            exact_term<T>(nd, e, psi, e.j0 + b % nj, e.k0 + b / nj, s[2], s[3]);
    } else {
        const RectQ q = cell_rect_i<T>(nd, p.x, p.y, cell_cq(nd, i));
        if (q.r > q.l && q.t > q.b) {
            const vec2<T> *exy = reinterpret_cast<const vec2<T> *>(base + L.exy);
            const double rqd = (double)nd.rq[i] * 0x1p-40;
            const int j0 = q.l / nd.bq, nj = (q.r - 1) / nd.bq - j0 + 1;
            const int k0 = q.b / nd.hq, nk = (q.t - 1) / nd.hq - k0 + 1;
            for (int b = threadIdx.x; b < nj * nk; b += kBlock) {
                const int k = k0 + b / nj, j = j0 + b % nj;
                const double qq = rqd * (double)overlap(q.l, q.r, j, nd.bq) *
                                  (double)overlap(q.b, q.t, k, nd.hq);
                const vec2<T> ev = exy[(size_t)k * nd.mx + j];
                s[2] -= qq * (double)ev.x;
                s[3] -= qq * (double)ev.y;
            }
        }
    }
    __shared__ double red[4 * 4];
    block_sum_n<4>(s, red);
    if (threadIdx.x == 0) {
        T *g = reinterpret_cast<T *>(base + L.g);
        T *gd = reinterpret_cast<T *>(base + L.gd);
        g[i] = (T)s[0];
        g[nd.n_mov + i] = (T)s[1];
        gd[i] = (T)s[2];
        gd[nd.n_mov + i] = (T)s[3];
    }
}

template <typename T>
hipError_t launch_big_grad(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                           int grad_mode, hipStream_t st) {
    if (nd.n_big == 0) return hipSuccess;
    HP_LAUNCH("big_grad_kernel", (big_grad_kernel<T, false>), dim3(nd.n_big, sa.n), dim3(kBlock), 0, st,
              nd, sa, L, grad_mode);
    return hipGetLastError();
}

// Four consecutive (xi_x, xi_y) pairs of a field row: two 16-byte loads in FP32 (the row
// start is 8-byte aligned; the part reads 16 bytes at any 4-byte alignment), four in FP64.
template <typename T>
__device__ __forceinline__ void load_row4(const vec2<T> *src, vec2<T> (&r)[4]) {
    if constexpr (sizeof(T) == 4) {
        float4 a, b;
        __builtin_memcpy(&a, src, 16);
        __builtin_memcpy(&b, src + 2, 16);
        r[0] = cmk2<T>(a.x, a.y);
        r[1] = cmk2<T>(a.z, a.w);
        r[2] = cmk2<T>(b.x, b.y);
        r[3] = cmk2<T>(b.z, b.w);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = src[k];
    }
}

// The same, loading only the first pair (lo) and / or the second pair (hi) of bins.
template <typename T>
__device__ __forceinline__ void load_row4_part(const vec2<T> *src, bool lo, bool hi,
                                               vec2<T> (&r)[4]) {
    if constexpr (sizeof(T) == 4) {
        if (lo) {
            float4 a;
            __builtin_memcpy(&a, src, 16);
            r[0] = cmk2<T>(a.x, a.y);
            r[1] = cmk2<T>(a.z, a.w);
        }
        if (hi) {
            float4 b;
            __builtin_memcpy(&b, src + 2, 16);
            r[2] = cmk2<T>(b.x, b.y);
            r[3] = cmk2<T>(b.z, b.w);
        }
    } else {
        if (lo) {
            r[0] = src[0];
            r[1] = src[1];
        }
        if (hi) {
            r[2] = src[2];
            r[3] = src[3];
        }
    }
}

// Fused cell gradient.  Wirelength part: the sum of the cell's pin gradients (fixed pin
// order -> deterministic).  Density part: the field force, dN/dx_i = -sum_b q_ib xi_x(b),
// with q_ib the cell's integer charge in bin b.  Steady state writes g = gWL + lambda gD;
// on a slot's first evaluation (lambda not yet derived) it writes gWL to g and gD to gd and
// the per-block L1 norms of both, from which lambda_0 is derived.  In steady state the block
// also forms its partials of the following Nesterov step's reductions.
// Cell block cb = xcd_remap(blockIdx.x) of nb blocks (the grid is nb rounded up to a multiple
// of 8), so that each XCD walks one contiguous eighth of the cells: the pin gradients that
// neighbouring cells share stay in that XCD's L2.  RAG: the slot's netlist and layout from its
// descriptor and nb its own block count (the grid: the largest slot's, rounded up).  Six
// waves per SIMD (80 registers): the pass waits on gathers, and at five it was 2-3% slower,
// at eight (spilling) 20% slower.
//
// The pin gradients of a wave's 64 cells are one contiguous range of the cell-ordered pin
// list.  The wave gathers that range in windows of kPinWin pins, every lane taking kPinPer of
// them (index loads coalesced, every gather slot used), stages each window in LDS, and each
// lane then adds its own cell's pins from LDS in pin order: the same additions in the same
// order as a lane walking its own pins, without the wave waiting on its longest pin list.
// On 2.2 M cells, 8 pins a lane took the pass from 85 us (a lane per cell's own pins) to 75.5 us;
// 4 gave 80 us, 2 gave 83 us, and 16 (LDS and registers then allow 4 waves per SIMD) 90 us.
// FP64 (16 bytes a pin) stages 32 KB a block and runs at 3 waves per SIMD without spilling.
constexpr int kPinPer = 8;
constexpr int kPinWin = 64 * kPinPer;

// LDS written by some lanes of a wave is read by others: order the accesses within the wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// The smallest v over the wave's 64 lanes, in every lane (as a scalar).
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return __builtin_amdgcn_readfirstlane(v);
}

template <typename T, bool RAG>
__global__ __launch_bounds__(kBlock, 6) void cell_grad_kernel(NetDev nda, SlotArgs sa, SlotLayout La,
                                                           double lam_fixed, int use_fixed,
                                                           int grad_mode, int nb_arg) {
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    const int nb = RAG ? max(1, cell_parts(nd)) : nb_arg;  // as launch_cell_grad
    const int cb = xcd_remap(blockIdx.x, gridDim.x);
    if (cb >= nb) return;  // whole block: no barrier is skipped by part of it
    Scalars *sc = scalars(base, L);
    const bool init = !use_fixed && sc->lambda_valid == 0;
    const int i = cb * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    T gwx = 0, gwy = 0, gdx = 0, gdy = 0;
    // the wave's pin range [p0, p1) (wave-uniform); none in a density-only evaluation (the
    // sweep did not run)
    const int c0 = __builtin_amdgcn_readfirstlane(cb * kBlock + (threadIdx.x & ~63));
    int p0 = 0, p1 = 0;
    if (!(grad_mode & GRAD_DENSITY_ONLY) && c0 < nd.n_mov) {
        p0 = nd.cell_pin_start[c0];
        p1 = nd.cell_pin_start[min(c0 + 64, nd.n_mov)];
    }
    const vec2<T> *pg = reinterpret_cast<const vec2<T> *>(base + L.pin_grad);
    const vec2<T> *exy = reinterpret_cast<const vec2<T> *>(base + L.exy);
    // Loads are issued in dependency rounds, each round's loads all in flight before any of
    // them is used: (1) the cell's pin range, position and charge constants, and the wave's
    // first window of pin indices; (2) the field at its charge footprint (a fixed 3 x 4 bin
    // window on clamped in-footprint indices) and the first window's pin gradients; then each
    // window's gradients with the next window's indices.  Sums keep pin order and row-major
    // bin order.
    int id[kPinPer];
    if (p1 > p0) {
#pragma unroll
        for (int u = 0; u < kPinPer; ++u) id[u] = nd.cell_pins[min(p0 + lane + 64 * u, p1 - 1)];
    }
    int j = 0, e = 0;  // the lane's own pins (none for a big cell or past the cells)
    bool big = false, has = false, small = false;
    int4 cc = make_int4(0, 0, 0, 0);
    vec2<T> p = cmk2<T>(T(0), T(0));
    T rqt = 0;
    RectQ q{};
    int j0 = 0, j1 = 0, k0 = 0, k1 = 0;
    constexpr int KR = 3, JC = 4;
    int js = 0, ks = 0;
    vec2<T> f[KR][JC];
    if (i < nd.n_mov) {
        cc = cell_cq(nd, i);
        big = is_big(nd, cc);  // both parts already reduced by its own block
        if (!big && p1 > p0) {
            j = nd.cell_pin_start[i];
            e = nd.cell_pin_start[i + 1];
        }
        p = reinterpret_cast<const vec2<T> *>(base + L.v)[i];
        // charge weight of a bin: rq ox oy 2^-40, formed in the compute type (exact in FP64;
        // in FP32 a relative rounding of ~1e-7, far inside the gradient tolerance)
        rqt = (T)nd.rq[i] * (T)0x1p-40;
        q = cell_rect_i<T>(nd, p.x, p.y, cc);
        has = !big && q.r > q.l && q.t > q.b;
        j0 = q.l / nd.bq;
        j1 = has ? (q.r - 1) / nd.bq : j0;
        k0 = q.b / nd.hq;
        k1 = has ? (q.t - 1) / nd.hq : k0;
        small = !(grad_mode & GRAD_EXACT) && has && k1 - k0 < KR && j1 - j0 < JC;
        // the window: rows ks .. ks+2 and columns js .. js+3 of the field, inside the grid
        // (sides >= 8 bins) and covering the footprint; each row is read as wide loads
        js = min(j0, nd.mx - JC);
        ks = min(k0, nd.my - KR);
        if (small) {  // only the rows and bin pairs of the window that the footprint covers
            const bool lo = j0 <= js + 1, hi = j1 >= js + 2;
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) {
                f[kk][0] = f[kk][1] = f[kk][2] = f[kk][3] = cmk2<T>(T(0), T(0));
                if (ks + kk >= k0 && ks + kk <= k1)
                    load_row4_part<T>(exy + (size_t)(ks + kk) * nd.mx + js, lo, hi, f[kk]);
            }
        }
    }
    // the wave's pin windows (indices clamped into the range; staged slots past it are never
    // read).  A big cell's pins are summed by its own block, not here: a wave holding one
    // trims its range to the first and last pin that its lanes add (a wave of big cells
    // gathers nothing; the pins of a big cell between two others are gathered and not added).
    if (p1 > p0) {
        __shared__ vec2<T> stage[kBlock / 64][kPinWin];
        if (__ballot(big) != 0) {  // wave-uniform
            const int b0 = wave_min(j < e ? j : p1), b1 = -wave_min(j < e ? -e : -p0);
            if (b0 != p0 && b0 < b1) {
#pragma unroll
                for (int u = 0; u < kPinPer; ++u)
                    id[u] = nd.cell_pins[min(b0 + lane + 64 * u, b1 - 1)];
            }
            p0 = b0;
            p1 = b1;
        }
        for (int wb = p0; wb < p1;) {
            vec2<T> gb[kPinPer];
#pragma unroll
            for (int u = 0; u < kPinPer; ++u) gb[u] = pg[id[u]];
            const int wn = wb + kPinWin;
            if (wn < p1) {
#pragma unroll
                for (int u = 0; u < kPinPer; ++u)
                    id[u] = nd.cell_pins[min(wn + lane + 64 * u, p1 - 1)];
            }
            wave_lds_sync();  // the previous window's reads come first
#pragma unroll
            for (int u = 0; u < kPinPer; ++u) stage[wv][lane + 64 * u] = gb[u];
            wave_lds_sync();
            const int qe = min(e, wn);
            for (int k = max(j, wb); k < qe; ++k) {
                const vec2<T> g = stage[wv][k - wb];
                gwx += g.x;
                gwy += g.y;
            }
            wb = wn;
        }
    }
    if (i < nd.n_mov) {
        if (big) {
            const T *gw = reinterpret_cast<const T *>(base + L.g);
            const T *gd = reinterpret_cast<const T *>(base + L.gd);
            gwx = gw[i];
            gwy = gw[nd.n_mov + i];
            gdx = gd[i];
            gdy = gd[nd.n_mov + i];
        } else if (grad_mode & GRAD_EXACT) {  // exact adjoint of the continuous charge rectangle
            exact_adjoint<T>(nd, reinterpret_cast<const T *>(base + L.psi), i, (double)p.x,
                             (double)p.y, gdx, gdy);
        } else if (small) {  // the footprint's bins of the window, row-major
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) {
                const int k = ks + kk;
                if (k < k0 || k > k1) continue;
                const T oy = (T)overlap(q.b, q.t, k, nd.hq) * rqt;
#pragma unroll
                for (int jj = 0; jj < JC; ++jj) {
                    const int jx = js + jj;
                    if (jx < j0 || jx > j1) continue;
                    const T qq = (T)overlap(q.l, q.r, jx, nd.bq) * oy;
                    gdx -= qq * f[kk][jj].x;
                    gdy -= qq * f[kk][jj].y;
                }
            }
        } else if (has) {  // footprints wider than the window: plain loop
            for (int k = k0; k <= k1; ++k) {
                const T oy = (T)overlap(q.b, q.t, k, nd.hq) * rqt;
                for (int jx = j0; jx <= j1; ++jx) {
                    const T qq = (T)overlap(q.l, q.r, jx, nd.bq) * oy;
                    const vec2<T> ev = exy[(size_t)k * nd.mx + jx];
                    gdx -= qq * ev.x;
                    gdy -= qq * ev.y;
                }
            }
        }
    }
    T *g = reinterpret_cast<T *>(base + L.g);
    if (!init) {
        const double lam_step = use_fixed ? lam_fixed : sc->lambda;
        // the step's lambda (no block of this pass reads the field; the closing reduction, when
        // it runs, writes the same value)
        if (cb == 0 && threadIdx.x == 0) sc->lambda_step = lam_step;
        const T lam = (T)lam_step;
        const T g0 = gwx + lam * gdx, g1 = gwy + lam * gdy;
        if (i < nd.n_mov) {
            g[i] = g0;
            g[nd.n_mov + i] = g1;
        }
        // the following step's reductions, from the gradient just formed
        __shared__ double red[4 * 3];
        step_block_norms<T>(nd, base, L, cb, i, i < nd.n_mov, g0, g1, lam_step, red);
    } else {
        T *gd = reinterpret_cast<T *>(base + L.gd);
        if (i < nd.n_mov) {
            g[i] = gwx;
            g[nd.n_mov + i] = gwy;
            gd[i] = gdx;
            gd[nd.n_mov + i] = gdy;
        }
        __shared__ double red[4 * 2];
        double n[2] = {(double)(fabs(gwx) + fabs(gwy)), (double)(fabs(gdx) + fabs(gdy))};
        block_sum_n<2>(n, red);
        if (threadIdx.x == 0) {
            double *part = reinterpret_cast<double *>(base + L.part);
            part[PART_N1 * L.pstride + cb] = n[0];
            part[PART_N2 * L.pstride + cb] = n[1];
        }
    }
}

// (x, y) pairs <-> separate x and y arrays of n elements of `rs` bytes, device to device (a
// strided 2-D copy with one tiny row per element is far slower).  Either of x, y may be null
// when splitting.
template <typename T>
__global__ __launch_bounds__(kBlock) void split_pairs_kernel(const T *pairs, T *x, T *y, int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (x) x[i] = pairs[2 * (size_t)i];
    if (y) y[i] = pairs[2 * (size_t)i + 1];
}
template <typename T>
__global__ __launch_bounds__(kBlock) void join_pairs_kernel(const T *x, const T *y, T *pairs, int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    pairs[2 * (size_t)i] = x[i];
    pairs[2 * (size_t)i + 1] = y[i];
}

hipError_t launch_split_pairs(const void *pairs, void *x, void *y, int n, size_t rs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 g((n + kBlock - 1) / kBlock);
    if (rs == 4)
        HP_LAUNCH("split_pairs_kernel", split_pairs_kernel<float>, g, dim3(kBlock), 0, st,
                  (const float *)pairs, (float *)x, (float *)y, n);
    else
        HP_LAUNCH("split_pairs_kernel", split_pairs_kernel<double>, g, dim3(kBlock), 0, st,
                  (const double *)pairs, (double *)x, (double *)y, n);
    return hipGetLastError();
}

hipError_t launch_join_pairs(const void *x, const void *y, void *pairs, int n, size_t rs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 g((n + kBlock - 1) / kBlock);
    if (rs == 4)
        HP_LAUNCH("join_pairs_kernel", join_pairs_kernel<float>, g, dim3(kBlock), 0, st,
                  (const float *)x, (const float *)y, (float *)pairs, n);
    else
        HP_LAUNCH("join_pairs_kernel", join_pairs_kernel<double>, g, dim3(kBlock), 0, st,
                  (const double *)x, (const double *)y, (double *)pairs, n);
    return hipGetLastError();
}

// ---- overflow of a prefix of the movable cells (filler cells excluded) ---------------------
// The overflow of Eq. 1's density constraint counts the real cells only when the last movable
// cells are ePlace fillers.  Off the iteration path: the counted cells' charge goes into the
// (zero) movable map with global atomics, then each bin's excess over the free capacity is
// summed (int64, order-free, so exact) and the map is zeroed again.
template <typename T>
__global__ __launch_bounds__(kBlock) void counted_scatter_kernel(NetDev nd, char *base, SlotLayout L,
                                                                 int n_counted) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) scalars(base, L)->ovf_tmp = 0;
    if (i >= n_counted) return;
    const vec2<T> p = reinterpret_cast<const vec2<T> *>(base + L.v)[i];
    const RectQ q = cell_rect_i<T>(nd, p.x, p.y, cell_cq(nd, i));
    if (q.r <= q.l || q.t <= q.b) return;
    const long long rq = nd.rq[i];
    unsigned long long *rho = reinterpret_cast<unsigned long long *>(base + L.rho);
    for (int k = q.b / nd.hq; k <= (q.t - 1) / nd.hq; ++k) {
        const long long oy = overlap(q.b, q.t, k, nd.hq);
        for (int j = q.l / nd.bq; j <= (q.r - 1) / nd.bq; ++j)
            atomicAdd(&rho[(size_t)k * nd.mx + j],
                      (unsigned long long)(rq * overlap(q.l, q.r, j, nd.bq) * oy));
    }
}

__global__ __launch_bounds__(kBlock) void counted_overflow_kernel(NetDev nd, char *base,
                                                                  SlotLayout L) {
    __shared__ long long red[4];
    long long *rho = reinterpret_cast<long long *>(base + L.rho);
    const size_t nb = (size_t)nd.mx * nd.my;
    long long s = 0;
    for (size_t b = (size_t)blockIdx.x * kBlock + threadIdx.x; b < nb; b += (size_t)gridDim.x * kBlock) {
        const long long cap = __double2ll_rn(nd.target_density * (double)(nd.area_q - nd.rho_fixed[b]));
        const long long over = rho[b] - cap;
        if (over > 0) s += over;
        rho[b] = 0;
    }
    s = group_sum<64>(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = (red[0] + red[1]) + (red[2] + red[3]);
        if (t) atomicAdd(reinterpret_cast<unsigned long long *>(&scalars(base, L)->ovf_tmp),
                         (unsigned long long)t);
    }
}

template <typename T>
hipError_t launch_overflow_of_cells(const NetDev &nd, char *base, const SlotLayout &L,
                                    int n_counted, hipStream_t st) {
    const int g = std::max(1, (n_counted + kBlock - 1) / kBlock);
    HP_LAUNCH("counted_scatter_kernel", counted_scatter_kernel<T>, dim3(g), dim3(kBlock), 0, st, nd,
              base, L, n_counted);
    HP_LAUNCH("counted_overflow_kernel", counted_overflow_kernel, dim3(256), dim3(kBlock), 0, st, nd,
              base, L);
    return hipGetLastError();
}

// Zero the slots' movable charge maps (after an evaluation that kept them for inspection).
__global__ __launch_bounds__(kBlock) void clear_rho_kernel(NetDev nd, SlotArgs sa, SlotLayout L) {
    long long *rho = reinterpret_cast<long long *>(sa.base[blockIdx.y] + L.rho);
    const size_t n = (size_t)nd.mx * nd.my;
    for (size_t b = (size_t)blockIdx.x * kBlock + threadIdx.x; b < n; b += (size_t)gridDim.x * kBlock)
        rho[b] = 0;
}

hipError_t launch_clear_rho(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                            hipStream_t st) {
    HP_LAUNCH("clear_rho_kernel", clear_rho_kernel, dim3(256, sa.n), dim3(kBlock), 0, st, nd, sa, L);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cell_grad(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                            double lambda_fixed, bool use_fixed, int grad_mode, int nwl, int ne,
                            int nov, int finish, uint32_t banks, hipStream_t st) {
    const int nb = std::max(1, cell_parts(nd));
    const int grid = (nb + kXcds - 1) / kXcds * kXcds;
    HP_LAUNCH("cell_grad_kernel", (cell_grad_kernel<T, false>), dim3(grid, sa.n), dim3(kBlock), 0, st, nd,
              sa, L, lambda_fixed, (int)use_fixed, grad_mode, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (finish < 0) return hipSuccess;
    return launch_eval_finish(nd, sa, L, nwl, ne, nov, nb, use_fixed, lambda_fixed, finish, banks, st);
}

// Over slots of different netlists in steady state: big cells, then the cell gradients with
// each slot's own lambda, grids from the largest slot.
template <typename T>
hipError_t rag_big_grad(const SlotArgs &sa, int grid_x, hipStream_t st) {
    if (grid_x == 0) return hipSuccess;
    HP_LAUNCH("big_grad_kernel", (big_grad_kernel<T, true>), dim3(grid_x, sa.n), dim3(kBlock), 0, st,
              NetDev{}, sa, SlotLayout{}, 0);
    return hipGetLastError();
}
template <typename T>
hipError_t rag_cell_grad(const SlotArgs &sa, int grid_x, hipStream_t st) {
    HP_LAUNCH("cell_grad_kernel", (cell_grad_kernel<T, true>), dim3(grid_x, sa.n), dim3(kBlock), 0,
              st, NetDev{}, sa, SlotLayout{}, 0.0, 0, 0, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fixed_map(const NetDev &nd, const double *fxy, const double *fwh,
                            int64_t *rho_fixed, hipStream_t st) {
    if (nd.n_fixed == 0) return hipSuccess;
    HP_LAUNCH("fixed_map_kernel", fixed_map_kernel, dim3((nd.n_fixed + kBlock - 1) / kBlock),
                       dim3(kBlock), 0, st, nd, fxy, fwh,
                       reinterpret_cast<unsigned long long *>(rho_fixed));
    return hipGetLastError();
}

#define HP_INST(T)                                                                          \
    template hipError_t launch_big_grad<T>(const NetDev &, const SlotArgs &,                \
                                           const SlotLayout &, int, hipStream_t);           \
    template hipError_t launch_overflow_of_cells<T>(const NetDev &, char *, const SlotLayout &, \
                                                    int, hipStream_t);                      \
    template hipError_t launch_cell_grad<T>(const NetDev &, const SlotArgs &,               \
                                            const SlotLayout &, double, bool, int, int, int, \
                                            int, int, uint32_t, hipStream_t);                              \
    template hipError_t launch_fixed_map<T>(const NetDev &, const double *, const double *, \
                                            int64_t *, hipStream_t);                        \
    template hipError_t rag_big_grad<T>(const SlotArgs &, int, hipStream_t);                \
    template hipError_t rag_cell_grad<T>(const SlotArgs &, int, hipStream_t);
HP_INST(float)
HP_INST(double)
#undef HP_INST

}  // namespace hp
