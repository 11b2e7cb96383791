// WireMask perturbation of Alg. 1 ("Perturb", Sec. 4.2): the listed macros, one after another
// in the given order, each move to the bin-corner position with the least increment of the
// exact HPWL of Eq. 1 (2^-16 grid), given every other cell where it currently is, among the
// positions where the macro overlaps neither another listed macro nor a fixed cell of nonzero
// area.  Ties go to the smaller displacement |dx| + |dy|, then to the lower candidate index
// j * nci + i; a macro without a free position stays.
//
// The increment is separable: for a net e of macro m with the other pins' extent [lo, hi] and
// m's pin offsets [omin, omax] on an axis, placing m at a gives
//   max(hi, a + omax) - min(lo, a + omin) - (hi - lo),
// so the mask over the nci x ncj candidates is X[i] + Y[j] with X and Y sums over m's nets.
// Per macro three launches on one stream:
//   wm_mask_kernel   one block: m's pins in chunks of 256 (a lane per pin slot; the lane of
//                    the first slot of each net scans the net), then X[i] and Y[j] over the
//                    chunk's nets, all in int64 (exact, order-free);
//   wm_cand_kernel   a lane per candidate: the overlap test against the listed macros and the
//                    fixed cells, the key (increment, displacement, index), block minimum;
//   wm_pick_kernel   one block: the minimum of the block minima; the macro moves there (u, v
//                    and v_prev), and the moved count in the slot's scalars goes up.
#include "hp_device.h"

namespace hp {

template <typename T>
hipError_t launch_perturb_restart(const NetDev &nd, char *base, const SlotLayout &L,
                                  hipStream_t st);

namespace {

__device__ __forceinline__ int64_t q16d(double v) { return __double2ll_rn(v * 65536.0); }

struct WmScratch {
    int64_t *X, *Y;      // [mx], [my] increments per candidate column / row
    int64_t *part;       // [3][cand_blocks] block minima (increment, displacement, index)
    const int32_t *pool; // [n_pool] the listed macros
};

__host__ __device__ inline size_t wm_cand_blocks(const NetDev &nd) {
    return ((size_t)nd.mx * nd.my + kBlock - 1) / kBlock;
}

__device__ __forceinline__ WmScratch wm_scratch(const NetDev &nd, char *base, const SlotLayout &L) {
    char *w = base + L.work;
    WmScratch s;
    s.X = reinterpret_cast<int64_t *>(w);
    s.Y = s.X + nd.mx;
    s.part = s.Y + nd.my;
    s.pool = reinterpret_cast<const int32_t *>(s.part + 3 * wm_cand_blocks(nd));
    return s;
}

struct WmGeom {
    int64_t bw, bh, wq, hq;
    int nci, ncj;
};
template <typename T>
__device__ __forceinline__ WmGeom wm_geom(const NetDev &nd, int m) {
    const T *wh = reinterpret_cast<const T *>(nd.cell_wh);
    WmGeom g;
    g.bw = q16d(nd.wb);
    g.bh = q16d(nd.hb);
    g.wq = q16d((double)wh[m]);
    g.hq = q16d((double)wh[nd.n_mov + m]);
    const int64_t Wq = q16d(nd.W), Hq = q16d(nd.H);
    g.nci = g.wq > Wq ? 0 : (int)min((Wq - g.wq) / g.bw + 1, (int64_t)nd.mx);
    g.ncj = g.hq > Hq ? 0 : (int)min((Hq - g.hq) / g.bh + 1, (int64_t)nd.my);
    return g;
}

// the q16 lower-left of cell c at the major solution (movable) or its fixed place
template <typename T>
__device__ __forceinline__ void cell_q16(const NetDev &nd, const vec2<T> *u, int c, int64_t &x,
                                         int64_t &y) {
    if (c < nd.n_mov) {
        const vec2<T> p = u[c];
        x = q16d((double)p.x);
        y = q16d((double)p.y);
    } else {
        x = q16d(nd.fixed_xy[c - nd.n_mov]);
        y = q16d(nd.fixed_xy[nd.n_fixed + c - nd.n_mov]);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void wm_mask_kernel(NetDev nd, char *base, SlotLayout L, int m) {
    // per net of the chunk: other pins' extent and m's offsets, both axes (valid: has others)
    __shared__ int64_t lox[kBlock], hix[kBlock], omnx[kBlock], omxx[kBlock];
    __shared__ int64_t loy[kBlock], hiy[kBlock], omny[kBlock], omxy[kBlock];
    __shared__ int valid[kBlock];
    const WmScratch S = wm_scratch(nd, base, L);
    const WmGeom G = wm_geom<T>(nd, m);
    const vec2<T> *u = reinterpret_cast<const vec2<T> *>(base + L.u);
    for (int i = threadIdx.x; i < G.nci; i += kBlock) S.X[i] = 0;
    for (int j = threadIdx.x; j < G.ncj; j += kBlock) S.Y[j] = 0;
    const int p0 = nd.cell_pin_start[m], p1 = nd.cell_pin_start[m + 1];
    for (int c0 = p0; c0 < p1; c0 += kBlock) {
        const int t = threadIdx.x;
        valid[t] = 0;
        if (c0 + t < p1) {
            const int slot = nd.cell_pins[c0 + t];
            // the net holding this pin slot: the last e with net_start[e] <= slot
            int a = 0, b = nd.ns;
            while (b - a > 1) {
                const int mid = (a + b) >> 1;
                if (nd.net_start[mid] <= slot) a = mid; else b = mid;
            }
            const int s0 = nd.net_start[a], s1 = nd.net_start[a + 1];
            bool first = true;
            for (int q = s0; q < slot && first; ++q) first = nd.pin_cell[q] != m;
            if (first) {
                int64_t lx = INT64_MAX, hx = INT64_MIN, ly = INT64_MAX, hy = INT64_MIN;
                int64_t mnx = INT64_MAX, mxx = INT64_MIN, mny = INT64_MAX, mxy = INT64_MIN;
                bool other = false;
                for (int q = s0; q < s1; ++q) {
                    const int c = nd.pin_cell[q];
                    if (c < 0) continue;  // padding of the net's slot range
                    const int2 o = nd.pin_offq[q];
                    if (c == m) {
                        mnx = min(mnx, (int64_t)o.x);
                        mxx = max(mxx, (int64_t)o.x);
                        mny = min(mny, (int64_t)o.y);
                        mxy = max(mxy, (int64_t)o.y);
                    } else {
                        int64_t cx, cy;
                        cell_q16<T>(nd, u, c, cx, cy);
                        lx = min(lx, cx + o.x);
                        hx = max(hx, cx + o.x);
                        ly = min(ly, cy + o.y);
                        hy = max(hy, cy + o.y);
                        other = true;
                    }
                }
                if (other) {
                    lox[t] = lx;
                    hix[t] = hx;
                    omnx[t] = mnx;
                    omxx[t] = mxx;
                    loy[t] = ly;
                    hiy[t] = hy;
                    omny[t] = mny;
                    omxy[t] = mxy;
                    valid[t] = 1;
                }
            }
        }
        __syncthreads();
        const int nk = min(kBlock, p1 - c0);
        for (int i = threadIdx.x; i < G.nci; i += kBlock) {
            const int64_t a = (int64_t)i * G.bw;
            int64_t acc = 0;
            for (int k = 0; k < nk; ++k) {
                if (!valid[k]) continue;
                const int64_t hi = max(hix[k], a + omxx[k]), lo = min(lox[k], a + omnx[k]);
                acc += (hi - lo) - (hix[k] - lox[k]);
            }
            S.X[i] += acc;
        }
        for (int j = threadIdx.x; j < G.ncj; j += kBlock) {
            const int64_t a = (int64_t)j * G.bh;
            int64_t acc = 0;
            for (int k = 0; k < nk; ++k) {
                if (!valid[k]) continue;
                const int64_t hi = max(hiy[k], a + omxy[k]), lo = min(loy[k], a + omny[k]);
                acc += (hi - lo) - (hiy[k] - loy[k]);
            }
            S.Y[j] += acc;
        }
        __syncthreads();
    }
}

// lexicographic minimum of (inc, disp, idx) keys over a block; idx < 0 marks "none"
__device__ __forceinline__ bool key_less(int64_t i1, int64_t d1, int64_t x1, int64_t i2, int64_t d2,
                                         int64_t x2) {
    if (x2 < 0) return x1 >= 0;
    if (x1 < 0) return false;
    if (i1 != i2) return i1 < i2;
    if (d1 != d2) return d1 < d2;
    return x1 < x2;
}
__device__ void block_min_key(int64_t &inc, int64_t &disp, int64_t &idx) {
    __shared__ int64_t ri[kBlock], rd[kBlock], rx[kBlock];
    ri[threadIdx.x] = inc;
    rd[threadIdx.x] = disp;
    rx[threadIdx.x] = idx;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const int o = threadIdx.x + h;
            if (key_less(ri[o], rd[o], rx[o], ri[threadIdx.x], rd[threadIdx.x], rx[threadIdx.x])) {
                ri[threadIdx.x] = ri[o];
                rd[threadIdx.x] = rd[o];
                rx[threadIdx.x] = rx[o];
            }
        }
        __syncthreads();
    }
    inc = ri[0];
    disp = rd[0];
    idx = rx[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void wm_cand_kernel(NetDev nd, char *base, SlotLayout L, int m,
                                                         int n_pool) {
    const WmScratch S = wm_scratch(nd, base, L);
    const WmGeom G = wm_geom<T>(nd, m);
    const vec2<T> *u = reinterpret_cast<const vec2<T> *>(base + L.u);
    const T *wh = reinterpret_cast<const T *>(nd.cell_wh);
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t inc = 0, disp = 0, idx = -1;
    if (c < (int64_t)G.nci * G.ncj) {
        const int i = (int)(c % G.nci), j = (int)(c / G.nci);
        const int64_t a = (int64_t)i * G.bw, b = (int64_t)j * G.bh;
        bool legal = true;
        for (int k = 0; k < n_pool && legal; ++k) {
            const int o = S.pool[k];
            if (o == m) continue;
            int64_t ox, oy;
            cell_q16<T>(nd, u, o, ox, oy);
            const int64_t ow = q16d((double)wh[o]), oh = q16d((double)wh[nd.n_mov + o]);
            legal = !(a < ox + ow && ox < a + G.wq && b < oy + oh && oy < b + G.hq);
        }
        for (int f = 0; f < nd.n_fixed && legal; ++f) {
            const double fw = nd.fixed_wh[f], fh = nd.fixed_wh[nd.n_fixed + f];
            if (!(fw > 0.0) || !(fh > 0.0)) continue;
            const int64_t ox = q16d(nd.fixed_xy[f]), oy = q16d(nd.fixed_xy[nd.n_fixed + f]);
            legal = !(a < ox + q16d(fw) && ox < a + G.wq && b < oy + q16d(fh) && oy < b + G.hq);
        }
        if (legal) {
            int64_t xm, ym;
            cell_q16<T>(nd, u, m, xm, ym);
            inc = S.X[i] + S.Y[j];
            disp = (a > xm ? a - xm : xm - a) + (b > ym ? b - ym : ym - b);
            idx = c;
        }
    }
    block_min_key(inc, disp, idx);
    if (threadIdx.x == 0) {
        const size_t nb = wm_cand_blocks(nd);
        S.part[blockIdx.x] = inc;
        S.part[nb + blockIdx.x] = disp;
        S.part[2 * nb + blockIdx.x] = idx;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void wm_pick_kernel(NetDev nd, char *base, SlotLayout L, int m,
                                                         int nblk) {
    const WmScratch S = wm_scratch(nd, base, L);
    const size_t nb = wm_cand_blocks(nd);
    int64_t inc = 0, disp = 0, idx = -1;
    for (int k = threadIdx.x; k < nblk; k += kBlock)
        if (key_less(S.part[k], S.part[nb + k], S.part[2 * nb + k], inc, disp, idx)) {
            inc = S.part[k];
            disp = S.part[nb + k];
            idx = S.part[2 * nb + k];
        }
    block_min_key(inc, disp, idx);
    if (threadIdx.x != 0 || idx < 0) return;
    const WmGeom G = wm_geom<T>(nd, m);
    const T nx = (T)((double)((idx % G.nci) * G.bw) / 65536.0);
    const T ny = (T)((double)((idx / G.nci) * G.bh) / 65536.0);
    vec2<T> *u = reinterpret_cast<vec2<T> *>(base + L.u);
    const vec2<T> old = u[m];
    if (old.x != nx || old.y != ny) scalars(base, L)->sel_count += 1;
    const vec2<T> p = cmk2<T>(nx, ny);
    u[m] = p;
    reinterpret_cast<vec2<T> *>(base + L.v)[m] = p;
    reinterpret_cast<vec2<T> *>(base + L.vprev)[m] = p;
}

}  // namespace

size_t wiremask_pool_offset(const NetDev &nd) {
    return 8 * ((size_t)nd.mx + nd.my) + 24 * wm_cand_blocks(nd);
}

template <typename T>
hipError_t launch_wiremask(const NetDev &nd, char *base, const SlotLayout &L, const int32_t *pool,
                           int n_pool, hipStream_t st) {
    hipError_t e = launch_perturb_restart<T>(nd, base, L, st);  // also zeroes the moved count
    if (e != hipSuccess) return e;
    const int nblk = (int)wm_cand_blocks(nd);
    for (int k = 0; k < n_pool; ++k) {
        const int m = pool[k];
        HP_LAUNCH("wm_mask_kernel", wm_mask_kernel<T>, dim3(1), dim3(kBlock), 0, st, nd, base, L, m);
        HP_LAUNCH("wm_cand_kernel", wm_cand_kernel<T>, dim3(nblk), dim3(kBlock), 0, st, nd, base, L, m,
                  n_pool);
        HP_LAUNCH("wm_pick_kernel", wm_pick_kernel<T>, dim3(1), dim3(kBlock), 0, st, nd, base, L, m, nblk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_wiremask<float>(const NetDev &, char *, const SlotLayout &, const int32_t *,
                                           int, hipStream_t);
template hipError_t launch_wiremask<double>(const NetDev &, char *, const SlotLayout &, const int32_t *,
                                            int, hipStream_t);

}  // namespace hp
