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
//   wm_mask_kernel   a wave per pin of m over the grid, scanning the pin's net (a net counts
//                    at the first of m's pins in it) and adding its increments to X[i] and Y[j]
//                    with int64 atomics (exact, order-free);
//   wm_cand_kernel   a lane per candidate: the overlap test against the listed macros and the
//                    fixed cells that meet the area the block's candidates span (staged in
//                    LDS), the key (increment, displacement, index), block minimum;
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

__device__ __forceinline__ int64_t wave_min64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (int64_t)__shfl_xor((long long)v, o));
    return v;
}
__device__ __forceinline__ int64_t wave_max64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (int64_t)__shfl_xor((long long)v, o));
    return v;
}

constexpr int kMaskBlocks = 128;  // waves over the macro's pins: kMaskBlocks * kBlock / 64

// X and Y start at zero for each macro: zeroed once before the pass, and by the pick kernel
// after each macro's candidates have read them.
__global__ __launch_bounds__(kBlock) void wm_zero_kernel(NetDev nd, char *base, SlotLayout L) {
    const WmScratch S = wm_scratch(nd, base, L);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nd.mx + nd.my; i += gridDim.x * kBlock)
        S.X[i] = 0;  // X and Y are adjacent
}

// A wave per pin of macro m (all of m's pins at once over the grid): the wave scans the pin's
// net four slots per lane and round (a net counts at the first of m's pins in it), reduces the
// other pins' extent and m's offsets, and adds the net's increment at every candidate column
// and row to X and Y with int64 atomics (exact and order-free).
template <typename T>
__global__ __launch_bounds__(kBlock) void wm_mask_kernel(NetDev nd, char *base, SlotLayout L, int m) {
    const WmScratch S = wm_scratch(nd, base, L);
    const WmGeom G = wm_geom<T>(nd, m);
    const vec2<T> *u = reinterpret_cast<const vec2<T> *>(base + L.u);
    const int lane = threadIdx.x & 63;
    const int gw = (blockIdx.x * kBlock + threadIdx.x) >> 6, nw = gridDim.x * (kBlock / 64);
    const int p0 = nd.cell_pin_start[m], p1 = nd.cell_pin_start[m + 1];
    for (int pi = p0 + gw; pi < p1; pi += nw) {  // wave-uniform
        const int slot = nd.cell_pins[pi], e = nd.cell_pin_net[pi];
        const int s0 = nd.net_start[e], s1 = nd.net_start[e + 1];
        int64_t lx = INT64_MAX, hx = INT64_MIN, ly = INT64_MAX, hy = INT64_MIN;
        int64_t mnx = INT64_MAX, mxx = INT64_MIN, mny = INT64_MAX, mxy = INT64_MIN;
        int dup = 0, other = 0;
        // four slots per lane and round, their loads (on clamped, in-range indices) all in
        // flight before any is used
        for (int q0 = s0 + lane; q0 < s1; q0 += 256) {
            int cc[4];
            int2 oo[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int q = min(q0 + 64 * k, s1 - 1);
                cc[k] = q0 + 64 * k < s1 ? nd.pin_cell[q] : -1;
                oo[k] = nd.pin_offq[q];
            }
            int64_t px[4], py[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int c = cc[k] < 0 ? m : cc[k];
                cell_q16<T>(nd, u, c, px[k], py[k]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int c = cc[k];
                if (c < 0) continue;  // padding of the net's slot range, or past its end
                const int2 o = oo[k];
                if (c == m) {
                    dup |= q0 + 64 * k < slot;  // an earlier pin of m in this net counts it
                    mnx = min(mnx, (int64_t)o.x);
                    mxx = max(mxx, (int64_t)o.x);
                    mny = min(mny, (int64_t)o.y);
                    mxy = max(mxy, (int64_t)o.y);
                } else {
                    lx = min(lx, px[k] + o.x);
                    hx = max(hx, px[k] + o.x);
                    ly = min(ly, py[k] + o.y);
                    hy = max(hy, py[k] + o.y);
                    other = 1;
                }
            }
        }
        lx = wave_min64(lx);
        hx = wave_max64(hx);
        ly = wave_min64(ly);
        hy = wave_max64(hy);
        mnx = wave_min64(mnx);
        mxx = wave_max64(mxx);
        mny = wave_min64(mny);
        mxy = wave_max64(mxy);
        if (__any(dup) || !__any(other)) continue;  // wave-uniform
        for (int i = lane; i < G.nci; i += 64) {
            const int64_t a = (int64_t)i * G.bw;
            const int64_t d = (max(hx, a + mxx) - min(lx, a + mnx)) - (hx - lx);
            if (d) atomicAdd(reinterpret_cast<unsigned long long *>(&S.X[i]), (unsigned long long)d);
        }
        for (int j = lane; j < G.ncj; j += 64) {
            const int64_t a = (int64_t)j * G.bh;
            const int64_t d = (max(hy, a + mxy) - min(ly, a + mny)) - (hy - ly);
            if (d) atomicAdd(reinterpret_cast<unsigned long long *>(&S.Y[j]), (unsigned long long)d);
        }
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

constexpr int kObstChunk = 512;  // obstacle rectangles staged in LDS at a time

template <typename T>
__global__ __launch_bounds__(kBlock) void wm_cand_kernel(NetDev nd, char *base, SlotLayout L, int m,
                                                         int n_pool) {
    __shared__ int64_t ob[4][kObstChunk];  // x, y, x + w, y + h of the kept obstacles (q16)
    __shared__ int n_kept;
    const WmScratch S = wm_scratch(nd, base, L);
    const WmGeom G = wm_geom<T>(nd, m);
    const vec2<T> *u = reinterpret_cast<const vec2<T> *>(base + L.u);
    const T *wh = reinterpret_cast<const T *>(nd.cell_wh);
    const int64_t ncand = (int64_t)G.nci * G.ncj;
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = c < ncand;
    const int i = live ? (int)(c % G.nci) : 0, j = live ? (int)(c / G.nci) : 0;
    const int64_t a = (int64_t)i * G.bw, b = (int64_t)j * G.bh;
    bool legal = live;
    // the area the block's candidates can cover: an obstacle outside it is dropped (legality
    // is an AND over obstacles, so the order in which the kept ones are staged is immaterial)
    int64_t bx0 = 0, bx1 = 0, by0 = 0, by1 = 0;
    {
        const int64_t c0 = (int64_t)blockIdx.x * kBlock;
        const int64_t c1 = min(c0 + kBlock, ncand) - 1;
        if (c1 >= c0) {
            const int j0 = (int)(c0 / G.nci), j1 = (int)(c1 / G.nci);
            const int i0 = j0 == j1 ? (int)(c0 % G.nci) : 0;
            const int i1 = j0 == j1 ? (int)(c1 % G.nci) : G.nci - 1;
            bx0 = (int64_t)i0 * G.bw;
            bx1 = (int64_t)i1 * G.bw + G.wq;
            by0 = (int64_t)j0 * G.bh;
            by1 = (int64_t)j1 * G.bh + G.hq;
        }
    }
    // obstacles: the other listed macros, then the fixed cells of nonzero area (a zero-area
    // rectangle overlaps nothing, so those are staged as empty)
    const int n_obst = n_pool + nd.n_fixed;
    for (int k0 = 0; k0 < n_obst; k0 += kObstChunk) {
        __syncthreads();
        if (threadIdx.x == 0) n_kept = 0;
        __syncthreads();
        for (int k = threadIdx.x; k < kObstChunk && k0 + k < n_obst; k += kBlock) {
            const int kk = k0 + k;
            int64_t ox = 0, oy = 0, ow = 0, oh = 0;
            if (kk < n_pool) {
                const int o = S.pool[kk];
                if (o != m) {
                    cell_q16<T>(nd, u, o, ox, oy);
                    ow = q16d((double)wh[o]);
                    oh = q16d((double)wh[nd.n_mov + o]);
                }
            } else {
                const int f = kk - n_pool;
                const double fw = nd.fixed_wh[f], fh = nd.fixed_wh[nd.n_fixed + f];
                if (fw > 0.0 && fh > 0.0) {
                    ox = q16d(nd.fixed_xy[f]);
                    oy = q16d(nd.fixed_xy[nd.n_fixed + f]);
                    ow = q16d(fw);
                    oh = q16d(fh);
                }
            }
            // keep a nonempty obstacle that meets the block's area
            if (ow > 0 && oh > 0 && bx0 < ox + ow && ox < bx1 && by0 < oy + oh && oy < by1) {
                const int at = atomicAdd(&n_kept, 1);
                ob[0][at] = ox;
                ob[1][at] = oy;
                ob[2][at] = ox + ow;
                ob[3][at] = oy + oh;
            }
        }
        __syncthreads();
        const int nk = n_kept;
        for (int k = 0; k < nk && legal; ++k)
            legal = !(a < ob[2][k] && ob[0][k] < a + G.wq && b < ob[3][k] && ob[1][k] < b + G.hq);
    }
    int64_t inc = 0, disp = 0, idx = -1;
    if (legal) {
        int64_t xm, ym;
        cell_q16<T>(nd, u, m, xm, ym);
        inc = S.X[i] + S.Y[j];
        disp = (a > xm ? a - xm : xm - a) + (b > ym ? b - ym : ym - b);
        idx = c;
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
    for (int k = threadIdx.x; k < nd.mx + nd.my; k += kBlock) S.X[k] = 0;  // for the next macro
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
    HP_LAUNCH("wm_zero_kernel", wm_zero_kernel, dim3(8), dim3(kBlock), 0, st, nd, base, L);
    for (int k = 0; k < n_pool; ++k) {
        const int m = pool[k];
        HP_LAUNCH("wm_mask_kernel", wm_mask_kernel<T>, dim3(kMaskBlocks), dim3(kBlock), 0, st, nd, base,
                  L, m);
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
