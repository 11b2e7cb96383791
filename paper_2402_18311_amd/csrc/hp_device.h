// Device-side helpers of libhybro: wave/block reductions and fixed-point conversions.
#pragma once
#include "hp_internal.h"

namespace hp {

template <typename T> __device__ __forceinline__ vec2<T> cmk2(T a, T b) {
    vec2<T> r;
    r.x = a;
    r.y = b;
    return r;
}

__device__ __forceinline__ int64_t q16(double v) { return __double2ll_rn(v * 65536.0); }
__device__ __forceinline__ int64_t q12(double v) { return __double2ll_rn(v * 4096.0); }

template <typename T> __device__ __forceinline__ T dev_exp(T v);
template <> __device__ __forceinline__ float dev_exp<float>(float v) { return expf(v); }
template <> __device__ __forceinline__ double dev_exp<double>(double v) { return exp(v); }

template <typename T> __device__ __forceinline__ T pos_inf();
template <> __device__ __forceinline__ float pos_inf<float>() { return __int_as_float(0x7f800000); }
template <> __device__ __forceinline__ double pos_inf<double>() {
    return __longlong_as_double(0x7ff0000000000000LL);
}

// Reductions inside aligned groups of G lanes (G a power of two <= 64); every lane of the
// group gets the result.  The xor butterfly is a fixed order, so results are reproducible.
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}
template <int G, typename T> __device__ __forceinline__ T group_max(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, G));
    return v;
}
template <int G, typename T> __device__ __forceinline__ T group_min(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, G));
    return v;
}

// Block-wide reductions for kBlock = 256 threads (4 waves); all threads get the result.
// `red` is a __shared__ scratch of >= 4 elements; the leading barrier makes reuse safe.
template <typename T> __device__ __forceinline__ T block_sum(T v, T *red) {
    v = group_sum<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}
template <typename T> __device__ __forceinline__ T block_max(T v, T *red) {
    v = group_max<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return max(max(red[0], red[1]), max(red[2], red[3]));
}
template <typename T> __device__ __forceinline__ T block_min(T v, T *red) {
    v = group_min<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return min(min(red[0], red[1]), min(red[2], red[3]));
}

// Fixed-order sums of n per-block partials by one block: thread t sums t, t+256, ... (the
// thread_* part), then the block tree.
template <typename T> __device__ __forceinline__ T thread_sum(const T *p, int n) {
    T s = 0;
    int i = threadIdx.x;
    for (; i + 3 * kBlock < n; i += 4 * kBlock) {  // four independent loads in flight
        const T a = p[i], b = p[i + kBlock], c = p[i + 2 * kBlock], d = p[i + 3 * kBlock];
        s += (a + b) + (c + d);
    }
    for (; i < n; i += kBlock) s += p[i];
    return s;
}
__device__ __forceinline__ double thread_max(const double *p, int n) {
    double s = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kBlock < n; i += 4 * kBlock)
        s = fmax(fmax(s, fmax(p[i], p[i + kBlock])), fmax(p[i + 2 * kBlock], p[i + 3 * kBlock]));
    for (; i < n; i += kBlock) s = fmax(s, p[i]);
    return s;
}
template <typename T> __device__ T sum_parts(const T *p, int n, T *red) {
    return block_sum(thread_sum(p, n), red);
}
__device__ inline double max_parts(const double *p, int n, double *red) {
    return block_max(thread_max(p, n), red);
}

// Preconditioner of the Nesterov step (ePlace reading): P_i = max(1, pins_i + lambda area_i),
// with the lambda of the evaluation that produced the gradient.
template <typename T>
__device__ __forceinline__ double precond(const T *cs, int n, int i, double lam) {
    const double P = (double)cs[i] + lam * (double)cs[n + i];
    return P < 1.0 ? 1.0 : P;
}

// The step's three reductions for the block's cells (cell i = blockIdx.x * 256 + threadIdx.x,
// gradient (g0, g1) of cell i, valid when `live`): |v - v_prev|^2, |g~ - g~_prev|^2 and
// max|g~| with g~ = g / P, stored as the block's partials.  Both the step kernels and the
// fused cell-gradient pass call this, so their partials are identical.
template <typename T>
__device__ __forceinline__ void step_block_norms(const NetDev &nd, char *base, const SlotLayout &L,
                                                 int i, bool live, T g0, T g1, double lam,
                                                 double *red) {
    double dv = 0.0, dg = 0.0, gm = 0.0;
    if (live) {
        const int n = nd.n_mov;
        const T *cs = reinterpret_cast<const T *>(nd.cstep);
        const double P = precond(cs, n, i, lam);
        const vec2<T> v = reinterpret_cast<const vec2<T> *>(base + L.v)[i];
        const vec2<T> vp = reinterpret_cast<const vec2<T> *>(base + L.vprev)[i];
        const T *gp = reinterpret_cast<const T *>(base + L.gprev);
        const double gx = (double)g0 / P, gy = (double)g1 / P;
        const double ax = (double)v.x - (double)vp.x;
        const double ay = (double)v.y - (double)vp.y;
        const double bx = gx - (double)gp[i], by = gy - (double)gp[n + i];
        dv = ax * ax + ay * ay;
        dg = bx * bx + by * by;
        gm = fmax(fabs(gx), fabs(gy));
    }
    dv = block_sum(dv, red);
    dg = block_sum(dg, red);
    gm = block_max(gm, red);
    if (threadIdx.x == 0) {
        double *part = reinterpret_cast<double *>(base + L.part);
        part[PART_DV * L.pstride + blockIdx.x] = dv;
        part[PART_DG * L.pstride + blockIdx.x] = dg;
        part[PART_GMAX * L.pstride + blockIdx.x] = gm;
    }
}

// Step proposal from the totals of the three reductions: alpha_0 = 0.1 bin / max|g~| on the
// first step, else alpha_k = |v - v_prev| / |g~ - g~_prev| (Barzilai-Borwein, the previous
// alpha when the gradient did not change); a' = (1 + sqrt(4 a^2 + 1)) / 2 and momentum
// (a - 1) / a'.  The step kernel commits it (a = a', k + 1, lambda times the ratio).
__device__ __forceinline__ void step_propose(Scalars *sc, double DV, double DG, double GM,
                                             double wb) {
    double alpha;
    if (sc->k == 0)
        alpha = 0.1 * wb / (GM > 1e-30 ? GM : 1e-30);
    else
        alpha = DG > 0.0 ? sqrt(DV) / sqrt(DG) : sc->alpha;
    const double a = sc->a;
    const double an = (1.0 + sqrt(4.0 * a * a + 1.0)) * 0.5;
    sc->step_alpha = alpha;
    sc->step_coef = (a - 1.0) / an;
    sc->step_a = an;
}

// Movable charge of bin (k, j) assembled from the binned scatter's chunk windows: the chunks
// of the bin's own tile, and of the tiles to its left / below / below-left whose windows
// reach into it (the bin lies within the halo of their far edges).
__device__ __forceinline__ long long binned_charge(const NetDev &nd, const char *base,
                                                   const SlotLayout &L, int k, int j) {
    const int *cstart = reinterpret_cast<const int *>(base + L.cstart);
    const unsigned long long *W = reinterpret_cast<const unsigned long long *>(base + L.wins);
    const int ts = 1 << nd.log_ts, ws = nd.win_side, nw = ws * ws;
    const int ty = k >> nd.log_ts, tx = j >> nd.log_ts, kk = k & (ts - 1), jj = j & (ts - 1);
    unsigned long long s = 0;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
        if (dy && (kk >= nd.halo || ty == 0)) continue;
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            if (dx && (jj >= nd.halo || tx == 0)) continue;
            const int t = (ty - dy) * nd.ntx + (tx - dx);
            const int off = (kk + dy * ts) * ws + jj + dx * ts;
            const int c1 = cstart[t + 1];
            int c = cstart[t];
            for (; c + 4 <= c1; c += 4) {  // independent loads in flight when a tile is crowded
                const unsigned long long a0 = W[(size_t)c * nw + off], a1 = W[(size_t)(c + 1) * nw + off];
                const unsigned long long a2 = W[(size_t)(c + 2) * nw + off], a3 = W[(size_t)(c + 3) * nw + off];
                s += (a0 + a1) + (a2 + a3);
            }
            for (; c < c1; ++c) s += W[(size_t)c * nw + off];
        }
    }
    return (long long)s;
}

// Map a block index inside a bucket of nb blocks (nb a multiple of kXcds) so that each XCD
// (which receives blocks i with i % 8 == xcd) works on one contiguous eighth of the bucket.
__device__ __forceinline__ int xcd_remap(int i, int nb) {
    const int q = nb / kXcds;
    return (i % kXcds) * q + i / kXcds;
}

}  // namespace hp
