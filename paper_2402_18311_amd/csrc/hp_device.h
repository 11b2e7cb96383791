// Device-side helpers of libhybro: wave/block reductions and fixed-point conversions.
#pragma once
#include <climits>

#include "hp_internal.h"

namespace hp {

template <typename T> __device__ __forceinline__ vec2<T> cmk2(T a, T b) {
    vec2<T> r;
    r.x = a;
    r.y = b;
    return r;
}

__device__ __forceinline__ int64_t q16(double v) { return __double2ll_rn(v * 65536.0); }
// The same quantization in int32 (exact: scaling by 2^16 is exact in either type and the
// result is rounded half to even once); valid for |v| < 2^15, which load-time validation of
// the die guarantees for positions and pin offsets.
template <typename T> __device__ __forceinline__ int q16i(T v);
template <> __device__ __forceinline__ int q16i<float>(float v) { return __float2int_rn(v * 65536.0f); }
template <> __device__ __forceinline__ int q16i<double>(double v) { return __double2int_rn(v * 65536.0); }
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
// group gets the result.  Partners are combined smallest stride first: lane ^ 1 and lane ^ 2 by
// DPP quad permutes, then the other quad of the 8-lane half-row (DPP half-row mirror), the
// other half of the 16-lane row (DPP row mirror), lane ^ 16 (ds_swizzle) and lane ^ 32
// (bpermute).  After each step every lane of a 2S-lane subgroup holds the same value (x + y
// and y + x are equal), so the result is uniform over the group and run-to-run identical.
template <int S> __device__ __forceinline__ int lane_partner32(int v) {
    if constexpr (S == 1)
        return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    else if constexpr (S == 2)
        return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    else if constexpr (S == 4)
        return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    else if constexpr (S == 8)
        return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    else if constexpr (S == 16)
        return __builtin_amdgcn_ds_swizzle(v, 0x401F);  // bitmask mode: lane ^ 16 within 32
    else
        return __shfl_xor(v, 32);
}
template <int S, typename T> __device__ __forceinline__ T lane_partner(T v) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, lane_partner32<S>(__builtin_bit_cast(int, v)));
    } else {
        static_assert(sizeof(T) == 8, "32- or 64-bit values");
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = lane_partner32<S>((int)(b & 0xffffffffLL));
        const int hi = lane_partner32<S>((int)(b >> 32));
        return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)hi << 32) |
                                                 (unsigned long long)(unsigned)lo));
    }
}
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int s = 1; s < G; s <<= 1) {
        if (s == 1) v += lane_partner<1>(v);
        if (s == 2) v += lane_partner<2>(v);
        if (s == 4) v += lane_partner<4>(v);
        if (s == 8) v += lane_partner<8>(v);
        if (s == 16) v += lane_partner<16>(v);
        if (s == 32) v += lane_partner<32>(v);
    }
    return v;
}
template <int G, typename T> __device__ __forceinline__ T group_max(T v) {
#pragma unroll
    for (int s = 1; s < G; s <<= 1) {
        if (s == 1) v = max(v, lane_partner<1>(v));
        if (s == 2) v = max(v, lane_partner<2>(v));
        if (s == 4) v = max(v, lane_partner<4>(v));
        if (s == 8) v = max(v, lane_partner<8>(v));
        if (s == 16) v = max(v, lane_partner<16>(v));
        if (s == 32) v = max(v, lane_partner<32>(v));
    }
    return v;
}
template <int G, typename T> __device__ __forceinline__ T group_min(T v) {
#pragma unroll
    for (int s = 1; s < G; s <<= 1) {
        if (s == 1) v = min(v, lane_partner<1>(v));
        if (s == 2) v = min(v, lane_partner<2>(v));
        if (s == 4) v = min(v, lane_partner<4>(v));
        if (s == 8) v = min(v, lane_partner<8>(v));
        if (s == 16) v = min(v, lane_partner<16>(v));
        if (s == 32) v = min(v, lane_partner<32>(v));
    }
    return v;
}

// Fast forms for the FP32 path of the WA sweep (exp via the hardware exp2, reciprocal by the
// hardware estimate, ~1 ulp); the FP64 path keeps the library functions.
template <typename T> __device__ __forceinline__ T wa_exp(T v);
template <> __device__ __forceinline__ float wa_exp<float>(float v) { return __expf(v); }
template <> __device__ __forceinline__ double wa_exp<double>(double v) { return exp(v); }
template <typename T> __device__ __forceinline__ T wa_rcp(T v);
template <> __device__ __forceinline__ float wa_rcp<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <> __device__ __forceinline__ double wa_rcp<double>(double v) { return 1.0 / v; }

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

// N block-wide reductions at once (one pair of barriers), each with the same tree as
// block_sum / block_max: xor butterfly in the wave, then (w0 op w1) op (w2 op w3).  `red`
// holds >= 4 * N elements; every thread gets the results in v.
template <int N, typename T> __device__ __forceinline__ void block_sum_n(T (&v)[N], T *red) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = group_sum<64>(v[j]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) red[(threadIdx.x >> 6) * N + j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = (red[j] + red[N + j]) + (red[2 * N + j] + red[3 * N + j]);
}
template <int N, typename T> __device__ __forceinline__ void block_max_n(T (&v)[N], T *red) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = group_max<64>(v[j]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) red[(threadIdx.x >> 6) * N + j] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j)
        v[j] = max(max(red[j], red[N + j]), max(red[2 * N + j], red[3 * N + j]));
}

// Fixed-order sums of n per-block partials by one block: thread t sums t, t+256, ... (the
// thread_* part), then the block tree.
template <typename T> __device__ __forceinline__ T thread_sum(const T *p, int n) {
    T s = 0;
    int i = threadIdx.x;
    for (; i + 7 * kBlock < n; i += 8 * kBlock) {  // eight independent loads in flight
        T a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = p[i + u * kBlock];
        s += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    for (; i + 3 * kBlock < n; i += 4 * kBlock) {
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
__device__ __forceinline__ double precond_of(T pins, T area, double lam) {
    const double P = (double)pins + lam * (double)area;
    return P < 1.0 ? 1.0 : P;
}
template <typename T>
__device__ __forceinline__ double precond(const T *cs, int n, int i, double lam) {
    return precond_of<T>(cs[i], cs[n + i], lam);
}

// The step's three reductions for cell block cb (cell i = cb * 256 + threadIdx.x, gradient
// (g0, g1) of cell i, valid when `live`): |v - v_prev|^2, |g~ - g~_prev|^2 and max|g~| with
// g~ = g / P, stored as partial cb.  `red` holds >= 12 doubles.  Both the step kernels and
// the fused cell-gradient pass call this, so their partials are identical.
template <typename T>
__device__ __forceinline__ void step_block_norms(const NetDev &nd, char *base, const SlotLayout &L,
                                                 int cb, int i, bool live, T g0, T g1, double lam,
                                                 double *red) {
    double dv = 0.0, dg = 0.0, gm = 0.0;
    if (live) {
        const int n = nd.n_mov;
        const T *cs = reinterpret_cast<const T *>(nd.cstep);
        const double iP = 1.0 / precond(cs, n, i, lam);
        const vec2<T> v = reinterpret_cast<const vec2<T> *>(base + L.v)[i];
        const vec2<T> vp = reinterpret_cast<const vec2<T> *>(base + L.vprev)[i];
        const T *gp = reinterpret_cast<const T *>(base + L.gprev);
        const double gx = (double)g0 * iP, gy = (double)g1 * iP;
        const double ax = (double)v.x - (double)vp.x;
        const double ay = (double)v.y - (double)vp.y;
        const double bx = gx - (double)gp[i], by = gy - (double)gp[n + i];
        dv = ax * ax + ay * ay;
        dg = bx * bx + by * by;
        gm = fmax(fabs(gx), fabs(gy));
    }
    // one pair of barriers for the three (trees as in block_sum / block_max)
    dv = group_sum<64>(dv);
    dg = group_sum<64>(dg);
    gm = group_max<64>(gm);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        red[w] = dv;
        red[4 + w] = dg;
        red[8 + w] = gm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *part = reinterpret_cast<double *>(base + L.part);
        part[PART_DV * L.pstride + cb] = (red[0] + red[1]) + (red[2] + red[3]);
        part[PART_DG * L.pstride + cb] = (red[4] + red[5]) + (red[6] + red[7]);
        part[PART_GMAX * L.pstride + cb] = fmax(fmax(red[8], red[9]), fmax(red[10], red[11]));
    }
}

// Step proposal from the totals of the three reductions: alpha_0 = 0.1 bin / max|g~| on the
// first step, else alpha_k = |v - v_prev| / |g~ - g~_prev| (Barzilai-Borwein, the previous
// alpha when the gradient did not change); a' = (1 + sqrt(4 a^2 + 1)) / 2 and momentum
// (a - 1) / a'.  k, a, a_prev and the previous alpha are the optimiser state of the current
// bank.  With backtracking (ePlace's Nesterov method with Lipschitz prediction, Lu et al.,
// TODAES 2015) and a start saved by the last accepted step: if alpha_k, the length predicted
// at the reached point, is below 0.95 of the length that reached it, that step is redone from
// its start with alpha_k (momentum (a_prev - 1) / a; k and a unchanged).
struct StepProposal {
    double alpha, coef, a, aprev;
    int64_t k;
    int reject;
};
__device__ __forceinline__ StepProposal propose_step(int64_t k, double a, double aprev,
                                                     double alpha_prev, bool ready, bool backtrack,
                                                     double DV, double DG, double GM, double wb) {
    StepProposal p;
    if (k == 0)
        p.alpha = 0.1 * wb / (GM > 1e-30 ? GM : 1e-30);
    else
        p.alpha = DG > 0.0 ? sqrt(DV) / sqrt(DG) : alpha_prev;
    p.reject = backtrack && ready && k > 0 && p.alpha < 0.95 * alpha_prev;
    if (p.reject) {
        p.a = a;
        p.aprev = aprev;
        p.coef = (aprev - 1.0) / a;
        p.k = k;
    } else {
        p.a = (1.0 + sqrt(4.0 * a * a + 1.0)) * 0.5;
        p.aprev = a;
        p.coef = (a - 1.0) / p.a;
        p.k = k + 1;
    }
    return p;
}
__device__ __forceinline__ StepProposal propose_from_bank(const Scalars *sc, int b, double DV,
                                                          double DG, double GM, double wb) {
    return propose_step(sc->kb[b], sc->ab[b], sc->aprevb[b], sc->alphab[b], sc->readyb[b] != 0,
                        sc->backtrack != 0, DV, DG, GM, wb);
}
// The proposal from bank b, stored for the step kernel, which commits it into bank 1 - b.
__device__ __forceinline__ void store_proposal(Scalars *sc, const StepProposal &p) {
    sc->step_alpha = p.alpha;
    sc->step_coef = p.coef;
    sc->step_a = p.a;
    sc->step_aprev = p.aprev;
    sc->step_k = p.k;
    sc->step_reject = p.reject;
}
__device__ __forceinline__ void step_propose(Scalars *sc, double DV, double DG, double GM,
                                             double wb, int b) {
    store_proposal(sc, propose_from_bank(sc, b, DV, DG, GM, wb));
}

// Movable charge of bin (k, j) assembled from the binned scatter's tile windows: its own
// tile's, and those of the tiles to its left / below / below-left that reach into it (the bin
// lies within the halo of their far edges).  Every window element inside the die belongs to
// exactly one bin, whose reader clears it (the next scatter adds into zeros).
__device__ __forceinline__ long long take_binned_charge(const NetDev &nd, char *base,
                                                        const SlotLayout &L, int k, int j) {
    unsigned long long *W = reinterpret_cast<unsigned long long *>(base + L.wins);
    const int ts = 1 << nd.log_ts, ws = nd.win_side, nw = ws * ws;
    const int ty = k >> nd.log_ts, tx = j >> nd.log_ts, kk = k & (ts - 1), jj = j & (ts - 1);
    const bool left = jj < nd.halo && tx > 0, below = kk < nd.halo && ty > 0;
    // own tile, left, below, below-left (an absent one reads the own element again, unused)
    const size_t a0 = (size_t)(ty * nd.ntx + tx) * nw + kk * ws + jj;
    const size_t a1 = left ? (size_t)(ty * nd.ntx + tx - 1) * nw + kk * ws + jj + ts : a0;
    const size_t a2 = below ? (size_t)((ty - 1) * nd.ntx + tx) * nw + (kk + ts) * ws + jj : a0;
    const size_t a3 = left && below
                          ? (size_t)((ty - 1) * nd.ntx + tx - 1) * nw + (kk + ts) * ws + jj + ts
                          : a0;
    const unsigned long long v0 = W[a0], v1 = left ? W[a1] : 0ull, v2 = below ? W[a2] : 0ull,
                             v3 = (left && below) ? W[a3] : 0ull;
    if (v0) W[a0] = 0;
    if (v1) W[a1] = 0;
    if (v2) W[a2] = 0;
    if (v3) W[a3] = 0;
    return (long long)((v0 + v1) + (v2 + v3));
}

// Map a block index inside a bucket of nb blocks (nb a multiple of kXcds) so that each XCD
// (which receives blocks i with i % 8 == xcd) works on one contiguous eighth of the bucket.
__device__ __forceinline__ int xcd_remap(int i, int nb) {
    const int q = nb / kXcds;
    return (i % kXcds) * q + i / kXcds;
}

}  // namespace hp
