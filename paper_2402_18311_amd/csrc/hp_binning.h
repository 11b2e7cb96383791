// Device bodies of the binned charge scatter, shared by its own kernels and by the fused first
// launch of an evaluation.  The scheme is described in k_binning.hip.
#pragma once
#include "hp_device.h"

namespace hp {

struct RectQ {
    int l, r, b, t;
};

// A cell's charge rectangle in 2^-12 units, clipped to the die: left edge q12(x) + dxq.  In
// 32-bit arithmetic: scaling a position by 2^12 is exact and rounded once (half to even) in
// either precision, and die validation keeps every coordinate below 2^26.
template <typename T> __device__ __forceinline__ int q12b(T v);
template <> __device__ __forceinline__ int q12b<float>(float v) { return __float2int_rn(v * 4096.0f); }
template <> __device__ __forceinline__ int q12b<double>(double v) { return __double2int_rn(v * 4096.0); }
template <typename T>
__device__ __forceinline__ RectQ cell_rect_b(const NetDev &nd, T x, T y, int4 c) {
    const int L = q12b<T>(x) + c.z, B = q12b<T>(y) + c.w;
    RectQ q;
    q.l = min(max(L, 0), nd.wq_die);
    q.r = min(max(L + c.x, 0), nd.wq_die);
    q.b = min(max(B, 0), nd.hq_die);
    q.t = min(max(B + c.y, 0), nd.hq_die);
    return q;
}

__device__ __forceinline__ int overlap_b(int lo, int hi, int idx, int w) {
    const int a = max(lo, idx * w), b = min(hi, (idx + 1) * w);
    return b > a ? b - a : 0;
}

// tile of cell i: the tile of its charge rectangle's lower-left bin (clamped into the die, so
// that a cell whose rectangle is clipped away still has a place in the order).  Also the
// cell's charge record for an accumulation in the same evaluation: (l, b, w | h << 16, rq)
// of its clipped rectangle, or w | h << 16 = -1 for a big cell or sides that do not pack
// (the accumulation then gathers the cell's data itself).
template <typename T>
__device__ __forceinline__ int cell_tile(const NetDev &nd, const vec2<T> *pos, int i, int4 &rec) {
    const vec2<T> p = pos[i];
    const int4 cc = cell_cq(nd, i);
    const RectQ q = cell_rect_b<T>(nd, p.x, p.y, cc);
    const int j = min(q.l / nd.bq, nd.mx - 1), k = min(q.b / nd.hq, nd.my - 1);
    const int w = max(q.r - q.l, 0), h = max(q.t - q.b, 0);
    rec = make_int4(q.l, q.b, (!is_big(nd, cc) && w < 65536 && h < 32768) ? (w | (h << 16)) : -1,
                    nd.rq[i]);
    return (k >> nd.log_ts) * nd.ntx + (j >> nd.log_ts);
}

// Counting pass of the grouping for block `blk` of the cells (dynamic LDS: int [ntiles]);
// `records`: also the cells' charge records, for an accumulation in the new order in the same
// evaluation.
template <typename T>
__device__ __forceinline__ void count_body(const NetDev &nd, char *base, const SlotLayout &L, int blk,
                                           bool records) {
    extern __shared__ int hist[];  // [ntiles]
    if (blk >= nd.sort_blocks) return;  // block-uniform (the launch may round the grid up)
    const vec2<T> *pos = reinterpret_cast<const vec2<T> *>(base + L.v);
    int *tile = reinterpret_cast<int *>(base + L.tile);
    int4 *crec = reinterpret_cast<int4 *>(base + L.crec);
    for (int t = threadIdx.x; t < nd.ntiles; t += kBlock) hist[t] = 0;
    __syncthreads();
    const int i0 = blk * nd.sort_cells, i1 = min(nd.n_mov, i0 + nd.sort_cells);
    // four cells per thread and round, their loads (clamped in range) all in flight first
    for (int i = i0 + threadIdx.x; i < i1; i += 4 * kBlock) {
        int t[4];
        int4 rec[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = cell_tile<T>(nd, pos, min(i + u * kBlock, i1 - 1), rec[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i + u * kBlock >= i1) break;
            tile[i + u * kBlock] = t[u];
            if (records) crec[i + u * kBlock] = rec[u];
            atomicAdd(&hist[t[u]], 1);
        }
    }
    __syncthreads();
    int *cnt = reinterpret_cast<int *>(base + L.scnt) + (size_t)blk * nd.ntiles;
    for (int t = threadIdx.x; t < nd.ntiles; t += kBlock) cnt[t] = hist[t];
}

// Accumulation of chunk c of the grouped order into its LDS window (dynamic LDS: uint64
// [win_side^2]), added into its tile's window; cells outside the window add to rho with global
// atomics.  REC: the order was counted in this evaluation, so each cell's charge record from
// the counting pass is current and one gather replaces those of its position, rectangle
// constants and charge.
constexpr int kAccBatch = 2;  // cells per thread and round of the accumulation (4: no faster)
template <typename T, bool REC>
__device__ __forceinline__ void accum_body(const NetDev &nd, char *base, const SlotLayout &L, int c) {
    extern __shared__ unsigned long long win[];  // [win_side^2]
    const int *cstart = reinterpret_cast<const int *>(base + L.cstart);
    if (c >= nd.max_chunks || c >= cstart[nd.ntiles]) return;  // block-uniform
    const int4 ck = reinterpret_cast<const int4 *>(base + L.chunk)[c];
    const int t = ck.x, s0 = ck.y, s1 = ck.z;
    const int ws = nd.win_side, nw = ws * ws;
    for (int b = threadIdx.x; b < nw; b += kBlock) win[b] = 0;
    __syncthreads();
    const int j00 = (t % nd.ntx) << nd.log_ts, k00 = (t / nd.ntx) << nd.log_ts;
    const vec2<T> *pos = reinterpret_cast<const vec2<T> *>(base + L.v);
    const int *sorted = reinterpret_cast<const int *>(base + L.sorted);
    unsigned long long *rho = reinterpret_cast<unsigned long long *>(base + L.rho);
    const int4 *crec = reinterpret_cast<const int4 *>(base + L.crec);
    // kAccBatch cells per thread and round: their ids, then their records, all in flight
    // together (indices clamped into the chunk; only cells in it add charge)
    for (int s = s0 + threadIdx.x; s < s1; s += kAccBatch * kBlock) {
        int ids[kAccBatch];
        int4 recs[kAccBatch];
#pragma unroll
        for (int u = 0; u < kAccBatch; ++u) ids[u] = sorted[min(s + u * kBlock, s1 - 1)];
#pragma unroll
        for (int u = 0; u < kAccBatch; ++u) recs[u] = REC ? crec[ids[u]] : make_int4(0, 0, -1, 0);
        for (int u = 0; u < kAccBatch; ++u) {
            if (s + u * kBlock >= s1) break;
            const int i = ids[u];
            const int4 rec = recs[u];
            RectQ q;
            long long rq;
            if (rec.z >= 0) {
                q.l = rec.x;
                q.b = rec.y;
                q.r = rec.x + (rec.z & 0xffff);
                q.t = rec.y + (rec.z >> 16);
                rq = rec.w;
            } else {
                const vec2<T> p = pos[i];
                const int4 cc = cell_cq(nd, i);
                if (is_big(nd, cc)) continue;  // scattered by a block of its own
                q = cell_rect_b<T>(nd, p.x, p.y, cc);
                rq = nd.rq[i];
            }
            if (q.r <= q.l || q.t <= q.b) continue;  // clipped away: no charge
            const int j0 = q.l / nd.bq, j1 = (q.r - 1) / nd.bq;
            const int k0 = q.b / nd.hq, k1 = (q.t - 1) / nd.hq;
            const bool inside = j0 >= j00 && j1 < j00 + ws && k0 >= k00 && k1 < k00 + ws;
            for (int k = k0; k <= k1; ++k) {
                const long long oy = overlap_b(q.b, q.t, k, nd.hq);
                for (int j = j0; j <= j1; ++j) {
                    const long long ox = overlap_b(q.l, q.r, j, nd.bq);
                    const unsigned long long c = (unsigned long long)(rq * ox * oy);
                    if (inside)
                        atomicAdd(&win[(k - k00) * ws + (j - j00)], c);
                    else  // moved out of the window since the order was built
                        atomicAdd(&rho[(size_t)k * nd.mx + j], c);
                }
            }
        }
    }
    __syncthreads();
    // one window per tile: the tile's only chunk stores it, several chunks add theirs (integer
    // sums, order-free); the row pass clears every element it reads, so the windows are zero
    // at the next accumulation
    unsigned long long *out = reinterpret_cast<unsigned long long *>(base + L.wins) + (size_t)t * nw;
    if (cstart[t + 1] - cstart[t] == 1) {
        for (int b = threadIdx.x; b < nw; b += kBlock) out[b] = win[b];
    } else {
        for (int b = threadIdx.x; b < nw; b += kBlock)
            if (win[b]) atomicAdd(&out[b], win[b]);
    }
}

// Charge of big cell big_ids[k] (a macro) added to rho by the whole block, one bin per thread
// and round, with global atomics (an integer sum: order-free and bit-exact).
template <typename T>
__device__ __forceinline__ void big_scatter_body(const NetDev &nd, char *base, const SlotLayout &L,
                                                 int k) {
    if (k >= nd.n_big) return;  // block-uniform (the range is rounded up)
    const int i = nd.big_ids[k];
    const vec2<T> p = reinterpret_cast<const vec2<T> *>(base + L.v)[i];
    const RectQ q = cell_rect_b<T>(nd, p.x, p.y, cell_cq(nd, i));
    if (q.r <= q.l || q.t <= q.b) return;  // clipped away: no charge
    const long long rq = nd.rq[i];
    const int j0 = q.l / nd.bq, nj = (q.r - 1) / nd.bq - j0 + 1;
    const int k0 = q.b / nd.hq, nk = (q.t - 1) / nd.hq - k0 + 1;
    unsigned long long *rho = reinterpret_cast<unsigned long long *>(base + L.rho);
    for (int b = threadIdx.x; b < nj * nk; b += kBlock) {
        const int kk = k0 + b / nj, j = j0 + b % nj;
        const long long c = rq * overlap_b(q.l, q.r, j, nd.bq) * overlap_b(q.b, q.t, kk, nd.hq);
        atomicAdd(&rho[(size_t)kk * nd.mx + j], (unsigned long long)c);
    }
}

}  // namespace hp
