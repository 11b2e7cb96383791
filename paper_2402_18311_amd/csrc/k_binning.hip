// Integer charge scatter (the density D of Eqs. 1-2, ePlace reading), built in LDS.
//
// Device-scope int64 atomics run at ~22 G/s on this part and serialise when cells clump, so
// the bulk of the map is built from LDS windows:
//   1. count: each block takes a contiguous run of cells, finds each cell's tile (the
//      ts x ts bin tile holding the lower-left bin of its charge rectangle), and writes its
//      per-tile histogram (LDS atomics only);
//   2. scan: one block turns the histograms into each (block, tile) output offset, the tiles'
//      cell ranges, and each tile's chunks of at most kChunk cells;
//   3. place: cells are written to the tile-sorted order (rank by LDS atomic);
//   4. accumulate: one block per chunk sums its cells' integer charges into an LDS window of
//      (ts + halo)^2 bins (halo = widest footprint - 1) and stores the window;
// and the row pass of the Poisson solve assembles each bin from the windows of its own tile
// and of the tiles left of / below it.
//
// Steps 1-3 are only a grouping: every cell is in the order exactly once, and a cell whose
// charge rectangle no longer fits its chunk's window (it moved since the order was built)
// adds its charge to the slot's movable map directly with global atomics; the row pass adds
// that map and clears it.  Integer sums do not depend on order, so the map is bit-identical
// however stale the order is, and the order is rebuilt only every few evaluations, when cells
// have drifted little.
#include "hp_device.h"

namespace hp {

struct RectQ {
    int l, r, b, t;
};

__device__ __forceinline__ RectQ cell_rect_b(const NetDev &nd, double x, double y, int4 c) {
    const long long L = q12(x) + c.z, B = q12(y) + c.w;
    RectQ q;
    q.l = (int)min(max(L, 0LL), (long long)nd.wq_die);
    q.r = (int)min(max(L + c.x, 0LL), (long long)nd.wq_die);
    q.b = (int)min(max(B, 0LL), (long long)nd.hq_die);
    q.t = (int)min(max(B + c.y, 0LL), (long long)nd.hq_die);
    return q;
}

__device__ __forceinline__ int overlap_b(int lo, int hi, int idx, int w) {
    const int a = max(lo, idx * w), b = min(hi, (idx + 1) * w);
    return b > a ? b - a : 0;
}

// tile of cell i: the tile of its charge rectangle's lower-left bin (clamped into the die, so
// that a cell whose rectangle is clipped away still has a place in the order)
template <typename T>
__device__ __forceinline__ int cell_tile(const NetDev &nd, const vec2<T> *pos, int i) {
    const vec2<T> p = pos[i];
    const RectQ q = cell_rect_b(nd, (double)p.x, (double)p.y, nd.cq[i]);
    const int j = min(q.l / nd.bq, nd.mx - 1), k = min(q.b / nd.hq, nd.my - 1);
    return (k >> nd.log_ts) * nd.ntx + (j >> nd.log_ts);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void bin_count_kernel(NetDev nd, SlotArgs sa, SlotLayout L) {
    extern __shared__ int hist[];  // [ntiles]
    char *base = sa.base[blockIdx.y];
    const vec2<T> *pos = reinterpret_cast<const vec2<T> *>(base + L.v);
    int *tile = reinterpret_cast<int *>(base + L.tile);
    for (int t = threadIdx.x; t < nd.ntiles; t += kBlock) hist[t] = 0;
    __syncthreads();
    const int i0 = blockIdx.x * nd.sort_cells, i1 = min(nd.n_mov, i0 + nd.sort_cells);
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const int t = cell_tile<T>(nd, pos, i);
        tile[i] = t;
        atomicAdd(&hist[t], 1);
    }
    __syncthreads();
    int *cnt = reinterpret_cast<int *>(base + L.scnt) + (size_t)blockIdx.x * nd.ntiles;
    for (int t = threadIdx.x; t < nd.ntiles; t += kBlock) cnt[t] = hist[t];
}

// One block of 1024 threads: column-wise exclusive scans of the per-block histograms (in
// place), tile starts, and chunk starts (ceil(cells / kChunk) chunks per tile).
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void bin_scan_kernel(NetDev nd, SlotArgs sa, SlotLayout L) {
    __shared__ int ws[kScanThreads / 64][2];
    char *base = sa.base[blockIdx.y];
    const int *__restrict__ cnt = reinterpret_cast<const int *>(base + L.scnt);
    int *__restrict__ off = reinterpret_cast<int *>(base + L.soff);
    int *tstart = reinterpret_cast<int *>(base + L.tstart);
    int *cstart = reinterpret_cast<int *>(base + L.cstart);
    const int T = nd.ntiles, nsb = nd.sort_blocks;
    const int per = (T + kScanThreads - 1) / kScanThreads;
    const int t0 = threadIdx.x * per, t1 = min(T, t0 + per);
    int sc = 0, sk = 0;  // this thread's cells and chunks
    for (int t = t0; t < t1; ++t) {
        int s = 0;
        int b = 0;
        for (; b + 8 <= nsb; b += 8) {  // eight independent loads in flight
            int c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = cnt[(size_t)(b + u) * T + t];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                off[(size_t)(b + u) * T + t] = s;
                s += c[u];
            }
        }
        for (; b < nsb; ++b) {
            const int c = cnt[(size_t)b * T + t];
            off[(size_t)b * T + t] = s;
            s += c;
        }
        tstart[t] = s;  // the tile's total for now
        sc += s;
        sk += (s + kChunk - 1) / kChunk;
    }
    // exclusive scan of (sc, sk) over the threads
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int ic = sc, ik = sk;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int a = __shfl_up(ic, o), b = __shfl_up(ik, o);
        if (lane >= o) {
            ic += a;
            ik += b;
        }
    }
    if (lane == 63) {
        ws[w][0] = ic;
        ws[w][1] = ik;
    }
    __syncthreads();
    int oc = ic - sc, ok = ik - sk;
    for (int i = 0; i < w; ++i) {
        oc += ws[i][0];
        ok += ws[i][1];
    }
    for (int t = t0; t < t1; ++t) {
        const int s = tstart[t];
        tstart[t] = oc;
        cstart[t] = ok;
        oc += s;
        ok += (s + kChunk - 1) / kChunk;
    }
    if (threadIdx.x == kScanThreads - 1) {
        tstart[T] = oc;
        cstart[T] = ok;
    }
}

__global__ __launch_bounds__(kBlock) void bin_place_kernel(NetDev nd, SlotArgs sa, SlotLayout L) {
    extern __shared__ int rank[];  // [ntiles]
    char *base = sa.base[blockIdx.y];
    for (int t = threadIdx.x; t < nd.ntiles; t += kBlock) rank[t] = 0;
    __syncthreads();
    const int *tile = reinterpret_cast<const int *>(base + L.tile);
    const int *cnt = reinterpret_cast<const int *>(base + L.soff) + (size_t)blockIdx.x * nd.ntiles;
    const int *tstart = reinterpret_cast<const int *>(base + L.tstart);
    int *sorted = reinterpret_cast<int *>(base + L.sorted);
    const int i0 = blockIdx.x * nd.sort_cells, i1 = min(nd.n_mov, i0 + nd.sort_cells);
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const int t = tile[i];
        const int r = atomicAdd(&rank[t], 1);
        sorted[tstart[t] + cnt[t] + r] = i;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void bin_accum_kernel(NetDev nd, SlotArgs sa, SlotLayout L) {
    extern __shared__ unsigned long long win[];  // [win_side^2]
    char *base = sa.base[blockIdx.y];
    const int *cstart = reinterpret_cast<const int *>(base + L.cstart);
    const int c = blockIdx.x;
    if (c >= cstart[nd.ntiles]) return;  // block-uniform
    // the tile owning chunk c: the last t with cstart[t] <= c
    int lo = 0, hi = nd.ntiles - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    const int t = lo;
    const int *tstart = reinterpret_cast<const int *>(base + L.tstart);
    const int s0 = tstart[t] + (c - cstart[t]) * kChunk;
    const int s1 = min(tstart[t + 1], s0 + kChunk);
    const int ws = nd.win_side, nw = ws * ws;
    for (int b = threadIdx.x; b < nw; b += kBlock) win[b] = 0;
    __syncthreads();
    const int j00 = (t % nd.ntx) << nd.log_ts, k00 = (t / nd.ntx) << nd.log_ts;
    const vec2<T> *pos = reinterpret_cast<const vec2<T> *>(base + L.v);
    const int *sorted = reinterpret_cast<const int *>(base + L.sorted);
    unsigned long long *rho = reinterpret_cast<unsigned long long *>(base + L.rho);
    for (int s = s0 + threadIdx.x; s < s1; s += kBlock) {
        const int i = sorted[s];
        const vec2<T> p = pos[i];
        const RectQ q = cell_rect_b(nd, (double)p.x, (double)p.y, nd.cq[i]);
        if (q.r <= q.l || q.t <= q.b) continue;  // clipped away: no charge
        const long long rq = nd.rq[i];
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
    __syncthreads();
    unsigned long long *out = reinterpret_cast<unsigned long long *>(base + L.wins) + (size_t)c * nw;
    for (int b = threadIdx.x; b < nw; b += kBlock) out[b] = win[b];
}

template <typename T>
hipError_t launch_scatter(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L, bool regroup,
                          hipStream_t st) {
    const size_t hsh = sizeof(int) * (size_t)nd.ntiles;
    hipError_t e;
    if (!regroup) goto accumulate;
    HP_LAUNCH("bin_count_kernel", bin_count_kernel<T>, dim3(nd.sort_blocks, sa.n), dim3(kBlock), hsh,
              st, nd, sa, L);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    HP_LAUNCH("bin_scan_kernel", bin_scan_kernel, dim3(1, sa.n), dim3(kScanThreads), 0, st, nd, sa, L);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    HP_LAUNCH("bin_place_kernel", bin_place_kernel, dim3(nd.sort_blocks, sa.n), dim3(kBlock), hsh, st,
              nd, sa, L);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
accumulate:
    const size_t wsh = sizeof(unsigned long long) * (size_t)nd.win_side * nd.win_side;
    HP_LAUNCH("bin_accum_kernel", bin_accum_kernel<T>, dim3(nd.max_chunks, sa.n), dim3(kBlock), wsh,
              st, nd, sa, L);
    return hipGetLastError();
}

template hipError_t launch_scatter<float>(const NetDev &, const SlotArgs &, const SlotLayout &,
                                          bool, hipStream_t);
template hipError_t launch_scatter<double>(const NetDev &, const SlotArgs &, const SlotLayout &,
                                           bool, hipStream_t);

}  // namespace hp
