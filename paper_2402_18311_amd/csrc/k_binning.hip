// Integer charge scatter (the density D of Eqs. 1-2, ePlace reading), built in LDS.
//
// Device-scope int64 atomics run at ~22 G/s on this part and serialise when cells clump, so
// the bulk of the map is built from LDS windows:
//   1. count: each block takes a contiguous run of cells, finds each cell's tile (the
//      ts x ts bin tile holding the lower-left bin of its charge rectangle), and writes its
//      per-tile histogram (LDS atomics only);
//   2. scan: column scans turn the histograms into each (block, tile) output offset, and one
//      block scans the tile totals into the tiles' cell ranges and chunks of <= kChunk cells;
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
#include "hp_binning.h"

namespace hp {

// The scan of a regroup: column scans in a launch of their own, then the tile scan inside
// every placement block.
//
// 1. Column scans (many blocks): a block takes 16 tiles; each tile's column of per-block counts
//    (sort_blocks <= 512 rows) is split into 16 bands of <= 32 rows, one thread per band, whose
//    counts are loaded in one round and kept in registers.  The band sums are scanned in LDS,
//    every (block, tile) gets its exclusive offset within the tile, and the tile's total goes
//    to tstart[t].
// 2. Tile scan (in each placement block, so no launch of its own): exclusive scans of the tile
//    totals and of their chunk counts (ceil(cells / kChunk) per tile) give the tile starts,
//    which the block places by, and the chunk starts and each chunk's tile and cell range,
//    which each block writes for its share of the tiles.
constexpr int kColTiles = 16, kColBands = kBlock / kColTiles, kColRows = 32;
static_assert(kColBands * kColRows >= kMaxSortBlocks, "the column scan covers every counting block");
template <bool RAG>
__global__ __launch_bounds__(kBlock) void bin_colscan_kernel(NetDev nda, SlotArgs sa, SlotLayout La) {
    __shared__ int band[kColBands][kColTiles];
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    if (RAG && blockIdx.x * kColTiles >= nd.ntiles) return;  // past the slot's own tiles
    const int *__restrict__ cnt = reinterpret_cast<const int *>(base + L.scnt);
    int *__restrict__ off = reinterpret_cast<int *>(base + L.soff);
    int *tot = reinterpret_cast<int *>(base + L.tstart);
    const int T = nd.ntiles, R = nd.sort_blocks;
    const int tl = threadIdx.x % kColTiles, bd = threadIdx.x / kColTiles;
    const int t = blockIdx.x * kColTiles + tl;
    const int rpb = (R + kColBands - 1) / kColBands;  // <= kColRows
    const int r0 = bd * rpb, r1 = min(R, r0 + rpb);
    int c[kColRows];
#pragma unroll
    for (int u = 0; u < kColRows; ++u) {
        const int r = r0 + u;
        c[u] = (t < T && r < r1) ? cnt[(size_t)r * T + t] : 0;
    }
    int sum = 0;
#pragma unroll
    for (int u = 0; u < kColRows; ++u) sum += c[u];
    band[bd][tl] = sum;
    __syncthreads();
    if (bd == 0) {
        int run = 0;
        for (int g = 0; g < kColBands; ++g) {
            const int v = band[g][tl];
            band[g][tl] = run;
            run += v;
        }
        if (t < T) tot[t] = run;
    }
    __syncthreads();
    int o = band[bd][tl];
#pragma unroll
    for (int u = 0; u < kColRows; ++u) {
        const int r = r0 + u;
        if (t < T && r < r1) off[(size_t)r * T + t] = o;
        o += c[u];
    }
}

// Threads of a placement block, NT: 1024 while a launch has at most two blocks per CU (one slot:
// one block per counting block, at most kMaxSortBlocks, so its threads take few rounds of
// cells), 256 for launches over many slots, where smaller blocks interleave better.  Tiles per
// thread of its scan: the tile grid has at most 8192 tiles (the tile side doubles until it does,
// or reaches the grid's short side, where at most 2048 / 8 remain).
template <bool RAG, int NT>
__global__ __launch_bounds__(NT) void bin_place_kernel(NetDev nda, SlotArgs sa, SlotLayout La) {
    constexpr int kPlaceRun = 8192 / NT;
    static_assert(NT * kPlaceRun >= 8192, "the placement pass's scan covers every tile");
    extern __shared__ int place_lds[];  // rank [ntiles], then the tile starts [ntiles]
    __shared__ int ws[NT / 64][2];
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    if (RAG && (int)blockIdx.x >= nd.sort_blocks) return;  // past the slot's own blocks
    const int T = nd.ntiles, nb = nd.sort_blocks, blk = blockIdx.x;
    int *rank = place_lds, *hs = place_lds + T;
    const int *tot = reinterpret_cast<const int *>(base + L.tstart);  // tile totals
    int *cstart = reinterpret_cast<int *>(base + L.cstart);
    int4 *chunk = reinterpret_cast<int4 *>(base + L.chunk);
    // the tile scan: each thread a contiguous run of at most kPlaceRun tiles (ntiles <= 8192),
    // its totals loaded into registers in one round, its (cells, chunks) sums scanned over the
    // block
    const int per = (T + NT - 1) / NT;
    const int t0 = min(T, (int)threadIdx.x * per), t1 = min(T, t0 + per);
    int v[kPlaceRun];
#pragma unroll
    for (int k = 0; k < kPlaceRun; ++k) v[k] = (k < per && t0 + k < t1) ? tot[t0 + k] : 0;
    for (int t = threadIdx.x; t < T; t += NT) rank[t] = 0;
    int sc = 0, sk = 0;
#pragma unroll
    for (int k = 0; k < kPlaceRun; ++k) {
        sc += v[k];
        sk += (v[k] + kChunk - 1) / kChunk;
    }
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
    // tile starts for this block's placement; the chunk tables of this block's share of the
    // tiles for the accumulation (every tile's entries written by exactly one block)
    const int w0 = (int)((long long)blk * T / nb), w1 = (int)((long long)(blk + 1) * T / nb);
#pragma unroll
    for (int k = 0; k < kPlaceRun; ++k) {
        const int tk = t0 + k;
        if (k >= per || tk >= t1) break;
        const int s = v[k], nck = (s + kChunk - 1) / kChunk;
        hs[tk] = oc;
        if (tk >= w0 && tk < w1) {
            cstart[tk] = ok;
            for (int c = 0; c < nck; ++c)
                chunk[ok + c] = make_int4(tk, oc + c * kChunk, min(oc + s, oc + (c + 1) * kChunk), 0);
        }
        oc += s;
        ok += nck;
    }
    if (blk == nb - 1 && threadIdx.x == NT - 1) cstart[T] = ok;  // the chunk count
    __syncthreads();
    const int *tile = reinterpret_cast<const int *>(base + L.tile);
    const int *cnt = reinterpret_cast<const int *>(base + L.soff) + (size_t)blk * T;
    int *sorted = reinterpret_cast<int *>(base + L.sorted);
    const int i0 = blk * nd.sort_cells, i1 = min(nd.n_mov, i0 + nd.sort_cells);
    // four cells per thread and round: tiles, then ranks, then offsets, each step's accesses
    // all in flight together (indices clamped in range; only valid cells take a rank)
    for (int i = i0 + threadIdx.x; i < i1; i += 4 * NT) {
        int tt[4], r[4], o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) tt[u] = tile[min(i + u * NT, i1 - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = i + u * NT < i1 ? atomicAdd(&rank[tt[u]], 1) : 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) o[u] = hs[tt[u]] + cnt[tt[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * NT < i1) sorted[o[u] + r[u]] = i + u * NT;
    }
}

// The accumulation right after its order was counted and placed; REC: the counting pass of
// this evaluation wrote the charge records.
template <typename T, bool RAG, bool REC>
__global__ __launch_bounds__(kBlock) void bin_accum_kernel(NetDev nda, SlotArgs sa, SlotLayout La) {
    char *base = sa.base[blockIdx.y];
    // accum_body returns for chunks past the slot's own
    accum_body<T, REC>(view_nd<RAG>(nda, base), base, view_L<RAG>(La, base), blockIdx.x);
}

size_t scatter_count_lds(const NetDev &nd) { return sizeof(int) * (size_t)nd.ntiles; }
size_t scatter_place_lds(const NetDev &nd) { return 2 * sizeof(int) * (size_t)nd.ntiles; }
size_t scatter_accum_lds(const NetDev &nd) {
    return sizeof(unsigned long long) * (size_t)nd.win_side * nd.win_side;
}

// The rest of a rebuild after its counting pass (which the evaluation's first launch runs):
// scan, place, then (accum) the accumulation of the fresh order.
template <typename T>
hipError_t launch_regroup_tail(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                               bool accum, bool records, hipStream_t st) {
    HP_LAUNCH("bin_colscan_kernel", bin_colscan_kernel<false>, dim3((nd.ntiles + kColTiles - 1) / kColTiles, sa.n),
              dim3(kBlock), 0, st, nd, sa, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((size_t)nd.sort_blocks * sa.n <= 2 * (size_t)nd.n_cu)
        HP_LAUNCH("bin_place_kernel", (bin_place_kernel<false, 1024>), dim3(nd.sort_blocks, sa.n),
                  dim3(1024), scatter_place_lds(nd), st, nd, sa, L);
    else
        HP_LAUNCH("bin_place_kernel", (bin_place_kernel<false, kBlock>), dim3(nd.sort_blocks, sa.n),
                  dim3(kBlock), scatter_place_lds(nd), st, nd, sa, L);
    e = hipGetLastError();
    if (e != hipSuccess || !accum) return e;
    if (records)
        HP_LAUNCH("bin_accum_kernel", (bin_accum_kernel<T, false, true>), dim3(nd.max_chunks, sa.n),
                  dim3(kBlock), scatter_accum_lds(nd), st, nd, sa, L);
    else
        HP_LAUNCH("bin_accum_kernel", (bin_accum_kernel<T, false, false>), dim3(nd.max_chunks, sa.n),
                  dim3(kBlock), scatter_accum_lds(nd), st, nd, sa, L);
    return hipGetLastError();
}

// The same over slots of different netlists (each slot's sizes and layout from its
// descriptor); grid.x from the largest slot, dynamic LDS the largest need.
template <typename T>
hipError_t rag_regroup_tail(const SlotArgs &sa, int colscan_x, int place_x, int accum_x,
                            size_t place_lds, size_t accum_lds, hipStream_t st) {
    const NetDev nd0{};
    const SlotLayout L0{};
    HP_LAUNCH("bin_colscan_kernel", bin_colscan_kernel<true>, dim3(colscan_x, sa.n), dim3(kBlock),
              0, st, nd0, sa, L0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    HP_LAUNCH("bin_place_kernel", (bin_place_kernel<true, kBlock>), dim3(place_x, sa.n), dim3(kBlock),
              place_lds, st, nd0, sa, L0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the first launch wrote every rebuilding slot's charge records
    HP_LAUNCH("bin_accum_kernel", (bin_accum_kernel<T, true, true>), dim3(accum_x, sa.n),
              dim3(kBlock), accum_lds, st, nd0, sa, L0);
    return hipGetLastError();
}
int colscan_blocks(const NetDev &nd) { return (nd.ntiles + kColTiles - 1) / kColTiles; }

template hipError_t rag_regroup_tail<float>(const SlotArgs &, int, int, int, size_t, size_t,
                                            hipStream_t);
template hipError_t rag_regroup_tail<double>(const SlotArgs &, int, int, int, size_t, size_t,
                                             hipStream_t);
template hipError_t launch_regroup_tail<float>(const NetDev &, const SlotArgs &, const SlotLayout &,
                                               bool, bool, hipStream_t);
template hipError_t launch_regroup_tail<double>(const NetDev &, const SlotArgs &,
                                                const SlotLayout &, bool, bool, hipStream_t);

}  // namespace hp
