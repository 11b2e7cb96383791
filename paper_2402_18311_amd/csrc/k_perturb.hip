// Perturbation of Alg. 1 ("Perturb", Sec. 4.2) on one slot's major solution u.
//
// Keys: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) as a counter-based generator, draw i of
// stream `seed` = mix64(seed + (i + 1) * 0x9e3779b97f4a7c15), the key of cell i (shifted right
// by one bit when the selection is restricted to a pool of cells, such as the macros).  The
// moved subset is the m cells with the smallest (key, index): an exact radix select finds the
// m-th smallest key T (eight 8-bit digit passes, each a block-privatised histogram), then a
// stable compaction in index order takes every key < T and the lowest-index keys == T.  GAUSS
// displaces them by a Box-Muller Gaussian from the two halves of mix64(draw); SHUFFLE
// permutes their centres with a
// keyed 4-round Feistel permutation of [0, m) with cycle walking (Black & Rogaway, CT-RSA
// 2002); UNIFORM redraws every cell.  The optimiser restarts at the result.
#include <algorithm>

#include "hp_device.h"

namespace hp {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t i) {
    return mix64(seed + (i + 1) * 0x9e3779b97f4a7c15ULL);
}

__device__ __forceinline__ uint64_t feistel(uint64_t x, int hb, uint64_t key) {
    const uint64_t mask = (1ULL << hb) - 1;
    uint64_t Lh = x >> hb, R = x & mask;
    for (uint64_t r = 0; r < 4; ++r) {
        const uint64_t f = mix64(key ^ ((4 * R + r + 1) * 0x9e3779b97f4a7c15ULL)) & mask;
        const uint64_t nr = Lh ^ f;
        Lh = R;
        R = nr;
    }
    return (Lh << hb) | R;
}

__device__ uint64_t shuffle_perm(uint64_t j, uint64_t m, uint64_t seed) {
    int bits = 2;
    while ((1ULL << bits) < m) bits += 2;
    const uint64_t key = mix64(seed ^ 0x5851f42d4c957f2dULL);
    uint64_t y = feistel(j, bits / 2, key);
    while (y >= m) y = feistel(y, bits / 2, key);  // a permutation: the walk returns into [0, m)
    return y;
}

// restart the optimiser at u; keys for the selection (with a pool, every key is all ones
// here and the pool's keys are written next)
template <typename T>
__global__ __launch_bounds__(kBlock) void perturb_init_kernel(NetDev nd, char *base, SlotLayout L,
                                                              uint64_t seed, int64_t m, int pooled) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    Scalars *sc = scalars(base, L);
    if (i == 0) {
        for (int b = 0; b < 2; ++b) {  // both banks of the optimiser state
            sc->kb[b] = 0;
            sc->ab[b] = 1.0;
            sc->alphab[b] = 0.0;
        }
        sc->lambda_valid = 0;
        sc->hpwl_valid = 0;
        sc->sel_prefix = 0;
        sc->sel_mask = 0;
        sc->sel_remaining = m;
        sc->sel_count = m;
    }
    if (i < 256) sc->hist[i] = 0;
    if (i >= nd.n_mov) return;
    const vec2<T> p = reinterpret_cast<const vec2<T> *>(base + L.u)[i];
    reinterpret_cast<vec2<T> *>(base + L.v)[i] = p;
    reinterpret_cast<vec2<T> *>(base + L.vprev)[i] = p;
    reinterpret_cast<uint64_t *>(base + L.keys)[i] = pooled ? ~0ULL : splitmix(seed, (uint64_t)i);
}

// Keys of a pool of cells (its ids in `work`): the draw shifted right by one bit, so that it
// stays below the all-ones key of every cell outside the pool.
__global__ __launch_bounds__(kBlock) void pool_keys_kernel(char *base, SlotLayout L, int n_pool,
                                                           uint64_t seed) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n_pool) return;
    const int c = reinterpret_cast<const int32_t *>(base + L.work)[j];
    reinterpret_cast<uint64_t *>(base + L.keys)[c] = splitmix(seed, (uint64_t)c) >> 1;
}

__global__ __launch_bounds__(kBlock) void select_hist_kernel(NetDev nd, char *base, SlotLayout L,
                                                             int shift) {
    __shared__ unsigned int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    Scalars *sc = scalars(base, L);
    const uint64_t prefix = sc->sel_prefix, mask = sc->sel_mask;
    const uint64_t *keys = reinterpret_cast<const uint64_t *>(base + L.keys);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nd.n_mov; i += gridDim.x * kBlock) {
        const uint64_t k = keys[i];
        if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&sc->hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void select_pick_kernel(char *base, SlotLayout L, int shift) {
    if (threadIdx.x != 0) return;
    Scalars *sc = scalars(base, L);
    int64_t r = sc->sel_remaining, cum = 0;
    int digit = 255;
    for (int b = 0; b < 256; ++b) {
        if (cum + (int64_t)sc->hist[b] >= r) {
            digit = b;
            break;
        }
        cum += sc->hist[b];
    }
    for (int b = 0; b < 256; ++b) sc->hist[b] = 0;
    sc->sel_remaining = r - cum;
    sc->sel_prefix |= (uint64_t)digit << shift;
    sc->sel_mask |= 255ULL << shift;
}

// exclusive block scan of an int (256 threads); returns the prefix, *total the block sum
__device__ int block_excl_scan(int v, int *total) {
    __shared__ int ws[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    __syncthreads();
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    int off = 0;
    for (int i = 0; i < w; ++i) off += ws[i];
    *total = ws[0] + ws[1] + ws[2] + ws[3];
    return off + inc - v;
}

__global__ __launch_bounds__(kBlock) void select_count_kernel(NetDev nd, char *base, SlotLayout L) {
    const Scalars *sc = scalars(base, L);
    const uint64_t T0 = sc->sel_prefix;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    int lt = 0, eq = 0;
    if (i < nd.n_mov) {
        const uint64_t k = reinterpret_cast<const uint64_t *>(base + L.keys)[i];
        lt = k < T0;
        eq = k == T0;
    }
    int tl, te;
    block_excl_scan(lt, &tl);
    block_excl_scan(eq, &te);
    if (threadIdx.x == 0) {
        int *cnt = reinterpret_cast<int *>(base + L.work);
        cnt[2 * blockIdx.x] = tl;
        cnt[2 * blockIdx.x + 1] = te;
    }
}

// exclusive scan of the per-block (lt, eq) counts, in place, by one block
__global__ __launch_bounds__(kBlock) void select_scan_kernel(char *base, SlotLayout L, int nblk) {
    int *cnt = reinterpret_cast<int *>(base + L.work);
    const int per = (nblk + kBlock - 1) / kBlock;
    const int b0 = threadIdx.x * per, b1 = min(nblk, b0 + per);
    int sl = 0, se = 0;
    for (int b = b0; b < b1; ++b) {
        sl += cnt[2 * b];
        se += cnt[2 * b + 1];
    }
    int tl, te;
    const int ol = block_excl_scan(sl, &tl), oe = block_excl_scan(se, &te);
    __syncthreads();
    int al = ol, ae = oe;
    for (int b = b0; b < b1; ++b) {
        const int l = cnt[2 * b], e = cnt[2 * b + 1];
        cnt[2 * b] = al;
        cnt[2 * b + 1] = ae;
        al += l;
        ae += e;
    }
}

__global__ __launch_bounds__(kBlock) void select_write_kernel(NetDev nd, char *base, SlotLayout L) {
    const Scalars *sc = scalars(base, L);
    const uint64_t T0 = sc->sel_prefix;
    const int64_t r = sc->sel_remaining;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    int lt = 0, eq = 0;
    if (i < nd.n_mov) {
        const uint64_t k = reinterpret_cast<const uint64_t *>(base + L.keys)[i];
        lt = k < T0;
        eq = k == T0;
    }
    int tl, te;
    const int *cnt = reinterpret_cast<const int *>(base + L.work);
    const int64_t lb = cnt[2 * blockIdx.x] + block_excl_scan(lt, &tl);
    const int64_t eb = cnt[2 * blockIdx.x + 1] + block_excl_scan(eq, &te);
    const int64_t pos = lb + (eb < r ? eb : r);
    if ((lt || (eq && eb < r)) && pos < sc->sel_count)
        reinterpret_cast<int32_t *>(base + L.sel)[pos] = i;
}

template <typename T>
__device__ __forceinline__ void put(char *base, const NetDev &nd, const SlotLayout &L, int c,
                                    double x, double y) {
    const T *cs = reinterpret_cast<const T *>(nd.cstep);
    const double hx = (double)cs[2 * nd.n_mov + c], hy = (double)cs[3 * nd.n_mov + c];
    x = x < 0.0 ? 0.0 : (x > hx ? hx : x);
    y = y < 0.0 ? 0.0 : (y > hy ? hy : y);
    const vec2<T> p = cmk2<T>((T)x, (T)y);
    reinterpret_cast<vec2<T> *>(base + L.u)[c] = p;
    reinterpret_cast<vec2<T> *>(base + L.v)[c] = p;
    reinterpret_cast<vec2<T> *>(base + L.vprev)[c] = p;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void apply_gauss_kernel(NetDev nd, char *base, SlotLayout L,
                                                             int64_t m, double sx, double sy,
                                                             uint64_t seed, int uniform) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    const int c = uniform ? j : reinterpret_cast<const int32_t *>(base + L.sel)[j];
    const uint64_t k2 = mix64(splitmix(seed, (uint64_t)c));
    const double u1 = ((double)(k2 >> 32) + 0.5) / 4294967296.0;
    const double u2 = ((double)(k2 & 0xffffffffULL) + 0.5) / 4294967296.0;
    const vec2<T> *u = reinterpret_cast<const vec2<T> *>(base + L.u);
    if (uniform) {
        const T *cs = reinterpret_cast<const T *>(nd.cstep);
        put<T>(base, nd, L, c, u1 * (double)cs[2 * nd.n_mov + c], u2 * (double)cs[3 * nd.n_mov + c]);
        reinterpret_cast<int32_t *>(base + L.sel)[j] = c;
    } else {
        const double rad = sqrt(-2.0 * log(u1));
        const double dx = sx * rad * cos(2.0 * M_PI * u2), dy = sy * rad * sin(2.0 * M_PI * u2);
        const vec2<T> p = u[c];
        put<T>(base, nd, L, c, (double)p.x + dx, (double)p.y + dy);
    }
}

// SHUFFLE, phase 1: the centre that selected cell j will take (from the unmodified u)
template <typename T>
__global__ __launch_bounds__(kBlock) void shuffle_gather_kernel(NetDev nd, char *base, SlotLayout L,
                                                                int64_t m, uint64_t seed) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    const int32_t *sel = reinterpret_cast<const int32_t *>(base + L.sel);
    const int s = sel[shuffle_perm((uint64_t)j, (uint64_t)m, seed)];
    const vec2<T> p = reinterpret_cast<const vec2<T> *>(base + L.u)[s];
    const T *wh = reinterpret_cast<const T *>(nd.cell_wh);
    double *cen = reinterpret_cast<double *>(base + L.work);
    cen[2 * j] = (double)p.x + 0.5 * (double)wh[s];
    cen[2 * j + 1] = (double)p.y + 0.5 * (double)wh[nd.n_mov + s];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void shuffle_apply_kernel(NetDev nd, char *base, SlotLayout L,
                                                               int64_t m) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    const int c = reinterpret_cast<const int32_t *>(base + L.sel)[j];
    const T *wh = reinterpret_cast<const T *>(nd.cell_wh);
    const double *cen = reinterpret_cast<const double *>(base + L.work);
    put<T>(base, nd, L, c, cen[2 * j] - 0.5 * (double)wh[c], cen[2 * j + 1] - 0.5 * (double)wh[nd.n_mov + c]);
}

size_t perturb_work_bytes(int n_mov, int mx, int my) {
    const size_t nblk = ((size_t)n_mov + kBlock - 1) / kBlock;
    const size_t a = 8 * nblk, b = 16 * (size_t)n_mov;
    // WireMask: per-axis increments, per-block candidate minima, the macro list
    const size_t cand_blocks = ((size_t)mx * my + kBlock - 1) / kBlock;
    const size_t c = 8 * ((size_t)mx + my) + 24 * cand_blocks + 256 + 4 * (size_t)n_mov;
    return std::max({a, b, c}) + 256;
}

// restart hook shared with the WireMask pass (k_wiremask.hip)
template <typename T>
hipError_t launch_perturb_restart(const NetDev &nd, char *base, const SlotLayout &L,
                                  hipStream_t st) {
    const int nblk = (nd.n_mov + kBlock - 1) / kBlock;
    HP_LAUNCH("perturb_init_kernel", perturb_init_kernel<T>, dim3(nblk > 0 ? nblk : 1), dim3(kBlock), 0, st,
              nd, base, L, 0ULL, (int64_t)0, 0);
    return hipGetLastError();
}
template hipError_t launch_perturb_restart<float>(const NetDev &, char *, const SlotLayout &, hipStream_t);
template hipError_t launch_perturb_restart<double>(const NetDev &, char *, const SlotLayout &, hipStream_t);

template <typename T>
hipError_t launch_perturb(const NetDev &nd, char *base, const SlotLayout &L, int mode, int64_t m,
                          double sigma_x, double sigma_y, uint64_t seed, int n_pool,
                          hipStream_t st) {
    const int nblk = (nd.n_mov + kBlock - 1) / kBlock;
    const int gb = nblk > 0 ? nblk : 1;
    const int pooled = n_pool >= 0;
    HP_LAUNCH("perturb_init_kernel", perturb_init_kernel<T>, dim3(gb), dim3(kBlock), 0, st, nd, base, L, seed, m,
              pooled);
    if (pooled && n_pool > 0)
        HP_LAUNCH("pool_keys_kernel", pool_keys_kernel, dim3((n_pool + kBlock - 1) / kBlock), dim3(kBlock), 0,
                  st, base, L, n_pool, seed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || m == 0) return e;
    const int mb = (int)((m + kBlock - 1) / kBlock);
    if (mode == 2) {
        HP_LAUNCH("apply_gauss_kernel", apply_gauss_kernel<T>, dim3(mb), dim3(kBlock), 0, st, nd, base, L, m, 0.0,
                           0.0, seed, 1);
        return hipGetLastError();
    }
    const int hb = nblk < 2048 ? nblk : 2048;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        HP_LAUNCH("select_hist_kernel", select_hist_kernel, dim3(hb), dim3(kBlock), 0, st, nd, base, L, shift);
        HP_LAUNCH("select_pick_kernel", select_pick_kernel, dim3(1), dim3(64), 0, st, base, L, shift);
    }
    HP_LAUNCH("select_count_kernel", select_count_kernel, dim3(nblk), dim3(kBlock), 0, st, nd, base, L);
    HP_LAUNCH("select_scan_kernel", select_scan_kernel, dim3(1), dim3(kBlock), 0, st, base, L, nblk);
    HP_LAUNCH("select_write_kernel", select_write_kernel, dim3(nblk), dim3(kBlock), 0, st, nd, base, L);
    if (mode == 0) {
        HP_LAUNCH("apply_gauss_kernel", apply_gauss_kernel<T>, dim3(mb), dim3(kBlock), 0, st, nd, base, L, m,
                           sigma_x, sigma_y, seed, 0);
    } else {
        HP_LAUNCH("shuffle_gather_kernel", shuffle_gather_kernel<T>, dim3(mb), dim3(kBlock), 0, st, nd, base, L, m,
                           seed);
        HP_LAUNCH("shuffle_apply_kernel", shuffle_apply_kernel<T>, dim3(mb), dim3(kBlock), 0, st, nd, base, L, m);
    }
    return hipGetLastError();
}

template hipError_t launch_perturb<float>(const NetDev &, char *, const SlotLayout &, int, int64_t,
                                          double, double, uint64_t, int, hipStream_t);
template hipError_t launch_perturb<double>(const NetDev &, char *, const SlotLayout &, int, int64_t,
                                           double, double, uint64_t, int, hipStream_t);

}  // namespace hp
