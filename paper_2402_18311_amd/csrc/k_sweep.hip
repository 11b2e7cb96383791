// Net sweeps over the pin CSR: the weighted-average wirelength of Eq. 3 with its per-pin
// gradient, and the exact HPWL of Eq. 1.
//
// Nets are grouped at load time by degree.  A net with d <= 64 pins is handled by an aligned
// group of G = nextpow2(d) lanes, one pin per lane: the pin loads of a wave are contiguous
// (coalesced), the cell-position loads (one interleaved (x, y) pair per pin) are the only
// gathers, and the max/min/exp-sum reductions are xor butterflies inside the group.  A larger
// net gets a whole block and streams its pins three times (max/min, exp sums, gradients); the
// repeats hit L2.  Within a bucket nets are ordered by their lowest cell, and the blocks of
// each bucket are remapped so that every XCD walks one contiguous eighth of it: neighbouring
// lanes then gather neighbouring cells, and each XCD's gathers stay in a compact cell range.
#include "hp_device.h"

namespace hp {

// ---- weighted-average wirelength ----------------------------------------------------------
//
// For one net and one axis with pin coordinates x_i, m+ = max x_i, m- = min x_i:
//   a+_i = exp((x_i - m+)/gamma), a-_i = exp(-(x_i - m-)/gamma)      (all exponents <= 0)
//   r+ = sum (x_i - m+) a+_i / sum a+_i,  r- = sum (x_i - m-) a-_i / sum a-_i
//   WL = (m+ - m-) + r+ - r-                                          (Eq. 3, rescaled)
//   dWL/dx_i = a+_i/b+ (1 + (x_i - m+ - r+)/gamma) - a-_i/b- (1 - (x_i - m- - r-)/gamma)
template <typename T, int G>
__device__ __forceinline__ void wa_groups(const NetDev &nd, int net0, int net1, int local,
                                          const vec2<T> *__restrict__ pos, T invg,
                                          vec2<T> *__restrict__ pg, double &wl) {
    constexpr int NPB = kBlock / G;
    const int lane = threadIdx.x & (G - 1);
    const int net = net0 + local * NPB + (int)threadIdx.x / G;
    const bool vnet = net < net1;
    int s = 0, d = 0;
    if (vnet) {
        s = nd.net_start[net];
        d = nd.net_start[net + 1] - s;
    }
    const bool act = lane < d;
    const int p = s + lane;
    T px = 0, py = 0;
    if (act) {
        const int c = nd.pin_cell[p];
        const vec2<T> o = reinterpret_cast<const vec2<T> *>(nd.pin_off)[p];
        const vec2<T> q = pos[c];
        px = q.x + o.x;
        py = q.y + o.y;
    }
    const T inf = pos_inf<T>();
    const T xmax = group_max<G>(act ? px : -inf), xmin = group_min<G>(act ? px : inf);
    const T ymax = group_max<G>(act ? py : -inf), ymin = group_min<G>(act ? py : inf);
    const T dxp = act ? px - xmax : T(0), dxm = act ? px - xmin : T(0);
    const T dyp = act ? py - ymax : T(0), dym = act ? py - ymin : T(0);
    const T axp = act ? dev_exp<T>(dxp * invg) : T(0), axm = act ? dev_exp<T>(-dxm * invg) : T(0);
    const T ayp = act ? dev_exp<T>(dyp * invg) : T(0), aym = act ? dev_exp<T>(-dym * invg) : T(0);
    const T bxp = group_sum<G>(axp), bxm = group_sum<G>(axm);
    const T byp = group_sum<G>(ayp), bym = group_sum<G>(aym);
    const T rxp = group_sum<G>(dxp * axp) / bxp, rxm = group_sum<G>(dxm * axm) / bxm;
    const T ryp = group_sum<G>(dyp * ayp) / byp, rym = group_sum<G>(dym * aym) / bym;
    const T w = (vnet && nd.net_w) ? reinterpret_cast<const T *>(nd.net_w)[net] : T(1);
    if (act) {
        const T gx = axp / bxp * (T(1) + (dxp - rxp) * invg) - axm / bxm * (T(1) - (dxm - rxm) * invg);
        const T gy = ayp / byp * (T(1) + (dyp - ryp) * invg) - aym / bym * (T(1) - (dym - rym) * invg);
        vec2<T> o;
        o.x = w * gx;
        o.y = w * gy;
        pg[p] = o;
    }
    wl = (vnet && lane == 0)
             ? (double)(w * (((xmax - xmin) + (rxp - rxm)) + ((ymax - ymin) + (ryp - rym))))
             : 0.0;
}

template <typename T>
__device__ void wa_block(const NetDev &nd, int net, const vec2<T> *__restrict__ pos, T invg,
                         vec2<T> *__restrict__ pg, double &wl) {
    __shared__ T red[4];
    const int s = nd.net_start[net], d = nd.net_start[net + 1] - s;
    const T inf = pos_inf<T>();
    const vec2<T> *off = reinterpret_cast<const vec2<T> *>(nd.pin_off);
    T lxM = -inf, lxm = inf, lyM = -inf, lym = inf;
    for (int i = threadIdx.x; i < d; i += kBlock) {
        const vec2<T> q = pos[nd.pin_cell[s + i]], o = off[s + i];
        const T px = q.x + o.x, py = q.y + o.y;
        lxM = max(lxM, px);
        lxm = min(lxm, px);
        lyM = max(lyM, py);
        lym = min(lym, py);
    }
    const T xmax = block_max(lxM, red), xmin = block_min(lxm, red);
    const T ymax = block_max(lyM, red), ymin = block_min(lym, red);
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0, s6 = 0, s7 = 0;
    for (int i = threadIdx.x; i < d; i += kBlock) {
        const vec2<T> q = pos[nd.pin_cell[s + i]], o = off[s + i];
        const T px = q.x + o.x, py = q.y + o.y;
        const T dxp = px - xmax, dxm = px - xmin, dyp = py - ymax, dym = py - ymin;
        const T axp = dev_exp<T>(dxp * invg), axm = dev_exp<T>(-dxm * invg);
        const T ayp = dev_exp<T>(dyp * invg), aym = dev_exp<T>(-dym * invg);
        s0 += axp;
        s1 += axm;
        s2 += ayp;
        s3 += aym;
        s4 += dxp * axp;
        s5 += dxm * axm;
        s6 += dyp * ayp;
        s7 += dym * aym;
    }
    const T bxp = block_sum(s0, red), bxm = block_sum(s1, red);
    const T byp = block_sum(s2, red), bym = block_sum(s3, red);
    const T rxp = block_sum(s4, red) / bxp, rxm = block_sum(s5, red) / bxm;
    const T ryp = block_sum(s6, red) / byp, rym = block_sum(s7, red) / bym;
    const T w = nd.net_w ? reinterpret_cast<const T *>(nd.net_w)[net] : T(1);
    for (int i = threadIdx.x; i < d; i += kBlock) {
        const vec2<T> q = pos[nd.pin_cell[s + i]], o = off[s + i];
        const T px = q.x + o.x, py = q.y + o.y;
        const T dxp = px - xmax, dxm = px - xmin, dyp = py - ymax, dym = py - ymin;
        const T axp = dev_exp<T>(dxp * invg), axm = dev_exp<T>(-dxm * invg);
        const T ayp = dev_exp<T>(dyp * invg), aym = dev_exp<T>(-dym * invg);
        vec2<T> g;
        g.x = w * (axp / bxp * (T(1) + (dxp - rxp) * invg) - axm / bxm * (T(1) - (dxm - rxm) * invg));
        g.y = w * (ayp / byp * (T(1) + (dyp - ryp) * invg) - aym / bym * (T(1) - (dym - rym) * invg));
        pg[s + i] = g;
    }
    wl = threadIdx.x == 0
             ? (double)(w * (((xmax - xmin) + (rxp - rxm)) + ((ymax - ymin) + (ryp - rym))))
             : 0.0;
}

// ---- exact HPWL ----------------------------------------------------------------------------
// Pin coordinate q16(cell) + q16(offset), both exact integers; per net the x and y extents.
template <typename T, int G>
__device__ __forceinline__ int64_t hpwl_groups(const NetDev &nd, int net0, int net1, int local,
                                               const vec2<T> *__restrict__ pos) {
    constexpr int NPB = kBlock / G;
    const int lane = threadIdx.x & (G - 1);
    const int net = net0 + local * NPB + (int)threadIdx.x / G;
    int s = 0, d = 0;
    if (net < net1) {
        s = nd.net_start[net];
        d = nd.net_start[net + 1] - s;
    }
    const bool act = lane < d;
    long long px = 0, py = 0;
    if (act) {
        const vec2<T> q = pos[nd.pin_cell[s + lane]];
        const int2 o = nd.pin_offq[s + lane];
        px = q16((double)q.x) + o.x;
        py = q16((double)q.y) + o.y;
    }
    const long long big = 0x3fffffffffffffffLL;
    const long long xM = group_max<G>(act ? px : -big), xm = group_min<G>(act ? px : big);
    const long long yM = group_max<G>(act ? py : -big), ym = group_min<G>(act ? py : big);
    return (act && lane == 0) ? (int64_t)((xM - xm) + (yM - ym)) : 0;
}

template <typename T>
__device__ int64_t hpwl_block(const NetDev &nd, int net, const vec2<T> *__restrict__ pos) {
    __shared__ long long red[4];
    const int s = nd.net_start[net], d = nd.net_start[net + 1] - s;
    const long long big = 0x3fffffffffffffffLL;
    long long xM = -big, xm = big, yM = -big, ym = big;
    for (int i = threadIdx.x; i < d; i += kBlock) {
        const vec2<T> q = pos[nd.pin_cell[s + i]];
        const int2 o = nd.pin_offq[s + i];
        const long long px = q16((double)q.x) + o.x, py = q16((double)q.y) + o.y;
        xM = max(xM, px);
        xm = min(xm, px);
        yM = max(yM, py);
        ym = min(ym, py);
    }
    xM = block_max(xM, red);
    xm = block_min(xm, red);
    yM = block_max(yM, red);
    ym = block_min(ym, red);
    return threadIdx.x == 0 ? (int64_t)((xM - xm) + (yM - ym)) : 0;
}

enum { MODE_WA = 0, MODE_HPWL = 1 };

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void sweep_kernel(NetDev nd, Buckets bk, SlotArgs sa,
                                                       SlotLayout L, T invg) {
    char *base = sa.base[blockIdx.y];
    int b = 0;
    while (b + 1 < bk.n && (int)blockIdx.x >= bk.blk0[b + 1]) ++b;
    const int local = xcd_remap((int)blockIdx.x - bk.blk0[b], bk.nblk[b]);
    const int net0 = bk.net0[b], net1 = bk.net1[b];
    const vec2<T> *pos = reinterpret_cast<const vec2<T> *>(base + (MODE == MODE_WA ? L.v : L.u));
    if constexpr (MODE == MODE_WA) {
        vec2<T> *pg = reinterpret_cast<vec2<T> *>(base + L.pin_grad);
        double wl = 0.0;
        switch (bk.G[b]) {
            case 2: wa_groups<T, 2>(nd, net0, net1, local, pos, invg, pg, wl); break;
            case 4: wa_groups<T, 4>(nd, net0, net1, local, pos, invg, pg, wl); break;
            case 8: wa_groups<T, 8>(nd, net0, net1, local, pos, invg, pg, wl); break;
            case 16: wa_groups<T, 16>(nd, net0, net1, local, pos, invg, pg, wl); break;
            case 32: wa_groups<T, 32>(nd, net0, net1, local, pos, invg, pg, wl); break;
            case 64: wa_groups<T, 64>(nd, net0, net1, local, pos, invg, pg, wl); break;
            default:
                if (net0 + local < net1) wa_block<T>(nd, net0 + local, pos, invg, pg, wl);
                break;
        }
        __shared__ double red[4];
        const double tot = block_sum(wl, red);
        if (threadIdx.x == 0)
            reinterpret_cast<double *>(base + L.part)[PART_WL * L.pstride + blockIdx.x] = tot;
    } else {
        int64_t h = 0;
        switch (bk.G[b]) {
            case 2: h = hpwl_groups<T, 2>(nd, net0, net1, local, pos); break;
            case 4: h = hpwl_groups<T, 4>(nd, net0, net1, local, pos); break;
            case 8: h = hpwl_groups<T, 8>(nd, net0, net1, local, pos); break;
            case 16: h = hpwl_groups<T, 16>(nd, net0, net1, local, pos); break;
            case 32: h = hpwl_groups<T, 32>(nd, net0, net1, local, pos); break;
            case 64: h = hpwl_groups<T, 64>(nd, net0, net1, local, pos); break;
            default:
                if (net0 + local < net1) h = hpwl_block<T>(nd, net0 + local, pos);
                break;
        }
        __shared__ long long red[4];
        const long long tot = block_sum((long long)h, red);
        if (threadIdx.x == 0)
            (reinterpret_cast<long long *>(base + L.part) + PART_HPWL * L.pstride)[blockIdx.x] = tot;
    }
}

int sweep_parts(const Buckets &bk) { return bk.total_blocks; }

template <typename T>
hipError_t launch_sweep_wa(const NetDev &nd, const Buckets &bk, const SlotArgs &sa,
                           const SlotLayout &L, double inv_gamma, hipStream_t st) {
    dim3 grid(bk.total_blocks, sa.n);
    HP_LAUNCH("sweep_wa", (sweep_kernel<T, MODE_WA>), grid, dim3(kBlock), 0, st, nd, bk, sa, L,
              (T)inv_gamma);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep_hpwl(const NetDev &nd, const Buckets &bk, const SlotArgs &sa,
                             const SlotLayout &L, hipStream_t st) {
    dim3 grid(bk.total_blocks, sa.n);
    HP_LAUNCH("sweep_hpwl", (sweep_kernel<T, MODE_HPWL>), grid, dim3(kBlock), 0, st, nd, bk, sa,
              L, (T)0);
    return hipGetLastError();
}

template hipError_t launch_sweep_wa<float>(const NetDev &, const Buckets &, const SlotArgs &,
                                           const SlotLayout &, double, hipStream_t);
template hipError_t launch_sweep_wa<double>(const NetDev &, const Buckets &, const SlotArgs &,
                                            const SlotLayout &, double, hipStream_t);
template hipError_t launch_sweep_hpwl<float>(const NetDev &, const Buckets &, const SlotArgs &,
                                             const SlotLayout &, hipStream_t);
template hipError_t launch_sweep_hpwl<double>(const NetDev &, const Buckets &,
                                              const SlotArgs &, const SlotLayout &,
                                              hipStream_t);

}  // namespace hp
