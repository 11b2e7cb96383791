// Net sweeps over the pin CSR: the weighted-average wirelength of Eq. 3 with its per-pin
// gradient, and the exact HPWL of Eq. 1.
//
// Nets are grouped at load time by degree.  A net with d <= 64 pins is handled by an aligned
// group of G = nextpow2(d) lanes, one pin per lane, in a padded layout (G pin slots per net)
// so that a lane finds its pin without reading the net's start: the pin loads of a wave are
// contiguous (coalesced), the cell-position loads (one interleaved (x, y) pair per pin) are
// the only gathers, and the max/min/exp-sum reductions are xor butterflies inside the group.
// A net with 65..256 pins gets one wave, in the same padded layout with S = 64 PPL slots
// (PPL = 2 or 4 pins per lane, lane l holding slots l, l + 64, ...), its reductions within the
// wave; a larger net gets a whole block, which stages up to 2048 of its pin coordinates in
// LDS for its three passes (max/min, exp sums, gradients).  Within a bucket nets are ordered by their
// lowest cell, and the blocks of each bucket are remapped so that every XCD walks one
// contiguous eighth of it: neighbouring lanes then gather neighbouring cells, and each XCD's
// gathers stay in a compact cell range.
#include "hp_binning.h"

namespace hp {

// ---- weighted-average wirelength ----------------------------------------------------------
//
// For one net and one axis with pin coordinates x_i, m+ = max x_i, m- = min x_i:
//   a+_i = exp((x_i - m+)/gamma), a-_i = exp(-(x_i - m-)/gamma)      (all exponents <= 0)
//   r+ = sum (x_i - m+) a+_i / sum a+_i,  r- = sum (x_i - m-) a-_i / sum a-_i
//   WL = (m+ - m-) + r+ - r-                                          (Eq. 3, rescaled)
//   dWL/dx_i = a+_i/b+ (1 + (x_i - m+ - r+)/gamma) - a-_i/b- (1 - (x_i - m- - r-)/gamma)
// Group buckets: nets of the bucket are laid out padded (net j owns pin slots pin0 + j G ...,
// padding lanes hold cell -1), so a lane's pin slot follows from its index: one round of
// loads (cell index, offset) and one of gathers (position).  A block takes R = kNetsPerLane
// consecutive runs of 256 / G nets; every lane issues the loads of its R nets before using any.
// With H, the same lanes also form the exact HPWL (Eq. 1) of the positions `posu` over the
// same nets (the pin loads are shared; see hpwl_groups for the arithmetic), added to h.  When
// every offset is a multiple of 2^-16 (nd.offq_exact), the quantized offset is formed from the
// float one (the same integer) instead of being loaded.
template <typename T, int G, bool H>
__device__ __forceinline__ void wa_groups(const NetDev &nd, const Buckets &bk, int b, int local,
                                          const vec2<T> *__restrict__ pos, T invg,
                                          vec2<T> *__restrict__ pg, double &wl,
                                          const vec2<T> *__restrict__ posu, int64_t &h) {
    constexpr int NPB = kBlock / G, R = kNetsPerLane;
    const int lane = threadIdx.x & (G - 1);
    const int net0 = bk.net0[b], net1 = bk.net1[b], pin0 = bk.pin0[b];
    const vec2<T> *off = reinterpret_cast<const vec2<T> *>(nd.pin_off);
    // all loads issued on clamped in-range indices before any use: a net past the bucket's end
    // reads the bucket's first slot, a padding lane's cell -1 reads cell 0; both are ignored
    int net[R], p[R], c[R];
    vec2<T> o[R];
    int2 oq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        net[r] = net0 + (local * R + r) * NPB + (int)threadIdx.x / G;
        p[r] = net[r] < net1 ? pin0 + (net[r] - net0) * G + lane : pin0;
        c[r] = nd.pin_cell[p[r]];
        o[r] = off[p[r]];
        if constexpr (H)
            oq[r] = nd.offq_exact ? make_int2(q16i<T>(o[r].x), q16i<T>(o[r].y)) : nd.pin_offq[p[r]];
    }
    vec2<T> q[R], qu[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        q[r] = pos[max(c[r], 0)];
        if constexpr (H) qu[r] = posu[max(c[r], 0)];
    }
    if constexpr (H) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool act = c[r] >= 0 && net[r] < net1;
            const int ux = act ? q16i<T>(qu[r].x) + oq[r].x : 0;
            const int uy = act ? q16i<T>(qu[r].y) + oq[r].y : 0;
            const int xM = group_max<G>(act ? ux : INT_MIN), xm = group_min<G>(act ? ux : INT_MAX);
            const int yM = group_max<G>(act ? uy : INT_MIN), ym = group_min<G>(act ? uy : INT_MAX);
            if (act && lane == 0) h += ((int64_t)xM - xm) + ((int64_t)yM - ym);
        }
    }
    T px[R], py[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (net[r] >= net1) c[r] = -1;
        px[r] = c[r] >= 0 ? q[r].x + o[r].x : T(0);
        py[r] = c[r] >= 0 ? q[r].y + o[r].y : T(0);
    }
    const T inf = pos_inf<T>();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool act = c[r] >= 0, vnet = net[r] < net1;
        const T xmax = group_max<G>(act ? px[r] : -inf), xmin = group_min<G>(act ? px[r] : inf);
        const T ymax = group_max<G>(act ? py[r] : -inf), ymin = group_min<G>(act ? py[r] : inf);
        const T dxp = act ? px[r] - xmax : T(0), dxm = act ? px[r] - xmin : T(0);
        const T dyp = act ? py[r] - ymax : T(0), dym = act ? py[r] - ymin : T(0);
        const T axp = act ? wa_exp<T>(dxp * invg) : T(0), axm = act ? wa_exp<T>(-dxm * invg) : T(0);
        const T ayp = act ? wa_exp<T>(dyp * invg) : T(0), aym = act ? wa_exp<T>(-dym * invg) : T(0);
        // b >= 1 for a real net (its extreme pin contributes exp(0)); padding-only groups are
        // never written or counted
        const T ibxp = wa_rcp<T>(group_sum<G>(axp)), ibxm = wa_rcp<T>(group_sum<G>(axm));
        const T ibyp = wa_rcp<T>(group_sum<G>(ayp)), ibym = wa_rcp<T>(group_sum<G>(aym));
        const T rxp = group_sum<G>(dxp * axp) * ibxp, rxm = group_sum<G>(dxm * axm) * ibxm;
        const T ryp = group_sum<G>(dyp * ayp) * ibyp, rym = group_sum<G>(dym * aym) * ibym;
        const T w = (vnet && nd.net_w) ? reinterpret_cast<const T *>(nd.net_w)[net[r]] : T(1);
        if (act) {
            const T gx = axp * ibxp * (T(1) + (dxp - rxp) * invg) - axm * ibxm * (T(1) - (dxm - rxm) * invg);
            const T gy = ayp * ibyp * (T(1) + (dyp - ryp) * invg) - aym * ibym * (T(1) - (dym - rym) * invg);
            pg[p[r]] = cmk2<T>(w * gx, w * gy);
        }
        if (vnet && lane == 0)
            wl += (double)(w * (((xmax - xmin) + (rxp - rxm)) + ((ymax - ymin) + (ryp - rym))));
    }
}

// Wave-per-net sweep of a padded bucket with S = 64 PPL slots per net: each wave takes one net
// and each lane PPL of its pins (all loads issued before use), sums over them in slot order,
// then the wave's butterflies.
template <typename T, int PPL, bool H>
__device__ __forceinline__ void wa_wave(const NetDev &nd, const Buckets &bk, int b, int local,
                                        const vec2<T> *__restrict__ pos, T invg,
                                        vec2<T> *__restrict__ pg, double &wl,
                                        const vec2<T> *__restrict__ posu, int64_t &h) {
    constexpr int S = 64 * PPL;
    const int lane = threadIdx.x & 63;
    const int net0 = bk.net0[b], net1 = bk.net1[b];
    const int net = net0 + local * (kBlock / 64) + (int)threadIdx.x / 64;
    const bool vnet = net < net1;
    const int p0 = bk.pin0[b] + (vnet ? (net - net0) * S : 0) + lane;
    const vec2<T> *off = reinterpret_cast<const vec2<T> *>(nd.pin_off);
    int c[PPL];
    vec2<T> o[PPL];
    int2 oq[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        c[k] = nd.pin_cell[p0 + 64 * k];
        o[k] = off[p0 + 64 * k];
        if constexpr (H)
            oq[k] = nd.offq_exact ? make_int2(q16i<T>(o[k].x), q16i<T>(o[k].y)) : nd.pin_offq[p0 + 64 * k];
    }
    vec2<T> q[PPL], qu[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        q[k] = pos[max(c[k], 0)];
        if constexpr (H) qu[k] = posu[max(c[k], 0)];
    }
    if constexpr (H) {  // exact HPWL of posu over the same pins (see hpwl_wave)
        int uM = INT_MIN, um = INT_MAX, vM = INT_MIN, vm = INT_MAX;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            if (vnet && c[k] >= 0) {
                const int ux = q16i<T>(qu[k].x) + oq[k].x, uy = q16i<T>(qu[k].y) + oq[k].y;
                uM = max(uM, ux);
                um = min(um, ux);
                vM = max(vM, uy);
                vm = min(vm, uy);
            }
        }
        uM = group_max<64>(uM);
        um = group_min<64>(um);
        vM = group_max<64>(vM);
        vm = group_min<64>(vm);
        if (vnet && lane == 0) h += ((int64_t)uM - um) + ((int64_t)vM - vm);
    }
    const T inf = pos_inf<T>();
    T px[PPL], py[PPL];
    T xM = -inf, xm = inf, yM = -inf, ym = inf;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        if (!vnet) c[k] = -1;
        px[k] = c[k] >= 0 ? q[k].x + o[k].x : T(0);
        py[k] = c[k] >= 0 ? q[k].y + o[k].y : T(0);
        if (c[k] >= 0) {
            xM = max(xM, px[k]);
            xm = min(xm, px[k]);
            yM = max(yM, py[k]);
            ym = min(ym, py[k]);
        }
    }
    xM = group_max<64>(xM);
    xm = group_min<64>(xm);
    yM = group_max<64>(yM);
    ym = group_min<64>(ym);
    // the exponentials are formed again in the gradient pass rather than held (register
    // pressure sets the occupancy of the whole first launch)
    T sm[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const bool act = c[k] >= 0;
        const T dxp = act ? px[k] - xM : T(0), dxm = act ? px[k] - xm : T(0);
        const T dyp = act ? py[k] - yM : T(0), dym = act ? py[k] - ym : T(0);
        const T axp = act ? wa_exp<T>(dxp * invg) : T(0), axm = act ? wa_exp<T>(-dxm * invg) : T(0);
        const T ayp = act ? wa_exp<T>(dyp * invg) : T(0), aym = act ? wa_exp<T>(-dym * invg) : T(0);
        sm[0] += axp;
        sm[1] += axm;
        sm[2] += ayp;
        sm[3] += aym;
        sm[4] += dxp * axp;
        sm[5] += dxm * axm;
        sm[6] += dyp * ayp;
        sm[7] += dym * aym;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) sm[j] = group_sum<64>(sm[j]);
    // an invalid wave (past the bucket's end) has only zero sums; it writes nothing
    const T ibxp = wa_rcp<T>(sm[0]), ibxm = wa_rcp<T>(sm[1]);
    const T ibyp = wa_rcp<T>(sm[2]), ibym = wa_rcp<T>(sm[3]);
    const T rxp = sm[4] * ibxp, rxm = sm[5] * ibxm, ryp = sm[6] * ibyp, rym = sm[7] * ibym;
    const T w = (vnet && nd.net_w) ? reinterpret_cast<const T *>(nd.net_w)[net] : T(1);
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        if (c[k] < 0) continue;
        const T dxp = px[k] - xM, dxm = px[k] - xm, dyp = py[k] - yM, dym = py[k] - ym;
        const T axp = wa_exp<T>(dxp * invg), axm = wa_exp<T>(-dxm * invg);
        const T ayp = wa_exp<T>(dyp * invg), aym = wa_exp<T>(-dym * invg);
        const T gx = axp * ibxp * (T(1) + (dxp - rxp) * invg) - axm * ibxm * (T(1) - (dxm - rxm) * invg);
        const T gy = ayp * ibyp * (T(1) + (dyp - ryp) * invg) - aym * ibym * (T(1) - (dym - rym) * invg);
        pg[p0 + 64 * k] = cmk2<T>(w * gx, w * gy);
    }
    if (vnet && lane == 0)
        wl += (double)(w * (((xM - xm) + (rxp - rxm)) + ((yM - ym) + (ryp - rym))));
}

// Block-per-net sweep.  The first kNetRegs * kBlock pins of the net are loaded once, with all
// of a thread's cell-index loads in flight together and then all its position loads, and kept
// in LDS for the three passes (each thread reads back only its own pins, so no barrier); pins
// beyond that (nets over 2048 pins) are re-streamed in each pass.  Per-thread sums run in pin
// order and the block trees are those of block_sum / block_max.
constexpr int kNetRegs = 8;

template <typename T>
__device__ __forceinline__ void net_pins_to_lds(const NetDev &nd, int s, int d,
                                                const vec2<T> *__restrict__ pos, vec2<T> *sp) {
    // Every load is issued unconditionally on a clamped in-range index and used only after all
    // are in flight (a load whose use sits inside its own branch would be waited for there).
    const vec2<T> *off = reinterpret_cast<const vec2<T> *>(nd.pin_off);
    int c[kNetRegs];
    vec2<T> o[kNetRegs];
#pragma unroll
    for (int k = 0; k < kNetRegs; ++k) {
        const int i = min((int)threadIdx.x + k * kBlock, d - 1);
        c[k] = nd.pin_cell[s + i];
        o[k] = off[s + i];
    }
    vec2<T> q[kNetRegs];
#pragma unroll
    for (int k = 0; k < kNetRegs; ++k) q[k] = pos[c[k]];
#pragma unroll
    for (int k = 0; k < kNetRegs; ++k) {
        const int i = threadIdx.x + k * kBlock;
        if (i < d) sp[i] = cmk2<T>(q[k].x + o[k].x, q[k].y + o[k].y);
    }
}

template <typename T>
__device__ void wa_block(const NetDev &nd, int net, const vec2<T> *__restrict__ pos, T invg,
                         vec2<T> *__restrict__ pg, double &wl) {
    __shared__ T red[4 * 8];
    // the staged pins live in the launch's dynamic LDS, which the scatter's blocks of the same
    // launch use for their histograms or windows (a block does one job), so a block reserves
    // the larger of the two rather than their sum
    extern __shared__ __align__(16) unsigned char sweep_lds[];
    vec2<T> *sp = reinterpret_cast<vec2<T> *>(sweep_lds);  // [kNetRegs * kBlock]
    const int s = nd.net_start[net], d = nd.net_start[net + 1] - s;
    const T inf = pos_inf<T>();
    const vec2<T> *off = reinterpret_cast<const vec2<T> *>(nd.pin_off);
    net_pins_to_lds<T>(nd, s, d, pos, sp);
    const int dr = min(d, kNetRegs * kBlock);  // pins held in LDS
    // every pass visits the thread's pins i = tid, tid + 256, ... in order: those in LDS, then
    // the tail in batches of 4 whose loads are all issued before use
    auto visit = [&](auto &&f) {
        int i = threadIdx.x;
        for (; i < dr; i += kBlock) f(i, sp[i]);
        for (; i < d; i += 4 * kBlock) {
            int c[4];
            vec2<T> o[4], q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = min(i + u * kBlock, d - 1);
                c[u] = nd.pin_cell[s + j];
                o[u] = off[s + j];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = pos[c[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (i + u * kBlock < d) f(i + u * kBlock, cmk2<T>(q[u].x + o[u].x, q[u].y + o[u].y));
        }
    };
    // pass 1: extents (max x, -min x, max y, -min y)
    T m[4] = {-inf, -inf, -inf, -inf};
    visit([&](int, vec2<T> p) {
        m[0] = max(m[0], p.x);
        m[1] = max(m[1], -p.x);
        m[2] = max(m[2], p.y);
        m[3] = max(m[3], -p.y);
    });
    block_max_n<4>(m, red);
    const T xmax = m[0], xmin = -m[1], ymax = m[2], ymin = -m[3];
    // pass 2: exponential sums
    T sm[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    visit([&](int, vec2<T> p) {
        const T dxp = p.x - xmax, dxm = p.x - xmin, dyp = p.y - ymax, dym = p.y - ymin;
        const T axp = wa_exp<T>(dxp * invg), axm = wa_exp<T>(-dxm * invg);
        const T ayp = wa_exp<T>(dyp * invg), aym = wa_exp<T>(-dym * invg);
        sm[0] += axp;
        sm[1] += axm;
        sm[2] += ayp;
        sm[3] += aym;
        sm[4] += dxp * axp;
        sm[5] += dxm * axm;
        sm[6] += dyp * ayp;
        sm[7] += dym * aym;
    });
    block_sum_n<8>(sm, red);
    const T ibxp = wa_rcp<T>(sm[0]), ibxm = wa_rcp<T>(sm[1]);
    const T ibyp = wa_rcp<T>(sm[2]), ibym = wa_rcp<T>(sm[3]);
    const T rxp = sm[4] * ibxp, rxm = sm[5] * ibxm, ryp = sm[6] * ibyp, rym = sm[7] * ibym;
    const T w = nd.net_w ? reinterpret_cast<const T *>(nd.net_w)[net] : T(1);
    // pass 3: per-pin gradients
    visit([&](int i, vec2<T> p) {
        const T dxp = p.x - xmax, dxm = p.x - xmin, dyp = p.y - ymax, dym = p.y - ymin;
        const T axp = wa_exp<T>(dxp * invg), axm = wa_exp<T>(-dxm * invg);
        const T ayp = wa_exp<T>(dyp * invg), aym = wa_exp<T>(-dym * invg);
        vec2<T> g;
        g.x = w * (axp * ibxp * (T(1) + (dxp - rxp) * invg) - axm * ibxm * (T(1) - (dxm - rxm) * invg));
        g.y = w * (ayp * ibyp * (T(1) + (dyp - ryp) * invg) - aym * ibym * (T(1) - (dym - rym) * invg));
        pg[s + i] = g;
    });
    wl = threadIdx.x == 0
             ? (double)(w * (((xmax - xmin) + (rxp - rxm)) + ((ymax - ymin) + (ryp - rym))))
             : 0.0;
}

// ---- exact HPWL ----------------------------------------------------------------------------
// Pin coordinate q16(cell) + q16(offset), both exact integers; per net the x and y extents.
template <typename T, int G>
__device__ __forceinline__ int64_t hpwl_groups(const NetDev &nd, const Buckets &bk, int b, int local,
                                               const vec2<T> *__restrict__ pos) {
    constexpr int NPB = kBlock / G, R = kNetsPerLane;
    const int lane = threadIdx.x & (G - 1);
    const int net0 = bk.net0[b], net1 = bk.net1[b], pin0 = bk.pin0[b];
    int p[R], c[R];
    int2 o[R];
    bool vn[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {  // loads on clamped indices first (see wa_groups)
        const int net = net0 + (local * R + r) * NPB + (int)threadIdx.x / G;
        vn[r] = net < net1;
        p[r] = vn[r] ? pin0 + (net - net0) * G + lane : pin0;
        c[r] = nd.pin_cell[p[r]];
        o[r] = nd.pin_offq[p[r]];
    }
    vec2<T> q[R];
#pragma unroll
    for (int r = 0; r < R; ++r) q[r] = pos[max(c[r], 0)];
    int px[R], py[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!vn[r]) c[r] = -1;
        px[r] = c[r] >= 0 ? q16i<T>(q[r].x) + o[r].x : 0;
        py[r] = c[r] >= 0 ? q16i<T>(q[r].y) + o[r].y : 0;
    }
    int64_t h = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool act = c[r] >= 0;
        const int xM = group_max<G>(act ? px[r] : INT_MIN), xm = group_min<G>(act ? px[r] : INT_MAX);
        const int yM = group_max<G>(act ? py[r] : INT_MIN), ym = group_min<G>(act ? py[r] : INT_MAX);
        if (act && lane == 0) h += ((int64_t)xM - xm) + ((int64_t)yM - ym);
    }
    return h;
}

// Wave-per-net HPWL of a padded bucket with S = 64 PPL slots per net (see wa_wave).
template <typename T, int PPL>
__device__ __forceinline__ int64_t hpwl_wave(const NetDev &nd, const Buckets &bk, int b, int local,
                                             const vec2<T> *__restrict__ pos) {
    constexpr int S = 64 * PPL;
    const int lane = threadIdx.x & 63;
    const int net0 = bk.net0[b], net1 = bk.net1[b];
    const int net = net0 + local * (kBlock / 64) + (int)threadIdx.x / 64;
    const bool vnet = net < net1;
    const int p0 = bk.pin0[b] + (vnet ? (net - net0) * S : 0) + lane;
    int c[PPL];
    int2 o[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        c[k] = nd.pin_cell[p0 + 64 * k];
        o[k] = nd.pin_offq[p0 + 64 * k];
    }
    vec2<T> q[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) q[k] = pos[max(c[k], 0)];
    int xM = INT_MIN, xm = INT_MAX, yM = INT_MIN, ym = INT_MAX;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        if (vnet && c[k] >= 0) {
            const int px = q16i<T>(q[k].x) + o[k].x, py = q16i<T>(q[k].y) + o[k].y;
            xM = max(xM, px);
            xm = min(xm, px);
            yM = max(yM, py);
            ym = min(ym, py);
        }
    }
    xM = group_max<64>(xM);
    xm = group_min<64>(xm);
    yM = group_max<64>(yM);
    ym = group_min<64>(ym);
    return (vnet && lane == 0) ? ((int64_t)xM - xm) + ((int64_t)yM - ym) : 0;
}

template <typename T>
__device__ int64_t hpwl_block(const NetDev &nd, int net, const vec2<T> *__restrict__ pos) {
    __shared__ int red[4 * 4];
    const int s = nd.net_start[net], d = nd.net_start[net + 1] - s;
    int m[4] = {-INT_MAX, -INT_MAX, -INT_MAX, -INT_MAX};  // max x, -min x, max y, -min y
    auto ext = [&](int i, int c) {
        const vec2<T> q = pos[c];
        const int2 o = nd.pin_offq[s + i];
        const int px = q16i<T>(q.x) + o.x, py = q16i<T>(q.y) + o.y;
        m[0] = max(m[0], px);
        m[1] = max(m[1], -px);
        m[2] = max(m[2], py);
        m[3] = max(m[3], -py);
    };
    // the first kNetRegs pins per thread: all loads in flight (clamped indices), then used
    int c[kNetRegs];
    int2 o[kNetRegs];
#pragma unroll
    for (int k = 0; k < kNetRegs; ++k) {
        const int i = min((int)threadIdx.x + k * kBlock, d - 1);
        c[k] = nd.pin_cell[s + i];
        o[k] = nd.pin_offq[s + i];
    }
    vec2<T> q[kNetRegs];
#pragma unroll
    for (int k = 0; k < kNetRegs; ++k) q[k] = pos[c[k]];
#pragma unroll
    for (int k = 0; k < kNetRegs; ++k) {
        if ((int)threadIdx.x + k * kBlock >= d) continue;
        const int px = q16i<T>(q[k].x) + o[k].x, py = q16i<T>(q[k].y) + o[k].y;
        m[0] = max(m[0], px);
        m[1] = max(m[1], -px);
        m[2] = max(m[2], py);
        m[3] = max(m[3], -py);
    }
    for (int i = threadIdx.x + kNetRegs * kBlock; i < d; i += 4 * kBlock) {  // tail, batches of 4
        int cc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) cc[u] = nd.pin_cell[s + min(i + u * kBlock, d - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * kBlock < d) ext(i + u * kBlock, cc[u]);
    }
    block_max_n<4>(m, red);
    return threadIdx.x == 0 ? ((int64_t)m[0] + m[1]) + ((int64_t)m[2] + m[3]) : 0;
}

enum { MODE_WA = 0, MODE_HPWL = 1 };

// This lane's share of the exact HPWL of block-local index `local` of bucket b.
template <typename T>
__device__ __forceinline__ int64_t hpwl_bucket(const NetDev &nd, const Buckets &bk, int b,
                                               int local, const vec2<T> *__restrict__ pos) {
    switch (bk.G[b]) {
        case 2: return hpwl_groups<T, 2>(nd, bk, b, local, pos);
        case 4: return hpwl_groups<T, 4>(nd, bk, b, local, pos);
        case 8: return hpwl_groups<T, 8>(nd, bk, b, local, pos);
        case 16: return hpwl_groups<T, 16>(nd, bk, b, local, pos);
        case 32: return hpwl_groups<T, 32>(nd, bk, b, local, pos);
        case 64: return hpwl_groups<T, 64>(nd, bk, b, local, pos);
        case 128: return hpwl_wave<T, 2>(nd, bk, b, local, pos);
        case 256: return hpwl_wave<T, 4>(nd, bk, b, local, pos);
        default:
            return bk.net0[b] + local < bk.net1[b] ? hpwl_block<T>(nd, bk.net0[b] + local, pos) : 0;
    }
}

// Block `bx` (0 <= bx < bk.total_blocks) of a sweep of one slot: WA over v, or HPWL over u.
// MODE_WA with H: the WA sweep of v and the HPWL sweep of u in the same blocks, both partials
// written.
template <typename T, int MODE, bool H = false>
__device__ __forceinline__ void sweep_body(const NetDev &nd, const Buckets &bk, char *base,
                                           const SlotLayout &L, T invg, int bx) {
    int b = 0;
    while (b + 1 < bk.n && bx >= bk.blk0[b + 1]) ++b;
    const int local = xcd_remap(bx - bk.blk0[b], bk.nblk[b]);
    const int net0 = bk.net0[b], net1 = bk.net1[b];
    const vec2<T> *pos = reinterpret_cast<const vec2<T> *>(base + (MODE == MODE_WA ? L.v : L.u));
    if constexpr (MODE == MODE_WA) {
        vec2<T> *pg = reinterpret_cast<vec2<T> *>(base + L.pin_grad);
        const vec2<T> *posu = reinterpret_cast<const vec2<T> *>(base + L.u);
        double wl = 0.0;
        int64_t h = 0;
        switch (bk.G[b]) {
            case 2: wa_groups<T, 2, H>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 4: wa_groups<T, 4, H>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 8: wa_groups<T, 8, H>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 16: wa_groups<T, 16, H>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 32: wa_groups<T, 32, H>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 64: wa_groups<T, 64, H>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 128: wa_wave<T, 2, H>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 256: wa_wave<T, 4, H>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            default:
                if (net0 + local < net1) {
                    wa_block<T>(nd, net0 + local, pos, invg, pg, wl);
                    if constexpr (H) h = hpwl_block<T>(nd, net0 + local, posu);
                }
                break;
        }
        __shared__ double red[4];
        const double tot = block_sum(wl, red);
        if (threadIdx.x == 0)
            reinterpret_cast<double *>(base + L.part)[PART_WL * L.pstride + bx] = tot;
        if constexpr (H) {
            __shared__ long long redh[4];
            const long long th = block_sum((long long)h, redh);
            if (threadIdx.x == 0)
                (reinterpret_cast<long long *>(base + L.part) + PART_HPWL * L.pstride)[bx] = th;
        }
    } else {
        __shared__ long long red[4];
        const long long tot = block_sum((long long)hpwl_bucket<T>(nd, bk, b, local, pos), red);
        if (threadIdx.x == 0)
            (reinterpret_cast<long long *>(base + L.part) + PART_HPWL * L.pstride)[bx] = tot;
    }
}

// The HPWL sweep on its own (a pending hp_hpwl that no evaluation absorbed).
template <typename T>
__global__ __launch_bounds__(kBlock) void sweep_hpwl_kernel(NetDev nd, Buckets bk, SlotArgs sa,
                                                            SlotLayout L) {
    sweep_body<T, MODE_HPWL>(nd, bk, sa.base[blockIdx.y], L, T(0), blockIdx.x);
}

// The first launch of an evaluation: independent jobs in disjoint block ranges of one grid,
// so that the net sweep and the charge scatter fill the machine together without a second
// stream or any cross-stream synchronisation.  Blocks are dispatched in index order, so the
// longest-latency work comes first:
//   [0, nacc)                 the accumulation of v's charge in the existing grouped order
//                             (nacc = 0 when the slot has no grouping yet);
//   [nacc, nacc + ncnt)       the counting pass of a new grouping from v (ncnt = 0 between
//                             rebuilds);
//   [.., .. + nbig)           the charge of the big cells (macros), one block per cell (nbig =
//                             0 without any);
//   [.., .. + nw)             the WA sweep of v (nw = the sweep's block count; its
//                             block-per-net bucket leads); for the slots in hmask (a deferred
//                             hp_hpwl) the same blocks also sweep the HPWL of u, sharing the pin
//                             loads.
// nacc, ncnt and nbig are multiples of 8, so the sweep keeps the XCD striping of its own blocks.
template <typename T>
__global__ __launch_bounds__(kBlock, 8) void eval_front_kernel(NetDev nd, Buckets bk, SlotArgs sa,
                                                            SlotLayout L, T invg, int nacc,
                                                            int ncnt, int nbig, uint32_t hmask) {
    char *base = sa.base[blockIdx.y];
    const int bx = blockIdx.x;
    const int s0 = nacc + ncnt + nbig;
    if (bx < nacc) {
        accum_body<T>(nd, base, L, bx);
    } else if (bx < nacc + ncnt) {
        count_body<T>(nd, base, L, bx - nacc);
    } else if (bx < s0) {
        big_scatter_body<T>(nd, base, L, bx - nacc - ncnt);
    } else if ((hmask >> blockIdx.y) & 1u) {
        sweep_body<T, MODE_WA, true>(nd, bk, base, L, invg, bx - s0);
    } else {
        sweep_body<T, MODE_WA, false>(nd, bk, base, L, invg, bx - s0);
    }
}

int sweep_parts(const Buckets &bk) { return bk.total_blocks; }

// Exact HPWL of positions the caller holds (pairs over all cells): one partial per block into
// `part`, then one block sums them into out[0].  Every partial is written, so `part` needs no
// clearing.
template <typename T>
__global__ __launch_bounds__(kBlock) void hpwl_pos_kernel(NetDev nd, Buckets bk, const vec2<T> *pos,
                                                          long long *part) {
    const int bx = blockIdx.x;
    int b = 0;
    while (b + 1 < bk.n && bx >= bk.blk0[b + 1]) ++b;
    const int local = xcd_remap(bx - bk.blk0[b], bk.nblk[b]);
    __shared__ long long red[4];
    const long long tot = block_sum((long long)hpwl_bucket<T>(nd, bk, b, local, pos), red);
    if (threadIdx.x == 0) part[bx] = tot;
}

__global__ __launch_bounds__(kBlock) void hpwl_pos_finish_kernel(const long long *part, int n,
                                                                 long long *out) {
    __shared__ long long red[4];
    const long long h = sum_parts(part, n, red);
    if (threadIdx.x == 0) out[0] = h;
}

template <typename T>
hipError_t launch_hpwl_positions(const NetDev &nd, const Buckets &bk, const void *pos,
                                 long long *part, long long *out, hipStream_t st) {
    if (bk.total_blocks > 0) {
        HP_LAUNCH("hpwl_pos_kernel", hpwl_pos_kernel<T>, dim3(bk.total_blocks), dim3(kBlock), 0, st,
                  nd, bk, reinterpret_cast<const vec2<T> *>(pos), part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    HP_LAUNCH("hpwl_pos_finish_kernel", hpwl_pos_finish_kernel, dim3(1), dim3(kBlock), 0, st, part,
              bk.total_blocks, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_eval_front(const NetDev &nd, const Buckets &bk, const SlotArgs &sa,
                             const SlotLayout &L, double inv_gamma, uint32_t hpwl_mask,
                             bool accum, bool count, hipStream_t st) {
    const int nacc = accum ? (nd.max_chunks + kXcds - 1) / kXcds * kXcds : 0;
    const int ncnt = count ? (nd.sort_blocks + kXcds - 1) / kXcds * kXcds : 0;
    const int nbig = (nd.n_big + kXcds - 1) / kXcds * kXcds;
    // dynamic LDS: the largest need of the jobs (a block does one of them; big cells need none)
    const size_t big = (bk.n > 0 && bk.G[0] == 0) ? sizeof(vec2<T>) * kNetRegs * kBlock : 0;
    const size_t lds = std::max({accum ? scatter_accum_lds(nd) : 0,
                                 count ? scatter_count_lds(nd) : 0, big});
    dim3 grid(nacc + ncnt + nbig + bk.total_blocks, sa.n);
    HP_LAUNCH("eval_front_kernel", eval_front_kernel<T>, grid, dim3(kBlock), lds, st, nd, bk, sa,
              L, (T)inv_gamma, nacc, ncnt, nbig, hpwl_mask);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep_hpwl(const NetDev &nd, const Buckets &bk, const SlotArgs &sa,
                             const SlotLayout &L, hipStream_t st) {
    HP_LAUNCH("sweep_hpwl", sweep_hpwl_kernel<T>, dim3(bk.total_blocks, sa.n), dim3(kBlock), 0, st,
              nd, bk, sa, L);
    return hipGetLastError();
}

#define HP_INST(T)                                                                             \
    template hipError_t launch_eval_front<T>(const NetDev &, const Buckets &, const SlotArgs &, \
                                             const SlotLayout &, double, uint32_t, bool, bool,  \
                                             hipStream_t);                                      \
    template hipError_t launch_sweep_hpwl<T>(const NetDev &, const Buckets &, const SlotArgs &, \
                                             const SlotLayout &, hipStream_t);                  \
    template hipError_t launch_hpwl_positions<T>(const NetDev &, const Buckets &, const void *, \
                                                 long long *, long long *, hipStream_t);
HP_INST(float)
HP_INST(double)
#undef HP_INST

}  // namespace hp
