// Net sweeps over the pin CSR: the weighted-average wirelength of Eq. 3 with its per-pin
// gradient, and the exact HPWL of Eq. 1.
//
// Nets are grouped at load time by degree into buckets laid out padded: a net of a bucket of
// G slots (G = next power of two >= its degree, at least 4 from three pins up) owns G
// consecutive pin slots, its pins first and the rest marked by cell -1, so a lane finds its
// slots from its index alone.  Two-pin nets (the largest bucket) take one lane each and the
// closed form of Eq. 3 for two pins; a net of G >= 4 slots spans LP = G / 4 consecutive lanes,
// each owning four consecutive slots that it loads with single 16-byte loads (cell ids,
// offsets), so every pin's exponentials are formed exactly once and the max / min / exp-sum
// reductions run over log2(LP) lane steps.  Nets over 256 pins get a whole block, which
// stages up to 2048 of its pin coordinates in LDS for its three passes (max/min, exp sums,
// gradients).  Within a bucket nets are ordered by their lowest cell, and the blocks of each
// bucket are remapped so that every XCD walks one contiguous eighth of it: neighbouring
// lanes then gather neighbouring cells, and each XCD's gathers stay in a compact cell range.
#include "hp_binning.h"

namespace hp {

// ---- weighted-average wirelength ----------------------------------------------------------
//
// For one net and one axis with pin coordinates x_i, m+ = max x_i, m- = min x_i:
//   a+_i = exp((x_i - m+)/gamma), a-_i = exp(-(x_i - m-)/gamma)      (all exponents <= 0)
//   r+ = sum (x_i - m+) a+_i / sum a+_i,  r- = sum (x_i - m-) a-_i / sum a-_i
//   WL = (m+ - m-) + r+ - r-                                          (Eq. 3, rescaled)
//   dWL/dx_i = a+_i/b+ (1 + (x_i - m+ - r+)/gamma) - a-_i/b- (1 - (x_i - m- - r-)/gamma)
// For two pins at distance D this is WL = D tanh(t), t = D / (2 gamma), and the pin further
// along the axis gets dWL/dx = tanh(t) + t (1 - tanh(t)^2), the other its negative.
//
// With H, the same lanes also form the exact HPWL (Eq. 1) of the positions `posu` over the
// same nets (the pin loads are shared): per pin q16(cell) + q16(offset) in integers, per net
// the x and y extents, added to h by the net's first lane.  When every offset is a multiple of
// 2^-16 (nd.offq_exact), the quantized offset is formed from the float one (the same integer)
// instead of being loaded.

// Native vector types for the non-temporal load and store builtins.
typedef int nt_v2i __attribute__((ext_vector_type(2)));
typedef int nt_v4i __attribute__((ext_vector_type(4)));
typedef float nt_v4f __attribute__((ext_vector_type(4)));

// 16 / 8 bytes of read-once pin data, with a non-temporal hint when NT.
template <bool NT>
__device__ __forceinline__ int4 ld4(const int32_t *p) {
    if constexpr (NT) {
        const nt_v4i v = __builtin_nontemporal_load(reinterpret_cast<const nt_v4i *>(p));
        return make_int4(v.x, v.y, v.z, v.w);
    }
    return *reinterpret_cast<const int4 *>(p);
}
template <bool NT>
__device__ __forceinline__ int2 ld2(const int32_t *p) {
    if constexpr (NT) {
        const nt_v2i v = __builtin_nontemporal_load(reinterpret_cast<const nt_v2i *>(p));
        return make_int2(v.x, v.y);
    }
    return *reinterpret_cast<const int2 *>(p);
}
// 16 bytes of pin gradients, with a non-temporal hint when NT.
template <bool NT>
__device__ __forceinline__ void st4f(float *p, float a, float b, float c, float d) {
    if constexpr (NT) {
        nt_v4f v;
        v.x = a;
        v.y = b;
        v.z = c;
        v.w = d;
        __builtin_nontemporal_store(v, reinterpret_cast<nt_v4f *>(p));
    } else {
        *reinterpret_cast<float4 *>(p) = make_float4(a, b, c, d);
    }
}

// One slot's compact offset (two int16 in units of 2^-off16_shift) as T: the same value as the
// full-width offset, exactly (an int16 times a power of two).
template <typename T>
__device__ __forceinline__ vec2<T> off16(int32_t w, T unit) {
    return cmk2<T>((T)(int)(int16_t)(w & 0xffff) * unit, (T)(w >> 16) * unit);
}

// Four consecutive pin slots (slot a multiple of 4): cell ids and offsets by 16-byte loads
// (one for the offsets when they are compact).
template <typename T, bool NT>
__device__ __forceinline__ void load_slots4(const NetDev &nd, int slot, int (&c)[4],
                                            vec2<T> (&o)[4]) {
    const int4 cc = ld4<NT>(nd.pin_cell + slot);
    c[0] = cc.x;
    c[1] = cc.y;
    c[2] = cc.z;
    c[3] = cc.w;
    if (nd.off16_shift >= 0) {
        const int4 w = ld4<NT>(nd.pin_off16 + slot);
        const T unit = (T)ldexp(1.0, -nd.off16_shift);
        o[0] = off16<T>(w.x, unit);
        o[1] = off16<T>(w.y, unit);
        o[2] = off16<T>(w.z, unit);
        o[3] = off16<T>(w.w, unit);
        return;
    }
    const vec2<T> *off = reinterpret_cast<const vec2<T> *>(nd.pin_off) + slot;
    if constexpr (sizeof(T) == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(off);
        const float4 b = *reinterpret_cast<const float4 *>(off + 2);
        o[0] = cmk2<T>(a.x, a.y);
        o[1] = cmk2<T>(a.z, a.w);
        o[2] = cmk2<T>(b.x, b.y);
        o[3] = cmk2<T>(b.z, b.w);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = off[k];
    }
}
__device__ __forceinline__ void load_offq4(const NetDev &nd, int slot, int2 (&q)[4]) {
    const int4 a = *reinterpret_cast<const int4 *>(nd.pin_offq + slot);
    const int4 b = *reinterpret_cast<const int4 *>(nd.pin_offq + slot + 2);
    q[0] = make_int2(a.x, a.y);
    q[1] = make_int2(a.z, a.w);
    q[2] = make_int2(b.x, b.y);
    q[3] = make_int2(b.z, b.w);
}
// Four gradient pairs to four consecutive slots.
template <typename T, bool NT>
__device__ __forceinline__ void store_grad4(vec2<T> *pg, const T (&gx)[4], const T (&gy)[4]) {
    if constexpr (sizeof(T) == 4) {
        st4f<NT>(reinterpret_cast<float *>(pg), gx[0], gy[0], gx[1], gy[1]);
        st4f<NT>(reinterpret_cast<float *>(pg + 2), gx[2], gy[2], gx[3], gy[3]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) pg[k] = cmk2<T>(gx[k], gy[k]);
    }
}

// tanh(t) of t = D / (2 gamma) >= 0 as (1 - e) / (1 + e), e = exp(-D / gamma), with 1 - e
// formed by expm1 so that short nets keep their relative accuracy.
template <typename T> __device__ __forceinline__ T wa_tanh2(T d_over_gamma);
template <> __device__ __forceinline__ float wa_tanh2<float>(float u) {
    return -expm1f(-u) * __builtin_amdgcn_rcpf(1.0f + __expf(-u));
}
template <> __device__ __forceinline__ double wa_tanh2<double>(double u) {
    return -expm1(-u) / (1.0 + exp(-u));
}

// Two-pin nets, one lane each, kPairNets per lane (net = net0 + (local kPairNets + r) kBlock +
// lane, so a wave's loads are contiguous): WL = D tanh(D / 2 gamma) per axis.
template <typename T, bool H, bool NT>
__device__ __forceinline__ void wa_pairs(const NetDev &nd, const Buckets &bk, int b, int local,
                                         const vec2<T> *__restrict__ pos, T invg,
                                         vec2<T> *__restrict__ pg, double &wl,
                                         const vec2<T> *__restrict__ posu, int64_t &h) {
    constexpr int R = kPairNets;
    const int net0 = bk.net0[b], net1 = bk.net1[b], pin0 = bk.pin0[b];
    const vec2<T> *off = reinterpret_cast<const vec2<T> *>(nd.pin_off);
    const T unit = (T)ldexp(1.0, -max(nd.off16_shift, 0));
    int net[R], slot[R];
    int2 c[R];
    vec2<T> o0[R], o1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {  // loads on clamped in-range slots first
        net[r] = net0 + (local * R + r) * kBlock + (int)threadIdx.x;
        slot[r] = pin0 + (net[r] < net1 ? 2 * (net[r] - net0) : 0);
        c[r] = ld2<NT>(nd.pin_cell + slot[r]);
        if (nd.off16_shift >= 0) {
            const int2 w = ld2<NT>(nd.pin_off16 + slot[r]);
            o0[r] = off16<T>(w.x, unit);
            o1[r] = off16<T>(w.y, unit);
        } else if constexpr (sizeof(T) == 4) {
            const float4 a = *reinterpret_cast<const float4 *>(off + slot[r]);
            o0[r] = cmk2<T>(a.x, a.y);
            o1[r] = cmk2<T>(a.z, a.w);
        } else {
            o0[r] = off[slot[r]];
            o1[r] = off[slot[r] + 1];
        }
    }
    vec2<T> q0[R], q1[R], u0[R], u1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        q0[r] = pos[c[r].x];
        q1[r] = pos[c[r].y];
        if constexpr (H) {
            u0[r] = posu[c[r].x];
            u1[r] = posu[c[r].y];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (net[r] >= net1) continue;
        if constexpr (H) {
            int2 oq0, oq1;
            if (nd.offq_exact) {
                oq0 = make_int2(q16i<T>(o0[r].x), q16i<T>(o0[r].y));
                oq1 = make_int2(q16i<T>(o1[r].x), q16i<T>(o1[r].y));
            } else {
                const int4 a = *reinterpret_cast<const int4 *>(nd.pin_offq + slot[r]);
                oq0 = make_int2(a.x, a.y);
                oq1 = make_int2(a.z, a.w);
            }
            const int dx = (q16i<T>(u0[r].x) + oq0.x) - (q16i<T>(u1[r].x) + oq1.x);
            const int dy = (q16i<T>(u0[r].y) + oq0.y) - (q16i<T>(u1[r].y) + oq1.y);
            h += (int64_t)abs(dx) + (int64_t)abs(dy);
        }
        const T dx = (q0[r].x + o0[r].x) - (q1[r].x + o1[r].x);
        const T dy = (q0[r].y + o0[r].y) - (q1[r].y + o1[r].y);
        const T ax = fabs(dx), ay = fabs(dy);
        const T thx = wa_tanh2<T>(ax * invg), thy = wa_tanh2<T>(ay * invg);
        const T tx = T(0.5) * ax * invg, ty = T(0.5) * ay * invg;
        const T w = nd.net_w ? reinterpret_cast<const T *>(nd.net_w)[net[r]] : T(1);
        const T gx = w * (thx + tx * (T(1) - thx * thx)), gy = w * (thy + ty * (T(1) - thy * thy));
        const T sx = dx >= T(0) ? gx : -gx, sy = dy >= T(0) ? gy : -gy;
        if constexpr (sizeof(T) == 4)
            st4f<NT>(reinterpret_cast<float *>(pg + slot[r]), sx, sy, -sx, -sy);
        else {
            pg[slot[r]] = cmk2<T>(sx, sy);
            pg[slot[r] + 1] = cmk2<T>(-sx, -sy);
        }
        wl += (double)(w * (ax * thx + ay * thy));
    }
}

// Nets of G = 4 LP slots, LP lanes each (LP = 1 .. 64), one net per lane group and block row:
// lane l of the group owns slots 4 l .. 4 l + 3 of its net.
template <typename T, int LP, bool H, bool NT>
__device__ __forceinline__ void wa_lanes(const NetDev &nd, const Buckets &bk, int b, int local,
                                         const vec2<T> *__restrict__ pos, T invg,
                                         vec2<T> *__restrict__ pg, double &wl,
                                         const vec2<T> *__restrict__ posu, int64_t &h) {
    constexpr int G = 4 * LP, NPB = kBlock / LP;
    const int l = threadIdx.x & (LP - 1);
    const int net0 = bk.net0[b], net1 = bk.net1[b];
    const int net = net0 + local * NPB + (int)threadIdx.x / LP;
    const bool vnet = net < net1;
    const int slot = bk.pin0[b] + (vnet ? (net - net0) * G : 0) + 4 * l;
    // every load issued on in-range slots before any use (a net past the bucket's end reads
    // its first net's slots, a padding slot's cell -1 reads cell 0; both are ignored)
    int c[4];
    vec2<T> o[4];
    load_slots4<T, NT>(nd, slot, c, o);
    int2 oq[4];
    if constexpr (H) {
        if (nd.offq_exact) {
#pragma unroll
            for (int k = 0; k < 4; ++k) oq[k] = make_int2(q16i<T>(o[k].x), q16i<T>(o[k].y));
        } else {
            load_offq4(nd, slot, oq);
        }
    }
    vec2<T> q[4], qu[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        q[k] = pos[max(c[k], 0)];
        if constexpr (H) qu[k] = posu[max(c[k], 0)];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (!vnet) c[k] = -1;
    if constexpr (H) {
        int xM = INT_MIN, xm = INT_MAX, yM = INT_MIN, ym = INT_MAX;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (c[k] < 0) continue;
            const int ux = q16i<T>(qu[k].x) + oq[k].x, uy = q16i<T>(qu[k].y) + oq[k].y;
            xM = max(xM, ux);
            xm = min(xm, ux);
            yM = max(yM, uy);
            ym = min(ym, uy);
        }
        xM = group_max<LP>(xM);
        xm = group_min<LP>(xm);
        yM = group_max<LP>(yM);
        ym = group_min<LP>(ym);
        if (vnet && l == 0) h += ((int64_t)xM - xm) + ((int64_t)yM - ym);
    }
    const T inf = pos_inf<T>();
    T px[4], py[4];
    T xM = -inf, xm = inf, yM = -inf, ym = inf;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        px[k] = c[k] >= 0 ? q[k].x + o[k].x : T(0);
        py[k] = c[k] >= 0 ? q[k].y + o[k].y : T(0);
        if (c[k] >= 0) {
            xM = max(xM, px[k]);
            xm = min(xm, px[k]);
            yM = max(yM, py[k]);
            ym = min(ym, py[k]);
        }
    }
    xM = group_max<LP>(xM);
    xm = group_min<LP>(xm);
    yM = group_max<LP>(yM);
    ym = group_min<LP>(ym);
    // the exponentials are formed again in the gradient pass rather than held (register
    // pressure sets the occupancy of the whole first launch)
    T sm[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
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
    for (int j = 0; j < 8; ++j) sm[j] = group_sum<LP>(sm[j]);
    // b >= 1 for a real net (its extreme pin contributes exp(0)); an invalid group has only
    // zero sums and writes nothing
    const T ibxp = wa_rcp<T>(sm[0]), ibxm = wa_rcp<T>(sm[1]);
    const T ibyp = wa_rcp<T>(sm[2]), ibym = wa_rcp<T>(sm[3]);
    const T rxp = sm[4] * ibxp, rxm = sm[5] * ibxm, ryp = sm[6] * ibyp, rym = sm[7] * ibym;
    const T w = (vnet && nd.net_w) ? reinterpret_cast<const T *>(nd.net_w)[net] : T(1);
    T gx[4], gy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T dxp = px[k] - xM, dxm = px[k] - xm, dyp = py[k] - yM, dym = py[k] - ym;
        const T axp = wa_exp<T>(dxp * invg), axm = wa_exp<T>(-dxm * invg);
        const T ayp = wa_exp<T>(dyp * invg), aym = wa_exp<T>(-dym * invg);
        gx[k] = c[k] < 0 ? T(0)
                         : w * (axp * ibxp * (T(1) + (dxp - rxp) * invg) -
                                axm * ibxm * (T(1) - (dxm - rxm) * invg));
        gy[k] = c[k] < 0 ? T(0)
                         : w * (ayp * ibyp * (T(1) + (dyp - ryp) * invg) -
                                aym * ibym * (T(1) - (dym - rym) * invg));
    }
    if (vnet) store_grad4<T, NT>(pg + slot, gx, gy);
    if (vnet && l == 0)
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
template <typename T>
__device__ __forceinline__ int64_t hpwl_pairs(const NetDev &nd, const Buckets &bk, int b, int local,
                                              const vec2<T> *__restrict__ pos) {
    constexpr int R = kPairNets;
    const int net0 = bk.net0[b], net1 = bk.net1[b], pin0 = bk.pin0[b];
    int net[R];
    int2 c[R];
    int4 oq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        net[r] = net0 + (local * R + r) * kBlock + (int)threadIdx.x;
        const int slot = pin0 + (net[r] < net1 ? 2 * (net[r] - net0) : 0);
        c[r] = *reinterpret_cast<const int2 *>(nd.pin_cell + slot);
        oq[r] = *reinterpret_cast<const int4 *>(nd.pin_offq + slot);
    }
    vec2<T> q0[R], q1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        q0[r] = pos[c[r].x];
        q1[r] = pos[c[r].y];
    }
    int64_t h = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (net[r] >= net1) continue;
        const int dx = (q16i<T>(q0[r].x) + oq[r].x) - (q16i<T>(q1[r].x) + oq[r].z);
        const int dy = (q16i<T>(q0[r].y) + oq[r].y) - (q16i<T>(q1[r].y) + oq[r].w);
        h += (int64_t)abs(dx) + (int64_t)abs(dy);
    }
    return h;
}

template <typename T, int LP>
__device__ __forceinline__ int64_t hpwl_lanes(const NetDev &nd, const Buckets &bk, int b, int local,
                                              const vec2<T> *__restrict__ pos) {
    constexpr int G = 4 * LP, NPB = kBlock / LP;
    const int l = threadIdx.x & (LP - 1);
    const int net0 = bk.net0[b], net1 = bk.net1[b];
    const int net = net0 + local * NPB + (int)threadIdx.x / LP;
    const bool vnet = net < net1;
    const int slot = bk.pin0[b] + (vnet ? (net - net0) * G : 0) + 4 * l;
    const int4 cc = *reinterpret_cast<const int4 *>(nd.pin_cell + slot);
    const int c[4] = {cc.x, cc.y, cc.z, cc.w};
    int2 oq[4];
    load_offq4(nd, slot, oq);
    vec2<T> q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = pos[max(c[k], 0)];
    int xM = INT_MIN, xm = INT_MAX, yM = INT_MIN, ym = INT_MAX;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!vnet || c[k] < 0) continue;
        const int px = q16i<T>(q[k].x) + oq[k].x, py = q16i<T>(q[k].y) + oq[k].y;
        xM = max(xM, px);
        xm = min(xm, px);
        yM = max(yM, py);
        ym = min(ym, py);
    }
    xM = group_max<LP>(xM);
    xm = group_min<LP>(xm);
    yM = group_max<LP>(yM);
    ym = group_min<LP>(ym);
    return (vnet && l == 0) ? ((int64_t)xM - xm) + ((int64_t)yM - ym) : 0;
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

// Bucket b and bucket-local block index of sweep block bx.  Default order: bucket after bucket,
// each padded bucket's blocks remapped so that XCD x (blocks bx with bx % 8 == x) walks one
// contiguous eighth of it.  Interleaved order: the block-per-net bucket first, then on every XCD the
// blocks of the padded buckets merged by their progress through their eighth (nd.sweep_map),
// so all buckets sweep the same cell range at the same time.
__device__ __forceinline__ void sweep_block(const NetDev &nd, const Buckets &bk, int bx, int &b,
                                            int &local) {
    if (nd.sweep_interleave && bx >= nd.sweep_lead) {
        const int r = bx - nd.sweep_lead;
        const int e = nd.sweep_map[r / kXcds];
        b = e >> 24;
        local = (r % kXcds) * (bk.nblk[b] / kXcds) + (e & 0xffffff);
        return;
    }
    b = 0;
    while (b + 1 < bk.n && bx >= bk.blk0[b + 1]) ++b;
    // The block-per-net bucket is ordered by decreasing size: its blocks take the nets in grid
    // order, so that consecutive (widest first) nets go to different XCDs and every XCD gets an
    // even share of the work; in the padded buckets each XCD takes a contiguous eighth, whose
    // nets gather a compact cell range.
    local = bk.G[b] == 0 ? bx - bk.blk0[b] : xcd_remap(bx - bk.blk0[b], bk.nblk[b]);
}

// This lane's share of the exact HPWL of block-local index `local` of bucket b.
template <typename T>
__device__ __forceinline__ int64_t hpwl_bucket(const NetDev &nd, const Buckets &bk, int b,
                                               int local, const vec2<T> *__restrict__ pos) {
    switch (bk.G[b]) {
        case 2: return hpwl_pairs<T>(nd, bk, b, local, pos);
        case 4: return hpwl_lanes<T, 1>(nd, bk, b, local, pos);
        case 8: return hpwl_lanes<T, 2>(nd, bk, b, local, pos);
        case 16: return hpwl_lanes<T, 4>(nd, bk, b, local, pos);
        case 32: return hpwl_lanes<T, 8>(nd, bk, b, local, pos);
        case 64: return hpwl_lanes<T, 16>(nd, bk, b, local, pos);
        case 128: return hpwl_lanes<T, 32>(nd, bk, b, local, pos);
        case 256: return hpwl_lanes<T, 64>(nd, bk, b, local, pos);
        default:
            return bk.net0[b] + local < bk.net1[b] ? hpwl_block<T>(nd, bk.net0[b] + local, pos) : 0;
    }
}

// Block `bx` (0 <= bx < bk.total_blocks) of a sweep of one slot: WA over v, or HPWL over u.
// MODE_WA with H: the WA sweep of v and the HPWL sweep of u in the same blocks, both partials
// written.
template <typename T, int MODE, bool H = false, bool NT = false>
__device__ __forceinline__ void sweep_body(const NetDev &nd, const Buckets &bk, char *base,
                                           const SlotLayout &L, T invg, int bx) {
    int b, local;
    sweep_block(nd, bk, bx, b, local);
    const int net0 = bk.net0[b], net1 = bk.net1[b];
    const vec2<T> *pos = reinterpret_cast<const vec2<T> *>(base + (MODE == MODE_WA ? L.v : L.u));
    if constexpr (MODE == MODE_WA) {
        vec2<T> *pg = reinterpret_cast<vec2<T> *>(base + L.pin_grad);
        const vec2<T> *posu = reinterpret_cast<const vec2<T> *>(base + L.u);
        double wl = 0.0;
        int64_t h = 0;
        switch (bk.G[b]) {
            case 2: wa_pairs<T, H, NT>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 4: wa_lanes<T, 1, H, NT>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 8: wa_lanes<T, 2, H, NT>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 16: wa_lanes<T, 4, H, NT>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 32: wa_lanes<T, 8, H, NT>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 64: wa_lanes<T, 16, H, NT>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 128: wa_lanes<T, 32, H, NT>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
            case 256: wa_lanes<T, 64, H, NT>(nd, bk, b, local, pos, invg, pg, wl, posu, h); break;
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
//                             rebuilds), with the cells' charge records when `records` (the
//                             new order accumulates in this evaluation);
//   [.., .. + nbig)           the charge of the big cells (macros), one block per cell (nbig =
//                             0 without any);
//   [.., .. + nw)             the WA sweep of v (nw = the sweep's block count; its
//                             block-per-net bucket leads); for the slots in hmask (a deferred
//                             hp_hpwl) the same blocks also sweep the HPWL of u, sharing the pin
//                             loads.
// nacc, ncnt and nbig are multiples of 8, so the sweep keeps the XCD striping of its own blocks.
template <typename T, bool NT>
__global__ __launch_bounds__(kBlock, 8) void eval_front_kernel(NetDev nd, Buckets bk, SlotArgs sa,
                                                            SlotLayout L, T invg, int nacc,
                                                            int ncnt, int nbig, uint32_t hmask,
                                                            int records) {
    char *base = sa.base[blockIdx.y];
    const int bx = blockIdx.x;
    const int s0 = nacc + ncnt + nbig;
    if (bx < nacc) {
        accum_body<T, false>(nd, base, L, bx);
    } else if (bx < nacc + ncnt) {
        count_body<T>(nd, base, L, bx - nacc, records != 0);
    } else if (bx < s0) {
        big_scatter_body<T>(nd, base, L, bx - nacc - ncnt);
    } else if ((hmask >> blockIdx.y) & 1u) {
        sweep_body<T, MODE_WA, true, NT>(nd, bk, base, L, invg, bx - s0);
    } else {
        sweep_body<T, MODE_WA, false, NT>(nd, bk, base, L, invg, bx - s0);
    }
}

// The first launch over steady-state slots of different netlists: each slot's netlist,
// buckets, layout and smoothing from its descriptor, its block ranges as above from its own
// sizes and the masks (bit blockIdx.y); blocks past the slot's own range return.
template <typename T>
__global__ __launch_bounds__(kBlock, 8) void rag_front_kernel(SlotArgs sa, SlotGammas g,
                                                              uint32_t accm, uint32_t cntm,
                                                              uint32_t hmask) {
    char *base = sa.base[blockIdx.y];
    const SlotDesc *d = slot_desc(base);
    const NetDev &nd = d->nd;
    const Buckets &bk = d->bk;
    const SlotLayout &L = d->L;
    const int nacc = ((accm >> blockIdx.y) & 1u) ? round8(nd.max_chunks) : 0;
    const int ncnt = ((cntm >> blockIdx.y) & 1u) ? round8(nd.sort_blocks) : 0;
    const int nbig = round8(nd.n_big);
    const int s0 = nacc + ncnt + nbig;
    const int bx = blockIdx.x;
    if (bx >= s0 + bk.total_blocks) return;  // whole block
    const T invg = (T)g.inv[blockIdx.y];
    if (bx < nacc) {
        accum_body<T, false>(nd, base, L, bx);
    } else if (bx < nacc + ncnt) {
        count_body<T>(nd, base, L, bx - nacc, true);  // the new order accumulates right after
    } else if (bx < s0) {
        big_scatter_body<T>(nd, base, L, bx - nacc - ncnt);
    } else if ((hmask >> blockIdx.y) & 1u) {
        sweep_body<T, MODE_WA, true>(nd, bk, base, L, invg, bx - s0);
    } else {
        sweep_body<T, MODE_WA, false>(nd, bk, base, L, invg, bx - s0);
    }
}

template <typename T>
hipError_t rag_front(const SlotArgs &sa, const SlotGammas &g, uint32_t accm, uint32_t cntm,
                     uint32_t hmask, int grid_x, size_t lds, hipStream_t st) {
    HP_LAUNCH("eval_front_kernel", rag_front_kernel<T>, dim3(grid_x, sa.n), dim3(kBlock), lds, st,
              sa, g, accm, cntm, hmask);
    return hipGetLastError();
}

// Blocks and dynamic LDS of one slot's share of a first launch (as launch_eval_front sizes them)
int front_blocks(const NetDev &nd, const Buckets &bk, bool accum, bool count) {
    return (accum ? round8(nd.max_chunks) : 0) + (count ? round8(nd.sort_blocks) : 0) +
           round8(nd.n_big) + bk.total_blocks;
}
template <typename T>
size_t front_lds(const NetDev &nd, const Buckets &bk, bool accum, bool count) {
    const size_t big = (bk.n > 0 && bk.G[0] == 0) ? sizeof(vec2<T>) * kNetRegs * kBlock : 0;
    return std::max({accum ? scatter_accum_lds(nd) : 0, count ? scatter_count_lds(nd) : 0, big});
}

int sweep_parts(const Buckets &bk) { return bk.total_blocks; }

// Exact HPWL of positions the caller holds (pairs over all cells): one partial per block into
// `part`, then one block sums them into out[0].  Every partial is written, so `part` needs no
// clearing.
template <typename T>
__global__ __launch_bounds__(kBlock) void hpwl_pos_kernel(NetDev nd, Buckets bk, const vec2<T> *pos,
                                                          long long *part) {
    int b, local;
    sweep_block(nd, bk, blockIdx.x, b, local);
    __shared__ long long red[4];
    const long long tot = block_sum((long long)hpwl_bucket<T>(nd, bk, b, local, pos), red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
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
                             bool accum, bool count, bool records, bool sweep, hipStream_t st) {
    const int nacc = accum ? (nd.max_chunks + kXcds - 1) / kXcds * kXcds : 0;
    const int ncnt = count ? (nd.sort_blocks + kXcds - 1) / kXcds * kXcds : 0;
    const int nbig = (nd.n_big + kXcds - 1) / kXcds * kXcds;
    // dynamic LDS: the largest need of the jobs (a block does one of them; big cells need none)
    const size_t big = (sweep && bk.n > 0 && bk.G[0] == 0) ? sizeof(vec2<T>) * kNetRegs * kBlock : 0;
    const size_t lds = std::max({accum ? scatter_accum_lds(nd) : 0,
                                 count ? scatter_count_lds(nd) : 0, big});
    dim3 grid(nacc + ncnt + nbig + (sweep ? bk.total_blocks : 0), sa.n);
    if (grid.x == 0) return hipSuccess;
    if (nd.sweep_nt)
        HP_LAUNCH("eval_front_kernel", (eval_front_kernel<T, true>), grid, dim3(kBlock), lds, st,
                  nd, bk, sa, L, (T)inv_gamma, nacc, ncnt, nbig, hpwl_mask, (int)records);
    else
        HP_LAUNCH("eval_front_kernel", (eval_front_kernel<T, false>), grid, dim3(kBlock), lds, st,
                  nd, bk, sa, L, (T)inv_gamma, nacc, ncnt, nbig, hpwl_mask, (int)records);
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
                                             bool, bool, hipStream_t);                          \
    template hipError_t launch_sweep_hpwl<T>(const NetDev &, const Buckets &, const SlotArgs &, \
                                             const SlotLayout &, hipStream_t);                  \
    template hipError_t launch_hpwl_positions<T>(const NetDev &, const Buckets &, const void *, \
                                                 long long *, long long *, hipStream_t);        \
    template size_t front_lds<T>(const NetDev &, const Buckets &, bool, bool);                  \
    template hipError_t rag_front<T>(const SlotArgs &, const SlotGammas &, uint32_t, uint32_t,  \
                                     uint32_t, int, size_t, hipStream_t);
HP_INST(float)
HP_INST(double)
#undef HP_INST

}  // namespace hp
