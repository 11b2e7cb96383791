// Closing reductions of an evaluation and of the HPWL sweep, the preconditioned Nesterov step,
// the first-evaluation gradient combination, and the best-of selection of Alg. 1.  Every total
// is a fixed-order reduction of per-block partials (thread t sums partials t, t + blockDim, ... then
// a fixed tree) by one block per slot, so repeated runs are bit-identical.
#include "hp_device.h"

namespace hp {

// Totals of one evaluation: WL (Eq. 3), energy N, overflow; lambda_0 on a slot's first
// evaluation with the scheduled lambda (scale * |grad WL|_1 / |grad N|_1); the lambda the
// following step preconditions with and, in steady state, that step's proposal from the
// reductions the cell-gradient pass formed.
// One 1024-thread block per slot: the partial counts reach tens of thousands at millions of
// cells, and a single block is latency bound, so it keeps 16 waves of loads in flight.
constexpr int kFinBlock = 1024;
constexpr int kFinWaves = kFinBlock / 64;

// RAG: the slot's netlist and layout from its descriptor, ncell its own cell-gradient block
// count (the steady-state step form only: nwl = ne = nov = 0).
template <bool RAG>
__global__ __launch_bounds__(kFinBlock) void eval_finish_kernel(NetDev nda, SlotArgs sa, SlotLayout La,
                                                               int nwl, int ne, int nov, int ncell_arg,
                                                               int use_fixed, double lam_fixed,
                                                               int mode, uint32_t banks) {
    __shared__ double rs[kFinWaves][4], rm[kFinWaves];
    __shared__ long long ri[kFinWaves];
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    const int ncell = RAG ? max(1, cell_parts(nd)) : ncell_arg;  // as launch_cell_grad
    Scalars *sc = scalars(base, L);
    const double *part = reinterpret_cast<const double *>(base + L.part);
    // mode FIN_TOTALS: the WL, energy and overflow of the last evaluation only; FIN_STEP: the
    // step's lambda and proposal only (the totals are reduced when read); FIN_FULL: both, and
    // lambda_0 on a first evaluation
    const bool totals = mode != FIN_STEP, full = mode != FIN_TOTALS;
    const bool init = full && !use_fixed && sc->lambda_valid == 0;
    const bool prop = full && !init && ncell > 0;
    // One pass over all partial arrays with their loads in flight together (thread t takes
    // elements t, t + 1024, ... of each, in order), then a fixed tree over the waves.
    const double *pw = part + PART_WL * L.pstride, *pe = part + PART_E * L.pstride;
    const double *pa = part + (init ? PART_N1 : PART_DV) * L.pstride;
    const double *pb = part + (init ? PART_N2 : PART_DG) * L.pstride;
    const double *pg = part + PART_GMAX * L.pstride;
    const long long *po = reinterpret_cast<const long long *>(part) + PART_OVF * L.pstride;
    const int nab = (init || prop) ? ncell : 0, ng = prop ? ncell : 0;
    const int nmax = max(max(nwl, ne), max(nov, nab));
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    double gm = 0.0;
    long long ov = 0;
    if (nwl == 0 && ne == 0 && nov == 0) {
        // The step's reductions alone (steady state above 1024 cell blocks): three arrays, so
        // each thread keeps 12 elements of each in flight per round (one round up to 12,288
        // partials).  The same elements in the same order as the general loop below.
        constexpr int U = 12;
        for (int i = threadIdx.x; i < nab; i += U * kFinBlock) {
            double a[U], b[U], c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = i + u * kFinBlock;
                a[u] = j < nab ? pa[j] : 0.0;
                b[u] = j < nab ? pb[j] : 0.0;
                c[u] = j < ng ? pg[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                v[2] += a[u];
                v[3] += b[u];
                gm = fmax(gm, c[u]);
            }
        }
    } else
    for (int i = threadIdx.x; i < nmax; i += 4 * kFinBlock) {
        double a[4][5];
        long long o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = i + u * kFinBlock;
            a[u][0] = j < nwl ? pw[j] : 0.0;
            a[u][1] = j < ne ? pe[j] : 0.0;
            a[u][2] = j < nab ? pa[j] : 0.0;
            a[u][3] = j < nab ? pb[j] : 0.0;
            a[u][4] = j < ng ? pg[j] : 0.0;
            o[u] = j < nov ? po[j] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] += a[u][k];
            gm = fmax(gm, a[u][4]);
            ov += o[u];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = group_sum<64>(v[j]);
    gm = group_max<64>(gm);
    ov = group_sum<64>(ov);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) rs[w][j] = v[j];
        rm[w] = gm;
        ri[w] = ov;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // Pairwise tree over the 16 wave totals.
        double t[4];
        double GM;
        long long OV;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double q[kFinWaves];
#pragma unroll
            for (int k = 0; k < kFinWaves; ++k) q[k] = rs[k][j];
#pragma unroll
            for (int h = kFinWaves / 2; h > 0; h >>= 1)
#pragma unroll
                for (int k = 0; k < h; ++k) q[k] += q[k + h];
            t[j] = q[0];
        }
        {
            double q[kFinWaves];
            long long qi[kFinWaves];
#pragma unroll
            for (int k = 0; k < kFinWaves; ++k) {
                q[k] = rm[k];
                qi[k] = ri[k];
            }
#pragma unroll
            for (int h = kFinWaves / 2; h > 0; h >>= 1)
#pragma unroll
                for (int k = 0; k < h; ++k) {
                    q[k] = fmax(q[k], q[k + h]);
                    qi[k] += qi[k + h];
                }
            GM = q[0];
            OV = qi[0];
        }
        if (totals) {
            sc->wl = t[0];
            sc->energy = 0.5 * nd.wb * nd.hb * t[1];
            sc->overflow_num = OV;
            sc->overflow = (double)OV / (double)nd.total_charge;
        }
        if (full) {
            sc->init_this_eval = init ? 1 : 0;
            if (init) {
                sc->lambda = sc->lambda0_scale * (t[3] > 0.0 ? t[2] / t[3] : 1.0);
                sc->lambda_valid = 1;
            }
            sc->lambda_step = use_fixed ? lam_fixed : sc->lambda;
            if (prop) step_propose(sc, t[2], t[3], GM, nd.wb, (banks >> blockIdx.y) & 1u);
        }
    }
}

// HPWL (Eq. 1) total of the per-block partials of the sweep.
__global__ __launch_bounds__(kBlock) void hpwl_finish_kernel(SlotArgs sa, SlotLayout L, int n) {
    __shared__ long long red[4];
    char *base = sa.base[blockIdx.x];
    const long long h =
        sum_parts(reinterpret_cast<const long long *>(base + L.part) + PART_HPWL * L.pstride, n, red);
    if (threadIdx.x == 0) {
        Scalars *sc = scalars(base, L);
        sc->hpwl_q = h;
        sc->hpwl_valid = 1;
    }
}

hipError_t launch_eval_finish(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L, int nwl,
                              int ne, int nov, int ncell, bool use_fixed, double lam_fixed,
                              int mode, uint32_t banks, hipStream_t st) {
    const bool totals = mode != FIN_STEP, full = mode != FIN_TOTALS;
    HP_LAUNCH("eval_finish_kernel", eval_finish_kernel<false>, dim3(1, sa.n), dim3(kFinBlock), 0, st, nd, sa,
              L, totals ? nwl : 0, totals ? ne : 0, totals ? nov : 0, full ? ncell : 0,
              (int)use_fixed, lam_fixed, mode, banks);
    return hipGetLastError();
}

hipError_t launch_hpwl_finish(const SlotArgs &sa, const SlotLayout &L, int nparts, hipStream_t st) {
    HP_LAUNCH("hpwl_finish_kernel", hpwl_finish_kernel, dim3(sa.n), dim3(kBlock), 0, st, sa, L,
              nparts);
    return hipGetLastError();
}

// First evaluation only: g = gWL + lambda_0 gD.
template <typename T>
__global__ __launch_bounds__(kBlock) void combine_kernel(NetDev nd, SlotArgs sa, SlotLayout L) {
    char *base = sa.base[blockIdx.y];
    const Scalars *sc = scalars(base, L);
    if (!sc->init_this_eval) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 2 * nd.n_mov) return;
    T *g = reinterpret_cast<T *>(base + L.g);
    const T *gd = reinterpret_cast<const T *>(base + L.gd);
    g[i] += (T)sc->lambda * gd[i];
}

// ---- Nesterov -------------------------------------------------------------------------------
// The step's reductions when the evaluation did not form them (a slot's first evaluation, or a
// second step on one gradient): per block |v - v_prev|^2, |g~ - g~_prev|^2, max|g~|.
template <typename T>
__global__ __launch_bounds__(kBlock) void step_norms_kernel(NetDev nd, SlotArgs sa, SlotLayout L) {
    __shared__ double red[4 * 3];
    char *base = sa.base[blockIdx.y];
    const Scalars *sc = scalars(base, L);
    const int n = nd.n_mov;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const T *g = reinterpret_cast<const T *>(base + L.g);
    const bool live = i < n;
    step_block_norms<T>(nd, base, L, blockIdx.x, i, live, live ? g[i] : (T)0, live ? g[n + i] : (T)0,
                        sc->lambda_step, red);
}

// Totals of those reductions and the step proposal.
__global__ __launch_bounds__(kBlock) void step_scalars_kernel(NetDev nd, SlotArgs sa, SlotLayout L,
                                                             int nb, uint32_t banks) {
    __shared__ double red[4];
    char *base = sa.base[blockIdx.y];
    Scalars *sc = scalars(base, L);
    const double *part = reinterpret_cast<const double *>(base + L.part);
    const double DV = sum_parts(part + PART_DV * L.pstride, nb, red);
    const double DG = sum_parts(part + PART_DG * L.pstride, nb, red);
    const double GM = max_parts(part + PART_GMAX * L.pstride, nb, red);
    if (threadIdx.x == 0) step_propose(sc, DV, DG, GM, nd.wb, (banks >> blockIdx.y) & 1u);
}

// Totals of the step's three reductions over the cell-gradient pass's n partials, formed by
// one block of NT threads (every thread gets them): thread t takes partials t, t + NT, ... of
// the three arrays in one pass, then the wave butterflies and a pairwise tree over the waves.
// red: >= 3 * NT / 64 doubles.
template <int NT>
__device__ __forceinline__ void step_totals(const double *part, const SlotLayout &L, int n,
                                            double *red, double &DV, double &DG, double &GM) {
    constexpr int W = NT / 64;
    const double *pv = part + PART_DV * L.pstride, *pg = part + PART_DG * L.pstride;
    const double *pm = part + PART_GMAX * L.pstride;
    double v = 0.0, g = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < n; i += 4 * NT) {
        double a[4], b[4], c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = i + u * NT;
            a[u] = j < n ? pv[j] : 0.0;
            b[u] = j < n ? pg[j] : 0.0;
            c[u] = j < n ? pm[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v += a[u];
            g += b[u];
            m = fmax(m, c[u]);
        }
    }
    v = group_sum<64>(v);
    g = group_sum<64>(g);
    m = group_max<64>(m);
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        red[w] = v;
        red[W + w] = g;
        red[2 * W + w] = m;
    }
    __syncthreads();
    double qv[W], qg[W], qm[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        qv[k] = red[k];
        qg[k] = red[W + k];
        qm[k] = red[2 * W + k];
    }
#pragma unroll
    for (int h = W / 2; h > 0; h >>= 1)
#pragma unroll
        for (int k = 0; k < h; ++k) {
            qv[k] += qv[k + h];
            qg[k] += qg[k + h];
            qm[k] = fmax(qm[k], qm[k + h]);
        }
    DV = qv[0];
    DG = qg[0];
    GM = qm[0];
}

constexpr int kStepThreads = 1024;  // cells per block of the update (fewer blocks, each of
                                    // which reduces the step's partials itself)

// u' = clamp(v - alpha g~), v' = clamp(u' + coef (u' - u)); v_prev = v, g~_prev = g~ (and
// u_prev = u with backtracking on).  A redo (a rejected step under backtracking) instead
// recomputes the last step from its start: u' = clamp(v_prev - alpha g~_prev),
// v' = clamp(u' + coef (u' - u_prev)), with v_prev, g~_prev, u_prev kept.  The proposal
// (alpha, coef, a', ...) is the one stored by the evaluation's closing reduction or the
// step-scalars kernel, or (fused) derived by every block itself from the cell-gradient pass's
// nc partials and the optimiser state of bank b.  One thread commits it into bank 1 - b and,
// for an accepted step, multiplies lambda by the schedule's ratio; no block reads what that
// thread writes.
// RAG: the slot's netlist and layout from its descriptor and nc its own cell-gradient block
// count; blocks past the slot's own cells return.
template <typename T, bool RAG>
__global__ __launch_bounds__(kStepThreads) void step_update_kernel(NetDev nda, SlotArgs sa, SlotLayout La,
                                                                   int fused, int nc_arg, uint32_t banks) {
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    if (RAG && (int)blockIdx.x * kStepThreads >= nd.n_mov) return;  // whole block
    const int nc = RAG ? max(1, cell_parts(nd)) : nc_arg;  // as launch_cell_grad
    Scalars *sc = scalars(base, L);
    const int b = (banks >> blockIdx.y) & 1u;
    const int n = nd.n_mov;
    const int i = blockIdx.x * kStepThreads + threadIdx.x;
    // the cell's own inputs first (clamped index), so that their loads are in flight while a
    // fused step reduces the partials
    const int ic = i < n ? i : max(n - 1, 0);  // the launcher skips n = 0
    const T *cs = reinterpret_cast<const T *>(nd.cstep);
    vec2<T> *u = reinterpret_cast<vec2<T> *>(base + L.u);
    vec2<T> *v = reinterpret_cast<vec2<T> *>(base + L.v);
    const T *g = reinterpret_cast<const T *>(base + L.g);
    const vec2<T> v0 = v[ic], u0 = u[ic];
    const T g0 = g[ic], g1 = g[(size_t)n + ic];
    const T c0 = cs[ic], c1 = cs[(size_t)n + ic], hx = cs[(size_t)2 * n + ic], hy = cs[(size_t)3 * n + ic];
    StepProposal pr;
    if (fused) {
        __shared__ double red[3 * kStepThreads / 64];
        double DV, DG, GM;
        step_totals<kStepThreads>(reinterpret_cast<const double *>(base + L.part), L, nc, red, DV,
                                  DG, GM);
        pr = propose_from_bank(sc, b, DV, DG, GM, nd.wb);
    } else {
        pr.alpha = sc->step_alpha;
        pr.coef = sc->step_coef;
        pr.a = sc->step_a;
        pr.aprev = sc->step_aprev;
        pr.k = sc->step_k;
        pr.reject = (int)sc->step_reject;
    }
    const bool save_start = sc->backtrack != 0;
    if (i == 0) {
        if (fused) store_proposal(sc, pr);
        sc->ab[1 - b] = pr.a;
        sc->aprevb[1 - b] = pr.aprev;
        sc->alphab[1 - b] = pr.alpha;
        sc->kb[1 - b] = pr.k;
        sc->readyb[1 - b] = pr.reject ? 1 : (save_start ? 1 : 0);
        if (pr.reject)
            sc->rejects += 1;
        else if (sc->lambda_valid)
            sc->lambda *= sc->lambda_ratio;
    }
    if (i >= n) return;
    const double alpha = pr.alpha, coef = pr.coef;
    vec2<T> *vp = reinterpret_cast<vec2<T> *>(base + L.vprev);
    vec2<T> *up = reinterpret_cast<vec2<T> *>(base + L.uprev);
    T *gp = reinterpret_cast<T *>(base + L.gprev);
    T un2[2], vn2[2];
    if (pr.reject) {  // redo the step that reached v, from its start, with the shorter alpha
        const vec2<T> vs = vp[i], us = up[i];
        const T gs[2] = {gp[i], gp[(size_t)n + i]};
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            const double hi = (double)(ax ? hy : hx);
            double un = (double)(ax ? vs.y : vs.x) - alpha * (double)gs[ax];
            un = un < 0.0 ? 0.0 : (un > hi ? hi : un);
            const T unt = (T)un;
            double vn = (double)unt + coef * ((double)unt - (double)(ax ? us.y : us.x));
            vn = vn < 0.0 ? 0.0 : (vn > hi ? hi : vn);
            un2[ax] = unt;
            vn2[ax] = (T)vn;
        }
        u[i] = cmk2<T>(un2[0], un2[1]);
        v[i] = cmk2<T>(vn2[0], vn2[1]);
        return;
    }
    const double P = precond_of<T>(c0, c1, sc->lambda_step);
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        const size_t ig = (size_t)ax * n + i;  // gradients: [2][n_mov]
        const double hi = (double)(ax ? hy : hx);
        const double gt = (double)(ax ? g1 : g0) / P;
        double un = (double)(ax ? v0.y : v0.x) - alpha * gt;
        un = un < 0.0 ? 0.0 : (un > hi ? hi : un);
        const T unt = (T)un;
        double vn = (double)unt + coef * ((double)unt - (double)(ax ? u0.y : u0.x));
        vn = vn < 0.0 ? 0.0 : (vn > hi ? hi : vn);
        gp[ig] = (T)gt;
        un2[ax] = unt;
        vn2[ax] = (T)vn;
    }
    vp[i] = v0;
    if (save_start) up[i] = u0;
    u[i] = cmk2<T>(un2[0], un2[1]);
    v[i] = cmk2<T>(vn2[0], vn2[1]);
}

// ---- best of Alg. 1 -------------------------------------------------------------------------
// Smallest HPWL among the slots (ties to the lowest list position), kept only if strictly
// better than the incumbent's (ties go to the incumbent).
__global__ void select_best_kernel(SlotArgs sa, char *inc, SlotLayout L) {
    if (threadIdx.x != 0) return;
    int best = -1;
    int64_t bv = 0;
    for (int s = 0; s < sa.n; ++s) {
        const Scalars *c = scalars(sa.base[s], L);
        if (!c->hpwl_valid) continue;
        if (best < 0 || c->hpwl_q < bv) {
            best = s;
            bv = c->hpwl_q;
        }
    }
    Scalars *is = scalars(inc, L);
    if (best >= 0 && is->hpwl_valid && is->hpwl_q <= bv) best = -1;
    is->best = best;
    if (best >= 0) {
        is->hpwl_q = bv;
        is->hpwl_valid = 1;
        for (int b = 0; b < 2; ++b) {  // the optimiser restarts (both banks)
            is->kb[b] = 0;
            is->ab[b] = 1.0;
            is->alphab[b] = 0.0;
        }
        is->lambda_valid = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void copy_best_kernel(NetDev nd, SlotArgs sa, char *inc,
                                                           SlotLayout L) {
    const int64_t best = scalars(inc, L)->best;
    if (best < 0) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nd.n_mov) return;
    const vec2<T> p = reinterpret_cast<const vec2<T> *>(sa.base[best] + L.u)[i];
    reinterpret_cast<vec2<T> *>(inc + L.u)[i] = p;
    reinterpret_cast<vec2<T> *>(inc + L.v)[i] = p;
    reinterpret_cast<vec2<T> *>(inc + L.vprev)[i] = p;
}

// ---- launchers ------------------------------------------------------------------------------
template <typename T>
hipError_t launch_combine(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                          hipStream_t st) {
    if (nd.n_mov == 0) return hipSuccess;
    HP_LAUNCH("combine_kernel", combine_kernel<T>, dim3((2 * nd.n_mov + kBlock - 1) / kBlock, sa.n),
              dim3(kBlock), 0, st, nd, sa, L);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L, bool proposed,
                       bool fused, uint32_t banks, hipStream_t st) {
    const int nc = cell_parts(nd);
    if (nc == 0) return hipSuccess;
    hipError_t e;
    fused = fused && proposed && nc <= kFusedStepParts;
    if (!proposed) {
        HP_LAUNCH("step_norms_kernel", step_norms_kernel<T>, dim3(nc, sa.n), dim3(kBlock), 0, st, nd,
                  sa, L);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        HP_LAUNCH("step_scalars_kernel", step_scalars_kernel, dim3(1, sa.n), dim3(kBlock), 0, st, nd,
                  sa, L, nc, banks);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int nu = (nd.n_mov + kStepThreads - 1) / kStepThreads;
    HP_LAUNCH("step_update_kernel", (step_update_kernel<T, false>), dim3(nu, sa.n), dim3(kStepThreads), 0, st, nd,
              sa, L, (int)fused, nc, banks);
    return hipGetLastError();
}

// Steady state over slots of different netlists: the closing reduction forms every slot's
// step (its lambda and proposal), then the update.
hipError_t rag_eval_finish(const SlotArgs &sa, uint32_t banks, hipStream_t st) {
    HP_LAUNCH("eval_finish_kernel", eval_finish_kernel<true>, dim3(1, sa.n), dim3(kFinBlock), 0, st,
              NetDev{}, sa, SlotLayout{}, 0, 0, 0, 0, 0, 0.0, FIN_STEP, banks);
    return hipGetLastError();
}
template <typename T>
hipError_t rag_step(const SlotArgs &sa, int grid_x, bool fused, uint32_t banks, hipStream_t st) {
    if (grid_x == 0) return hipSuccess;
    HP_LAUNCH("step_update_kernel", (step_update_kernel<T, true>), dim3(grid_x, sa.n),
              dim3(kStepThreads), 0, st, NetDev{}, sa, SlotLayout{}, (int)fused, 0, banks);
    return hipGetLastError();
}
int step_blocks(const NetDev &nd) { return (nd.n_mov + kStepThreads - 1) / kStepThreads; }

template <typename T>
hipError_t launch_select_best(const NetDev &nd, const SlotArgs &sa, char *incumbent,
                              const SlotLayout &L, hipStream_t st) {
    HP_LAUNCH("select_best_kernel", select_best_kernel, dim3(1), dim3(64), 0, st, sa, incumbent, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nd.n_mov == 0) return e;
    HP_LAUNCH("copy_best_kernel", copy_best_kernel<T>, dim3(cell_parts(nd)), dim3(kBlock), 0, st, nd,
              sa, incumbent, L);
    return hipGetLastError();
}

#define HP_INST(T)                                                                              \
    template hipError_t launch_combine<T>(const NetDev &, const SlotArgs &, const SlotLayout &,  \
                                          hipStream_t);                                         \
    template hipError_t launch_step<T>(const NetDev &, const SlotArgs &, const SlotLayout &,     \
                                       bool, bool, uint32_t, hipStream_t);                      \
    template hipError_t launch_select_best<T>(const NetDev &, const SlotArgs &, char *,          \
                                              const SlotLayout &, hipStream_t);                 \
    template hipError_t rag_step<T>(const SlotArgs &, int, bool, uint32_t, hipStream_t);
HP_INST(float)
HP_INST(double)
#undef HP_INST

}  // namespace hp
