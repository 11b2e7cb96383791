// Spectral Poisson solve on the bin grid (the electrostatic density term; cosine basis,
// Neumann walls), in three LDS-staged passes over the [my][mx] maps:
//
//   R1 (rows):    rho = (movable + fixed charge) * unit; T1[k][u] = sum_j rho_kj C_x(u, j)
//                 also the overflow sum, and the movable map is cleared for the next call
//   C  (columns): a_uv = c_u c_v / (mx my) sum_k T1[k][u] C_y(v, k); energy partial sums;
//                 Bx[k][u] = sum_v a_uv w_u/den C_y(v, k), By[k][u] = sum_v a_uv w_v/den S_y(v, k),
//                 Bp[k][u] = sum_v a_uv/den C_y(v, k)
//   R2 (rows):    xi_x[k][j] = sum_u Bx[k][u] S_x(u, j), xi_y = sum_u By C_x, psi = sum_u Bp C_x
//
// with C_x(u, j) = cos(pi u (2j+1) / (2 mx)), S_x its sine, den = d_x[u] + d_y[v] (w_u^2 + w_v^2,
// or the 5-point Laplacian's eigenvalues), and the (0,0) term dropped.  Every 1-D cosine sum
// of length M is computed with one complex FFT of length M (Makhoul's reordering): forward,
//   v_n = f_2n, v_{M-1-n} = f_{2n+1};  F_u = Re(exp(-i pi u / 2M) FFT(v)_u);
// inverse, V_u = exp(i pi u / 2M)(A'_u - i A'_{M-u}) with A'_0 = A_0, A'_u = A_u / 2, A'_M = 0,
//   v = IFFT(V) is real and x_2n = v_n, x_{2n+1} = v_{M-1-n};
// and a sine sum is a cosine sum of the reversed coefficients times (-1)^j.  Two real lines
// share one complex FFT.  The FFT is a radix-2 decimation-in-time transform in LDS over a
// batch of lines, with twiddles from a table built on the host in double precision.
#include "hp_device.h"

namespace hp {

template <typename T>
__device__ __forceinline__ vec2<T> cmk(T a, T b) {
    vec2<T> r;
    r.x = a;
    r.y = b;
    return r;
}

__device__ __forceinline__ int brev(int n, int logM) { return (int)(__brev((unsigned)n) >> (32 - logM)); }
// position of element j in Makhoul's reordered sequence (and of output j in the inverse)
__device__ __forceinline__ int mperm(int j, int M) { return (j & 1) ? (M - 1 - (j >> 1)) : (j >> 1); }

template <typename T>
__device__ void fft_lds(vec2<T> *buf, int nlines, int M, int logM, const vec2<T> *__restrict__ tw,
                        bool inverse) {
    const int hm = M >> 1;
    const int total = nlines * hm;
    for (int s = 0; s < logM; ++s) {
        const int half = 1 << s;
        const int tsh = logM - 1 - s;
        for (int b = threadIdx.x; b < total; b += kBlock) {
            const int line = b >> (logM - 1);
            const int t = b & (hm - 1);
            const int pos = t & (half - 1);
            const int i0 = ((t >> s) << (s + 1)) | pos;
            vec2<T> w = tw[pos << tsh];
            if (inverse) w.y = -w.y;
            vec2<T> *Lb = buf + (size_t)line * M;
            const vec2<T> a = Lb[i0], c0 = Lb[i0 + half];
            const T cr = c0.x * w.x - c0.y * w.y, ci = c0.x * w.y + c0.y * w.x;
            Lb[i0] = cmk<T>(a.x + cr, a.y + ci);
            Lb[i0 + half] = cmk<T>(a.x - cr, a.y - ci);
        }
        __syncthreads();
    }
}

// Split a packed forward FFT Z of two real sequences and apply the DCT post-twiddle:
// returns (F_a(u), F_b(u)).
template <typename T>
__device__ __forceinline__ vec2<T> dct_post(const vec2<T> *line, int u, int M, vec2<T> ph) {
    const vec2<T> Z = line[u], Zm = line[(M - u) & (M - 1)];
    const T var = (Z.x + Zm.x) * T(0.5), vai = (Z.y - Zm.y) * T(0.5);
    const T vbr = (Z.y + Zm.y) * T(0.5), vbi = -(Z.x - Zm.x) * T(0.5);
    return cmk<T>(ph.x * var + ph.y * vai, ph.x * vbr + ph.y * vbi);
}

// Makhoul inverse input for one real coefficient sequence at frequency v: p = A'(v),
// q = A'(M - v) -> exp(i phi)(p - i q).
template <typename T>
__device__ __forceinline__ vec2<T> idct_pre(T p, T q, vec2<T> ph) {
    return cmk<T>(p * ph.x + q * ph.y, p * ph.y - q * ph.x);
}

// ---- R1 ---------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void spec_rows_fwd(NetDev nd, SlotArgs sa, SlotLayout L,
                                                        int lpb, int keep) {
    extern __shared__ __align__(16) unsigned char smem[];
    vec2<T> *buf = reinterpret_cast<vec2<T> *>(smem);
    char *base = sa.base[blockIdx.y];
    const int M = nd.mx, logM = nd.logmx;
    int64_t *rho = reinterpret_cast<int64_t *>(base + L.rho);
    T *t1 = reinterpret_cast<T *>(base + L.t1);
    long long over = 0;
    for (int idx = threadIdx.x; idx < lpb * M; idx += kBlock) {
        const int l = idx >> logM, j = idx & (M - 1);
        const int ra = (blockIdx.x * lpb + l) * 2;
        const size_t ia = (size_t)ra * M + j, ib = ia + M;
        const int64_t ma = binned_charge(nd, base, L, ra, j), mb = binned_charge(nd, base, L, ra + 1, j);
        const int64_t fa = nd.rho_fixed[ia], fb = nd.rho_fixed[ib];
        const int64_t ca = __double2ll_rn(nd.target_density * (double)(nd.area_q - fa));
        const int64_t cb = __double2ll_rn(nd.target_density * (double)(nd.area_q - fb));
        if (ma > ca) over += ma - ca;
        if (mb > cb) over += mb - cb;
        if (keep) {  // the movable map itself is only materialised for inspection
            rho[ia] = ma;
            rho[ib] = mb;
        }
        buf[l * M + brev(mperm(j, M), logM)] =
            cmk<T>((T)((double)(ma + fa) * nd.density_unit), (T)((double)(mb + fb) * nd.density_unit));
    }
    __syncthreads();
    fft_lds<T>(buf, lpb, M, logM, reinterpret_cast<const vec2<T> *>(nd.tw_x), false);
    const vec2<T> *ph = reinterpret_cast<const vec2<T> *>(nd.ph_x);
    for (int idx = threadIdx.x; idx < lpb * M; idx += kBlock) {
        const int l = idx >> logM, u = idx & (M - 1);
        const int ra = (blockIdx.x * lpb + l) * 2;
        const vec2<T> F = dct_post<T>(buf + l * M, u, M, ph[u]);
        t1[(size_t)ra * M + u] = F.x;
        t1[(size_t)(ra + 1) * M + u] = F.y;
    }
    __shared__ long long red[4];
    over = block_sum(over, red);
    if (threadIdx.x == 0)
        (reinterpret_cast<long long *>(base + L.part) + PART_OVF * L.pstride)[blockIdx.x] = over;
}

// ---- C ----------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void spec_cols(NetDev nd, SlotArgs sa, SlotLayout L, int C,
                                                    int logC, int want_psi) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = nd.my, logM = nd.logmy, mx = nd.mx;
    T *acol = reinterpret_cast<T *>(smem);                                  // [C][M]
    vec2<T> *work = reinterpret_cast<vec2<T> *>(smem + sizeof(T) * (size_t)C * M);  // [C/2][M]
    char *base = sa.base[blockIdx.y];
    const int u0 = blockIdx.x * C;
    const T *t1 = reinterpret_cast<const T *>(base + L.t1);
    const vec2<T> *tw = reinterpret_cast<const vec2<T> *>(nd.tw_y);
    const vec2<T> *ph = reinterpret_cast<const vec2<T> *>(nd.ph_y);
    T *wr = reinterpret_cast<T *>(work);
    // load the column strip, two columns per complex line, Makhoul-reordered, bit-reversed
    for (int idx = threadIdx.x; idx < C * M; idx += kBlock) {
        const int k = idx >> logC, c = idx & (C - 1);
        wr[2 * ((c >> 1) * M + brev(mperm(k, M), logM)) + (c & 1)] = t1[(size_t)k * mx + u0 + c];
    }
    __syncthreads();
    fft_lds<T>(work, C / 2, M, logM, tw, false);
    const double norm = 1.0 / ((double)nd.mx * nd.my);
    double e = 0.0;
    for (int idx = threadIdx.x; idx < (C / 2) * M; idx += kBlock) {
        const int l = idx >> logM, v = idx & (M - 1);
        const vec2<T> F = dct_post<T>(work + l * M, v, M, ph[v]);
        const double cv = v ? 2.0 : 1.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = 2 * l + h, u = u0 + c;
            const double cu = u ? 2.0 : 1.0;
            const double a = cu * cv * norm * (double)(h ? F.y : F.x);
            acol[c * M + v] = (T)a;
            if (u | v) e += a * a * ((double)nd.mx * nd.my) / (cu * cv * (nd.den1[u] + nd.den1[mx + v]));
        }
    }
    __syncthreads();
    __shared__ double red[4];
    e = block_sum(e, red);
    if (threadIdx.x == 0)
        reinterpret_cast<double *>(base + L.part)[PART_E * L.pstride + blockIdx.x] = e;

    T *bx = reinterpret_cast<T *>(base + L.bx);
    T *by = reinterpret_cast<T *>(base + L.by);
    T *bp = reinterpret_cast<T *>(base + L.bp);
    const int hc = C / 2;
    // (Bx, By) of one column per complex line; two batches of C/2 columns
    for (int h = 0; h < 2; ++h) {
        for (int idx = threadIdx.x; idx < hc * M; idx += kBlock) {
            const int l = idx >> logM, v = idx & (M - 1);
            const int c = h * hc + l, u = u0 + c;
            const T *ac = acol + c * M;
            const T wu = (T)nd.omega[u], du = (T)nd.den1[u];
            // X(v) = a_uv w_u / den ; cosine sum in y
            auto X = [&](int vv) -> T {
                if ((u | vv) == 0) return T(0);
                return ac[vv] * wu / (du + (T)nd.den1[mx + vv]);
            };
            // Y(v) = a_uv w_v / den ; sine sum in y -> reversed coefficients
            auto Y = [&](int vv) -> T {
                if ((u | vv) == 0) return T(0);
                return ac[vv] * (T)nd.omega[mx + vv] / (du + (T)nd.den1[mx + vv]);
            };
            const T xp = v ? T(0.5) * X(v) : X(0);
            const T xq = v ? T(0.5) * X(M - v) : T(0);
            // reversed: Yt(0) = 0, Yt(w) = Y(M - w)
            const T yp = v ? T(0.5) * Y(M - v) : T(0);
            const T yq = v ? T(0.5) * Y(v) : T(0);
            const vec2<T> VX = idct_pre<T>(xp, xq, ph[v]);
            const vec2<T> VY = idct_pre<T>(yp, yq, ph[v]);
            work[l * M + brev(v, logM)] = cmk<T>(VX.x - VY.y, VX.y + VY.x);
        }
        __syncthreads();
        fft_lds<T>(work, hc, M, logM, tw, true);
        for (int idx = threadIdx.x; idx < hc * M; idx += kBlock) {
            const int k = idx / hc, l = idx - k * hc;
            const vec2<T> z = work[l * M + mperm(k, M)];
            const size_t o = (size_t)k * mx + u0 + h * hc + l;
            bx[o] = z.x;
            by[o] = (k & 1) ? -z.y : z.y;
        }
        __syncthreads();
    }
    if (want_psi) {
        for (int idx = threadIdx.x; idx < hc * M; idx += kBlock) {
            const int l = idx >> logM, v = idx & (M - 1);
            vec2<T> V2v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = 2 * l + h, u = u0 + c;
                const T *ac = acol + c * M;
                const T du = (T)nd.den1[u];
                auto P = [&](int vv) -> T {
                    if ((u | vv) == 0) return T(0);
                    return ac[vv] / (du + (T)nd.den1[mx + vv]);
                };
                const T pp = v ? T(0.5) * P(v) : P(0);
                const T pq = v ? T(0.5) * P(M - v) : T(0);
                V2v[h] = idct_pre<T>(pp, pq, ph[v]);
            }
            work[l * M + brev(v, logM)] = cmk<T>(V2v[0].x - V2v[1].y, V2v[0].y + V2v[1].x);
        }
        __syncthreads();
        fft_lds<T>(work, hc, M, logM, tw, true);
        for (int idx = threadIdx.x; idx < C * M; idx += kBlock) {
            const int k = idx >> logC, c = idx & (C - 1);
            const vec2<T> z = work[(c >> 1) * M + mperm(k, M)];
            bp[(size_t)k * mx + u0 + c] = (c & 1) ? z.y : z.x;
        }
    }
}

// ---- R2 ---------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void spec_rows_inv(NetDev nd, SlotArgs sa, SlotLayout L,
                                                        int want_psi) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int M = nd.mx, logM = nd.logmx;
    const int nst = want_psi ? 3 : 2;
    T *stage = reinterpret_cast<T *>(smem);  // [nst][2][M]
    vec2<T> *work = reinterpret_cast<vec2<T> *>(smem + sizeof(T) * (size_t)nst * 2 * M);
    char *base = sa.base[blockIdx.y];
    const int k0 = blockIdx.x * 2;
    const T *src[3] = {reinterpret_cast<const T *>(base + L.bx), reinterpret_cast<const T *>(base + L.by),
                       reinterpret_cast<const T *>(base + L.bp)};
    for (int idx = threadIdx.x; idx < nst * 2 * M; idx += kBlock) {
        const int a = idx / (2 * M), rem = idx - a * 2 * M;
        stage[idx] = src[a][(size_t)k0 * M + rem];
    }
    __syncthreads();
    const vec2<T> *ph = reinterpret_cast<const vec2<T> *>(nd.ph_x);
    const int nlines = want_psi ? 3 : 2;
    for (int idx = threadIdx.x; idx < 2 * M; idx += kBlock) {
        const int r = idx >> logM, u = idx & (M - 1);
        const T *sbx = stage + r * M, *sby = stage + 2 * M + r * M;
        // xi_x: sine sum of Bx -> cosine sum of the reversed row
        const T xp = u ? T(0.5) * sbx[M - u] : T(0);
        const T xq = u ? T(0.5) * sbx[u] : T(0);
        const T yp = u ? T(0.5) * sby[u] : sby[0];
        const T yq = u ? T(0.5) * sby[M - u] : T(0);
        const vec2<T> VX = idct_pre<T>(xp, xq, ph[u]), VY = idct_pre<T>(yp, yq, ph[u]);
        work[r * M + brev(u, logM)] = cmk<T>(VX.x - VY.y, VX.y + VY.x);
    }
    if (want_psi) {
        for (int u = threadIdx.x; u < M; u += kBlock) {
            const T *s0 = stage + 4 * M, *s1 = stage + 5 * M;
            const vec2<T> A = idct_pre<T>(u ? T(0.5) * s0[u] : s0[0], u ? T(0.5) * s0[M - u] : T(0), ph[u]);
            const vec2<T> B = idct_pre<T>(u ? T(0.5) * s1[u] : s1[0], u ? T(0.5) * s1[M - u] : T(0), ph[u]);
            work[2 * M + brev(u, logM)] = cmk<T>(A.x - B.y, A.y + B.x);
        }
    }
    __syncthreads();
    fft_lds<T>(work, nlines, M, logM, reinterpret_cast<const vec2<T> *>(nd.tw_x), true);
    vec2<T> *exy = reinterpret_cast<vec2<T> *>(base + L.exy);
    T *psi = reinterpret_cast<T *>(base + L.psi);
    for (int idx = threadIdx.x; idx < 2 * M; idx += kBlock) {
        const int r = idx >> logM, j = idx & (M - 1);
        const int n = mperm(j, M);
        const vec2<T> z = work[r * M + n];
        const size_t o = (size_t)(k0 + r) * M + j;
        exy[o] = cmk<T>((j & 1) ? -z.x : z.x, z.y);
        if (want_psi) {
            const vec2<T> zp = work[2 * M + n];
            psi[o] = r ? zp.y : zp.x;
        }
    }
}

// Columns per block of the C pass: one complex line (two real columns) per block gives
// mx / 2 blocks; the strided 8-byte row segments it reads come from L2/MALL, where the
// intermediate maps live, so parallelism wins over coalescing here.
template <typename T>
static int cols_per_block(const NetDev &nd) {
    int C = 2;
    while (C > 2 && 2ull * C * nd.my * sizeof(T) > (unsigned long long)nd.lds_budget) C /= 2;
    return C < nd.mx ? C : nd.mx;
}

// R1 takes lpb complex lines (2 rows each) per block
static int rows_fwd_lines(const NetDev &nd) {
    int lpb = 512 / nd.mx;
    if (lpb < 1) lpb = 1;
    if (lpb > nd.my / 2) lpb = nd.my / 2;
    return lpb;
}

int spectral_overflow_parts(const NetDev &nd) { return nd.my / 2 / rows_fwd_lines(nd); }

template <typename T>
hipError_t launch_spectral(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                           bool keep_maps, bool want_psi, hipStream_t st) {
    const int lpb = rows_fwd_lines(nd);
    size_t sh1 = sizeof(vec2<T>) * (size_t)lpb * nd.mx;
    HP_LAUNCH("spec_rows_fwd", spec_rows_fwd<T>, dim3(nd.my / 2 / lpb, sa.n), dim3(kBlock), sh1, st, nd,
                       sa, L, lpb, (int)keep_maps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int C = cols_per_block<T>(nd);
    int logC = 0;
    while ((1 << logC) < C) ++logC;
    size_t sh2 = 2 * sizeof(T) * (size_t)C * nd.my;
    HP_LAUNCH("spec_cols", spec_cols<T>, dim3(nd.mx / C, sa.n), dim3(kBlock), sh2, st, nd, sa, L, C,
                       logC, (int)want_psi);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nst = want_psi ? 3 : 2;
    size_t sh3 = sizeof(T) * (size_t)nst * 2 * nd.mx + sizeof(vec2<T>) * (size_t)nst * nd.mx;
    HP_LAUNCH("spec_rows_inv", spec_rows_inv<T>, dim3(nd.my / 2, sa.n), dim3(kBlock), sh3, st, nd, sa, L,
                       (int)want_psi);
    return hipGetLastError();
}

template <typename T>
int spectral_energy_parts(const NetDev &nd) { return nd.mx / cols_per_block<T>(nd); }

template <typename T>
size_t spectral_max_lds(const NetDev &nd) {
    const int C = cols_per_block<T>(nd);
    size_t a = sizeof(vec2<T>) * (size_t)std::max(1, std::min(512 / nd.mx, nd.my / 2)) * nd.mx;
    size_t b = 2 * sizeof(T) * (size_t)C * nd.my;
    size_t c = sizeof(T) * 6 * (size_t)nd.mx + sizeof(vec2<T>) * 3 * (size_t)nd.mx;
    return std::max(a, std::max(b, c));
}

// Ask for `bytes` of dynamic LDS per block on the three passes (above the 64 KB default).
template <typename T>
hipError_t spectral_prepare(int bytes) {
    hipError_t e = hipFuncSetAttribute((const void *)spec_rows_fwd<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)spec_cols<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)spec_rows_inv<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

#define HP_INST(T)                                                                            \
    template hipError_t launch_spectral<T>(const NetDev &, const SlotArgs &, const SlotLayout &, \
                                           bool, bool, hipStream_t);                          \
    template int spectral_energy_parts<T>(const NetDev &);                                    \
    template size_t spectral_max_lds<T>(const NetDev &);                                      \
    template hipError_t spectral_prepare<T>(int);
HP_INST(float)
HP_INST(double)
#undef HP_INST

}  // namespace hp
