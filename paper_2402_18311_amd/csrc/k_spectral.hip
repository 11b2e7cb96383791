// Spectral Poisson solve on the bin grid (the electrostatic density term; cosine basis,
// Neumann walls), in three LDS-staged passes over the [my][mx] maps:
//
//   R1 (rows):    rho = (movable + fixed charge) * unit; T1[k][u] = sum_j rho_kj C_x(u, j);
//                 the movable charge is assembled from the binned scatter's windows, and the
//                 overflow partial sums are taken on the way
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
// share one complex FFT.  The FFT is a decimation-in-time transform in LDS (radix-4 passes,
// one radix-2 pass for odd log M) over a batch of lines.  Each block copies the twiddles, DCT
// phases and per-axis symbols (tables built on the host in FP64) to LDS.  In the column and
// inverse-row passes the complex line buffers and the twiddles are stored with one spare slot
// after every 32 elements (fpad): the bit-reversed and power-of-two-strided accesses of a
// transform then spread over the LDS banks instead of meeting in a few of them.
//
// With M <= 1024 each pass has only M/2 blocks (one per CU or fewer), so a block's latency is
// the pass's time: blocks are wide (1024 threads; 512 for C and R2 in launches with more
// blocks than CUs) and every global load of a block, tables included, is issued before the
// first one is waited for.
#include "hp_device.h"

namespace hp {

template <typename T>
__device__ __forceinline__ vec2<T> cmk(T a, T b) {
    vec2<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__device__ __forceinline__ vec2<T> cmul(vec2<T> a, vec2<T> b) {
    return cmk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ vec2<T> cadd(vec2<T> a, vec2<T> b) { return cmk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ vec2<T> csub(vec2<T> a, vec2<T> b) { return cmk<T>(a.x - b.x, a.y - b.y); }

// LDS position of element i of a padded array (one spare slot after every 32 elements), and
// the elements such an array of n needs; lpos: the position in a padded (PAD) or plain array.
__host__ __device__ inline int fpad(int i) { return i + (i >> 5); }
__host__ __device__ inline size_t fpad_n(size_t n) { return n + (n >> 5) + 1; }
template <bool PAD> __device__ __forceinline__ int lpos(int i) { return PAD ? fpad(i) : i; }

__device__ __forceinline__ int brev(int n, int logM) { return (int)(__brev((unsigned)n) >> (32 - logM)); }
// position of element j in Makhoul's reordered sequence (and of output j in the inverse)
__device__ __forceinline__ int mperm(int j, int M) { return (j & 1) ? (M - 1 - (j >> 1)) : (j >> 1); }

// In-place FFT of nlines lines of length M held in bit-reversed order, line l's element i at
// buf[lpos<PAD>(l M + i)]; tw[lpos<PAD>(k)] = exp(-2 pi i k/M) (conjugated for the inverse).
// A radix-4 pass performs DIT stages s and s+1 at once: with
// h = 2^s, w1 = W_{2h}^pos and w2 = W_{4h}^pos, and W_{4h}^h = -i (forward) or +i (inverse).
template <typename T, int NT, bool PAD>
__device__ void fft_lds(vec2<T> *buf, int nlines, int M, int logM, const vec2<T> *tw, bool inverse) {
    int s = 0;
    for (; s + 1 < logM; s += 2) {
        const int h = 1 << s;
        const int q = M >> 2;
        const int total = nlines * q;
        const int sh1 = logM - 1 - s, sh2 = logM - 2 - s;
        for (int b = threadIdx.x; b < total; b += NT) {
            const int line = b >> (logM - 2);
            const int t = b & (q - 1);
            const int pos = t & (h - 1);
            const int i0 = ((t >> s) << (s + 2)) | pos;
            vec2<T> w1 = tw[lpos<PAD>(pos << sh1)], w2 = tw[lpos<PAD>(pos << sh2)];
            if (inverse) {
                w1.y = -w1.y;
                w2.y = -w2.y;
            }
            const int g = line * M + i0;
            const int a0 = lpos<PAD>(g), a1 = lpos<PAD>(g + h), a2 = lpos<PAD>(g + 2 * h),
                      a3 = lpos<PAD>(g + 3 * h);
            const vec2<T> x0 = buf[a0], x1 = buf[a1], x2 = buf[a2], x3 = buf[a3];
            const vec2<T> c1 = cmul<T>(w1, x1), c3 = cmul<T>(w1, x3);
            const vec2<T> b0 = cadd<T>(x0, c1), b1 = csub<T>(x0, c1);
            const vec2<T> b2 = cadd<T>(x2, c3), b3 = csub<T>(x2, c3);
            const vec2<T> d2 = cmul<T>(w2, b2), d3 = cmul<T>(w2, b3);
            const vec2<T> e3 = inverse ? cmk<T>(-d3.y, d3.x) : cmk<T>(d3.y, -d3.x);
            buf[a0] = cadd<T>(b0, d2);
            buf[a2] = csub<T>(b0, d2);
            buf[a1] = cadd<T>(b1, e3);
            buf[a3] = csub<T>(b1, e3);
        }
        __syncthreads();
    }
    if (s < logM) {  // one radix-2 stage left
        const int half = 1 << s, hm = M >> 1, total = nlines * hm, tsh = logM - 1 - s;
        for (int b = threadIdx.x; b < total; b += NT) {
            const int line = b >> (logM - 1);
            const int t = b & (hm - 1);
            const int pos = t & (half - 1);
            const int i0 = ((t >> s) << (s + 1)) | pos;
            vec2<T> w = tw[lpos<PAD>(pos << tsh)];
            if (inverse) w.y = -w.y;
            const int a0 = lpos<PAD>(line * M + i0), a1 = lpos<PAD>(line * M + i0 + half);
            const vec2<T> a = buf[a0], c = cmul<T>(w, buf[a1]);
            buf[a0] = cadd<T>(a, c);
            buf[a1] = csub<T>(a, c);
        }
        __syncthreads();
    }
}

// Split a packed forward FFT Z of two real sequences (the line at index lb of buf, laid out as
// lpos<PAD>) and apply the DCT post-twiddle: returns (F_a(u), F_b(u)).
template <typename T, bool PAD>
__device__ __forceinline__ vec2<T> dct_post(const vec2<T> *buf, int lb, int u, int M, vec2<T> ph) {
    const vec2<T> Z = buf[lpos<PAD>(lb + u)], Zm = buf[lpos<PAD>(lb + ((M - u) & (M - 1)))];
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

// Register prefetch of up to K elements per thread of a table of n (thread t takes t, t + NT,
// ...), so that several tables' loads are in flight together; put() stores them to LDS.
template <typename V, int NT, int K>
struct Prefetch {
    V r[K];
    __device__ __forceinline__ void get(const V *g, int n) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < n) r[k] = g[i];
        }
    }
    template <typename S>
    __device__ __forceinline__ void put(S *s, int n) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < n) s[i] = (S)r[k];
        }
    }
    // into a padded array (element i at s[fpad(i)])
    __device__ __forceinline__ void put_pad(V *s, int n) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = threadIdx.x + k * NT;
            if (i < n) s[fpad(i)] = r[k];
        }
    }
};

// Sum over a block of NT threads (all get the result): wave butterflies, then a pairwise tree
// over the NT / 64 wave totals.  red: >= NT / 64 elements.
template <int NT, typename T>
__device__ __forceinline__ T block_sum_nt(T v, T *red) {
    constexpr int NW = NT / 64;
    v = group_sum<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T q[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) q[k] = red[k];
#pragma unroll
    for (int h = NW / 2; h > 0; h >>= 1)
#pragma unroll
        for (int k = 0; k < h; ++k) q[k] += q[k + h];
    return q[0];
}

// The block's line (pair) index: neighbouring lines go to the same XCD (each XCD takes one
// contiguous eighth of the grid when the grid is a multiple of 8), so the column pass's 8-byte
// reads and writes of neighbouring columns meet in one L2 and leave it as whole lines, and the
// row passes' neighbouring rows share their tiles' charge windows.
// nb: the slot's block count (the grid's, except in a launch over slots of different
// netlists, whose blocks past nb return first).
__device__ __forceinline__ int spec_block(int nb) {
    return (nb % kXcds) ? (int)blockIdx.x : xcd_remap(blockIdx.x, nb);
}

// LDS layout helpers (16-byte aligned sections)
__host__ __device__ inline size_t al16(size_t v) { return (v + 15) & ~size_t(15); }

// ---- R1 ---------------------------------------------------------------------------------
// lds: tw [M/2] | ph [M] | buf [lpb][M] (not padded: here the padding's extra index arithmetic
// cost more than the bank conflicts it removes)
// A block takes 2 lpb consecutive rows (lpb complex lines), one bin per thread and round.
constexpr int kRowsFwdThreads = 1024;

// R1 takes lpb complex lines (2 rows each) per block
__host__ __device__ inline int rows_fwd_lines(const NetDev &nd) {
    int lpb = 512 / nd.mx;
    if (lpb < 1) lpb = 1;
    if (lpb > nd.my / 2) lpb = nd.my / 2;
    return lpb;
}

// RAG: the slot's netlist, layout and lpb from its descriptor (every pass below likewise)
template <typename T, bool RAG>
__global__ __launch_bounds__(kRowsFwdThreads) void spec_rows_fwd(NetDev nda, SlotArgs sa, SlotLayout La,
                                                                 int lpb_arg, int keep) {
    constexpr int NT = kRowsFwdThreads;
    extern __shared__ __align__(16) unsigned char smem[];
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    const int lpb = RAG ? rows_fwd_lines(nd) : lpb_arg;
    const int nb = RAG ? nd.my / 2 / lpb : (int)gridDim.x;
    if ((int)blockIdx.x >= nb) return;
    const int M = nd.mx, logM = nd.logmx;
    vec2<T> *s_tw = reinterpret_cast<vec2<T> *>(smem);
    vec2<T> *s_ph = reinterpret_cast<vec2<T> *>(smem + al16(sizeof(vec2<T>) * (M / 2)));
    vec2<T> *buf = reinterpret_cast<vec2<T> *>(smem + al16(sizeof(vec2<T>) * (M / 2)) +
                                               al16(sizeof(vec2<T>) * M));
    T *bufr = reinterpret_cast<T *>(buf);  // line l, element n: real part 2 (l M + n), imag + 1
    Prefetch<vec2<T>, NT, 1> ptw;  // M / 2 <= 1024
    Prefetch<vec2<T>, NT, 2> pph;  // M <= 2048
    ptw.get(reinterpret_cast<const vec2<T> *>(nd.tw_x), M / 2);
    pph.get(reinterpret_cast<const vec2<T> *>(nd.ph_x), M);
    int64_t *rho = reinterpret_cast<int64_t *>(base + L.rho);
    T *t1 = reinterpret_cast<T *>(base + L.t1);
    const int nel = 2 * lpb * M;
    const int bid = spec_block(nb);
    const size_t g0 = (size_t)bid * nel;  // first bin: row 2 lpb bid, column 0
    long long over = 0;
    for (int e = threadIdx.x; e < nel; e += NT) {
        const int rl = e >> logM, j = e & (M - 1);  // row within the block (line rl / 2)
        const size_t ia = g0 + e;
        const int row = (int)(ia >> logM);
        // tile windows of the binned scatter (cleared as they are read), plus the charge its
        // out-of-window cells added to rho
        const int64_t oa = rho[ia];
        const int64_t fa = nd.rho_fixed[ia];
        const int64_t ma = take_binned_charge(nd, base, L, row, j) + oa;
        const int64_t ca = __double2ll_rn(nd.target_density * (double)(nd.area_q - fa));
        if (ma > ca) over += ma - ca;
        if (keep)  // the whole movable map, for inspection (cleared before the next scatter)
            rho[ia] = ma;
        else if (oa)  // leave rho zero for the next scatter
            rho[ia] = 0;
        bufr[2 * ((rl >> 1) * M + brev(mperm(j, M), logM)) + (rl & 1)] =
            (T)((double)(ma + fa) * nd.density_unit);
    }
    ptw.put(s_tw, M / 2);
    pph.put(s_ph, M);
    __syncthreads();
    fft_lds<T, NT, false>(buf, lpb, M, logM, s_tw, false);
    for (int idx = threadIdx.x; idx < lpb * M; idx += NT) {
        const int l = idx >> logM, u = idx & (M - 1);
        const size_t ra = g0 + (size_t)(2 * l) * M;
        const vec2<T> F = dct_post<T, false>(buf, l * M, u, M, s_ph[u]);
        t1[ra + u] = F.x;
        t1[ra + M + u] = F.y;
    }
    __shared__ long long red[NT / 64];
    over = block_sum_nt<NT>(over, red);
    if (threadIdx.x == 0)
        (reinterpret_cast<long long *>(base + L.part) + PART_OVF * L.pstride)[bid] = over;
}

// ---- C: two columns per block -------------------------------------------------------------
// lds: tw [M/2, padded] | ph [M] | den_y [M] | om_y [M] | acol [2][M] | inv [2][M] |
// work [2][M, padded]
// (inv[h][v] = 1 / (d_x[u0 + h] + d_y[v]), 0 for the dropped (0, 0) term: every term of the
// column shares these denominators, so each is divided once)
template <typename T>
__host__ __device__ inline size_t cols_lds(int M) {
    return al16(sizeof(vec2<T>) * fpad_n(M / 2)) + al16(sizeof(vec2<T>) * M) +
           2 * al16(sizeof(T) * M) + 2 * al16(sizeof(T) * 2 * M) +
           al16(sizeof(vec2<T>) * fpad_n(2 * M));
}

// C and R2 run 1024-thread blocks when a launch has at most one block per CU (a single slot:
// the block's latency is the pass's time), 512-thread blocks when it has more (batched slots:
// smaller blocks interleave better); see wide_spectral.
template <typename T, int NT, bool RAG>
__global__ __launch_bounds__(NT) void spec_cols(NetDev nda, SlotArgs sa, SlotLayout La, int want_psi) {
    extern __shared__ __align__(16) unsigned char smem[];
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    const int nb = RAG ? nd.mx / 2 : (int)gridDim.x;
    if ((int)blockIdx.x >= nb) return;
    const int M = nd.my, logM = nd.logmy, mx = nd.mx;
    size_t o = 0;
    vec2<T> *s_tw = reinterpret_cast<vec2<T> *>(smem + o);
    o += al16(sizeof(vec2<T>) * fpad_n(M / 2));
    vec2<T> *s_ph = reinterpret_cast<vec2<T> *>(smem + o);
    o += al16(sizeof(vec2<T>) * M);
    T *s_den = reinterpret_cast<T *>(smem + o);
    o += al16(sizeof(T) * M);
    T *s_om = reinterpret_cast<T *>(smem + o);
    o += al16(sizeof(T) * M);
    T *acol = reinterpret_cast<T *>(smem + o);  // [2][M]
    o += al16(sizeof(T) * 2 * M);
    T *inv = reinterpret_cast<T *>(smem + o);  // [2][M]
    o += al16(sizeof(T) * 2 * M);
    vec2<T> *work = reinterpret_cast<vec2<T> *>(smem + o);  // [2][M], padded
    const int bid = spec_block(nb);
    const int u0 = bid * 2;
    // every global load first: the two columns (as one complex line), the y tables and
    // symbols (M <= 2048: at most 4 elements of each per thread)
    const T *t1 = reinterpret_cast<const T *>(base + L.t1);
    vec2<T> col[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = threadIdx.x + q * NT;
        if (k < M) col[q] = *reinterpret_cast<const vec2<T> *>(t1 + (size_t)k * mx + u0);
    }
    Prefetch<vec2<T>, NT, 2> ptw;
    Prefetch<vec2<T>, NT, 4> pph;
    Prefetch<double, NT, 4> pden, pom;
    ptw.get(reinterpret_cast<const vec2<T> *>(nd.tw_y), M / 2);
    pph.get(reinterpret_cast<const vec2<T> *>(nd.ph_y), M);
    pden.get(nd.den1 + mx, M);
    pom.get(nd.omega + mx, M);
    const T dux0 = (T)nd.den1[u0], dux1 = (T)nd.den1[u0 + 1];
    const T wux[2] = {(T)nd.omega[u0], (T)nd.omega[u0 + 1]};
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // Makhoul-reordered, bit-reversed
        const int k = threadIdx.x + q * NT;
        if (k < M) work[fpad(brev(mperm(k, M), logM))] = col[q];
    }
    ptw.put_pad(s_tw, M / 2);
    pph.put(s_ph, M);
    pden.put(s_den, M);
    pom.put(s_om, M);
    __syncthreads();
    fft_lds<T, NT, true>(work, 1, M, logM, s_tw, false);
    const T norm = (T)(1.0 / ((double)nd.mx * nd.my));
    const T cu0 = u0 ? T(2) : T(1);  // u0 + 1 > 0 always
    const double mm = (double)nd.mx * nd.my;
    double e = 0.0;
    for (int v = threadIdx.x; v < M; v += NT) {
        const vec2<T> F = dct_post<T, true>(work, 0, v, M, s_ph[v]);
        const T cv = v ? T(2) : T(1);
        const T a0 = cu0 * cv * norm * F.x, a1 = T(2) * cv * norm * F.y;
        acol[v] = a0;
        acol[M + v] = a1;
        const T i0 = (u0 | v) ? T(1) / (dux0 + s_den[v]) : T(0), i1 = T(1) / (dux1 + s_den[v]);
        inv[v] = i0;
        inv[M + v] = i1;
        // energy by Parseval: a^2 mx my / (c_u c_v den), accumulated in FP64
        e += (double)(a0 * a0 * i0 / (cu0 * cv)) * mm + (double)(a1 * a1 * i1 / (T(2) * cv)) * mm;
    }
    __shared__ double red[NT / 64];
    e = block_sum_nt<NT>(e, red);  // its barriers also publish acol / inv
    if (threadIdx.x == 0)
        reinterpret_cast<double *>(base + L.part)[PART_E * L.pstride + bid] = e;

    // (Bx + i By) of column h on complex line h: X(v) = a_uv w_u / den (cosine sum in y),
    // Y(v) = a_uv w_v / den (sine sum in y -> reversed coefficients)
    for (int idx = threadIdx.x; idx < 2 * M; idx += NT) {
        const int h = idx >> logM, v = idx & (M - 1);
        const T *ac = acol + h * M, *iv = inv + h * M;
        const T wu = wux[h];
        auto X = [&](int vv) -> T { return ac[vv] * wu * iv[vv]; };
        auto Y = [&](int vv) -> T { return ac[vv] * s_om[vv] * iv[vv]; };
        const T xp = v ? T(0.5) * X(v) : X(0);
        const T xq = v ? T(0.5) * X(M - v) : T(0);
        const T yp = v ? T(0.5) * Y(M - v) : T(0);
        const T yq = v ? T(0.5) * Y(v) : T(0);
        const vec2<T> VX = idct_pre<T>(xp, xq, s_ph[v]), VY = idct_pre<T>(yp, yq, s_ph[v]);
        work[fpad(h * M + brev(v, logM))] = cmk<T>(VX.x - VY.y, VX.y + VY.x);
    }
    __syncthreads();
    fft_lds<T, NT, true>(work, 2, M, logM, s_tw, true);
    T *bx = reinterpret_cast<T *>(base + L.bx);
    T *by = reinterpret_cast<T *>(base + L.by);
    for (int k = threadIdx.x; k < M; k += NT) {
        const int n = mperm(k, M);
        const vec2<T> z0 = work[fpad(n)], z1 = work[fpad(M + n)];
        const T sg = (k & 1) ? T(-1) : T(1);
        *reinterpret_cast<vec2<T> *>(bx + (size_t)k * mx + u0) = cmk<T>(z0.x, z1.x);
        *reinterpret_cast<vec2<T> *>(by + (size_t)k * mx + u0) = cmk<T>(sg * z0.y, sg * z1.y);
    }
    if (want_psi) {
        __syncthreads();
        for (int v = threadIdx.x; v < M; v += NT) {
            vec2<T> V2v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const T *ac = acol + h * M, *iv = inv + h * M;
                auto P = [&](int vv) -> T { return ac[vv] * iv[vv]; };
                const T pp = v ? T(0.5) * P(v) : P(0);
                const T pq = v ? T(0.5) * P(M - v) : T(0);
                V2v[h] = idct_pre<T>(pp, pq, s_ph[v]);
            }
            work[fpad(brev(v, logM))] = cmk<T>(V2v[0].x - V2v[1].y, V2v[0].y + V2v[1].x);
        }
        __syncthreads();
        fft_lds<T, NT, true>(work, 1, M, logM, s_tw, true);
        T *bp = reinterpret_cast<T *>(base + L.bp);
        for (int k = threadIdx.x; k < M; k += NT)
            *reinterpret_cast<vec2<T> *>(bp + (size_t)k * mx + u0) = work[fpad(mperm(k, M))];
    }
}

// ---- R2 ---------------------------------------------------------------------------------
// lds: tw [M/2, padded] | ph [M] | stage [nst][2][M] | work [nst][M, padded]
template <typename T, int NT, bool RAG>
__global__ __launch_bounds__(NT) void spec_rows_inv(NetDev nda, SlotArgs sa, SlotLayout La,
                                                    int want_psi) {
    extern __shared__ __align__(16) unsigned char smem[];
    char *base = sa.base[blockIdx.y];
    const NetDev &nd = view_nd<RAG>(nda, base);
    const SlotLayout &L = view_L<RAG>(La, base);
    const int nb = RAG ? nd.my / 2 : (int)gridDim.x;
    if ((int)blockIdx.x >= nb) return;
    const int M = nd.mx, logM = nd.logmx;
    const int nst = want_psi ? 3 : 2;
    size_t o = 0;
    vec2<T> *s_tw = reinterpret_cast<vec2<T> *>(smem + o);
    o += al16(sizeof(vec2<T>) * fpad_n(M / 2));
    vec2<T> *s_ph = reinterpret_cast<vec2<T> *>(smem + o);
    o += al16(sizeof(vec2<T>) * M);
    T *stage = reinterpret_cast<T *>(smem + o);  // [nst][2][M]
    o += al16(sizeof(T) * (size_t)nst * 2 * M);
    vec2<T> *work = reinterpret_cast<vec2<T> *>(smem + o);
    const int k0 = spec_block(nb) * 2;
    // every global load first: the two rows of Bx, By (and Bp) and the x tables; the rows in
    // rounds of 8 elements per thread (one round for M <= 1024 without psi)
    const T *src[3] = {reinterpret_cast<const T *>(base + L.bx), reinterpret_cast<const T *>(base + L.by),
                       reinterpret_cast<const T *>(base + L.bp)};
    Prefetch<vec2<T>, NT, 2> ptw;
    Prefetch<vec2<T>, NT, 4> pph;
    ptw.get(reinterpret_cast<const vec2<T> *>(nd.tw_x), M / 2);
    pph.get(reinterpret_cast<const vec2<T> *>(nd.ph_x), M);
    const int nall = nst * 2 * M;
    for (int i0 = 0; i0 < nall; i0 += 8 * NT) {
        T r[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = i0 + threadIdx.x + q * NT;
            if (idx < nall) {
                const int a = idx >> (logM + 1), rem = idx & (2 * M - 1);
                r[q] = src[a][(size_t)k0 * M + rem];
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = i0 + threadIdx.x + q * NT;
            if (idx < nall) stage[idx] = r[q];
        }
    }
    ptw.put_pad(s_tw, M / 2);
    pph.put(s_ph, M);
    __syncthreads();
    const int nlines = want_psi ? 3 : 2;
    for (int idx = threadIdx.x; idx < 2 * M; idx += NT) {
        const int r = idx >> logM, u = idx & (M - 1);
        const T *sbx = stage + r * M, *sby = stage + 2 * M + r * M;
        // xi_x: sine sum of Bx -> cosine sum of the reversed row
        const T xp = u ? T(0.5) * sbx[M - u] : T(0);
        const T xq = u ? T(0.5) * sbx[u] : T(0);
        const T yp = u ? T(0.5) * sby[u] : sby[0];
        const T yq = u ? T(0.5) * sby[M - u] : T(0);
        const vec2<T> VX = idct_pre<T>(xp, xq, s_ph[u]), VY = idct_pre<T>(yp, yq, s_ph[u]);
        work[fpad(r * M + brev(u, logM))] = cmk<T>(VX.x - VY.y, VX.y + VY.x);
    }
    if (want_psi) {
        for (int u = threadIdx.x; u < M; u += NT) {
            const T *s0 = stage + 4 * M, *s1 = stage + 5 * M;
            const vec2<T> A = idct_pre<T>(u ? T(0.5) * s0[u] : s0[0], u ? T(0.5) * s0[M - u] : T(0), s_ph[u]);
            const vec2<T> B = idct_pre<T>(u ? T(0.5) * s1[u] : s1[0], u ? T(0.5) * s1[M - u] : T(0), s_ph[u]);
            work[fpad(2 * M + brev(u, logM))] = cmk<T>(A.x - B.y, A.y + B.x);
        }
    }
    __syncthreads();
    fft_lds<T, NT, true>(work, nlines, M, logM, s_tw, true);
    vec2<T> *exy = reinterpret_cast<vec2<T> *>(base + L.exy);
    T *psi = reinterpret_cast<T *>(base + L.psi);
    for (int idx = threadIdx.x; idx < 2 * M; idx += NT) {
        const int r = idx >> logM, j = idx & (M - 1);
        const int n = mperm(j, M);
        const vec2<T> z = work[fpad(r * M + n)];
        const size_t oo = (size_t)(k0 + r) * M + j;
        exy[oo] = cmk<T>((j & 1) ? -z.x : z.x, z.y);
        if (want_psi) {
            const vec2<T> zp = work[fpad(2 * M + n)];
            psi[oo] = r ? zp.y : zp.x;
        }
    }
}

int spectral_overflow_parts(const NetDev &nd) { return nd.my / 2 / rows_fwd_lines(nd); }

template <typename T>
static size_t rows_fwd_lds(const NetDev &nd) {
    return al16(sizeof(vec2<T>) * (nd.mx / 2)) + al16(sizeof(vec2<T>) * nd.mx) +
           sizeof(vec2<T>) * (size_t)rows_fwd_lines(nd) * nd.mx;
}
template <typename T>
static size_t rows_inv_lds(const NetDev &nd, int nst) {
    return al16(sizeof(vec2<T>) * fpad_n(nd.mx / 2)) + al16(sizeof(vec2<T>) * nd.mx) +
           al16(sizeof(T) * (size_t)nst * 2 * nd.mx) + sizeof(vec2<T>) * fpad_n((size_t)nst * nd.mx);
}

// 1024-thread C and R2 blocks while a launch has at most one block per CU, unless the
// netlist's tunable fixes the width
static bool wide_spectral(const NetDev &nd, const SlotArgs &sa) {
    if (nd.spec_threads) return nd.spec_threads == 1024;
    return (size_t)std::max(nd.mx, nd.my) / 2 * sa.n <= (size_t)nd.n_cu;
}

template <typename T>
hipError_t launch_spectral(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                           bool keep_maps, bool want_psi, hipStream_t st) {
    const int lpb = rows_fwd_lines(nd);
    HP_LAUNCH("spec_rows_fwd", (spec_rows_fwd<T, false>), dim3(nd.my / 2 / lpb, sa.n), dim3(kRowsFwdThreads),
              rows_fwd_lds<T>(nd), st, nd, sa, L, lpb, (int)keep_maps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nst = want_psi ? 3 : 2;
    if (wide_spectral(nd, sa)) {
        HP_LAUNCH("spec_cols", (spec_cols<T, 1024, false>), dim3(nd.mx / 2, sa.n), dim3(1024),
                  cols_lds<T>(nd.my), st, nd, sa, L, (int)want_psi);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        HP_LAUNCH("spec_rows_inv", (spec_rows_inv<T, 1024, false>), dim3(nd.my / 2, sa.n), dim3(1024),
                  rows_inv_lds<T>(nd, nst), st, nd, sa, L, (int)want_psi);
    } else {
        HP_LAUNCH("spec_cols", (spec_cols<T, 512, false>), dim3(nd.mx / 2, sa.n), dim3(512),
                  cols_lds<T>(nd.my), st, nd, sa, L, (int)want_psi);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        HP_LAUNCH("spec_rows_inv", (spec_rows_inv<T, 512, false>), dim3(nd.my / 2, sa.n), dim3(512),
                  rows_inv_lds<T>(nd, nst), st, nd, sa, L, (int)want_psi);
    }
    return hipGetLastError();
}

// The three passes over slots of different netlists (no kept maps, no potential): 512-thread
// column and inverse-row blocks (many slots share the launch); grids from the largest slot.
template <typename T>
hipError_t rag_spectral(const SlotArgs &sa, int rows_x, int cols_x, int inv_x, size_t lds_rows,
                        size_t lds_cols, size_t lds_inv, hipStream_t st) {
    const NetDev nd0{};
    const SlotLayout L0{};
    HP_LAUNCH("spec_rows_fwd", (spec_rows_fwd<T, true>), dim3(rows_x, sa.n), dim3(kRowsFwdThreads),
              lds_rows, st, nd0, sa, L0, 0, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    HP_LAUNCH("spec_cols", (spec_cols<T, 512, true>), dim3(cols_x, sa.n), dim3(512), lds_cols, st,
              nd0, sa, L0, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    HP_LAUNCH("spec_rows_inv", (spec_rows_inv<T, 512, true>), dim3(inv_x, sa.n), dim3(512), lds_inv,
              st, nd0, sa, L0, 0);
    return hipGetLastError();
}
int rows_fwd_blocks(const NetDev &nd) { return nd.my / 2 / rows_fwd_lines(nd); }
template <typename T> size_t rows_fwd_lds_of(const NetDev &nd) { return rows_fwd_lds<T>(nd); }
template <typename T> size_t cols_lds_of(const NetDev &nd) { return cols_lds<T>(nd.my); }
template <typename T> size_t rows_inv_lds_of(const NetDev &nd) { return rows_inv_lds<T>(nd, 2); }

template <typename T>
int spectral_energy_parts(const NetDev &nd) { return nd.mx / 2; }

template <typename T>
size_t spectral_max_lds(const NetDev &nd) {
    return std::max(rows_fwd_lds<T>(nd), std::max(cols_lds<T>(nd.my), rows_inv_lds<T>(nd, 3)));
}

// Ask for `bytes` of dynamic LDS per block on the three passes (above the 64 KB default).
template <typename T>
hipError_t spectral_prepare(int bytes) {
    const void *fs[] = {(const void *)spec_rows_fwd<T, false>, (const void *)spec_rows_fwd<T, true>,
                        (const void *)spec_cols<T, 512, false>, (const void *)spec_cols<T, 1024, false>,
                        (const void *)spec_rows_inv<T, 512, false>,
                        (const void *)spec_rows_inv<T, 1024, false>,
                        (const void *)spec_cols<T, 512, true>, (const void *)spec_rows_inv<T, 512, true>};
    hipError_t e = hipSuccess;
    for (const void *f : fs) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#define HP_INST(T)                                                                            \
    template hipError_t launch_spectral<T>(const NetDev &, const SlotArgs &, const SlotLayout &, \
                                           bool, bool, hipStream_t);                          \
    template int spectral_energy_parts<T>(const NetDev &);                                    \
    template size_t spectral_max_lds<T>(const NetDev &);                                      \
    template hipError_t spectral_prepare<T>(int);                                             \
    template hipError_t rag_spectral<T>(const SlotArgs &, int, int, int, size_t, size_t, size_t, \
                                        hipStream_t);                                         \
    template size_t rows_fwd_lds_of<T>(const NetDev &);                                       \
    template size_t cols_lds_of<T>(const NetDev &);                                           \
    template size_t rows_inv_lds_of<T>(const NetDev &);
HP_INST(float)
HP_INST(double)
#undef HP_INST

}  // namespace hp
