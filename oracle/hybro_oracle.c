/*
 * Hybro placer hot path -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load this file; the device library never links, calls or includes it, and it
 * includes nothing of the device library.  Everything here is a slow, direct transcription of
 * the definitions, in double precision, with no fusion or blocking beyond what a definition
 * states, so that it can be checked against the paper by eye.
 *
 * Sources (paper: "Escaping Local Optima in Global Placement", Hybro):
 *   - HPWL, Eq. 1 (Sec. 3, Preliminaries): per net, x-extent plus y-extent of its pins.
 *   - Penalised objective, Eq. 2: sum of smooth wirelengths plus lambda times the density D.
 *   - Weighted-average wirelength, Eq. 3: ratio of exp-weighted sums with smoothing gamma.
 *   - The density D, the optimiser and lambda's schedule are only named by the paper; they are
 *     the ePlace/DREAMPlace electrostatic system the paper builds on (Sec. 3.1).  The readings
 *     used here (bin grid, charge stretching, cosine-basis Poisson solve, preconditioned
 *     Nesterov with a Barzilai-Borwein step, a log-linear lambda ramp) are listed with the
 *     functions that implement them.
 *   - Perturbation, Alg. 1 step "Perturb" and Sec. 4.2: select p% of the cells, or of the
 *     macros only, and exchange their places (Shuffle (all), Shuffle); move each macro to
 *     the grid position of least HPWL increment (WireMask); a seeded Gaussian displacement of
 *     a subset; and the fully random restart that Sec. 4.2 identifies with multiple-restart
 *     gradient descent.
 *   - Best solution, Alg. 1 return step: the candidate with the smallest HPWL.
 *
 * Integer contracts (so that the FP32 device path can be compared bit for bit):
 *   q16(v) = llrint(v * 2^16) for HPWL, q12(v) = llrint(v * 2^12) for density coordinates;
 *   density charge in int64 units of 2^-40 area (2^16 charge scale times 2^12 x 2^12).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC (see oracle.py).
 * OpenMP is used only on loops whose iterations own disjoint outputs; every floating-point
 * sum is accumulated serially in a fixed order, so results do not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#ifndef M_SQRT2
#define M_SQRT2 1.41421356237309504880
#endif

typedef struct {
    int32_t n_cells, n_movable, n_nets, n_pins;
    int32_t mx, my;          /* bins along x and y */
    double W, H;             /* die [0,W] x [0,H] */
    const double *cell_w, *cell_h;     /* [n_cells] */
    const double *fixed_x, *fixed_y;   /* [n_cells - n_movable], lower-left */
    const int32_t *net_start;          /* [n_nets + 1] */
    const int32_t *pin_cell;           /* [n_pins] */
    const double *pin_ox, *pin_oy;     /* [n_pins], offsets from the cell's lower-left */
    const double *net_weight;          /* [n_nets] or NULL (all 1) */
    int32_t stretch;                   /* 1: stretch small cells' charge to sqrt(2) bins */
} orc_netlist;

/* ------------------------------------------------------------------------------------------ */
/* Positions.  x, y hold the movable cells only; fixed cells sit at fixed_x/fixed_y.          */

static double cx(const orc_netlist *n, const double *x, int c)
{
    return c < n->n_movable ? x[c] : n->fixed_x[c - n->n_movable];
}
static double cy(const orc_netlist *n, const double *y, int c)
{
    return c < n->n_movable ? y[c] : n->fixed_y[c - n->n_movable];
}

static int64_t q16(double v) { return llrint(v * 65536.0); }
static int64_t q12(double v) { return llrint(v * 4096.0); }

/* ------------------------------------------------------------------------------------------ */
/* HPWL, Eq. 1: sum over nets of (max x - min x) + (max y - min y) over the net's pins.      */

double orc_hpwl(const orc_netlist *n, const double *x, const double *y)
{
    double total = 0.0;
    for (int e = 0; e < n->n_nets; ++e) {
        int s = n->net_start[e], t = n->net_start[e + 1];
        if (t - s < 2) continue;
        double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        for (int p = s; p < t; ++p) {
            double px = cx(n, x, n->pin_cell[p]) + n->pin_ox[p];
            double py = cy(n, y, n->pin_cell[p]) + n->pin_oy[p];
            if (px < xmin) xmin = px;
            if (px > xmax) xmax = px;
            if (py < ymin) ymin = py;
            if (py > ymax) ymax = py;
        }
        total += (xmax - xmin) + (ymax - ymin);
    }
    return total;
}

/* Exact HPWL of Eq. 1 on pin coordinates quantized to 2^-16: q16(cell) + q16(offset). */
int64_t orc_hpwl_q(const orc_netlist *n, const double *x, const double *y, int64_t *per_net)
{
    int64_t total = 0;
    for (int e = 0; e < n->n_nets; ++e) {
        int s = n->net_start[e], t = n->net_start[e + 1];
        int64_t h = 0;
        if (t - s >= 2) {
            int64_t xmin = INT64_MAX, xmax = INT64_MIN, ymin = INT64_MAX, ymax = INT64_MIN;
            for (int p = s; p < t; ++p) {
                int c = n->pin_cell[p];
                int64_t px = q16(cx(n, x, c)) + q16(n->pin_ox[p]);
                int64_t py = q16(cy(n, y, c)) + q16(n->pin_oy[p]);
                if (px < xmin) xmin = px;
                if (px > xmax) xmax = px;
                if (py < ymin) ymin = py;
                if (py > ymax) ymax = py;
            }
            h = (xmax - xmin) + (ymax - ymin);
        }
        if (per_net) per_net[e] = h;
        total += h;
    }
    return total;
}

/* ------------------------------------------------------------------------------------------ */
/* Weighted-average wirelength, Eq. 3, for one net and one axis.
 *
 * Eq. 3 is the difference of two exp-weighted means of the pin coordinates.  Dividing the
 * numerator and denominator of each mean by exp(max/gamma) (resp. exp(-min/gamma)) leaves the
 * value unchanged and keeps every exponent <= 0; the weighted means are then
 *   WL+ = m+ + sum (x_i - m+) a+_i / sum a+_i,  a+_i = exp((x_i - m+)/gamma)
 *   WL- = m- + sum (x_i - m-) a-_i / sum a-_i,  a-_i = exp(-(x_i - m-)/gamma)
 * and WL = WL+ - WL-.  Differentiating Eq. 3 gives, with s+-_i = a+-_i / sum a+-,
 *   dWL/dx_i = s+_i (1 + (x_i - WL+)/gamma) - s-_i (1 - (x_i - WL-)/gamma).
 */
static double wa_axis(const double *px, int d, double gamma, double *dpx)
{
    double mp = px[0], mm = px[0];
    for (int i = 1; i < d; ++i) {
        if (px[i] > mp) mp = px[i];
        if (px[i] < mm) mm = px[i];
    }
    double bp = 0.0, bm = 0.0, cp = 0.0, cm = 0.0;
    for (int i = 0; i < d; ++i) {
        double ap = exp((px[i] - mp) / gamma);
        double am = exp(-(px[i] - mm) / gamma);
        bp += ap;
        bm += am;
        cp += (px[i] - mp) * ap;
        cm += (px[i] - mm) * am;
    }
    double wlp = mp + cp / bp;
    double wlm = mm + cm / bm;
    if (dpx) {
        for (int i = 0; i < d; ++i) {
            double sp = exp((px[i] - mp) / gamma) / bp;
            double sm = exp(-(px[i] - mm) / gamma) / bm;
            dpx[i] = sp * (1.0 + (px[i] - wlp) / gamma) - sm * (1.0 - (px[i] - wlm) / gamma);
        }
    }
    return wlp - wlm;
}

/* The same value written literally as Eq. 3 (no shift); used only by tests on small inputs. */
double orc_wa_literal(const double *px, int d, double gamma)
{
    double np = 0, dp = 0, nm = 0, dm = 0;
    for (int i = 0; i < d; ++i) {
        np += px[i] * exp(px[i] / gamma);
        dp += exp(px[i] / gamma);
        nm += px[i] * exp(-px[i] / gamma);
        dm += exp(-px[i] / gamma);
    }
    return np / dp - nm / dm;
}

double orc_wa_net_axis(const double *px, int d, double gamma, double *dpx)
{
    return wa_axis(px, d, gamma, dpx);
}

/* Total weighted WA wirelength (sum over nets, x plus y) and its gradient with respect to the
 * movable cells' positions: the gradient of a cell is the sum of its pins' gradients. */
double orc_wa(const orc_netlist *n, const double *x, const double *y, double gamma,
              double *gx, double *gy, double *per_net)
{
    int maxd = 0;
    for (int e = 0; e < n->n_nets; ++e) {
        int d = n->net_start[e + 1] - n->net_start[e];
        if (d > maxd) maxd = d;
    }
    double *pin_gx = malloc(sizeof(double) * (size_t)(n->n_pins > 0 ? n->n_pins : 1));
    double *pin_gy = malloc(sizeof(double) * (size_t)(n->n_pins > 0 ? n->n_pins : 1));
    double *net_wl = malloc(sizeof(double) * (size_t)(n->n_nets > 0 ? n->n_nets : 1));
#pragma omp parallel
    {
        double *px = malloc(sizeof(double) * (size_t)(maxd + 1));
        double *py = malloc(sizeof(double) * (size_t)(maxd + 1));
#pragma omp for schedule(dynamic, 256)
        for (int e = 0; e < n->n_nets; ++e) {
            int s = n->net_start[e], t = n->net_start[e + 1], d = t - s;
            double we = n->net_weight ? n->net_weight[e] : 1.0;
            if (d < 2) {
                for (int p = s; p < t; ++p) pin_gx[p] = pin_gy[p] = 0.0;
                net_wl[e] = 0.0;
                continue;
            }
            for (int i = 0; i < d; ++i) {
                int c = n->pin_cell[s + i];
                px[i] = cx(n, x, c) + n->pin_ox[s + i];
                py[i] = cy(n, y, c) + n->pin_oy[s + i];
            }
            double wlx = wa_axis(px, d, gamma, pin_gx + s);
            double wly = wa_axis(py, d, gamma, pin_gy + s);
            for (int p = s; p < t; ++p) {
                pin_gx[p] *= we;
                pin_gy[p] *= we;
            }
            net_wl[e] = we * (wlx + wly);
        }
        free(px);
        free(py);
    }
    double total = 0.0;
    for (int e = 0; e < n->n_nets; ++e) {
        total += net_wl[e];
        if (per_net) per_net[e] = net_wl[e];
    }
    if (gx) {
        for (int i = 0; i < n->n_movable; ++i) gx[i] = gy[i] = 0.0;
        for (int p = 0; p < n->n_pins; ++p) {
            int c = n->pin_cell[p];
            if (c < n->n_movable) {
                gx[c] += pin_gx[p];
                gy[c] += pin_gy[p];
            }
        }
    }
    free(pin_gx);
    free(pin_gy);
    free(net_wl);
    return total;
}

/* ------------------------------------------------------------------------------------------ */
/* Density map (the D of Eqs. 1-2; ePlace electrostatic reading).
 *
 * The die is cut into mx x my bins of size wb x hb.  A movable cell is a charge spread over a
 * rectangle centred on the cell: its sides are stretched to at least sqrt(2) bins (ePlace's
 * local smoothing) and its charge density is scaled by r = w h / (w' h') so the total charge
 * equals the cell area.  Fixed cells put their true rectangle into a static map.  The map is
 * integer: rectangle edges are quantized to 2^-12, r to 2^-16, and the charge a cell puts in
 * bin (j,k) is r_q * ox_j * oy_k (units of 2^-40 area), exact in int64.  Map layout: row k
 * (y bin) major, [k * mx + j].
 */
typedef struct {
    int64_t wq, hq, dxq, dyq, rq;
} cellq;

static void cell_charge(const orc_netlist *n, int i, cellq *c)
{
    double w = n->cell_w[i], h = n->cell_h[i];
    double wb = n->W / n->mx, hb = n->H / n->my;
    double ws = w, hs = h, r = 1.0;
    if (i < n->n_movable && n->stretch) {
        ws = fmax(w, M_SQRT2 * wb);
        hs = fmax(h, M_SQRT2 * hb);
        r = (w * h) / (ws * hs);
    }
    c->wq = llrint(ws * 4096.0);
    c->hq = llrint(hs * 4096.0);
    c->dxq = llrint((w - ws) * 0.5 * 4096.0);
    c->dyq = llrint((h - hs) * 0.5 * 4096.0);
    c->rq = llrint(r * 65536.0);
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Overlap of [lo, hi) with bin j of width bq: max(0, min(hi, (j+1) bq) - max(lo, j bq)). */
static int64_t overlap_q(int64_t lo, int64_t hi, int64_t j, int64_t bq)
{
    int64_t a = lo > j * bq ? lo : j * bq;
    int64_t b = hi < (j + 1) * bq ? hi : (j + 1) * bq;
    return b > a ? b - a : 0;
}

/* Quantized rectangle of cell i at (x, y): [*l, *r) x [*b, *t), clipped to the die. */
static void cell_rect_q(const orc_netlist *n, int i, double x, double y, const cellq *c,
                        int64_t *l, int64_t *r, int64_t *b, int64_t *t)
{
    int64_t bq = llrint(n->W / n->mx * 4096.0), hq = llrint(n->H / n->my * 4096.0);
    int64_t Wq = bq * n->mx, Hq = hq * n->my;
    int64_t L = q12(x) + c->dxq, B = q12(y) + c->dyq;
    *l = clampi(L, 0, Wq);
    *r = clampi(L + c->wq, 0, Wq);
    *b = clampi(B, 0, Hq);
    *t = clampi(B + c->hq, 0, Hq);
    (void)i;
}

static void add_cell_q(const orc_netlist *n, int i, double x, double y, int64_t *rho)
{
    cellq c;
    cell_charge(n, i, &c);
    int64_t bq = llrint(n->W / n->mx * 4096.0), hq = llrint(n->H / n->my * 4096.0);
    int64_t l, r, b, t;
    cell_rect_q(n, i, x, y, &c, &l, &r, &b, &t);
    if (r <= l || t <= b) return;
    for (int64_t k = b / hq; k <= (t - 1) / hq; ++k) {
        int64_t oy = overlap_q(b, t, k, hq);
        for (int64_t j = l / bq; j <= (r - 1) / bq; ++j) {
            int64_t ox = overlap_q(l, r, j, bq);
            rho[k * n->mx + j] += c.rq * ox * oy;
        }
    }
}

/* Movable and fixed integer maps (either pointer may be NULL). */
void orc_density_q(const orc_netlist *n, const double *x, const double *y, int64_t *rho_mov,
                   int64_t *rho_fixed)
{
    size_t nb = (size_t)n->mx * (size_t)n->my;
    if (rho_mov) {
        memset(rho_mov, 0, nb * sizeof(int64_t));
        for (int i = 0; i < n->n_movable; ++i) add_cell_q(n, i, x[i], y[i], rho_mov);
    }
    if (rho_fixed) {
        memset(rho_fixed, 0, nb * sizeof(int64_t));
        for (int i = n->n_movable; i < n->n_cells; ++i) {
            if (n->cell_w[i] <= 0.0 || n->cell_h[i] <= 0.0) continue; /* pads carry no charge */
            add_cell_q(n, i, n->fixed_x[i - n->n_movable], n->fixed_y[i - n->n_movable],
                       rho_fixed);
        }
    }
}

/* Total movable charge sum_i r_q w'_q h'_q (the map's sum when no rectangle is clipped). */
int64_t orc_total_charge_q(const orc_netlist *n)
{
    int64_t s = 0;
    for (int i = 0; i < n->n_movable; ++i) {
        cellq c;
        cell_charge(n, i, &c);
        s += c.rq * c.wq * c.hq;
    }
    return s;
}

/* Overflow: the movable charge above the free capacity of each bin, summed, as an integer
 * (numerator) and divided by the total movable charge.  This measures D(s) <= eps of Eq. 1. */
double orc_overflow(const orc_netlist *n, const int64_t *rho_mov, const int64_t *rho_fixed,
                    double target_density, int64_t *out_num)
{
    int64_t bq = llrint(n->W / n->mx * 4096.0), hq = llrint(n->H / n->my * 4096.0);
    int64_t area_q = bq * hq * 65536;
    int64_t num = 0;
    for (int64_t b = 0; b < (int64_t)n->mx * n->my; ++b) {
        int64_t cap = llrint(target_density * (double)(area_q - rho_fixed[b]));
        int64_t over = rho_mov[b] - cap;
        if (over > 0) num += over;
    }
    if (out_num) *out_num = num;
    return (double)num / (double)orc_total_charge_q(n);
}

/* Continuous (unquantized) density map in area units, movable plus fixed; for the
 * finite-difference checks of the exact adjoint. */
static double overlap_f(double lo, double hi, double a, double b)
{
    double s = lo > a ? lo : a, t = hi < b ? hi : b;
    return t > s ? t - s : 0.0;
}

static void cell_rect_f(const orc_netlist *n, int i, double x, double y, double *l, double *r,
                        double *b, double *t, double *rr)
{
    double w = n->cell_w[i], h = n->cell_h[i];
    double wb = n->W / n->mx, hb = n->H / n->my;
    double ws = w, hs = h, sc = 1.0;
    if (i < n->n_movable && n->stretch) {
        ws = fmax(w, M_SQRT2 * wb);
        hs = fmax(h, M_SQRT2 * hb);
        sc = (w * h) / (ws * hs);
    }
    double L = x + (w - ws) * 0.5, B = y + (h - hs) * 0.5;
    *l = fmin(fmax(L, 0.0), n->W);
    *r = fmin(fmax(L + ws, 0.0), n->W);
    *b = fmin(fmax(B, 0.0), n->H);
    *t = fmin(fmax(B + hs, 0.0), n->H);
    *rr = sc;
}

void orc_density_float(const orc_netlist *n, const double *x, const double *y, double *rho)
{
    double wb = n->W / n->mx, hb = n->H / n->my;
    memset(rho, 0, sizeof(double) * (size_t)n->mx * n->my);
    for (int i = 0; i < n->n_cells; ++i) {
        if (n->cell_w[i] <= 0.0 || n->cell_h[i] <= 0.0) continue;
        double px = i < n->n_movable ? x[i] : n->fixed_x[i - n->n_movable];
        double py = i < n->n_movable ? y[i] : n->fixed_y[i - n->n_movable];
        double l, r, b, t, sc;
        cell_rect_f(n, i, px, py, &l, &r, &b, &t, &sc);
        for (int k = 0; k < n->my; ++k) {
            double oy = overlap_f(b, t, k * hb, (k + 1) * hb);
            if (oy <= 0.0) continue;
            for (int j = 0; j < n->mx; ++j) {
                double ox = overlap_f(l, r, j * wb, (j + 1) * wb);
                if (ox > 0.0) rho[k * n->mx + j] += sc * ox * oy;
            }
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Poisson solve on the bin grid in the cosine basis (ePlace electrostatics; Neumann walls).
 *
 * Bin centres are x_j = (j + 1/2) wb.  The cosine coefficients of the normalized density
 * rho_bar are
 *   a_uv = c_u c_v / (mx my) sum_{j,k} rho_bar_kj cos(pi u (j+1/2)/mx) cos(pi v (k+1/2)/my),
 * c_0 = 1, c_{>0} = 2, so that rho_bar = sum a_uv cos cos exactly.  Dropping a_00 (zero net
 * charge), with w_u = pi u / W, w_v = pi v / H and den_uv = w_u^2 + w_v^2:
 *   psi  = sum a_uv / den_uv  cos cos                       (potential, -lap psi = rho_bar - mean)
 *   xi_x = sum a_uv w_u / den_uv sin(w_u x) cos(w_v y)      (field, xi = -grad psi)
 *   xi_y = sum a_uv w_v / den_uv cos(w_u x) sin(w_v y)
 *   N    = 1/2 wb hb sum_kj rho_bar psi = 1/2 wb hb sum_{uv != 0} a_uv^2 mx my /(c_u c_v den_uv)
 * With fd5 = 1 the denominators use the 5-point Laplacian's eigenvalues
 * l_u = (2/wb)^2 sin^2(pi u / (2 mx)) instead of w_u^2.
 */
static double cos_idx(int64_t num, int M) /* cos(pi num / (2M)) with exact range reduction */
{
    int64_t r = num % (4 * (int64_t)M);
    if (r < 0) r += 4 * (int64_t)M;
    return cos(M_PI * (double)r / (2.0 * M));
}
static double sin_idx(int64_t num, int M)
{
    int64_t r = num % (4 * (int64_t)M);
    if (r < 0) r += 4 * (int64_t)M;
    return sin(M_PI * (double)r / (2.0 * M));
}

/* a_uv by the double sum written out (O(M^4)); only for small grids. Layout a[v*mx + u]. */
void orc_dct2_brute(int mx, int my, const double *rho, double *a)
{
    for (int v = 0; v < my; ++v)
        for (int u = 0; u < mx; ++u) {
            double s = 0.0;
            for (int k = 0; k < my; ++k)
                for (int j = 0; j < mx; ++j)
                    s += rho[k * mx + j] * cos_idx((int64_t)u * (2 * j + 1), mx) *
                         cos_idx((int64_t)v * (2 * k + 1), my);
            a[v * mx + u] = (u ? 2.0 : 1.0) * (v ? 2.0 : 1.0) / ((double)mx * my) * s;
        }
}

/* The same a_uv as two 1-D cosine sums (rows, then columns). */
void orc_dct2(int mx, int my, const double *rho, double *a)
{
    double *cxt = malloc(sizeof(double) * (size_t)mx * mx);
    double *cyt = malloc(sizeof(double) * (size_t)my * my);
    double *t = malloc(sizeof(double) * (size_t)mx * my);
    for (int u = 0; u < mx; ++u)
        for (int j = 0; j < mx; ++j) cxt[u * mx + j] = cos_idx((int64_t)u * (2 * j + 1), mx);
    for (int v = 0; v < my; ++v)
        for (int k = 0; k < my; ++k) cyt[v * my + k] = cos_idx((int64_t)v * (2 * k + 1), my);
#pragma omp parallel for
    for (int k = 0; k < my; ++k)
        for (int u = 0; u < mx; ++u) {
            double s = 0.0;
            for (int j = 0; j < mx; ++j) s += rho[k * mx + j] * cxt[u * mx + j];
            t[k * mx + u] = s;
        }
#pragma omp parallel for
    for (int v = 0; v < my; ++v)
        for (int u = 0; u < mx; ++u) {
            double s = 0.0;
            for (int k = 0; k < my; ++k) s += cyt[v * my + k] * t[k * mx + u];
            a[v * mx + u] = (u ? 2.0 : 1.0) * (v ? 2.0 : 1.0) / ((double)mx * my) * s;
        }
    free(cxt);
    free(cyt);
    free(t);
}

/* ---- FFT path of the same transforms (for timing; cross-checked against the sums above) ----
 * fft_inplace: X_k = sum_n x_n exp(sign 2 pi i k n / n_len), n_len a power of two (iterative
 * radix-2 decimation in time: bit-reversal permutation, then butterflies of doubling span).
 * dct_makhoul: X_u = sum_j x_j cos(pi u (2 j + 1) / (2 M)) by Makhoul's reordering (IEEE
 *   Trans. ASSP 1980): v_n = x_{2n}, v_{M-1-n} = x_{2n+1}, V = FFT_M(v), X_u = Re(e^{-i pi u/(2M)} V_u).
 * synth_fft: z_j = sum_{u<M} A_u e^{i pi u (2 j + 1)/(2 M)} as the 2M-point inverse DFT of
 *   A_u e^{i pi u/(2M)} padded with M zeros; Re z_j is the cosine synthesis, Im z_j the sine
 *   synthesis sum_u A_u sin(pi u (2 j + 1)/(2 M)). */
static void fft_inplace(double complex *x, int n, int sign)
{
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j |= bit;
        if (i < j) {
            double complex t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                double ang = sign * 2.0 * M_PI * k / len;
                double complex w = cos(ang) + I * sin(ang);
                double complex a = x[i + k], b = x[i + k + len / 2] * w;
                x[i + k] = a + b;
                x[i + k + len / 2] = a - b;
            }
    }
}

static void dct_makhoul(const double *x, int M, double *X, double complex *work)
{
    for (int n = 0; n < M / 2; ++n) {
        work[n] = x[2 * n];
        work[M - 1 - n] = x[2 * n + 1];
    }
    if (M == 1) work[0] = x[0];
    fft_inplace(work, M, -1);
    for (int u = 0; u < M; ++u) {
        double ang = -M_PI * u / (2.0 * M);
        X[u] = creal((cos(ang) + I * sin(ang)) * work[u]);
    }
}

static void synth_fft(const double *A, int M, int want_sin, double *y, double complex *work)
{
    for (int u = 0; u < M; ++u) {
        double ang = M_PI * u / (2.0 * M);
        work[u] = A[u] * (cos(ang) + I * sin(ang));
        work[M + u] = 0.0;
    }
    fft_inplace(work, 2 * M, +1);
    for (int j = 0; j < M; ++j) y[j] = want_sin ? cimag(work[j]) : creal(work[j]);
}

/* a_uv of orc_dct2, rows then columns through dct_makhoul. */
void orc_dct2_fft(int mx, int my, const double *rho, double *a)
{
    double *t = malloc(sizeof(double) * (size_t)mx * my);
#pragma omp parallel
    {
        double *in = malloc(sizeof(double) * (size_t)(mx > my ? mx : my));
        double *out = malloc(sizeof(double) * (size_t)(mx > my ? mx : my));
        double complex *w = malloc(sizeof(double complex) * (size_t)(mx > my ? mx : my));
#pragma omp for
        for (int k = 0; k < my; ++k) dct_makhoul(rho + (size_t)k * mx, mx, t + (size_t)k * mx, w);
#pragma omp for
        for (int u = 0; u < mx; ++u) {
            for (int k = 0; k < my; ++k) in[k] = t[(size_t)k * mx + u];
            dct_makhoul(in, my, out, w);
            for (int v = 0; v < my; ++v)
                a[(size_t)v * mx + u] = (u ? 2.0 : 1.0) * (v ? 2.0 : 1.0) / ((double)mx * my) * out[v];
        }
        free(in);
        free(out);
        free(w);
    }
    free(t);
}

/* out_kj = sum_{u,v} A_vu Bx(u, j) By(v, k) (as synth2) through synth_fft: rows, then columns. */
static void synth2_fft(int mx, int my, const double *A, int sin_x, int sin_y, double *out)
{
    double *s = malloc(sizeof(double) * (size_t)mx * my);
#pragma omp parallel
    {
        int mm = mx > my ? mx : my;
        double *in = malloc(sizeof(double) * (size_t)mm);
        double *o = malloc(sizeof(double) * (size_t)mm);
        double complex *w = malloc(sizeof(double complex) * 2 * (size_t)mm);
#pragma omp for
        for (int v = 0; v < my; ++v) synth_fft(A + (size_t)v * mx, mx, sin_x, s + (size_t)v * mx, w);
#pragma omp for
        for (int j = 0; j < mx; ++j) {
            for (int v = 0; v < my; ++v) in[v] = s[(size_t)v * mx + j];
            synth_fft(in, my, sin_y, o, w);
            for (int k = 0; k < my; ++k) out[(size_t)k * mx + j] = o[k];
        }
        free(in);
        free(o);
        free(w);
    }
    free(s);
}

/* Cosine synthesis (inverse of orc_dct2 up to its scale) and the sine variants, exposed for
 * the cross-checks: mode 0 cos-cos, 1 sin(x)-cos(y), 2 cos(x)-sin(y); fft selects the path. */
void orc_synth2(int mx, int my, const double *A, int mode, int fft, double *out);

/* out_kj = sum_{u,v} A_vu Bx(u, j) By(v, k) where Bx, By are cos or sin of pi u (j+1/2)/M. */
static void synth2(int mx, int my, const double *A, int sin_x, int sin_y, double *out)
{
    double *bx = malloc(sizeof(double) * (size_t)mx * mx);
    double *by = malloc(sizeof(double) * (size_t)my * my);
    double *s = malloc(sizeof(double) * (size_t)mx * my);
    for (int u = 0; u < mx; ++u)
        for (int j = 0; j < mx; ++j)
            bx[u * mx + j] = sin_x ? sin_idx((int64_t)u * (2 * j + 1), mx)
                                   : cos_idx((int64_t)u * (2 * j + 1), mx);
    for (int v = 0; v < my; ++v)
        for (int k = 0; k < my; ++k)
            by[v * my + k] = sin_y ? sin_idx((int64_t)v * (2 * k + 1), my)
                                   : cos_idx((int64_t)v * (2 * k + 1), my);
#pragma omp parallel for
    for (int v = 0; v < my; ++v)
        for (int j = 0; j < mx; ++j) {
            double acc = 0.0;
            for (int u = 0; u < mx; ++u) acc += A[v * mx + u] * bx[u * mx + j];
            s[v * mx + j] = acc;
        }
#pragma omp parallel for
    for (int k = 0; k < my; ++k)
        for (int j = 0; j < mx; ++j) {
            double acc = 0.0;
            for (int v = 0; v < my; ++v) acc += by[v * my + k] * s[v * mx + j];
            out[k * mx + j] = acc;
        }
    free(bx);
    free(by);
    free(s);
}

void orc_synth2(int mx, int my, const double *A, int mode, int fft, double *out)
{
    if (fft)
        synth2_fft(mx, my, A, mode == 1, mode == 2, out);
    else
        synth2(mx, my, A, mode == 1, mode == 2, out);
}

/* Solve for psi / xi_x / xi_y (each may be NULL) from rho_bar; returns the energy N.
 * a_out (may be NULL) receives the cosine coefficients a_uv. */
double orc_poisson(int mx, int my, double W, double H, const double *rho_bar, int fd5, int fft,
                   double *a_out, double *psi, double *ex, double *ey)
{
    size_t nb = (size_t)mx * my;
    double wb = W / mx, hb = H / my;
    double *a = malloc(sizeof(double) * nb);
    double *A = malloc(sizeof(double) * nb);
    if (fft)
        orc_dct2_fft(mx, my, rho_bar, a);
    else
        orc_dct2(mx, my, rho_bar, a);
    double energy = 0.0;
    for (int v = 0; v < my; ++v)
        for (int u = 0; u < mx; ++u) {
            if (u == 0 && v == 0) continue;
            double den = fd5 ? (4.0 / (wb * wb)) * pow(sin(M_PI * u / (2.0 * mx)), 2) +
                                   (4.0 / (hb * hb)) * pow(sin(M_PI * v / (2.0 * my)), 2)
                             : pow(M_PI * u / W, 2) + pow(M_PI * v / H, 2);
            double c = (u ? 2.0 : 1.0) * (v ? 2.0 : 1.0);
            energy += a[v * mx + u] * a[v * mx + u] * (double)mx * my / (c * den);
        }
    energy *= 0.5 * wb * hb;
    for (int pass = 0; pass < 3; ++pass) {
        double *out = pass == 0 ? psi : (pass == 1 ? ex : ey);
        if (!out) continue;
        for (int v = 0; v < my; ++v)
            for (int u = 0; u < mx; ++u) {
                double val = 0.0;
                if (u || v) {
                    double wu = M_PI * u / W, wv = M_PI * v / H;
                    double den = fd5 ? (4.0 / (wb * wb)) * pow(sin(M_PI * u / (2.0 * mx)), 2) +
                                           (4.0 / (hb * hb)) * pow(sin(M_PI * v / (2.0 * my)), 2)
                                     : wu * wu + wv * wv;
                    double num = pass == 0 ? 1.0 : (pass == 1 ? wu : wv);
                    val = a[v * mx + u] * num / den;
                }
                A[v * mx + u] = val;
            }
        if (fft)
            synth2_fft(mx, my, A, pass == 1, pass == 2, out);
        else
            synth2(mx, my, A, pass == 1, pass == 2, out);
    }
    if (a_out) memcpy(a_out, a, sizeof(double) * nb);
    free(a);
    free(A);
    return energy;
}

/* ------------------------------------------------------------------------------------------ */
/* Density gradient.
 * Field mode (the electrostatic force): dN/dx_i = - sum_b q_ib xi_x(b), q_ib the charge cell i
 * puts in bin b (from the integer map, in area units); likewise y.
 * Exact mode: dN/dx_i = sum_b psi_b dq_ib/dx_i on the continuous map, with right-hand
 * derivatives at kinks; this is the true derivative of the binned energy. */
void orc_density_grad_field(const orc_netlist *n, const double *x, const double *y,
                            const double *ex, const double *ey, double *gx, double *gy)
{
    int64_t bq = llrint(n->W / n->mx * 4096.0), hq = llrint(n->H / n->my * 4096.0);
    const double unit = ldexp(1.0, -40);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n->n_movable; ++i) {
        cellq c;
        cell_charge(n, i, &c);
        int64_t l, r, b, t;
        cell_rect_q(n, i, x[i], y[i], &c, &l, &r, &b, &t);
        double sx = 0.0, sy = 0.0;
        if (r > l && t > b) {
            for (int64_t k = b / hq; k <= (t - 1) / hq; ++k) {
                int64_t oy = overlap_q(b, t, k, hq);
                for (int64_t j = l / bq; j <= (r - 1) / bq; ++j) {
                    int64_t ox = overlap_q(l, r, j, bq);
                    double q = (double)(c.rq * ox * oy) * unit;
                    sx += q * ex[k * n->mx + j];
                    sy += q * ey[k * n->mx + j];
                }
            }
        }
        gx[i] = -sx;
        gy[i] = -sy;
    }
}

/* right derivative of overlap(lo(x), hi(x)) with bin [a, b) when lo, hi both move with x,
 * each clamped to [0, Wd] (the clamp derivative is 1 on [0, Wd) and 0 outside). */
static double doverlap(double lo_raw, double hi_raw, double a, double b, double Wd)
{
    double lo = fmin(fmax(lo_raw, 0.0), Wd), hi = fmin(fmax(hi_raw, 0.0), Wd);
    double dlo = (lo_raw >= 0.0 && lo_raw < Wd) ? 1.0 : 0.0;
    double dhi = (hi_raw >= 0.0 && hi_raw < Wd) ? 1.0 : 0.0;
    double s = lo >= a ? lo : a, ds = lo >= a ? dlo : 0.0;
    double t = hi < b ? hi : b, dt = hi < b ? dhi : 0.0;
    double o = t - s, d = dt - ds;
    if (o > 0.0) return d;
    if (o == 0.0) return d > 0.0 ? d : 0.0;
    return 0.0;
}

void orc_density_grad_exact(const orc_netlist *n, const double *x, const double *y,
                            const double *psi, double *gx, double *gy)
{
    double wb = n->W / n->mx, hb = n->H / n->my;
    for (int i = 0; i < n->n_movable; ++i) {
        double w = n->cell_w[i], h = n->cell_h[i];
        double ws = w, hs = h, sc = 1.0;
        if (n->stretch) {
            ws = fmax(w, M_SQRT2 * wb);
            hs = fmax(h, M_SQRT2 * hb);
            sc = (w * h) / (ws * hs);
        }
        double L = x[i] + (w - ws) * 0.5, B = y[i] + (h - hs) * 0.5;
        double l = fmin(fmax(L, 0.0), n->W), r = fmin(fmax(L + ws, 0.0), n->W);
        double b = fmin(fmax(B, 0.0), n->H), t = fmin(fmax(B + hs, 0.0), n->H);
        double sx = 0.0, sy = 0.0;
        for (int k = 0; k < n->my; ++k) {
            double oy = overlap_f(b, t, k * hb, (k + 1) * hb);
            double doy = doverlap(B, B + hs, k * hb, (k + 1) * hb, n->H);
            for (int j = 0; j < n->mx; ++j) {
                double ox = overlap_f(l, r, j * wb, (j + 1) * wb);
                double dox = doverlap(L, L + ws, j * wb, (j + 1) * wb, n->W);
                double p = psi[k * n->mx + j];
                sx += p * sc * dox * oy;
                sy += p * sc * ox * doy;
            }
        }
        gx[i] = sx;
        gy[i] = sy;
    }
}

/* Energy of the continuous map (for finite differences of the exact adjoint). */
double orc_density_energy_float(const orc_netlist *n, const double *x, const double *y, int fd5)
{
    size_t nb = (size_t)n->mx * n->my;
    double wb = n->W / n->mx, hb = n->H / n->my;
    double *rho = malloc(sizeof(double) * nb);
    orc_density_float(n, x, y, rho);
    for (size_t b = 0; b < nb; ++b) rho[b] /= wb * hb;
    double e = orc_poisson(n->mx, n->my, n->W, n->H, rho, fd5, 0, NULL, NULL, NULL, NULL);
    free(rho);
    return e;
}

/* ------------------------------------------------------------------------------------------ */
/* Objective of Eq. 2 and its gradient parts at positions (x, y):
 *   wl = sum_e WL_e (Eq. 3), energy = N (density term D), overflow = D(s) as a fraction,
 *   g_wl = d wl / d pos, g_d = dN / d pos (field or exact mode), all over movable cells.
 * rho_mov/rho_fixed/psi/ex/ey (may be NULL) receive the intermediate maps. */
typedef struct {
    double gamma;
    double target_density;
    int32_t grad_mode; /* 0 field, 1 exact */
    int32_t fd5;
    int32_t fft;       /* 1: the Poisson solve's transforms through the FFT path (timing) */
} orc_eval_params;

void orc_eval(const orc_netlist *n, const double *x, const double *y, const orc_eval_params *p,
              double *wl, double *energy, double *overflow, int64_t *overflow_num,
              double *gwx, double *gwy, double *gdx, double *gdy,
              int64_t *rho_mov_out, int64_t *rho_fixed_out, double *psi_out, double *ex_out,
              double *ey_out)
{
    size_t nb = (size_t)n->mx * n->my;
    double wb = n->W / n->mx, hb = n->H / n->my;
    *wl = orc_wa(n, x, y, p->gamma, gwx, gwy, NULL);
    int64_t *rm = malloc(sizeof(int64_t) * nb), *rf = malloc(sizeof(int64_t) * nb);
    double *rb = malloc(sizeof(double) * nb), *psi = malloc(sizeof(double) * nb);
    double *ex = malloc(sizeof(double) * nb), *ey = malloc(sizeof(double) * nb);
    orc_density_q(n, x, y, rm, rf);
    const double unit = ldexp(1.0, -40);
    for (size_t b = 0; b < nb; ++b) rb[b] = (double)(rm[b] + rf[b]) * unit / (wb * hb);
    *energy = orc_poisson(n->mx, n->my, n->W, n->H, rb, p->fd5, p->fft, NULL, psi, ex, ey);
    *overflow = orc_overflow(n, rm, rf, p->target_density, overflow_num);
    if (gdx) {
        if (p->grad_mode == 1)
            orc_density_grad_exact(n, x, y, psi, gdx, gdy);
        else
            orc_density_grad_field(n, x, y, ex, ey, gdx, gdy);
    }
    if (rho_mov_out) memcpy(rho_mov_out, rm, sizeof(int64_t) * nb);
    if (rho_fixed_out) memcpy(rho_fixed_out, rf, sizeof(int64_t) * nb);
    if (psi_out) memcpy(psi_out, psi, sizeof(double) * nb);
    if (ex_out) memcpy(ex_out, ex, sizeof(double) * nb);
    if (ey_out) memcpy(ey_out, ey, sizeof(double) * nb);
    free(rm);
    free(rf);
    free(rb);
    free(psi);
    free(ex);
    free(ey);
}

/* ------------------------------------------------------------------------------------------ */
/* Preconditioned Nesterov step (the gradient descent of Sec. 3.1, in ePlace's
 * accelerated form).  State over the 2*n_movable coordinates (x block then y block):
 *   u (major solution), v (reference point where the gradient is taken), v_prev, gp_prev
 *   (preconditioned gradient at v_prev), a (momentum), alpha (last step length), k.
 *   P_i = max(1, pins_i + lambda area_i);  gt = g / P
 *   alpha_0 = 0.1 wb / max|gt|;  alpha_k = |v - v_prev| / |gt - gp_prev|  (Barzilai-Borwein)
 *   u' = clamp(v - alpha gt);  a' = (1 + sqrt(4 a^2 + 1)) / 2;
 *   v' = clamp(u' + (a - 1)/a' (u' - u));  clamp keeps the cell inside the die. */
typedef struct {
    int32_t k;
    double a, alpha;
} orc_nesterov_scalars;

void orc_nesterov_step(const orc_netlist *n, double lambda, const double *g, double *u,
                       double *v, double *v_prev, double *gp_prev, orc_nesterov_scalars *s)
{
    int N = n->n_movable;
    double wb = n->W / n->mx;
    int32_t *pins = calloc((size_t)(N > 0 ? N : 1), sizeof(int32_t));
    for (int p = 0; p < n->n_pins; ++p)
        if (n->pin_cell[p] < N) pins[n->pin_cell[p]]++;
    double *gt = malloc(sizeof(double) * 2 * (size_t)(N > 0 ? N : 1));
    for (int i = 0; i < N; ++i) {
        double P = pins[i] + lambda * n->cell_w[i] * n->cell_h[i];
        if (P < 1.0) P = 1.0;
        gt[i] = g[i] / P;
        gt[N + i] = g[N + i] / P;
    }
    double alpha;
    if (s->k == 0) {
        double gmax = 0.0;
        for (int i = 0; i < 2 * N; ++i)
            if (fabs(gt[i]) > gmax) gmax = fabs(gt[i]);
        alpha = 0.1 * wb / (gmax > 1e-30 ? gmax : 1e-30);
    } else {
        double dv = 0.0, dg = 0.0;
        for (int i = 0; i < 2 * N; ++i) {
            dv += (v[i] - v_prev[i]) * (v[i] - v_prev[i]);
            dg += (gt[i] - gp_prev[i]) * (gt[i] - gp_prev[i]);
        }
        alpha = dg > 0.0 ? sqrt(dv) / sqrt(dg) : s->alpha;
    }
    double a_next = (1.0 + sqrt(4.0 * s->a * s->a + 1.0)) * 0.5;
    double coef = (s->a - 1.0) / a_next;
    for (int i = 0; i < 2 * N; ++i) {
        int c = i < N ? i : i - N;
        double hi = i < N ? n->W - n->cell_w[c] : n->H - n->cell_h[c];
        double un = v[i] - alpha * gt[i];
        un = un < 0.0 ? 0.0 : (un > hi ? hi : un);
        double vn = un + coef * (un - u[i]);
        vn = vn < 0.0 ? 0.0 : (vn > hi ? hi : vn);
        v_prev[i] = v[i];
        gp_prev[i] = gt[i];
        u[i] = un;
        v[i] = vn;
    }
    s->a = a_next;
    s->alpha = alpha;
    s->k += 1;
    free(pins);
    free(gt);
}

/* The same step with ePlace's backtracking on the predicted step length (Lu et al., ePlace,
 * TODAES 2015: Nesterov's method with Lipschitz-constant prediction).  alpha above is the step
 * length predicted at the reached point v; the step that reached v had length s->alpha.  When
 * k >= 1 and the new prediction is below 0.95 of that length, the step that reached v was too
 * long: it is redone from its own start with the new length,
 *   u = clamp(v_prev - alpha gp_prev),  v = clamp(u + (a_prev - 1)/a (u - u_prev)),
 * leaving v_prev, gp_prev, u_prev, a, a_prev and k as they were (s->rejected = 1; the gradient
 * taken at the rejected point is dropped).  Otherwise the step is the plain one above, and
 * u_prev, a_prev keep the start of this step for a later redo.  s->alpha is the length used. */
typedef struct {
    int32_t k;
    double a, a_prev, alpha;
    int32_t rejected;
} orc_nesterov_bt_scalars;

void orc_nesterov_step_bt(const orc_netlist *n, double lambda, const double *g, double *u,
                          double *v, double *v_prev, double *gp_prev, double *u_prev,
                          orc_nesterov_bt_scalars *s)
{
    int N = n->n_movable;
    double wb = n->W / n->mx;
    int32_t *pins = calloc((size_t)(N > 0 ? N : 1), sizeof(int32_t));
    for (int p = 0; p < n->n_pins; ++p)
        if (n->pin_cell[p] < N) pins[n->pin_cell[p]]++;
    double *gt = malloc(sizeof(double) * 2 * (size_t)(N > 0 ? N : 1));
    for (int i = 0; i < N; ++i) {
        double P = pins[i] + lambda * n->cell_w[i] * n->cell_h[i];
        if (P < 1.0) P = 1.0;
        gt[i] = g[i] / P;
        gt[N + i] = g[N + i] / P;
    }
    double alpha;
    if (s->k == 0) {
        double gmax = 0.0;
        for (int i = 0; i < 2 * N; ++i)
            if (fabs(gt[i]) > gmax) gmax = fabs(gt[i]);
        alpha = 0.1 * wb / (gmax > 1e-30 ? gmax : 1e-30);
    } else {
        double dv = 0.0, dg = 0.0;
        for (int i = 0; i < 2 * N; ++i) {
            dv += (v[i] - v_prev[i]) * (v[i] - v_prev[i]);
            dg += (gt[i] - gp_prev[i]) * (gt[i] - gp_prev[i]);
        }
        alpha = dg > 0.0 ? sqrt(dv) / sqrt(dg) : s->alpha;
    }
    s->rejected = s->k >= 1 && alpha < 0.95 * s->alpha;
    if (s->rejected) {
        double coef = (s->a_prev - 1.0) / s->a;
        for (int i = 0; i < 2 * N; ++i) {
            int c = i < N ? i : i - N;
            double hi = i < N ? n->W - n->cell_w[c] : n->H - n->cell_h[c];
            double un = v_prev[i] - alpha * gp_prev[i];
            un = un < 0.0 ? 0.0 : (un > hi ? hi : un);
            double vn = un + coef * (un - u_prev[i]);
            vn = vn < 0.0 ? 0.0 : (vn > hi ? hi : vn);
            u[i] = un;
            v[i] = vn;
        }
    } else {
        double a_next = (1.0 + sqrt(4.0 * s->a * s->a + 1.0)) * 0.5;
        double coef = (s->a - 1.0) / a_next;
        for (int i = 0; i < 2 * N; ++i) {
            int c = i < N ? i : i - N;
            double hi = i < N ? n->W - n->cell_w[c] : n->H - n->cell_h[c];
            double un = v[i] - alpha * gt[i];
            un = un < 0.0 ? 0.0 : (un > hi ? hi : un);
            double vn = un + coef * (un - u[i]);
            vn = vn < 0.0 ? 0.0 : (vn > hi ? hi : vn);
            u_prev[i] = u[i];
            v_prev[i] = v[i];
            gp_prev[i] = gt[i];
            u[i] = un;
            v[i] = vn;
        }
        s->a_prev = s->a;
        s->a = a_next;
        s->k += 1;
    }
    s->alpha = alpha;
    free(pins);
    free(gt);
}

/* ------------------------------------------------------------------------------------------ */
/* The placer: T iterations of [objective + gradient at v, Nesterov step], from (x, y).
 * lambda_0 = scale * |g_wl|_1 / |g_d|_1 at the first evaluation, then multiplied by
 * ratio = 10^(decades / T) each iteration (Eq. 2's lambda starts small and grows, Sec. 3).
 * On return x, y hold u_T; hpwl_trace[k] (may be NULL) is HPWL_q(u_{k+1}), lambda_trace[k]
 * the lambda of step k. */
typedef struct {
    orc_eval_params ev;
    int32_t iters;
    double lambda0_scale;
    double lambda_decades;
} orc_place_params;

double orc_lambda_ratio(double decades, int iters) { return pow(10.0, decades / iters); }

void orc_place(const orc_netlist *n, const orc_place_params *pp, double *x, double *y,
               int64_t *hpwl_trace, double *wl_trace, double *ovf_trace, double *lambda_trace)
{
    int N = n->n_movable;
    size_t N2 = 2 * (size_t)(N > 0 ? N : 1);
    double *u = malloc(sizeof(double) * N2), *v = malloc(sizeof(double) * N2);
    double *vp = malloc(sizeof(double) * N2), *gp = calloc(N2, sizeof(double));
    double *g = malloc(sizeof(double) * N2), *gd = malloc(sizeof(double) * N2);
    for (int i = 0; i < N; ++i) {
        u[i] = v[i] = vp[i] = x[i];
        u[N + i] = v[N + i] = vp[N + i] = y[i];
    }
    orc_nesterov_scalars s = {0, 1.0, 0.0};
    double lambda = 0.0, ratio = orc_lambda_ratio(pp->lambda_decades, pp->iters);
    for (int it = 0; it < pp->iters; ++it) {
        double wl, en, ovf;
        int64_t on;
        orc_eval(n, v, v + N, &pp->ev, &wl, &en, &ovf, &on, g, g + N, gd, gd + N, NULL, NULL,
                 NULL, NULL, NULL);
        if (it == 0) {
            double nw = 0.0, nd = 0.0;
            for (size_t i = 0; i < 2 * (size_t)N; ++i) {
                nw += fabs(g[i]);
                nd += fabs(gd[i]);
            }
            lambda = pp->lambda0_scale * (nd > 0.0 ? nw / nd : 1.0);
        } else {
            lambda *= ratio;
        }
        for (size_t i = 0; i < 2 * (size_t)N; ++i) g[i] += lambda * gd[i];
        orc_nesterov_step(n, lambda, g, u, v, vp, gp, &s);
        if (lambda_trace) lambda_trace[it] = lambda;
        if (wl_trace) wl_trace[it] = wl;
        if (ovf_trace) ovf_trace[it] = ovf;
        if (hpwl_trace) hpwl_trace[it] = orc_hpwl_q(n, u, u + N, NULL);
    }
    for (int i = 0; i < N; ++i) {
        x[i] = u[i];
        y[i] = u[N + i];
    }
    free(u);
    free(v);
    free(vp);
    free(gp);
    free(g);
    free(gd);
}

/* ------------------------------------------------------------------------------------------ */
/* Perturbation (Alg. 1 "Perturb"; Sec. 4.2).
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) used as a counter-based
 * generator: draw i of stream `seed` is mix64(seed + (i + 1) * 0x9e3779b97f4a7c15).
 * Subset: the m = floor(p * n_movable + 1/2) movable cells with the smallest (key_i, i).
 * SHUFFLE (the selected cells exchange places): the selected cells, in ascending index order
 *   S[0..m-1], exchange centres by a keyed permutation pi of [0, m): S[j] takes the centre of
 *   S[pi(j)].  pi is a 4-round balanced Feistel network on the smallest even bit width
 *   covering m, with cycle walking back into [0, m) (Black & Rogaway, CT-RSA 2002).
 * GAUSS: each selected cell moves by sigma * sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2)
 *   (Box-Muller), u1, u2 from the two 32-bit halves of mix64(key_i), sigma in bins.
 * UNIFORM: every movable cell is redrawn uniformly in the die (random restart).
 * Every moved cell is clamped inside the die.  Indices of moved cells go to idx (ascending). */
static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
uint64_t orc_splitmix(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * 0x9e3779b97f4a7c15ULL); }

static uint64_t feistel(uint64_t x, int half_bits, uint64_t key)
{
    uint64_t mask = (1ULL << half_bits) - 1;
    uint64_t L = x >> half_bits, R = x & mask;
    for (uint64_t r = 0; r < 4; ++r) {
        uint64_t f = mix64(key ^ ((4 * R + r + 1) * 0x9e3779b97f4a7c15ULL)) & mask;
        uint64_t nl = R, nr = L ^ f;
        L = nl;
        R = nr;
    }
    return (L << half_bits) | R;
}

uint64_t orc_shuffle_perm(uint64_t j, uint64_t m, uint64_t seed)
{
    int bits = 2;
    while ((1ULL << bits) < m) bits += 2;
    uint64_t key = mix64(seed ^ 0x5851f42d4c957f2dULL);
    uint64_t y = feistel(j, bits / 2, key);
    while (y >= m) y = feistel(y, bits / 2, key);
    return y;
}

typedef struct {
    uint64_t key;
    int32_t idx;
} keyidx;
static int cmp_keyidx(const void *a, const void *b)
{
    const keyidx *p = a, *q = b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}
static int cmp_i32(const void *a, const void *b)
{
    int32_t p = *(const int32_t *)a, q = *(const int32_t *)b;
    return (p > q) - (p < q);
}

enum { ORC_GAUSS = 0, ORC_SHUFFLE = 1, ORC_UNIFORM = 2 };

/* Perturbation among a pool of movable cells: every movable cell (cells == NULL), or the
 * n_pool distinct cells listed in `cells` (the macros of Hybro-Shuffle, Sec. 4.2: p% of the
 * macros are selected and shuffled).  A pooled cell's key is its SplitMix64 draw shifted right
 * by one bit, so that no key of the pool can equal the all-ones key of a cell outside it. */
int32_t orc_perturb_among(const orc_netlist *n, double *x, double *y, int mode, double fraction,
                          double sigma_bins, uint64_t seed, const int32_t *cells, int32_t n_pool,
                          int32_t *idx)
{
    int N = n->n_movable;
    int P = cells ? n_pool : N;
    double wb = n->W / n->mx, hb = n->H / n->my;
    int32_t m;
    int32_t *sel = malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    if (mode == ORC_UNIFORM) {
        m = N;
        for (int i = 0; i < N; ++i) sel[i] = i;
    } else {
        m = (int32_t)floor(fraction * P + 0.5);
        if (m > P) m = P;
        if (m < 0) m = 0;
        keyidx *ki = malloc(sizeof(keyidx) * (size_t)(P > 0 ? P : 1));
        for (int j = 0; j < P; ++j) {
            int c = cells ? cells[j] : j;
            ki[j].key = cells ? orc_splitmix(seed, (uint64_t)c) >> 1 : orc_splitmix(seed, (uint64_t)c);
            ki[j].idx = c;
        }
        qsort(ki, (size_t)P, sizeof(keyidx), cmp_keyidx);
        for (int j = 0; j < m; ++j) sel[j] = ki[j].idx;
        qsort(sel, (size_t)m, sizeof(int32_t), cmp_i32);
        free(ki);
    }
    if (mode == ORC_SHUFFLE) {
        double *cxs = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
        double *cys = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
        for (int j = 0; j < m; ++j) {
            int c = sel[j];
            cxs[j] = x[c] + 0.5 * n->cell_w[c];
            cys[j] = y[c] + 0.5 * n->cell_h[c];
        }
        for (int j = 0; j < m; ++j) {
            int c = sel[j];
            uint64_t src = orc_shuffle_perm((uint64_t)j, (uint64_t)m, seed);
            x[c] = cxs[src] - 0.5 * n->cell_w[c];
            y[c] = cys[src] - 0.5 * n->cell_h[c];
        }
        free(cxs);
        free(cys);
    } else {
        for (int j = 0; j < m; ++j) {
            int c = sel[j];
            uint64_t k2 = mix64(orc_splitmix(seed, (uint64_t)c));
            double u1 = ((double)(k2 >> 32) + 0.5) / 4294967296.0;
            double u2 = ((double)(k2 & 0xffffffffULL) + 0.5) / 4294967296.0;
            if (mode == ORC_GAUSS) {
                double rad = sqrt(-2.0 * log(u1));
                x[c] += sigma_bins * wb * rad * cos(2.0 * M_PI * u2);
                y[c] += sigma_bins * hb * rad * sin(2.0 * M_PI * u2);
            } else {
                x[c] = u1 * (n->W - n->cell_w[c]);
                y[c] = u2 * (n->H - n->cell_h[c]);
            }
        }
    }
    for (int j = 0; j < m; ++j) {
        int c = sel[j];
        double hx = n->W - n->cell_w[c], hy = n->H - n->cell_h[c];
        x[c] = x[c] < 0.0 ? 0.0 : (x[c] > hx ? hx : x[c]);
        y[c] = y[c] < 0.0 ? 0.0 : (y[c] > hy ? hy : y[c]);
        if (idx) idx[j] = c;
    }
    free(sel);
    return m;
}

int32_t orc_perturb(const orc_netlist *n, double *x, double *y, int mode, double fraction,
                    double sigma_bins, uint64_t seed, int32_t *idx)
{
    return orc_perturb_among(n, x, y, mode, fraction, sigma_bins, seed, NULL, 0, idx);
}

/* WireMask perturbation (Alg. 1 "Perturb", Sec. 4.2): the macros, in the given order, each move
 * to the bin-grid position with the least increment of HPWL (Eq. 1), given every other cell
 * where it is (macros earlier in the order already moved), among the positions where the macro
 * overlaps none of the other listed macros and no fixed cell of nonzero area.  Readings:
 *   - candidates are lower-left corners on bin corners, (i wb, j hb), with the macro inside the
 *     die;
 *   - the increment is the HPWL of the macro's nets with its pins at the candidate minus their
 *     HPWL without its pins, on the 2^-16 grid of the exact HPWL (nets whose only pins are the
 *     macro's add a constant and are left out);
 *   - ties go to the smaller displacement |dx| + |dy| from the macro's position, then to the
 *     lower index j * (candidates per row) + i; a macro with no free candidate stays.
 * Returns how many macros changed position. */
int32_t orc_wiremask(const orc_netlist *n, double *x, double *y, const int32_t *macros,
                     int32_t n_macros)
{
    int64_t bw = q16(n->W / n->mx), bh = q16(n->H / n->my), Wq = q16(n->W), Hq = q16(n->H);
    int32_t moved = 0;
    int64_t *X = malloc(sizeof(int64_t) * (size_t)n->mx);
    int64_t *Y = malloc(sizeof(int64_t) * (size_t)n->my);
    for (int k = 0; k < n_macros; ++k) {
        int m = macros[k];
        int64_t wq = q16(n->cell_w[m]), hq = q16(n->cell_h[m]);
        if (wq > Wq || hq > Hq) continue;
        int nci = (int)((Wq - wq) / bw) + 1, ncj = (int)((Hq - hq) / bh) + 1;
        if (nci > n->mx) nci = n->mx;
        if (ncj > n->my) ncj = n->my;
        memset(X, 0, sizeof(int64_t) * (size_t)nci);
        memset(Y, 0, sizeof(int64_t) * (size_t)ncj);
        for (int e = 0; e < n->n_nets; ++e) {
            int s = n->net_start[e], t = n->net_start[e + 1];
            if (t - s < 2) continue;
            int has_m = 0, has_other = 0;
            int64_t lox = INT64_MAX, hix = INT64_MIN, loy = INT64_MAX, hiy = INT64_MIN;
            int64_t omnx = INT64_MAX, omxx = INT64_MIN, omny = INT64_MAX, omxy = INT64_MIN;
            for (int p = s; p < t; ++p) {
                int c = n->pin_cell[p];
                int64_t ox = q16(n->pin_ox[p]), oy = q16(n->pin_oy[p]);
                if (c == m) {
                    has_m = 1;
                    if (ox < omnx) omnx = ox;
                    if (ox > omxx) omxx = ox;
                    if (oy < omny) omny = oy;
                    if (oy > omxy) omxy = oy;
                } else {
                    has_other = 1;
                    int64_t px = q16(cx(n, x, c)) + ox, py = q16(cy(n, y, c)) + oy;
                    if (px < lox) lox = px;
                    if (px > hix) hix = px;
                    if (py < loy) loy = py;
                    if (py > hiy) hiy = py;
                }
            }
            if (!has_m || !has_other) continue;
            for (int i = 0; i < nci; ++i) {
                int64_t a = (int64_t)i * bw;
                int64_t hi = a + omxx > hix ? a + omxx : hix, lo = a + omnx < lox ? a + omnx : lox;
                X[i] += (hi - lo) - (hix - lox);
            }
            for (int j = 0; j < ncj; ++j) {
                int64_t a = (int64_t)j * bh;
                int64_t hi = a + omxy > hiy ? a + omxy : hiy, lo = a + omny < loy ? a + omny : loy;
                Y[j] += (hi - lo) - (hiy - loy);
            }
        }
        int64_t xm = q16(x[m]), ym = q16(y[m]);
        int64_t b_inc = 0, b_disp = 0, b_idx = -1;
        for (int j = 0; j < ncj; ++j) {
            for (int i = 0; i < nci; ++i) {
                int64_t a = (int64_t)i * bw, b = (int64_t)j * bh;
                int legal = 1;
                for (int k2 = 0; k2 < n_macros && legal; ++k2) {
                    int o = macros[k2];
                    if (o == m) continue;
                    int64_t ox = q16(x[o]), oy = q16(y[o]), ow = q16(n->cell_w[o]), oh = q16(n->cell_h[o]);
                    if (a < ox + ow && ox < a + wq && b < oy + oh && oy < b + hq) legal = 0;
                }
                for (int f = 0; f < n->n_cells - n->n_movable && legal; ++f) {
                    int c = n->n_movable + f;
                    if (!(n->cell_w[c] > 0.0) || !(n->cell_h[c] > 0.0)) continue;
                    int64_t ox = q16(n->fixed_x[f]), oy = q16(n->fixed_y[f]);
                    int64_t ow = q16(n->cell_w[c]), oh = q16(n->cell_h[c]);
                    if (a < ox + ow && ox < a + wq && b < oy + oh && oy < b + hq) legal = 0;
                }
                if (!legal) continue;
                int64_t inc = X[i] + Y[j];
                int64_t disp = (a > xm ? a - xm : xm - a) + (b > ym ? b - ym : ym - b);
                int64_t idx = (int64_t)j * nci + i;
                if (b_idx < 0 || inc < b_inc || (inc == b_inc && (disp < b_disp ||
                                                                  (disp == b_disp && idx < b_idx)))) {
                    b_inc = inc;
                    b_disp = disp;
                    b_idx = idx;
                }
            }
        }
        if (b_idx < 0) continue;
        double nx = (double)((b_idx % nci) * bw) / 65536.0, ny = (double)((b_idx / nci) * bh) / 65536.0;
        if (nx != x[m] || ny != y[m]) moved++;
        x[m] = nx;
        y[m] = ny;
    }
    free(X);
    free(Y);
    return moved;
}

/* Best of Alg. 1: index of the smallest HPWL; ties go to the lowest index. */
int32_t orc_argmin_i64(const int64_t *v, int32_t n)
{
    int32_t b = -1;
    for (int32_t i = 0; i < n; ++i)
        if (b < 0 || v[i] < v[b]) b = i;
    return b;
}

/* Threads the oracle's parallel loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
/* Thread count of later parallel loops (timing only; results do not depend on it). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int orc_num_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif
