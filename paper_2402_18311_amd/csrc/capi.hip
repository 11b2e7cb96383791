// Host side of libhybro: argument validation, netlist preprocessing (degree buckets, cell ->
// pin CSR, quantized per-cell charge constants, spectral tables), buffer layouts, and the
// launch sequences of every C-ABI entry point.  No device memory is allocated here: all of
// it lives in buffers the caller lends.
#include <algorithm>
#include <atomic>
#include <deque>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "hp_internal.h"
#include "hybro.h"

using namespace hp;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HP_CHECK(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(HP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Propagate a failed HP_* return code of a helper.
#define HP_TRY(call)                 \
    do {                             \
        const int r_ = (call);       \
        if (r_ != HP_OK) return r_;  \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// f(lo, hi) over [0, n) split into contiguous ranges on up to 16 host threads (a single call
// for small n); the ranges own disjoint outputs.
// The context lock of an entry point (see hp_ctx::mu).
#define HP_GUARD(ctx)                                                          \
    if (!(ctx)) return fail(HP_EINVAL, "ctx is NULL");                         \
    std::unique_lock<std::recursive_mutex> hp_guard_((ctx)->mu)
// Wait for the context's stream without holding its lock (other threads keep queueing work
// meanwhile); the caller's slot and netlist stay in place, as slots and netlists are only
// appended or marked dead.
#define HP_SYNC_UNLOCKED(ctx)                                                  \
    do {                                                                       \
        ++(ctx)->stream_users;                                                 \
        hp_guard_.unlock();                                                    \
        const hipError_t e_ = hipStreamSynchronize((ctx)->stream);             \
        --(ctx)->stream_users;                                                 \
        hp_guard_.lock();                                                      \
        if (e_ != hipSuccess)                                                  \
            return fail(HP_EDEVICE, std::string("hipStreamSynchronize: ") +    \
                                        hipGetErrorString(e_));                \
    } while (0)

template <typename F>
void parallel_ranges(int64_t n, F &&f) {
    const int64_t grain = 1 << 16;
    int nt = (int)std::min<int64_t>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())),
                                    (n + grain - 1) / grain);
    if (nt <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] { f(n * t / nt, n * (t + 1) / nt); });
    for (auto &x : th) x.join();
}

// ---- static scratch of the allocation-free entry point (hp_hpwl_noalloc) --------------------
// Per-block partial sums of the exact-HPWL sweep live in this file-scope device array, one
// copy per GPU, held until the process ends.  In host code its name is only a stand-in: the
// device address of each GPU's copy is looked up once per device (with that device current) at
// context creation and kept in g_scratch, and only that address is handed to kernels.
constexpr int kNoAllocParts = 131072;  // 1 MiB of int64 partials
static __device__ __align__(256) long long scratch[kNoAllocParts];
std::mutex g_scratch_mu;
std::vector<void *> g_scratch;  // [device] address of that device's copy, or null

int scratch_setup(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch.size() <= device) g_scratch.resize(device + 1, nullptr);
    if (g_scratch[device]) return HP_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(HP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = ptr;
    return HP_OK;
}

void *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device < (int)g_scratch.size() ? g_scratch[device] : nullptr;
}

// Pin slots of the sweep order: a net of d <= 64 pins takes G = nextpow2(d) < 2d slots (the
// unused ones padded), a larger net exactly d, so 2 * n_pins bounds them.
size_t sweep_slots_bound(const hp_shape &s) { return 2 * (size_t)s.n_pins + 64; }

// v is held exactly in T and v * 2^16 is an integer: its 2^-16 quantization is then the
// exact product, which the device can form from the T value itself.
template <typename T>
static bool q16_exact(double v) {
    const double q = v * 65536.0;
    return (double)(T)v == v && std::nearbyint(q) == q && std::fabs(q) < 2147483648.0;
}

struct NetBuf {
    size_t net_start, pin_cell, pin_off, pin_off16, pin_offq, net_w, cell_pin_start, cell_pins, cq, cq16, rq,
        cstep, cell_wh, rho_fixed, tw_x, tw_y, ph_x, ph_y, omega, den1, fixed_pos, fxy, fwh,
        big_ids, cell_pin_net, sweep_map, total;
};

size_t part_stride(const hp_shape &s, const hp_die &d);

NetBuf net_layout(const hp_shape &s, const hp_die &d, size_t rs) {
    NetBuf b{};
    size_t o = 0;
    auto put = [&](size_t &f, size_t bytes) {
        f = o;
        o = align256(o + bytes);
    };
    const size_t E = s.n_nets, P = s.n_pins, Nm = s.n_movable, Nf = s.n_cells - s.n_movable;
    const size_t mx = d.mx, my = d.my, PS = sweep_slots_bound(s);
    put(b.net_start, 4 * (E + 1));
    put(b.pin_cell, 4 * PS);
    put(b.pin_off, 2 * rs * PS);
    put(b.pin_offq, 8 * PS);
    put(b.pin_off16, 4 * PS);
    put(b.net_w, rs * E);
    put(b.cell_pin_start, 4 * (Nm + 1));
    put(b.cell_pins, 4 * P);
    put(b.cq, 16 * Nm);
    put(b.cq16, 8 * Nm);
    put(b.rq, 4 * Nm);
    put(b.cstep, 4 * rs * Nm);
    put(b.cell_wh, 2 * rs * Nm);
    put(b.rho_fixed, 8 * mx * my);
    put(b.tw_x, 2 * rs * (mx / 2));
    put(b.tw_y, 2 * rs * (my / 2));
    put(b.ph_x, 2 * rs * mx);
    put(b.ph_y, 2 * rs * my);
    put(b.omega, 8 * (mx + my));
    put(b.den1, 8 * (mx + my));
    put(b.fixed_pos, 2 * rs * Nf);
    put(b.fxy, 16 * Nf);
    put(b.fwh, 16 * Nf);
    put(b.big_ids, 4 * Nm);
    put(b.cell_pin_net, 4 * P);
    put(b.sweep_map, 4 * (part_stride(s, d) / kXcds + 1));
    b.total = o;
    return b;
}

// Upper bound of the blocks of any per-slot reduction (sweep, cells, spectral columns).
size_t part_stride(const hp_shape &s, const hp_die &d) {
    const size_t sweep = (size_t)s.n_pins / 65 + (size_t)s.n_nets / 4 + 8 * kMaxBuckets + 8;
    const size_t cells = ((size_t)s.n_movable + kBlock - 1) / kBlock;
    return std::max<size_t>({sweep, cells, (size_t)d.mx, 1});
}

// Geometry of the tile-binned scatter that depends only on the grid and the cell count.
struct BinGeom {
    int log_ts, ntx, nty, ntiles, sort_cells, sort_blocks, max_chunks;
};

BinGeom bin_geom(const hp_shape &s, const hp_die &d) {
    BinGeom g{};
    int ts = 16;
    while (ts < std::min(d.mx, d.my) && (d.mx / ts) * (d.my / ts) > 8192) ts *= 2;
    ts = std::min(ts, std::min(d.mx, d.my));
    g.log_ts = 0;
    while ((1 << g.log_ts) < ts) ++g.log_ts;
    g.ntx = d.mx / ts;
    g.nty = d.my / ts;
    g.ntiles = g.ntx * g.nty;
    const int n = std::max(1, s.n_movable);
    // a multiple of 2048 cells, enough that there are at most kMaxSortBlocks blocks
    g.sort_cells = 2048 * ((n + 2048 * kMaxSortBlocks - 1) / (2048 * kMaxSortBlocks));
    g.sort_blocks = (n + g.sort_cells - 1) / g.sort_cells;
    g.max_chunks = (n + kChunk - 1) / kChunk + g.ntiles;
    return g;
}

// halo: widest charge footprint in bins minus one (at most the tile size); the byte-size
// bound used before a netlist is known takes the largest allowed halo.
SlotLayout slot_layout(const hp_shape &s, const hp_die &d, size_t rs, int halo = -1) {
    SlotLayout L{};
    const BinGeom g = bin_geom(s, d);
    if (halo < 0) halo = 1 << g.log_ts;
    const size_t ws = (size_t)(1 << g.log_ts) + halo;
    size_t o = kDescBytes;  // the slot's descriptor (SlotDesc) first
    auto put = [&](size_t &f, size_t bytes) {
        f = o;
        o = align256(o + bytes);
    };
    const size_t Nc = s.n_cells, Nm = s.n_movable, P = s.n_pins, nb = (size_t)d.mx * d.my;
    put(L.u, 2 * rs * Nc);
    put(L.v, 2 * rs * Nc);
    put(L.vprev, 2 * rs * Nm);
    put(L.uprev, 2 * rs * Nm);
    put(L.gprev, 2 * rs * Nm);
    put(L.g, 2 * rs * Nm);
    put(L.gd, 2 * rs * Nm);
    put(L.pin_grad, 2 * rs * sweep_slots_bound(s));
    put(L.rho, 8 * nb);
    put(L.t1, rs * nb);
    put(L.bx, rs * nb);
    put(L.by, rs * nb);
    put(L.bp, rs * nb);
    put(L.psi, rs * nb);
    put(L.exy, 2 * rs * nb);
    put(L.scal, sizeof(Scalars));
    L.pstride = part_stride(s, d);
    put(L.part, 8 * PART_COUNT * L.pstride);
    put(L.keys, 8 * Nm);
    put(L.sel, 4 * Nm);
    put(L.work, perturb_work_bytes((int)Nm, d.mx, d.my));
    put(L.tile, 4 * Nm);
    put(L.sorted, 4 * Nm);
    put(L.crec, 16 * Nm);
    put(L.scnt, 4 * (size_t)g.sort_blocks * g.ntiles);
    put(L.soff, 4 * (size_t)g.sort_blocks * g.ntiles);
    put(L.tstart, 4 * ((size_t)g.ntiles + 1));
    put(L.cstart, 4 * ((size_t)g.ntiles + 1));
    put(L.chunk, 16 * (size_t)g.max_chunks);
    put(L.wins, 8 * (size_t)g.ntiles * ws * ws);
    L.total = o;
    return L;
}

struct Netlist {
    bool alive = false;
    hp_shape shape{};
    hp_die die{};
    NetDev nd{};
    Buckets bk{};
    SlotLayout L{};
    char *buf = nullptr;
    int e_parts = 0;
    // scatter grouping policy (hp_set_scatter_policy): rebuild every `regroup_every`
    // evaluations; `deferred`: the rebuilding evaluation accumulates in the existing order
    int regroup_every = kRegroupEvery;
    bool deferred = true;
    // hp_set_tunable: most cell-gradient partials for which the update reduces them itself
    int fused_parts = kFusedStepParts;
    // hp_set_tunable: a rebuild accumulated in the same evaluation reads charge records
    bool charge_records = true;
    std::vector<int64_t> charge_prefix;  // [n_mov + 1] integer charge of cells [0, i)
};

struct Slot {
    bool alive = false;
    int netlist = -1;
    char *base = nullptr;
    bool lambda_valid = false;  // host mirror of the device flag
    bool maps_valid = false;
    bool hpwl_requested = false; // hp_hpwl was called; its sweep is not launched yet
    bool hpwl_pending = false;  // an HPWL sweep was launched; its partials are not yet reduced
    bool step_proposed = false; // the last evaluation formed the next step's proposal...
    bool step_fused = false;    // ... or only its partials, for the fused step to reduce
    bool totals_pending = false; // the last evaluation's WL / energy / overflow not yet reduced
    int bank = 0;               // current bank of the optimiser state (Scalars::kb, ab, alphab)
    int since_group = -1;       // evaluations since the scatter's tile order was built (-1: none)
    bool rho_dirty = false;     // rho holds a kept map, not zeros
};

// Every field of the host state of a slot that decides the launches of its next iterations.
bool same_state(const Slot &a, const Slot &b) {
    return a.alive == b.alive && a.netlist == b.netlist && a.base == b.base &&
           a.lambda_valid == b.lambda_valid && a.maps_valid == b.maps_valid &&
           a.hpwl_requested == b.hpwl_requested && a.hpwl_pending == b.hpwl_pending &&
           a.step_proposed == b.step_proposed && a.step_fused == b.step_fused &&
           a.totals_pending == b.totals_pending && a.bank == b.bank &&
           a.since_group == b.since_group && a.rho_dirty == b.rho_dirty;
}

// A captured block of hp_iterate or hp_iterate_multi (HP_ITER_GRAPH): its launches, the call's
// slots, its key (which call; smoothing, flags and the launch settings of the slots' netlists),
// and the host state of the slots at the block's start, which the block returns them to.
struct GraphBlock {
    bool valid = false;
    std::vector<int32_t> slots;
    std::vector<double> key;
    int len = 0;
    std::vector<Slot> start;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void drop_graph(GraphBlock &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = GraphBlock{};
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

struct hp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int precision = 32;
    int lds_budget = 65536;
    int n_cu = 256;  // compute units of the device
    // deques: references to an element stay valid while other threads append (a call may
    // release the lock while it waits for the stream, see HP_SYNC_UNLOCKED)
    std::deque<Netlist> nets;
    std::deque<Slot> slots;
    GraphBlock graph;  // the last captured block of hp_iterate (HP_ITER_GRAPH)
    int64_t graph_captures = 0, graph_replays = 0;
    // Entry points hold it for their whole call (a netlist load only while it registers the
    // netlist), so that threads may share a context: e.g. one loads arriving jobs while another
    // iterates the resident ones.
    std::recursive_mutex mu;
    // Threads using the stream without holding mu (a netlist load's uploads, a wait for the
    // stream), counted up while holding mu: no graph capture starts while it is non-zero, as
    // the stream must not be used by another thread while it is being captured.
    std::atomic<int> stream_users{0};
};

namespace {

size_t rsize(const hp_ctx *c) { return c->precision == 64 ? 8 : 4; }

int max_bins(const hp_ctx *c) { return c->precision == 64 ? 1024 : 2048; }

int check_die(const hp_ctx *ctx, const hp_die *d) {
    if (!d) return fail(HP_EINVAL, "die is NULL");
    if (!(std::isfinite(d->W) && std::isfinite(d->H) && d->W > 0 && d->H > 0))
        return fail(HP_EINVAL, "die W/H must be finite and positive");
    if (!is_pow2(d->mx) || !is_pow2(d->my) || d->mx < 8 || d->my < 8 || d->mx > max_bins(ctx) ||
        d->my > max_bins(ctx))
        return fail(HP_EINVAL, "bins mx/my must be powers of two in [8, " +
                                   std::to_string(max_bins(ctx)) + "]");
    const double bq = d->W / d->mx * 4096.0, hq = d->H / d->my * 4096.0;
    if (bq != std::floor(bq) || hq != std::floor(hq) || bq < 1 || hq < 1)
        return fail(HP_EINVAL, "bin width and height must be multiples of 2^-12");
    if (d->W > 16384.0 || d->H > 16384.0)  // pin coordinates in 2^-16 units stay below 2^31
        return fail(HP_EINVAL, "die sides must be at most 16384 (32-bit exact HPWL coordinates)");
    if (!(d->target_density > 0 && d->target_density <= 1e6))
        return fail(HP_EINVAL, "target_density must be positive");
    return HP_OK;
}

int check_shape(const hp_shape *s) {
    if (!s) return fail(HP_EINVAL, "shape is NULL");
    if (s->n_cells < 0 || s->n_movable < 0 || s->n_movable > s->n_cells || s->n_nets < 0 ||
        s->n_pins < 0)
        return fail(HP_EINVAL, "bad shape counts");
    if (s->n_movable == 0) return fail(HP_EINVAL, "no movable cell: nothing to place");
    return HP_OK;
}

template <typename T>
int load_netlist(hp_ctx *ctx, const hp_shape &S, const hp_die &D, const double *cell_w,
                 const double *cell_h, const double *fixed_x, const double *fixed_y,
                 const int32_t *net_start, const int32_t *pin_cell, const double *pin_ox,
                 const double *pin_oy, const double *net_weight, char *buf, Netlist &NL) {
    const int Nc = S.n_cells, Nm = S.n_movable, Nf = Nc - Nm, E = S.n_nets, P = S.n_pins;
    // ---- validation (host) ----------------------------------------------------------------
    if ((Nc && (!cell_w || !cell_h)) || (Nf && (!fixed_x || !fixed_y)) || !net_start ||
        (P && (!pin_cell || !pin_ox || !pin_oy)))
        return fail(HP_EINVAL, "required netlist array is NULL");
    if (net_start[0] != 0 || net_start[E] != P) return fail(HP_EINVAL, "net_start[0] must be 0 and net_start[n_nets] == n_pins");
    for (int e = 0; e < E; ++e)
        if (net_start[e + 1] < net_start[e]) return fail(HP_EINVAL, "net_start must be non-decreasing");
    {
        // the first bad pin in each range (ranges in order, so the first bad pin overall wins)
        std::vector<std::pair<int64_t, int>> bad;
        std::mutex mu;
        parallel_ranges(P, [&](int64_t lo, int64_t hi) {
            for (int64_t p = lo; p < hi; ++p) {
                int why = 0;
                if (pin_cell[p] < 0 || pin_cell[p] >= Nc) why = 1;
                else if (!std::isfinite(pin_ox[p]) || !std::isfinite(pin_oy[p])) why = 2;
                else if (std::fabs(pin_ox[p]) * 65536.0 >= 2147483647.0 ||
                         std::fabs(pin_oy[p]) * 65536.0 >= 2147483647.0)
                    why = 3;
                if (why) {
                    std::lock_guard<std::mutex> lk(mu);
                    bad.push_back({p, why});
                    return;
                }
            }
        });
        if (!bad.empty()) {
            const auto first = *std::min_element(bad.begin(), bad.end());
            if (first.second == 1)
                return fail(HP_EINVAL, "pin_cell[" + std::to_string(first.first) + "] out of range");
            if (first.second == 2) return fail(HP_EINVAL, "pin offsets must be finite");
            return fail(HP_EINVAL, "pin offset too large");
        }
    }
    for (int i = 0; i < Nc; ++i) {
        const double w = cell_w[i], h = cell_h[i];
        if (!std::isfinite(w) || !std::isfinite(h) || w < 0 || h < 0)
            return fail(HP_EINVAL, "cell sizes must be finite and >= 0");
        if (i < Nm && (w <= 0 || h <= 0 || w > D.W || h > D.H))
            return fail(HP_EINVAL, "movable cell " + std::to_string(i) + " must have 0 < size <= die");
    }
    for (int i = 0; i < Nf; ++i)
        if (!std::isfinite(fixed_x[i]) || !std::isfinite(fixed_y[i]))
            return fail(HP_EINVAL, "fixed positions must be finite");
    if (net_weight)
        for (int e = 0; e < E; ++e)
            if (!std::isfinite(net_weight[e])) return fail(HP_EINVAL, "net weights must be finite");

    const NetBuf B = net_layout(S, D, sizeof(T));
    NetDev &nd = NL.nd;
    nd = NetDev{};
    nd.n_cells = Nc;
    nd.n_mov = Nm;
    nd.n_fixed = Nf;
    nd.mx = D.mx;
    nd.my = D.my;
    nd.logmx = ilog2(D.mx);
    nd.logmy = ilog2(D.my);
    nd.W = D.W;
    nd.H = D.H;
    nd.wb = D.W / D.mx;
    nd.hb = D.H / D.my;
    nd.bq = (int)std::llrint(nd.wb * 4096.0);
    nd.hq = (int)std::llrint(nd.hb * 4096.0);
    nd.wq_die = nd.bq * D.mx;
    nd.hq_die = nd.hq * D.my;
    nd.density_unit = std::ldexp(1.0, -40) / (nd.wb * nd.hb);
    nd.area_q = (int64_t)nd.bq * nd.hq * 65536;
    nd.target_density = D.target_density;
    nd.lds_budget = ctx->lds_budget;
    nd.n_cu = ctx->n_cu;
    nd.spec_threads = 0;
    if (spectral_max_lds<T>(nd) > (size_t)nd.lds_budget)
        return fail(HP_EINVAL, "bin grid too large for this device's LDS at this precision");

    // ---- degree buckets -------------------------------------------------------------------
    // G = 0: nets over 256 pins, a block each; G = 256, 128, ..., 4: G = next power of two >= d
    // (d >= 3) slots per net, spread over G / 4 lanes; G = 2: two-pin nets, a lane each.
    constexpr int NB = 9;
    const int Gs[NB] = {0, 256, 128, 64, 32, 16, 8, 4, 2};
    // Every bucket but the first is laid out padded: net j of the bucket owns pin slots
    // [pin0 + j G, pin0 + (j + 1) G), its pins first, the rest marked by cell -1, so a lane
    // finds its pin slots from its index alone (G < 2d, so at most 2P slots).  The padded
    // buckets come first in memory, largest G first, so every net's slots start at a multiple
    // of 4 (of 2 for G = 2) and lanes load four slots at once; the block-per-net bucket comes
    // last in memory but first in the grid (its long nets start early).  Each block takes
    // 4 kBlock / G nets of a padded bucket with G >= 4, kPairNets kBlock two-pin nets, or one
    // net of the first bucket.
    std::vector<std::vector<int>> members(NB);
    for (int e = 0; e < E; ++e) {
        const int d = net_start[e + 1] - net_start[e];
        if (d < 2) continue;
        int b = 0;
        if (d <= 256) {
            int G = 2;
            while (G < d) G <<= 1;
            b = 1 + (8 - ilog2(G));
        }
        members[b].push_back(e);
    }
    std::stable_sort(members[0].begin(), members[0].end(), [&](int a, int b) {
        return net_start[a + 1] - net_start[a] > net_start[b + 1] - net_start[b];
    });
    // padded buckets: order nets by their lowest cell, so neighbouring lanes gather
    // neighbouring cells and each XCD's share of a bucket covers a compact cell range (a
    // stable counting sort by lowest cell: ties keep net order)
    {
        std::vector<int32_t> minc(E, 0);
        parallel_ranges(E, [&](int64_t lo, int64_t hi) {
            for (int64_t e = lo; e < hi; ++e) {
                int32_t m = INT32_MAX;
                for (int p = net_start[e]; p < net_start[e + 1]; ++p) m = std::min(m, pin_cell[p]);
                minc[e] = m;
            }
        });
        std::vector<int32_t> start((size_t)Nc + 1, 0), sorted;
        for (int b = 1; b < NB; ++b)
            for (int e : members[b]) ++start[(size_t)minc[e] + 1];
        for (int c = 0; c < Nc; ++c) start[c + 1] += start[c];
        sorted.resize(start[Nc]);
        for (int b = 1; b < NB; ++b)  // nets of every padded bucket, in net order
            for (int e : members[b]) sorted[start[minc[e]]++] = e;
        std::vector<int> bucket_of(E, -1);
        for (int b = 1; b < NB; ++b) {
            for (int e : members[b]) bucket_of[e] = b;
            members[b].clear();
        }
        for (int e : sorted) members[bucket_of[e]].push_back(e);
    }
    // sweep order of the nets (memory order): padded buckets by decreasing G, then the
    // block-per-net bucket
    const int mem_order[NB] = {1, 2, 3, 4, 5, 6, 7, 8, 0};
    std::vector<int> order, first(NB, 0);
    for (int m = 0; m < NB; ++m) {
        const int b = mem_order[m];
        first[b] = (int)order.size();
        order.insert(order.end(), members[b].begin(), members[b].end());
    }
    // bucket entries in grid order: the block-per-net bucket, then G = 256 ... 2
    Buckets bk{};
    int blk = 0;
    for (int b = 0; b < NB; ++b) {
        if (members[b].empty()) continue;
        const int G = Gs[b];
        const int npb = G == 0 ? 1 : G == 2 ? kPairNets * kBlock : 4 * kBlock / G;
        int nblk = ((int)members[b].size() + npb - 1) / npb;
        nblk = (nblk + kXcds - 1) / kXcds * kXcds;
        bk.G[bk.n] = G;
        bk.net0[bk.n] = first[b];
        bk.net1[bk.n] = first[b] + (int)members[b].size();
        bk.blk0[bk.n] = blk;
        bk.nblk[bk.n] = nblk;
        blk += nblk;
        ++bk.n;
    }
    if (bk.n == 0) {  // no net with two pins: one idle bucket so the reductions still run
        bk.n = 1;
        bk.G[0] = 0;
        bk.nblk[0] = kXcds;
        blk = kXcds;
    }
    bk.total_blocks = blk;
    if ((size_t)blk > part_stride(S, D)) return fail(HP_EINVAL, "internal: sweep block bound");
    // Interleaved block order of the padded buckets (hp_set_tunable HP_TUNE_SWEEP_INTERLEAVE):
    // an XCD's blocks of every bucket merged by their progress through the bucket, so that all
    // buckets sweep the same cell range at the same time.  Entry (bucket << 24 | i): the i-th
    // of that bucket's blocks on the XCD.  The block-per-net bucket leads, in its own order.
    std::vector<int32_t> h_smap;
    int lead = 0;
    {
        std::vector<std::pair<double, int32_t>> keys;
        for (int b = 0; b < bk.n; ++b) {
            if (bk.G[b] == 0) {
                lead += bk.nblk[b];
                continue;
            }
            const int q = bk.nblk[b] / kXcds;
            for (int i = 0; i < q; ++i) keys.push_back({(i + 0.5) / q, (b << 24) | i});
        }
        std::stable_sort(keys.begin(), keys.end(),
                         [](const auto &a, const auto &c) { return a.first < c.first; });
        for (const auto &k : keys) h_smap.push_back(k.second);
    }
    nd.sweep_lead = lead;
    nd.sweep_interleave = 0;
    nd.sweep_nt = 0;
    const int ns = (int)order.size();
    nd.ns = ns;

    std::vector<int32_t> h_ns(ns + 1);
    std::vector<T> h_w;
    bool any_w = false;
    if (net_weight)
        for (int e = 0; e < E; ++e) any_w |= net_weight[e] != 1.0;
    // entries in memory order (by their first sweep net); each sweep net's first pin slot: its
    // G slots in a padded bucket, its own pins in the block-per-net bucket
    std::vector<int> by_mem(bk.n);
    std::iota(by_mem.begin(), by_mem.end(), 0);
    std::sort(by_mem.begin(), by_mem.end(), [&](int a, int c) { return bk.net0[a] < bk.net0[c]; });
    {
        int32_t slot = 0;
        for (int m = 0, i = 0; m < bk.n; ++m) {
            const int b = by_mem[m];
            bk.pin0[b] = slot;
            for (; i < bk.net1[b]; ++i) {
                h_ns[i] = slot;
                const int d = net_start[order[i] + 1] - net_start[order[i]];
                slot += bk.G[b] ? bk.G[b] : d;
            }
        }
        h_ns[ns] = slot;
    }
    const int ps = h_ns[ns];
    std::vector<int32_t> h_pc(ps), h_pq(2 * (size_t)ps);
    std::vector<T> h_po(2 * (size_t)ps);
    std::atomic<bool> all_exact{true};
    parallel_ranges(ns, [&](int64_t lo, int64_t hi) {
        bool ex = true;
        for (int64_t i = lo; i < hi; ++i) {
            const int e = order[i];
            int32_t q = h_ns[i];
            for (int p = net_start[e]; p < net_start[e + 1]; ++p, ++q) {
                ex = ex && q16_exact<T>(pin_ox[p]) && q16_exact<T>(pin_oy[p]);
                h_pc[q] = pin_cell[p];
                h_po[2 * (size_t)q] = (T)pin_ox[p];
                h_po[2 * (size_t)q + 1] = (T)pin_oy[p];
                h_pq[2 * (size_t)q] = (int32_t)std::llrint(pin_ox[p] * 65536.0);
                h_pq[2 * (size_t)q + 1] = (int32_t)std::llrint(pin_oy[p] * 65536.0);
            }
            for (; q < h_ns[i + 1]; ++q) {  // padding slots
                h_pc[q] = -1;
                h_po[2 * (size_t)q] = h_po[2 * (size_t)q + 1] = T(0);
                h_pq[2 * (size_t)q] = h_pq[2 * (size_t)q + 1] = 0;
            }
        }
        if (!ex) all_exact = false;
    });
    const bool offq_exact = all_exact;
    // the compact offsets: the finest power-of-two unit 2^-s (s <= 15) of which every offset is
    // a multiple, if every offset then fits an int16; the sweeps decode them to the same values
    int off16_shift = -1;
    {
        // per value: a multiple of 2^-15 of magnitude below 2^52 (else no compaction), needing
        // 15 - (trailing zero bits of its 2^-15 count) fractional bits
        std::mutex mu;
        int need = 0;
        double amax = 0.0;
        std::atomic<bool> ok{true};
        parallel_ranges(P, [&](int64_t lo, int64_t hi) {
            int nd_ = 0;
            double am = 0.0;
            for (int64_t p = lo; p < hi && ok.load(std::memory_order_relaxed); ++p)
                for (const double o : {pin_ox[p], pin_oy[p]}) {
                    const double q = std::ldexp(o, 15);
                    if (!(std::fabs(q) < 0x1p52) || q != std::nearbyint(q)) {
                        ok = false;
                        break;
                    }
                    const long long qi = std::llabs(std::llrint(q));
                    if (qi) nd_ = std::max(nd_, 15 - std::min(15, __builtin_ctzll((unsigned long long)qi)));
                    am = std::max(am, std::fabs(o));
                }
            std::lock_guard<std::mutex> lk(mu);
            need = std::max(need, nd_);
            amax = std::max(amax, am);
        });
        if (ok && std::ldexp(amax, need) <= 32767.0) off16_shift = need;
    }
    std::vector<int32_t> h_po16;
    if (off16_shift >= 0) {
        h_po16.assign(ps, 0);
        for (int q = 0; q < ps; ++q) {
            const int x = (int)std::llrint(std::ldexp((double)h_po[2 * (size_t)q], off16_shift));
            const int y = (int)std::llrint(std::ldexp((double)h_po[2 * (size_t)q + 1], off16_shift));
            h_po16[q] = (int32_t)(((uint32_t)(uint16_t)(int16_t)y << 16) | (uint16_t)(int16_t)x);
        }
    }
    if (any_w)
        for (int i = 0; i < ns; ++i) h_w.push_back((T)net_weight[order[i]]);
    nd.ps = ps;
    nd.offq_exact = offq_exact ? 1 : 0;
    nd.off16_shift = off16_shift;
    if ((size_t)ps > sweep_slots_bound(S)) return fail(HP_EINVAL, "internal: sweep slot bound");

    // cell -> sweep-pin CSR (movable cells), and pin counts over all nets for the
    // preconditioner
    std::vector<int32_t> h_cps(Nm + 1, 0), cnt_all(Nm, 0);
    for (int p = 0; p < P; ++p)
        if (pin_cell[p] < Nm) cnt_all[pin_cell[p]]++;
    for (int q = 0; q < ps; ++q)
        if (h_pc[q] >= 0 && h_pc[q] < Nm) h_cps[h_pc[q] + 1]++;
    for (int i = 0; i < Nm; ++i) h_cps[i + 1] += h_cps[i];
    std::vector<int32_t> h_cp(h_cps[Nm]), h_cpn(h_cps[Nm]);
    {
        std::vector<int32_t> fill(h_cps.begin(), h_cps.end() - 1);
        for (int e = 0; e < ns; ++e)  // the sweep net of each of those pin slots
            for (int q = h_ns[e]; q < h_ns[e + 1]; ++q)
                if (h_pc[q] >= 0 && h_pc[q] < Nm) {
                    h_cpn[fill[h_pc[q]]] = e;
                    h_cp[fill[h_pc[q]]++] = q;
                }
    }

    // per-cell charge constants (2^-12 / 2^-16 integers, computed in FP64 once)
    std::vector<int32_t> h_cq(4 * (size_t)Nm), h_rq(Nm);
    std::vector<T> h_cs(4 * (size_t)Nm), h_wh(2 * (size_t)Nm);
    int64_t total_charge = 0;
    long long halo = 0;
    // big cells: a footprint that can span more than kBigHalo + 1 bins on an axis, i.e.
    // (b + w'q - 2) / b > kBigHalo for bin size b (all in 2^-12 units), or an area of
    // kBigArea bins or more
    nd.big_wq = kBigHalo * nd.bq + 2;
    nd.big_hq = kBigHalo * nd.hq + 2;
    nd.big_aq = (int64_t)kBigArea * nd.bq * nd.hq;
    std::vector<int32_t> h_big;
    NL.charge_prefix.assign((size_t)Nm + 1, 0);
    {
#pragma clang fp contract(off)
        for (int i = 0; i < Nm; ++i) {
            const double w = cell_w[i], h = cell_h[i];
            double ws = w, hs = h, r = 1.0;
            if (D.stretch) {
                ws = std::fmax(w, M_SQRT2 * nd.wb);
                hs = std::fmax(h, M_SQRT2 * nd.hb);
                r = (w * h) / (ws * hs);
            }
            const long long wq = std::llrint(ws * 4096.0), hq = std::llrint(hs * 4096.0);
            const long long dxq = std::llrint((w - ws) * 0.5 * 4096.0);
            const long long dyq = std::llrint((h - hs) * 0.5 * 4096.0);
            const long long rq = std::llrint(r * 65536.0);
            h_cq[4 * (size_t)i + 0] = (int32_t)wq;
            h_cq[4 * (size_t)i + 1] = (int32_t)hq;
            h_cq[4 * (size_t)i + 2] = (int32_t)dxq;
            h_cq[4 * (size_t)i + 3] = (int32_t)dyq;
            h_rq[i] = (int32_t)rq;
            total_charge += rq * wq * hq;
            NL.charge_prefix[(size_t)i + 1] = total_charge;
            h_cs[i] = (T)cnt_all[i];
            h_cs[(size_t)Nm + i] = (T)(w * h);
            h_cs[2 * (size_t)Nm + i] = (T)(D.W - w);
            h_cs[3 * (size_t)Nm + i] = (T)(D.H - h);
            h_wh[i] = (T)w;
            h_wh[(size_t)Nm + i] = (T)h;
            // bins a rectangle of this width can span, minus one (big cells stay out of the
            // tile windows)
            if (is_big(nd, make_int4((int)wq, (int)hq, 0, 0)))
                h_big.push_back(i);
            else
                halo = std::max<long long>(halo, std::max((nd.bq + wq - 2) / nd.bq, (nd.hq + hq - 2) / nd.hq));
        }
    }
    nd.n_big = (int32_t)h_big.size();
    nd.total_charge = total_charge > 0 ? total_charge : 1;
    nd.stretch = D.stretch;
    {
        const BinGeom g = bin_geom(S, D);
        if (halo > (1 << g.log_ts))
            return fail(HP_EINVAL, "a movable cell's charge spans more bins than the scatter tile");
        nd.log_ts = g.log_ts;
        nd.ntx = g.ntx;
        nd.nty = g.nty;
        nd.ntiles = g.ntiles;
        nd.halo = (int)halo;
        nd.win_side = (1 << g.log_ts) + (int)halo;
        nd.sort_cells = g.sort_cells;
        nd.sort_blocks = g.sort_blocks;
        nd.max_chunks = g.max_chunks;
    }

    // spectral tables: FFT twiddles exp(-2 pi i k / M), DCT phases (cos, sin)(pi u / 2M),
    // w_u = pi u / W and the per-axis Laplacian symbol
    auto twid = [](int M) {
        std::vector<T> t(M);
        for (int k = 0; k < M / 2; ++k) {
            t[2 * k] = (T)std::cos(2.0 * M_PI * k / M);
            t[2 * k + 1] = (T)(-std::sin(2.0 * M_PI * k / M));
        }
        return t;
    };
    auto phase = [](int M) {
        std::vector<T> t(2 * (size_t)M);
        for (int u = 0; u < M; ++u) {
            t[2 * u] = (T)std::cos(M_PI * u / (2.0 * M));
            t[2 * u + 1] = (T)std::sin(M_PI * u / (2.0 * M));
        }
        return t;
    };
    std::vector<double> h_om(D.mx + D.my), h_den(D.mx + D.my);
    for (int u = 0; u < D.mx; ++u) {
        h_om[u] = M_PI * u / D.W;
        h_den[u] = D.fd5 ? (4.0 / (nd.wb * nd.wb)) * std::pow(std::sin(M_PI * u / (2.0 * D.mx)), 2)
                         : std::pow(M_PI * u / D.W, 2);
    }
    for (int v = 0; v < D.my; ++v) {
        h_om[D.mx + v] = M_PI * v / D.H;
        h_den[D.mx + v] = D.fd5 ? (4.0 / (nd.hb * nd.hb)) * std::pow(std::sin(M_PI * v / (2.0 * D.my)), 2)
                                : std::pow(M_PI * v / D.H, 2);
    }
    std::vector<T> h_fp(2 * (size_t)Nf);
    std::vector<double> h_fxy(2 * (size_t)Nf), h_fwh(2 * (size_t)Nf);
    for (int i = 0; i < Nf; ++i) {
        h_fp[2 * (size_t)i] = (T)fixed_x[i];  // (x, y) pairs, the layout of slot positions
        h_fp[2 * (size_t)i + 1] = (T)fixed_y[i];
        h_fxy[i] = fixed_x[i];
        h_fxy[(size_t)Nf + i] = fixed_y[i];
        h_fwh[i] = cell_w[Nm + i];
        h_fwh[(size_t)Nf + i] = cell_h[Nm + i];
    }

    // ---- upload ---------------------------------------------------------------------------
    hipStream_t st = ctx->stream;
    auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(buf + off, src, bytes, hipMemcpyHostToDevice, st);
    };
    HP_CHECK(up(B.net_start, h_ns.data(), 4 * h_ns.size()));
    HP_CHECK(up(B.pin_cell, h_pc.data(), 4 * h_pc.size()));
    HP_CHECK(up(B.pin_off, h_po.data(), sizeof(T) * h_po.size()));
    HP_CHECK(up(B.pin_offq, h_pq.data(), 4 * h_pq.size()));
    if (!h_po16.empty()) HP_CHECK(up(B.pin_off16, h_po16.data(), 4 * h_po16.size()));
    if (any_w) HP_CHECK(up(B.net_w, h_w.data(), sizeof(T) * h_w.size()));
    HP_CHECK(up(B.cell_pin_start, h_cps.data(), 4 * h_cps.size()));
    HP_CHECK(up(B.cell_pins, h_cp.data(), 4 * h_cp.size()));
    HP_CHECK(up(B.cell_pin_net, h_cpn.data(), 4 * h_cpn.size()));
    HP_CHECK(up(B.cq, h_cq.data(), 4 * h_cq.size()));
    // the compact charge constants, when every cell's four values fit an int16 (the host
    // copy lives to the end of the load, like the others)
    std::vector<int32_t> h_cq16;
    {
        bool fits = true;
        for (const int32_t v : h_cq) fits = fits && v >= -32768 && v <= 32767;
        nd.cq_compact = fits ? 1 : 0;
        if (fits) {
            h_cq16.assign(2 * (size_t)Nm, 0);
            for (int i = 0; i < Nm; ++i) {
                const int32_t *c = &h_cq[4 * (size_t)i];
                h_cq16[2 * (size_t)i] = (int32_t)(((uint32_t)(uint16_t)(int16_t)c[1] << 16) |
                                                  (uint16_t)(int16_t)c[0]);
                h_cq16[2 * (size_t)i + 1] = (int32_t)(((uint32_t)(uint16_t)(int16_t)c[3] << 16) |
                                                      (uint16_t)(int16_t)c[2]);
            }
            HP_CHECK(up(B.cq16, h_cq16.data(), 4 * h_cq16.size()));
        }
    }
    HP_CHECK(up(B.rq, h_rq.data(), 4 * h_rq.size()));
    HP_CHECK(up(B.cstep, h_cs.data(), sizeof(T) * h_cs.size()));
    HP_CHECK(up(B.cell_wh, h_wh.data(), sizeof(T) * h_wh.size()));
    std::vector<T> twx = twid(D.mx), twy = twid(D.my), phx = phase(D.mx), phy = phase(D.my);
    HP_CHECK(up(B.tw_x, twx.data(), sizeof(T) * (size_t)D.mx));
    HP_CHECK(up(B.tw_y, twy.data(), sizeof(T) * (size_t)D.my));
    HP_CHECK(up(B.ph_x, phx.data(), sizeof(T) * phx.size()));
    HP_CHECK(up(B.ph_y, phy.data(), sizeof(T) * phy.size()));
    HP_CHECK(up(B.omega, h_om.data(), 8 * h_om.size()));
    HP_CHECK(up(B.den1, h_den.data(), 8 * h_den.size()));
    HP_CHECK(up(B.fixed_pos, h_fp.data(), sizeof(T) * h_fp.size()));
    HP_CHECK(up(B.fxy, h_fxy.data(), 8 * h_fxy.size()));
    HP_CHECK(up(B.fwh, h_fwh.data(), 8 * h_fwh.size()));
    HP_CHECK(up(B.big_ids, h_big.data(), 4 * h_big.size()));
    if (!h_smap.empty()) HP_CHECK(up(B.sweep_map, h_smap.data(), 4 * h_smap.size()));
    HP_CHECK(hipMemsetAsync(buf + B.rho_fixed, 0, 8 * (size_t)D.mx * D.my, st));

    nd.net_start = reinterpret_cast<const int32_t *>(buf + B.net_start);
    nd.pin_cell = reinterpret_cast<const int32_t *>(buf + B.pin_cell);
    nd.pin_off = buf + B.pin_off;
    nd.pin_offq = reinterpret_cast<const int2 *>(buf + B.pin_offq);
    nd.pin_off16 = reinterpret_cast<const int32_t *>(buf + B.pin_off16);
    nd.net_w = any_w ? buf + B.net_w : nullptr;
    nd.cell_pin_start = reinterpret_cast<const int32_t *>(buf + B.cell_pin_start);
    nd.cell_pins = reinterpret_cast<const int32_t *>(buf + B.cell_pins);
    nd.cq = reinterpret_cast<const int4 *>(buf + B.cq);
    nd.cq16 = reinterpret_cast<const int2 *>(buf + B.cq16);
    nd.rq = reinterpret_cast<const int32_t *>(buf + B.rq);
    nd.cstep = buf + B.cstep;
    nd.cell_wh = buf + B.cell_wh;
    nd.rho_fixed = reinterpret_cast<const int64_t *>(buf + B.rho_fixed);
    nd.tw_x = buf + B.tw_x;
    nd.tw_y = buf + B.tw_y;
    nd.ph_x = buf + B.ph_x;
    nd.ph_y = buf + B.ph_y;
    nd.omega = reinterpret_cast<const double *>(buf + B.omega);
    nd.den1 = reinterpret_cast<const double *>(buf + B.den1);
    nd.fixed_pos = buf + B.fixed_pos;
    nd.big_ids = reinterpret_cast<const int32_t *>(buf + B.big_ids);
    nd.cell_pin_net = reinterpret_cast<const int32_t *>(buf + B.cell_pin_net);
    nd.sweep_map = reinterpret_cast<const int32_t *>(buf + B.sweep_map);
    nd.fixed_xy = reinterpret_cast<const double *>(buf + B.fxy);
    nd.fixed_wh = reinterpret_cast<const double *>(buf + B.fwh);
    HP_CHECK(launch_fixed_map<T>(nd, reinterpret_cast<const double *>(buf + B.fxy),
                                 reinterpret_cast<const double *>(buf + B.fwh),
                                 reinterpret_cast<int64_t *>(buf + B.rho_fixed), st));
    HP_CHECK(hipStreamSynchronize(st));  // host staging vectors die at return

    NL.alive = true;
    NL.shape = S;
    NL.die = D;
    NL.bk = bk;
    NL.L = slot_layout(S, D, sizeof(T), nd.halo);
    NL.buf = buf;
    NL.e_parts = spectral_energy_parts<T>(nd);
    return HP_OK;
}

int get_slot(hp_ctx *ctx, int32_t id, Slot **s, Netlist **n) {
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (id < 0 || id >= (int)ctx->slots.size() || !ctx->slots[id].alive)
        return fail(HP_ESTATE, "unknown slot " + std::to_string(id));
    *s = &ctx->slots[id];
    *n = &ctx->nets[(*s)->netlist];
    return HP_OK;
}

// Write the descriptor (SlotDesc) of NL into the head of every listed slot buffer, on the
// context's stream, and wait for it: slot allocation and launch-setting changes only.
int write_descs(hp_ctx *ctx, const Netlist &NL, const std::vector<char *> &bases) {
    const SlotDesc d{NL.nd, NL.bk, NL.L};
    for (char *b : bases)
        HP_CHECK(hipMemcpyAsync(b, &d, sizeof(d), hipMemcpyHostToDevice, ctx->stream));
    HP_CHECK(hipStreamSynchronize(ctx->stream));
    return HP_OK;
}
int rewrite_descs(hp_ctx *ctx, int netlist) {
    std::vector<char *> bases;
    for (const Slot &s : ctx->slots)
        if (s.alive && s.netlist == netlist) bases.push_back(s.base);
    return write_descs(ctx, ctx->nets[netlist], bases);
}

// Resolve a slot list into launch chunks (all on one netlist).
int resolve(hp_ctx *ctx, const int32_t *slots, int32_t n, Netlist **net,
            std::vector<SlotArgs> &chunks, std::vector<Slot *> &ss) {
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (!slots || n <= 0) return fail(HP_EINVAL, "empty slot list");
    *net = nullptr;
    ss.clear();
    chunks.clear();
    for (int i = 0; i < n; ++i) {
        Slot *s;
        Netlist *nl;
        int rc = get_slot(ctx, slots[i], &s, &nl);
        if (rc) return rc;
        if (*net && nl != *net) return fail(HP_ESTATE, "slots of one call must share a netlist");
        for (Slot *o : ss)
            if (o == s) return fail(HP_EINVAL, "slot " + std::to_string(slots[i]) + " listed twice");
        *net = nl;
        ss.push_back(s);
        if (i % kMaxSlots == 0) chunks.push_back(SlotArgs{});
        SlotArgs &c = chunks.back();
        c.base[c.n++] = s->base;
    }
    return HP_OK;
}

// hp_hpwl only records the request; the sweep of u runs inside the next evaluation's first
// launch, or here, before anything that would change u or read the result.
int launch_requested_hpwl(hp_ctx *ctx, Netlist *NL, const std::vector<Slot *> &ss) {
    SlotArgs sa{};
    auto go = [&]() -> int {
        if (ctx->precision == 32)
            HP_CHECK(launch_sweep_hpwl<float>(NL->nd, NL->bk, sa, NL->L, ctx->stream));
        else
            HP_CHECK(launch_sweep_hpwl<double>(NL->nd, NL->bk, sa, NL->L, ctx->stream));
        sa.n = 0;
        return HP_OK;
    };
    for (Slot *s : ss) {
        if (!s->hpwl_requested) continue;
        s->hpwl_requested = false;
        s->hpwl_pending = true;
        sa.base[sa.n++] = s->base;
        if (sa.n == kMaxSlots) HP_TRY(go());
    }
    if (sa.n) HP_TRY(go());
    return HP_OK;
}

// Reduce the HPWL partials of slots whose sweep has not been totalled yet.
int finish_hpwl(hp_ctx *ctx, Netlist *NL, const std::vector<Slot *> &ss) {
    HP_TRY(launch_requested_hpwl(ctx, NL, ss));
    SlotArgs sa{};
    for (Slot *s : ss) {
        if (!s->hpwl_pending) continue;
        s->hpwl_pending = false;
        sa.base[sa.n++] = s->base;
        if (sa.n == kMaxSlots) {
            HP_CHECK(launch_hpwl_finish(sa, NL->L, NL->bk.total_blocks, ctx->stream));
            sa.n = 0;
        }
    }
    if (sa.n) HP_CHECK(launch_hpwl_finish(sa, NL->L, NL->bk.total_blocks, ctx->stream));
    return HP_OK;
}

// The WL / energy / overflow totals of evaluations that left them to be reduced when read
// (fused steady state), from the partials the evaluation wrote (no later launch writes them
// before the slot's next evaluation).
int finish_totals(hp_ctx *ctx, Netlist *NL, const std::vector<Slot *> &ss) {
    SlotArgs sa{};
    auto flush = [&]() -> int {
        HP_CHECK(launch_eval_finish(NL->nd, sa, NL->L, NL->bk.total_blocks, NL->e_parts,
                                    spectral_overflow_parts(NL->nd), 0, false, 0.0, FIN_TOTALS,
                                    0, ctx->stream));
        sa.n = 0;
        return HP_OK;
    };
    for (Slot *s : ss) {
        if (!s->totals_pending) continue;
        s->totals_pending = false;
        sa.base[sa.n++] = s->base;
        if (sa.n == kMaxSlots) HP_TRY(flush());
    }
    if (sa.n) HP_TRY(flush());
    return HP_OK;
}

int check_eval_params(const hp_eval_params *p) {
    if (!p) return fail(HP_EINVAL, "params is NULL");
    if (!(p->gamma > 0) || !std::isfinite(p->gamma)) return fail(HP_EINVAL, "gamma must be > 0");
    if (p->grad_mode < 0 || p->grad_mode > 3) return fail(HP_EINVAL, "grad_mode must be 0..3");
    if ((p->grad_mode & GRAD_DENSITY_ONLY) && !(p->lambda >= 0))
        return fail(HP_EINVAL, "a density-only evaluation needs lambda >= 0 given");
    if (p->lambda >= 0 && !std::isfinite(p->lambda)) return fail(HP_EINVAL, "lambda must be finite");
    return HP_OK;
}

// The launches of one evaluation of resolved slots (parameters already checked).
template <typename T>
int eval_resolved(hp_ctx *ctx, Netlist *NL, const std::vector<SlotArgs> &chunks,
                  const std::vector<Slot *> &ss, const hp_eval_params *p) {
    const bool use_fixed = p->lambda >= 0;
    const bool wl_on = !(p->grad_mode & GRAD_DENSITY_ONLY);
    hipStream_t st = ctx->stream;
    const NetDev &nd = NL->nd;
    const SlotLayout &L = NL->L;
    // a density-only evaluation has no sweep for a pending HPWL request to ride in
    if (!wl_on) HP_TRY(launch_requested_hpwl(ctx, NL, ss));
    for (size_t c = 0; c < chunks.size(); ++c) {
        const SlotArgs &sa = chunks[c];
        bool any_init = false;
        bool fresh = false, due = false, dirty = false;
        uint32_t hmask = 0;  // slots whose requested HPWL sweep rides along
        for (int i = 0; i < sa.n; ++i) {
            Slot *s = ss[c * kMaxSlots + i];
            any_init |= !use_fixed && !s->lambda_valid;
            fresh |= s->since_group < 0;
            due |= s->since_group >= NL->regroup_every;
            dirty |= s->rho_dirty;
            if (s->hpwl_requested) {
                hmask |= 1u << i;
                s->hpwl_requested = false;
                s->hpwl_pending = true;
            }
        }
        uint32_t banks = 0;
        for (int i = 0; i < sa.n; ++i) banks |= (uint32_t)ss[c * kMaxSlots + i]->bank << i;
        // steady state: the totals are reduced when first read; with few enough cell-gradient
        // partials there is no closing reduction at all (the step derives its proposal itself),
        // else it forms the step only
        // (density only: the totals now, with no wirelength partials)
        const bool fused = !any_init && wl_on && cell_parts(nd) <= NL->fused_parts;
        const int finish = (any_init || !wl_on) ? FIN_FULL : (fused ? -1 : FIN_STEP);
        const int nwl = wl_on ? NL->bk.total_blocks : 0;
        if (dirty) HP_CHECK(launch_clear_rho(nd, sa, L, st));
        // The scatter's grouping.  A slot without one (fresh), or a periodic rebuild (due) of
        // a netlist whose policy is not deferred, counts for a new order in the first launch
        // and accumulates in it right after (regroup tail with accumulation).  A deferred
        // periodic rebuild accumulates in the existing order in the first launch and counts
        // for the new order in the same launch; the rest of the rebuild (scans, place) runs
        // after the row pass, the last reader of the existing order's windows, so the next
        // evaluation accumulates in the new order.
        const bool rebuild_now = fresh || (due && !NL->deferred);
        const bool accum_now = !rebuild_now, count_now = fresh || due;
        const bool records = rebuild_now && NL->charge_records;
        // WA sweep, HPWL sweep and the scatter's accumulation and/or counting in one launch
        HP_CHECK(launch_eval_front<T>(nd, NL->bk, sa, L, 1.0 / p->gamma, hmask, accum_now,
                                      count_now, records, wl_on, st));
        if (rebuild_now) HP_CHECK(launch_regroup_tail<T>(nd, sa, L, true, records, st));
        HP_CHECK(launch_spectral<T>(nd, sa, L, p->keep_maps != 0,
                                    p->keep_maps != 0 || (p->grad_mode & GRAD_EXACT), st));
        if (!rebuild_now && due) HP_CHECK(launch_regroup_tail<T>(nd, sa, L, false, false, st));
        HP_CHECK(launch_big_grad<T>(nd, sa, L, p->grad_mode, st));
        HP_CHECK(launch_cell_grad<T>(nd, sa, L, use_fixed ? p->lambda : 0.0, use_fixed, p->grad_mode,
                                     nwl, NL->e_parts, spectral_overflow_parts(nd), finish, banks,
                                     st));
        if (any_init) HP_CHECK(launch_combine<T>(nd, sa, L, st));
        for (int i = 0; i < sa.n; ++i) {
            Slot *s = ss[c * kMaxSlots + i];
            s->maps_valid = p->keep_maps != 0;
            // a steady-state evaluation (lambda known) also proposed the next step (or, fused,
            // left its partials for the step to reduce)
            s->step_proposed = use_fixed || s->lambda_valid;
            s->step_fused = fused && s->step_proposed;
            s->totals_pending = finish != FIN_FULL;
            if (!use_fixed) s->lambda_valid = true;
            s->since_group = count_now ? 1 : s->since_group + 1;
            s->rho_dirty = p->keep_maps != 0;
        }
    }
    return HP_OK;
}

template <typename T>
int eval_impl(hp_ctx *ctx, const int32_t *slots, int32_t n, const hp_eval_params *p, double *wl,
              double *energy, double *overflow, void *gx, void *gy) {
    Netlist *NL;
    std::vector<SlotArgs> chunks;
    std::vector<Slot *> ss;
    int rc = resolve(ctx, slots, n, &NL, chunks, ss);
    if (rc) return rc;
    HP_TRY(check_eval_params(p));
    HP_TRY(eval_resolved<T>(ctx, NL, chunks, ss, p));
    hipStream_t st = ctx->stream;
    const SlotLayout &L = NL->L;
    const size_t rs = sizeof(T), Nm = NL->nd.n_mov;
    for (int i = 0; i < n; ++i) {
        if (gx) HP_CHECK(hipMemcpyAsync((char *)gx + i * Nm * rs, ss[i]->base + L.g, Nm * rs,
                                        hipMemcpyDeviceToDevice, st));
        if (gy) HP_CHECK(hipMemcpyAsync((char *)gy + i * Nm * rs, ss[i]->base + L.g + Nm * rs,
                                        Nm * rs, hipMemcpyDeviceToDevice, st));
    }
    if (wl || energy || overflow) {
        HP_TRY(finish_totals(ctx, NL, ss));
        std::vector<Scalars> h(n);
        for (int i = 0; i < n; ++i)
            HP_CHECK(hipMemcpyAsync(&h[i], ss[i]->base + L.scal, sizeof(Scalars), hipMemcpyDeviceToHost, st));
        HP_CHECK(hipStreamSynchronize(st));
        for (int i = 0; i < n; ++i) {
            if (wl) wl[i] = h[i].wl;
            if (energy) energy[i] = h[i].energy;
            if (overflow) overflow[i] = h[i].overflow;
        }
    }
    return HP_OK;
}

void init_scalars(Scalars &s, double scale, double decades, int iters) {
    std::memset(&s, 0, sizeof(s));
    s.ab[0] = s.ab[1] = 1.0;
    s.lambda0_scale = scale;
    s.lambda_ratio = std::pow(10.0, decades / iters);
    s.best = -1;
}

}  // namespace

// ---- per-kernel timing (process-wide; the on flag is read lock-free at every launch, the rest
// is guarded so that threads sharing or not sharing a context may launch while it is on) ------
namespace hp {
namespace {
std::atomic<bool> g_prof_on{false};
std::mutex g_prof_mu;      // guards everything below
std::string g_prof_only;  // empty: every kernel
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
struct ProfAcc {
    std::string name;
    int64_t count = 0;
    double ms = 0.0;
};
std::vector<ProfAcc> g_prof_acc;
}  // namespace
bool prof_want(const char *name) {
    if (!g_prof_on.load(std::memory_order_relaxed)) return false;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_only.empty() || g_prof_only == name;
}
hipEvent_t prof_event() {
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_pool.empty()) {
            hipEvent_t e = g_prof_pool.back();
            g_prof_pool.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}
void prof_push(const char *name, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back({name, a, b});
}
}  // namespace hp

namespace {
int step_resolved(hp_ctx *ctx, Netlist *NL, const std::vector<SlotArgs> &chunks,
                  const std::vector<Slot *> &ss) {
    HP_TRY(launch_requested_hpwl(ctx, NL, ss));  // the step changes u
    for (size_t c = 0; c < chunks.size(); ++c) {
        const SlotArgs &sa = chunks[c];
        // all proposed by their closing reductions: update only; all fused: the update derives
        // the proposals; otherwise (a second step on one gradient, or a mix): reductions and
        // proposals again from the gradient
        bool proposed = true, fused = true, any_fused = false;
        uint32_t banks = 0;
        for (int i = 0; i < sa.n; ++i) {
            const Slot *s = ss[c * kMaxSlots + i];
            proposed &= s->step_proposed;
            fused &= s->step_fused;
            any_fused |= s->step_fused;
            banks |= (uint32_t)s->bank << i;
        }
        if (any_fused && !fused) proposed = false;
        if (ctx->precision == 32)
            HP_CHECK(launch_step<float>(NL->nd, sa, NL->L, proposed, fused, banks, ctx->stream));
        else
            HP_CHECK(launch_step<double>(NL->nd, sa, NL->L, proposed, fused, banks, ctx->stream));
    }
    for (Slot *s : ss) {
        s->step_proposed = false;
        s->step_fused = false;
        s->bank ^= 1;  // the step committed into the other bank
    }
    return HP_OK;
}

// An HPWL request of resolved slots: the sweep of u reads only u and writes only its own
// partials, so it is deferred into the next evaluation's first launch (where it fills the
// machine beside the WA sweep) or launched before anything that changes u or reads it; the
// total is reduced from the partials when first needed.
int hpwl_resolved(hp_ctx *, Netlist *, const std::vector<SlotArgs> &,
                  const std::vector<Slot *> &ss) {
    for (Slot *s : ss) s->hpwl_requested = true;
    return HP_OK;
}
}  // namespace

// ============================================================================================
namespace {
// Iterations over slots of different netlists in shared launches: every launch of an
// iteration covers all slots (blockIdx.y), each block finding its slot's netlist, layout and
// sizes in the descriptor at the head of the slot buffer.  The launches and their arithmetic
// are those of hp_iterate's steady state, with the scatter's grouping rebuilt inside the
// rebuilding evaluation, and the step in its fused form when every slot's netlist takes it,
// else in its closing-reduction form (all of these bit-identical to the other forms).
// Runs iterations of `one` (the launches of one iteration and the host-state updates that go with
// them) from `done` towards `iters`, replaying steady blocks of L iterations from the context's
// cached graph.  A block is captured by running the same launch logic under stream capture and
// replayed while every slot's host state (the only input of that logic besides the call's
// parameters, which `key` records with the slots) equals the state the block was captured
// from; a block whose end state differs from its start (not yet steady) is thrown away and the
// iterations run eagerly.  No capture while another thread uses the stream outside the lock
// (the iterations then run as they are; replays need no capture and stay allowed).  Returns
// with fewer than L iterations left; the caller runs those eagerly.
// the longest block of iterations captured as one graph (longer cycles iterate eagerly)
constexpr int kMaxGraphBlock = 64;

template <class One>
int run_graph_blocks(hp_ctx *ctx, const std::vector<int32_t> &sl, const std::vector<Slot *> &ss,
                     const std::vector<double> &key, int L, int iters, int &done, One one) {
    GraphBlock &G = ctx->graph;
    const int n = (int)ss.size();
    auto state_is = [&](const std::vector<Slot> &st) {
        for (int i = 0; i < n; ++i)
            if (!same_state(*ss[i], st[i])) return false;
        return true;
    };
    bool have = G.valid && G.slots == sl && G.key == key && G.len == L;
    int attempts = 0, eager_run = 0;
    while (iters - done >= L) {
        if (have && state_is(G.start)) {
            HP_CHECK(hipGraphLaunch(G.exec, ctx->stream));
            ++ctx->graph_replays;
            done += L;
            eager_run = 0;
            continue;
        }
        // A call starts in the state left by whatever read the slots last (pending
        // reductions done), which no block returns to: one eager iteration brings the
        // slots into the steady cycle.  With a block for these parameters at hand, eager
        // iterations run until the slots reach its start (at most L); capture only without
        // one, or when that does not happen.
        bool steady = true;
        for (const Slot *s : ss) steady &= s->lambda_valid && !s->rho_dirty && s->since_group >= 0;
        if (steady && eager_run >= 1 && attempts < 2 && (!have || eager_run > L) &&
            ctx->stream_users.load() == 0) {
            ++attempts;
            std::vector<Slot> snap;
            for (const Slot *s : ss) snap.push_back(*s);
            HP_CHECK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            int crc = HP_OK;
            for (int k = 0; k < L && crc == HP_OK; ++k) crc = one();
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(ctx->stream, &g);
            const bool periodic = crc == HP_OK && ce == hipSuccess && state_is(snap);
            for (int i = 0; i < n; ++i) *ss[i] = snap[i];  // the capture ran nothing
            if (crc != HP_OK) {
                if (g) (void)hipGraphDestroy(g);
                return crc;
            }
            if (ce != hipSuccess) return fail(HP_EDEVICE, std::string("hipStreamEndCapture: ") +
                                                              hipGetErrorString(ce));
            if (periodic) {
                hipGraphExec_t ex = nullptr;
                const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                if (ie != hipSuccess) {
                    (void)hipGraphDestroy(g);
                    return fail(HP_EDEVICE, std::string("hipGraphInstantiate: ") +
                                                hipGetErrorString(ie));
                }
                if (G.valid) HP_CHECK(hipStreamSynchronize(ctx->stream));  // no replay pending
                drop_graph(G);
                G.valid = true;
                G.slots = sl;
                G.key = key;
                G.len = L;
                G.start = snap;
                G.graph = g;
                G.exec = ex;
                ++ctx->graph_captures;
                have = true;
                continue;  // the next pass finds the state matching and replays
            }
            (void)hipGraphDestroy(g);
        }
        HP_TRY(one());
        ++done;
        ++eager_run;
    }
    return HP_OK;
}

template <typename T>
int iterate_multi(hp_ctx *ctx, const std::vector<int32_t> &sl, const std::vector<Slot *> &ss,
                  const std::vector<Netlist *> &nls, const SlotGammas &g, int32_t flags,
                  int32_t iters) {
    hipStream_t st = ctx->stream;
    const int n = (int)ss.size();
    SlotArgs sa{};
    for (Slot *s : ss) sa.base[sa.n++] = s->base;
    // grids of the passes whose sizes do not change between iterations: the largest slot's;
    // the fused step form when every slot's netlist takes it (no closing reduction launch)
    int big_x = 0, cg_x = 0, rows_x = 0, cols_x = 0, inv_x = 0, step_x = 0;
    size_t l_rows = 0, l_cols = 0, l_inv = 0;
    bool fused = true;
    for (const Netlist *N : nls) {
        fused &= cell_parts(N->nd) <= N->fused_parts;
        const NetDev &nd = N->nd;
        big_x = std::max(big_x, nd.n_big);
        cg_x = std::max(cg_x, round8(std::max(1, cell_parts(nd))));
        rows_x = std::max(rows_x, rows_fwd_blocks(nd));
        cols_x = std::max(cols_x, nd.mx / 2);
        inv_x = std::max(inv_x, nd.my / 2);
        step_x = std::max(step_x, step_blocks(nd));
        l_rows = std::max(l_rows, rows_fwd_lds_of<T>(nd));
        l_cols = std::max(l_cols, cols_lds_of<T>(nd));
        l_inv = std::max(l_inv, rows_inv_lds_of<T>(nd));
    }
    auto one = [&]() -> int {
        uint32_t accm = 0, cntm = 0, hmask = 0, banks = 0;
        int front_x = 0, cs_x = 0, pl_x = 0, ac_x = 0;
        size_t l_front = 0, l_pl = 0, l_ac = 0;
        SlotArgs due{};  // slots whose grouping is rebuilt in this evaluation
        for (int i = 0; i < n; ++i) {
            Slot *s = ss[i];
            const Netlist &N = *nls[i];
            const bool rebuild = s->since_group >= N.regroup_every;
            if (rebuild) {
                cntm |= 1u << i;
                due.base[due.n++] = s->base;
                cs_x = std::max(cs_x, colscan_blocks(N.nd));
                pl_x = std::max(pl_x, N.nd.sort_blocks);
                ac_x = std::max(ac_x, N.nd.max_chunks);
                l_pl = std::max(l_pl, scatter_place_lds(N.nd));
                l_ac = std::max(l_ac, scatter_accum_lds(N.nd));
            } else {
                accm |= 1u << i;
            }
            if (s->hpwl_requested) {  // rides in this evaluation's sweep
                hmask |= 1u << i;
                s->hpwl_requested = false;
                s->hpwl_pending = true;
            }
            banks |= (uint32_t)s->bank << i;
            front_x = std::max(front_x, front_blocks(N.nd, N.bk, !rebuild, rebuild));
            l_front = std::max(l_front, front_lds<T>(N.nd, N.bk, !rebuild, rebuild));
        }
        HP_CHECK(rag_front<T>(sa, g, accm, cntm, hmask, front_x, l_front, st));
        if (due.n) HP_CHECK(rag_regroup_tail<T>(due, cs_x, pl_x, ac_x, l_pl, l_ac, st));
        HP_CHECK(rag_spectral<T>(sa, rows_x, cols_x, inv_x, l_rows, l_cols, l_inv, st));
        HP_CHECK(rag_big_grad<T>(sa, big_x, st));
        HP_CHECK(rag_cell_grad<T>(sa, cg_x, st));
        if (!fused) HP_CHECK(rag_eval_finish(sa, banks, st));
        HP_CHECK(rag_step<T>(sa, step_x, fused, banks, st));
        for (int i = 0; i < n; ++i) {
            Slot *s = ss[i];
            s->since_group = (cntm >> i) & 1u ? 1 : s->since_group + 1;
            // (the fused update stored its proposal; either form leaves the same state)
            s->maps_valid = false;
            s->rho_dirty = false;
            s->step_proposed = false;
            s->step_fused = false;
            s->totals_pending = true;
            s->bank ^= 1;  // the step committed into the other bank
            if (flags & HP_ITER_HPWL) s->hpwl_requested = true;
        }
        return HP_OK;
    };
    int done = 0;
    // graph replay of steady blocks: each slot's state comes back after twice its netlist's
    // rebuild interval, all of them after the least common multiple of those
    if ((flags & HP_ITER_GRAPH) && !hp::g_prof_on) {
        std::vector<double> key = {1.0, (double)flags};
        int L = 2;
        for (int i = 0; i < n; ++i) {
            const Netlist &N = *nls[i];
            key.insert(key.end(), {g.inv[i], (double)N.regroup_every, (double)N.fused_parts,
                                   (double)N.nd.spec_threads, (double)N.nd.sweep_interleave,
                                   (double)N.nd.sweep_nt});
            L = std::lcm(L, 2 * N.regroup_every);
        }
        if (L <= kMaxGraphBlock) HP_TRY(run_graph_blocks(ctx, sl, ss, key, L, iters, done, one));
    }
    for (; done < iters; ++done) HP_TRY(one());
    if (iters > 0 && !(flags & HP_ITER_HPWL) && (flags & HP_ITER_HPWL_LAST))
        for (Slot *s : ss) s->hpwl_requested = true;
    return HP_OK;
}

}  // namespace

extern "C" {

int hp_profile_enable(hp_ctx *ctx, int on, const char *only_kernel) {
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(hp::g_prof_mu);
    hp::g_prof_only = only_kernel ? only_kernel : "";
    hp::g_prof_on.store(on != 0);
    return HP_OK;
}

int hp_profile_read(hp_ctx *ctx, hp_kernel_time *out, int32_t max, int32_t *n_out, int reset) {
    if (!ctx || !n_out) return fail(HP_EINVAL, "ctx/n_out is NULL");
    HP_CHECK(hipStreamSynchronize(ctx->stream));
    HP_CHECK(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(hp::g_prof_mu);
    for (const ProfRec &r : hp::g_prof_pending) {
        float ms = 0.f;
        HP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
        auto it = std::find_if(hp::g_prof_acc.begin(), hp::g_prof_acc.end(),
                               [&](const hp::ProfAcc &a) { return a.name == r.name; });
        if (it == hp::g_prof_acc.end()) {
            hp::g_prof_acc.push_back({r.name, 0, 0.0});
            it = hp::g_prof_acc.end() - 1;
        }
        it->count += 1;
        it->ms += ms;
        hp::g_prof_pool.push_back(r.a);
        hp::g_prof_pool.push_back(r.b);
    }
    hp::g_prof_pending.clear();
    int32_t n = 0;
    for (const hp::ProfAcc &a : hp::g_prof_acc) {
        if (out && n < max) {
            std::memset(&out[n], 0, sizeof(hp_kernel_time));
            std::strncpy(out[n].name, a.name.c_str(), sizeof(out[n].name) - 1);
            out[n].count = a.count;
            out[n].total_ms = a.ms;
        }
        ++n;
    }
    *n_out = n;
    if (reset) hp::g_prof_acc.clear();
    return HP_OK;
}

const char *hp_last_error(void) { return g_err.c_str(); }

int hp_create(hp_ctx **out, int device, void *hip_stream, int precision) {
    if (!out) return fail(HP_EINVAL, "out is NULL");
    if (precision != 32 && precision != 64) return fail(HP_EINVAL, "precision must be 32 or 64");
    int ndev = 0;
    HP_CHECK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(HP_EINVAL, "no such device");
    HP_CHECK(hipSetDevice(device));
    // LDS a block may take: the device limit if the runtime lets the spectral passes opt in
    // to more than the 64 KB default, else 64 KB
    int lds = 65536;
    HP_CHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    if (lds > 65536) {
        const hipError_t e = precision == 32 ? spectral_prepare<float>(lds)
                                             : spectral_prepare<double>(lds);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            lds = 65536;
        }
    }
    int n_cu = 256;
    HP_CHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
    HP_TRY(scratch_setup(device));  // the device is current here
    hp_ctx *c = new hp_ctx;
    c->device = device;
    c->n_cu = n_cu > 0 ? n_cu : 1;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->precision = precision;
    c->lds_budget = lds;
    *out = c;
    return HP_OK;
}

int hp_destroy(hp_ctx *ctx) {
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    drop_graph(ctx->graph);
    delete ctx;
    if (e != hipSuccess) return fail(HP_EDEVICE, hipGetErrorString(e));
    return HP_OK;
}

size_t hp_netlist_bytes(const hp_ctx *ctx, const hp_shape *s, const hp_die *d) {
    if (!ctx || check_shape(s) || check_die(ctx, d)) return 0;
    return net_layout(*s, *d, rsize(ctx)).total;
}

size_t hp_slot_bytes(const hp_ctx *ctx, const hp_shape *s, const hp_die *d) {
    if (!ctx || check_shape(s) || check_die(ctx, d)) return 0;
    return slot_layout(*s, *d, rsize(ctx)).total;
}

int hp_load_netlist_csr(hp_ctx *ctx, const hp_shape *shape, const hp_die *die, const double *cell_w,
                        const double *cell_h, const double *fixed_x, const double *fixed_y,
                        const int32_t *net_start, const int32_t *pin_cell, const double *pin_ox,
                        const double *pin_oy, const double *net_weight, void *dev_buf,
                        size_t dev_bytes, int32_t *out_netlist) {
    if (!ctx || !out_netlist) return fail(HP_EINVAL, "ctx/out is NULL");
    int rc = check_shape(shape);
    if (rc) return rc;
    rc = check_die(ctx, die);
    if (rc) return rc;
    if (!dev_buf || ((uintptr_t)dev_buf & 255)) return fail(HP_EINVAL, "dev_buf must be 256-byte aligned");
    const size_t need = net_layout(*shape, *die, rsize(ctx)).total;
    if (dev_bytes < need)
        return fail(HP_ENOMEM, "netlist buffer needs " + std::to_string(need) + " bytes");
    HP_CHECK(hipSetDevice(ctx->device));
    {  // the preparation and uploads below use the stream without the lock
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        ++ctx->stream_users;
    }
    struct Leave {
        hp_ctx *c;
        ~Leave() { --c->stream_users; }
    } leave{ctx};
    Netlist NL;
    rc = ctx->precision == 32
             ? load_netlist<float>(ctx, *shape, *die, cell_w, cell_h, fixed_x, fixed_y, net_start,
                                   pin_cell, pin_ox, pin_oy, net_weight, (char *)dev_buf, NL)
             : load_netlist<double>(ctx, *shape, *die, cell_w, cell_h, fixed_x, fixed_y, net_start,
                                    pin_cell, pin_ox, pin_oy, net_weight, (char *)dev_buf, NL);
    if (rc) return rc;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->nets.push_back(NL);
    *out_netlist = (int32_t)ctx->nets.size() - 1;
    return HP_OK;
}

int hp_slot_alloc(hp_ctx *ctx, int32_t netlist, void *dev_buf, size_t dev_bytes, int32_t *out_slot) {
    HP_GUARD(ctx);
    if (!ctx || !out_slot) return fail(HP_EINVAL, "ctx/out is NULL");
    if (netlist < 0 || netlist >= (int)ctx->nets.size() || !ctx->nets[netlist].alive)
        return fail(HP_ESTATE, "unknown netlist");
    Netlist &NL = ctx->nets[netlist];
    if (!dev_buf || ((uintptr_t)dev_buf & 255)) return fail(HP_EINVAL, "dev_buf must be 256-byte aligned");
    if (dev_bytes < NL.L.total)
        return fail(HP_ENOMEM, "slot buffer needs " + std::to_string(NL.L.total) + " bytes");
    char *base = (char *)dev_buf;
    hipStream_t st = ctx->stream;
    const size_t rs = rsize(ctx);
    const size_t Nm = NL.nd.n_mov, Nf = NL.nd.n_fixed;
    HP_CHECK(hipMemsetAsync(base, 0, NL.L.total, st));
    for (size_t off : {NL.L.u, NL.L.v})  // fixed cells' (x, y) pairs after the movable ones
        if (Nf)
            HP_CHECK(hipMemcpyAsync(base + off + 2 * Nm * rs, NL.nd.fixed_pos, 2 * Nf * rs,
                                    hipMemcpyDeviceToDevice, st));
    Scalars s;
    init_scalars(s, 1e-4, 4.0, 1000);
    HP_CHECK(hipMemcpyAsync(base + NL.L.scal, &s, sizeof(s), hipMemcpyHostToDevice, st));
    const SlotDesc d{NL.nd, NL.bk, NL.L};  // the descriptor at the head of the slot buffer
    HP_CHECK(hipMemcpyAsync(base, &d, sizeof(d), hipMemcpyHostToDevice, st));
    HP_SYNC_UNLOCKED(ctx);  // s and d are read by then
    if (!NL.alive) return fail(HP_ESTATE, "netlist released while a slot was being allocated");
    if (NL.nd.spec_threads != d.nd.spec_threads || NL.nd.sweep_interleave != d.nd.sweep_interleave)
        HP_TRY(write_descs(ctx, NL, {base}));  // a launch setting changed meanwhile
    Slot sl;
    sl.alive = true;
    sl.netlist = netlist;
    sl.base = base;
    ctx->slots.push_back(sl);
    *out_slot = (int32_t)ctx->slots.size() - 1;
    return HP_OK;
}

int hp_slot_free(hp_ctx *ctx, int32_t slot) {
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    std::unique_lock<std::recursive_mutex> lk(ctx->mu);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    const auto &gs = ctx->graph.slots;
    if (std::find(gs.begin(), gs.end(), slot) != gs.end()) {
        HP_CHECK(hipStreamSynchronize(ctx->stream));  // no replay of its graph pending
        drop_graph(ctx->graph);
    }
    s->alive = false;  // no further work for it can be queued ...
    s->base = nullptr;
    ++ctx->stream_users;
    lk.unlock();
    // ... and once the work queued so far has finished, its buffer may be released (the wait
    // holds no lock, so other threads keep queueing work meanwhile)
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    --ctx->stream_users;
    if (e != hipSuccess) return fail(HP_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    return HP_OK;
}

int hp_set_positions(hp_ctx *ctx, int32_t slot, const void *x, const void *y, int on_device) {
    HP_GUARD(ctx);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    if (!x || !y) return fail(HP_EINVAL, "x/y is NULL");
    HP_TRY(launch_requested_hpwl(ctx, n, std::vector<Slot *>{s}));  // before u changes
    const size_t rs = rsize(ctx), Nm = n->nd.n_mov;
    hipStream_t st = ctx->stream;
    const SlotLayout &L = n->L;
    std::vector<char> staged;  // host pairs; lives until the synchronisation below
    if (Nm) {
        // interleave into u's (x, y) pairs (on the host, or by a kernel for device inputs: one
        // contiguous transfer either way), then copy u to v and v_prev
        if (on_device) {
            HP_CHECK(launch_join_pairs(x, y, s->base + L.u, (int)Nm, rs, st));
        } else {
            staged.resize(2 * Nm * rs);
            for (size_t i = 0; i < Nm; ++i) {
                std::memcpy(&staged[(2 * i) * rs], (const char *)x + i * rs, rs);
                std::memcpy(&staged[(2 * i + 1) * rs], (const char *)y + i * rs, rs);
            }
            HP_CHECK(hipMemcpyAsync(s->base + L.u, staged.data(), staged.size(),
                                    hipMemcpyHostToDevice, st));
        }
        HP_CHECK(hipMemcpyAsync(s->base + L.v, s->base + L.u, 2 * Nm * rs, hipMemcpyDeviceToDevice, st));
        HP_CHECK(hipMemcpyAsync(s->base + L.vprev, s->base + L.u, 2 * Nm * rs, hipMemcpyDeviceToDevice,
                                st));
    }
    Scalars h;
    HP_CHECK(hipMemcpyAsync(&h, s->base + L.scal, sizeof(h), hipMemcpyDeviceToHost, st));
    HP_SYNC_UNLOCKED(ctx);
    for (int b = 0; b < 2; ++b) {  // the optimiser restarts (both banks)
        h.kb[b] = 0;
        h.ab[b] = 1.0;
        h.alphab[b] = 0.0;
    }
    h.lambda_valid = 0;
    h.hpwl_valid = 0;
    HP_CHECK(hipMemcpyAsync(s->base + L.scal, &h, sizeof(h), hipMemcpyHostToDevice, st));
    HP_SYNC_UNLOCKED(ctx);
    s->lambda_valid = false;
    s->hpwl_pending = false;
    s->step_proposed = false;
    s->step_fused = false;
    s->since_group = -1;
    return HP_OK;
}

namespace {
int get_pos(hp_ctx *ctx, int32_t slot, size_t which, void *x, void *y, int on_device) {
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    const size_t rs = rsize(ctx), Nm = n->nd.n_mov;
    const char *src = s->base + which;  // (x, y) pairs
    if (!Nm || (!x && !y)) return HP_OK;
    if (on_device) return launch_split_pairs(src, x, y, (int)Nm, rs, ctx->stream) == hipSuccess
                              ? HP_OK
                              : fail(HP_EDEVICE, "split_pairs launch failed");
    // one contiguous copy, split on the host
    std::vector<char> h(2 * Nm * rs);
    HP_CHECK(hipMemcpyAsync(h.data(), src, h.size(), hipMemcpyDeviceToHost, ctx->stream));
    HP_CHECK(hipStreamSynchronize(ctx->stream));
    for (size_t i = 0; i < Nm; ++i) {
        if (x) std::memcpy((char *)x + i * rs, &h[(2 * i) * rs], rs);
        if (y) std::memcpy((char *)y + i * rs, &h[(2 * i + 1) * rs], rs);
    }
    return HP_OK;
}
}  // namespace

int hp_get_positions(hp_ctx *ctx, int32_t slot, void *x, void *y, int on_device) {
    HP_GUARD(ctx);
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (slot < 0 || slot >= (int)ctx->slots.size() || !ctx->slots[slot].alive)
        return fail(HP_ESTATE, "unknown slot " + std::to_string(slot));
    return get_pos(ctx, slot, ctx->nets[ctx->slots[slot].netlist].L.u, x, y, on_device);
}

int hp_get_eval_positions(hp_ctx *ctx, int32_t slot, void *x, void *y, int on_device) {
    HP_GUARD(ctx);
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (slot < 0 || slot >= (int)ctx->slots.size() || !ctx->slots[slot].alive)
        return fail(HP_ESTATE, "unknown slot " + std::to_string(slot));
    return get_pos(ctx, slot, ctx->nets[ctx->slots[slot].netlist].L.v, x, y, on_device);
}

int hp_set_schedule(hp_ctx *ctx, int32_t slot, double lambda0_scale, double decades, int32_t total_iters) {
    HP_GUARD(ctx);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    if (!(lambda0_scale > 0) || !std::isfinite(decades) || total_iters <= 0)
        return fail(HP_EINVAL, "bad schedule");
    Scalars h;
    HP_CHECK(hipMemcpyAsync(&h, s->base + n->L.scal, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HP_SYNC_UNLOCKED(ctx);
    h.lambda0_scale = lambda0_scale;
    h.lambda_ratio = std::pow(10.0, decades / total_iters);
    HP_CHECK(hipMemcpyAsync(s->base + n->L.scal, &h, sizeof(h), hipMemcpyHostToDevice, ctx->stream));
    HP_SYNC_UNLOCKED(ctx);
    return HP_OK;
}

int hp_set_scatter_policy(hp_ctx *ctx, int32_t netlist, int32_t regroup_every, int32_t deferred) {
    HP_GUARD(ctx);
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (netlist < 0 || netlist >= (int)ctx->nets.size() || !ctx->nets[netlist].alive)
        return fail(HP_ESTATE, "unknown netlist");
    if (regroup_every < 1 || regroup_every > 64)
        return fail(HP_EINVAL, "regroup_every must be in [1, 64]");
    if (deferred != 0 && deferred != 1) return fail(HP_EINVAL, "deferred must be 0 or 1");
    ctx->nets[netlist].regroup_every = regroup_every;
    ctx->nets[netlist].deferred = deferred != 0;
    return HP_OK;
}

int hp_set_tunable(hp_ctx *ctx, int32_t netlist, int32_t which, int32_t value) {
    HP_GUARD(ctx);
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (netlist < 0 || netlist >= (int)ctx->nets.size() || !ctx->nets[netlist].alive)
        return fail(HP_ESTATE, "unknown netlist");
    Netlist &NL = ctx->nets[netlist];
    switch (which) {
        case HP_TUNE_FUSED_STEP_PARTS:
            if (value < 0 || value > kFusedStepParts)
                return fail(HP_EINVAL, "fused step partials must be in [0, " +
                                           std::to_string(kFusedStepParts) + "]");
            NL.fused_parts = value;
            return HP_OK;
        case HP_TUNE_SPECTRAL_THREADS:
            if (value != 0 && value != 512 && value != 1024)
                return fail(HP_EINVAL, "spectral threads must be 0, 512 or 1024");
            NL.nd.spec_threads = value;
            return rewrite_descs(ctx, netlist);
        case HP_TUNE_SWEEP_INTERLEAVE:
            if (value != 0 && value != 1) return fail(HP_EINVAL, "sweep interleave must be 0 or 1");
            NL.nd.sweep_interleave = value;
            return rewrite_descs(ctx, netlist);
        case HP_TUNE_CHARGE_RECORDS:
            if (value != 0 && value != 1) return fail(HP_EINVAL, "charge records must be 0 or 1");
            NL.charge_records = value != 0;
            return HP_OK;
        case HP_TUNE_NONTEMPORAL:
            if (value != 0 && value != 1) return fail(HP_EINVAL, "non-temporal must be 0 or 1");
            NL.nd.sweep_nt = value;  // chosen by the host at launch; descriptors do not carry it
            return HP_OK;
        default:
            return fail(HP_EINVAL, "unknown tunable");
    }
}

int hp_get_tunable(hp_ctx *ctx, int32_t netlist, int32_t which, int32_t *value) {
    HP_GUARD(ctx);
    if (!ctx || !value) return fail(HP_EINVAL, "ctx/out is NULL");
    if (netlist < 0 || netlist >= (int)ctx->nets.size() || !ctx->nets[netlist].alive)
        return fail(HP_ESTATE, "unknown netlist");
    const Netlist &NL = ctx->nets[netlist];
    switch (which) {
        case HP_TUNE_FUSED_STEP_PARTS: *value = NL.fused_parts; return HP_OK;
        case HP_TUNE_SPECTRAL_THREADS: *value = NL.nd.spec_threads; return HP_OK;
        case HP_TUNE_SWEEP_INTERLEAVE: *value = NL.nd.sweep_interleave; return HP_OK;
        case HP_TUNE_CHARGE_RECORDS: *value = NL.charge_records ? 1 : 0; return HP_OK;
        case HP_TUNE_NONTEMPORAL: *value = NL.nd.sweep_nt; return HP_OK;
        default: return fail(HP_EINVAL, "unknown tunable");
    }
}

int hp_get_scatter_policy(hp_ctx *ctx, int32_t netlist, int32_t *regroup_every, int32_t *deferred) {
    HP_GUARD(ctx);
    if (!ctx || !regroup_every || !deferred) return fail(HP_EINVAL, "ctx/out is NULL");
    if (netlist < 0 || netlist >= (int)ctx->nets.size() || !ctx->nets[netlist].alive)
        return fail(HP_ESTATE, "unknown netlist");
    *regroup_every = ctx->nets[netlist].regroup_every;
    *deferred = ctx->nets[netlist].deferred ? 1 : 0;
    return HP_OK;
}

int hp_set_lambda_ratio(hp_ctx *ctx, int32_t slot, double ratio) {
    HP_GUARD(ctx);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    if (!(ratio > 0) || !std::isfinite(ratio)) return fail(HP_EINVAL, "ratio must be finite and > 0");
    HP_CHECK(hipMemcpyAsync(s->base + n->L.scal + offsetof(Scalars, lambda_ratio), &ratio,
                            sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HP_CHECK(hipStreamSynchronize(ctx->stream));
    return HP_OK;
}

int hp_overflow_of_cells(hp_ctx *ctx, int32_t slot, int32_t n_counted, int64_t *out_num,
                         double *out) {
    HP_GUARD(ctx);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    if (n_counted < 0 || n_counted > n->nd.n_mov) return fail(HP_EINVAL, "n_counted out of range");
    hipStream_t st = ctx->stream;
    if (s->rho_dirty) {  // a kept map: clear it first (the pass needs zeros)
        SlotArgs sa{};
        sa.base[0] = s->base;
        sa.n = 1;
        HP_CHECK(launch_clear_rho(n->nd, sa, n->L, st));
        s->rho_dirty = false;
        s->maps_valid = false;
    }
    if (ctx->precision == 32)
        HP_CHECK(launch_overflow_of_cells<float>(n->nd, s->base, n->L, n_counted, st));
    else
        HP_CHECK(launch_overflow_of_cells<double>(n->nd, s->base, n->L, n_counted, st));
    int64_t num = 0;
    HP_CHECK(hipMemcpyAsync(&num, s->base + n->L.scal + offsetof(Scalars, ovf_tmp), sizeof(num),
                            hipMemcpyDeviceToHost, st));
    HP_CHECK(hipStreamSynchronize(st));
    const int64_t den = n->charge_prefix[(size_t)n_counted];
    if (out_num) *out_num = num;
    if (out) *out = den > 0 ? (double)num / (double)den : 0.0;
    return HP_OK;
}

int hp_set_backtracking(hp_ctx *ctx, int32_t slot, int32_t on) {
    HP_GUARD(ctx);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    if (on != 0 && on != 1) return fail(HP_EINVAL, "on must be 0 or 1");
    const int64_t vals[2] = {on, 0};  // backtrack, rejects (adjacent fields)
    static_assert(offsetof(Scalars, rejects) == offsetof(Scalars, backtrack) + 8, "layout");
    HP_CHECK(hipMemcpyAsync(s->base + n->L.scal + offsetof(Scalars, backtrack), vals, sizeof(vals),
                            hipMemcpyHostToDevice, ctx->stream));
    HP_CHECK(hipStreamSynchronize(ctx->stream));
    return HP_OK;
}

int hp_eval_objective_grad(hp_ctx *ctx, const int32_t *slots, int32_t n, const hp_eval_params *p,
                           double *wl, double *energy, double *overflow, void *gx, void *gy) {
    HP_GUARD(ctx);
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    return ctx->precision == 32 ? eval_impl<float>(ctx, slots, n, p, wl, energy, overflow, gx, gy)
                                : eval_impl<double>(ctx, slots, n, p, wl, energy, overflow, gx, gy);
}

int hp_nesterov_step(hp_ctx *ctx, const int32_t *slots, int32_t n) {
    HP_GUARD(ctx);
    Netlist *NL;
    std::vector<SlotArgs> chunks;
    std::vector<Slot *> ss;
    int rc = resolve(ctx, slots, n, &NL, chunks, ss);
    if (rc) return rc;
    return step_resolved(ctx, NL, chunks, ss);
}

int hp_hpwl_noalloc(hp_ctx *ctx, int32_t netlist, const void *xy, int64_t *out_q) {
    HP_GUARD(ctx);
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (!xy || !out_q) return fail(HP_EINVAL, "xy and out_q must be device pointers");
    if (((uintptr_t)xy & (2 * rsize(ctx) - 1)) || ((uintptr_t)out_q & 7))
        return fail(HP_EINVAL, "xy must be aligned to a position pair, out_q to 8 bytes");
    if (netlist < 0 || netlist >= (int)ctx->nets.size() || !ctx->nets[netlist].alive)
        return fail(HP_ESTATE, "unknown netlist");
    const Netlist &NL = ctx->nets[netlist];
    if (NL.bk.total_blocks > kNoAllocParts)
        return fail(HP_ENOMEM, "the netlist's sweep has " + std::to_string(NL.bk.total_blocks) +
                                   " blocks; the static scratch holds " +
                                   std::to_string(kNoAllocParts) + " partials");
    long long *part = static_cast<long long *>(scratch_of(ctx->device));
    if (!part) return fail(HP_EDEVICE, "no static scratch address for this device");
    if (ctx->precision == 32)
        HP_CHECK(launch_hpwl_positions<float>(NL.nd, NL.bk, xy, part,
                                              reinterpret_cast<long long *>(out_q), ctx->stream));
    else
        HP_CHECK(launch_hpwl_positions<double>(NL.nd, NL.bk, xy, part,
                                               reinterpret_cast<long long *>(out_q), ctx->stream));
    return HP_OK;
}

int hp_hpwl(hp_ctx *ctx, const int32_t *slots, int32_t n, int64_t *out_q, double *out) {
    HP_GUARD(ctx);
    Netlist *NL;
    std::vector<SlotArgs> chunks;
    std::vector<Slot *> ss;
    int rc = resolve(ctx, slots, n, &NL, chunks, ss);
    if (rc) return rc;
    HP_TRY(hpwl_resolved(ctx, NL, chunks, ss));
    if (out_q || out) {
        rc = finish_hpwl(ctx, NL, ss);
        if (rc) return rc;
        std::vector<int64_t> h(n);
        for (int i = 0; i < n; ++i)
            HP_CHECK(hipMemcpyAsync(&h[i], ss[i]->base + NL->L.scal + offsetof(Scalars, hpwl_q), 8,
                                    hipMemcpyDeviceToHost, ctx->stream));
        HP_CHECK(hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < n; ++i) {
            if (out_q) out_q[i] = h[i];
            if (out) out[i] = std::ldexp((double)h[i], -16);
        }
    }
    return HP_OK;
}


int hp_iterate(hp_ctx *ctx, const int32_t *slots, int32_t n, const hp_iter_params *p,
               int32_t iters) {
    HP_GUARD(ctx);
    Netlist *NL;
    std::vector<SlotArgs> chunks;
    std::vector<Slot *> ss;
    int rc = resolve(ctx, slots, n, &NL, chunks, ss);
    if (rc) return rc;
    if (!p) return fail(HP_EINVAL, "params is NULL");
    if (iters < 0) return fail(HP_EINVAL, "iters must be >= 0");
    if (p->flags & ~(HP_ITER_HPWL | HP_ITER_GRAPH | HP_ITER_HPWL_LAST))
        return fail(HP_EINVAL, "unknown flags");
    const bool graph = (p->flags & HP_ITER_GRAPH) != 0;
    if (graph && ctx->stream == nullptr)
        return fail(HP_EINVAL, "HP_ITER_GRAPH needs a context stream other than the null stream "
                               "(the legacy default stream cannot be captured)");
    const hp_eval_params ep{p->gamma, -1.0, 0, 0};
    HP_TRY(check_eval_params(&ep));
    const bool with_hpwl = (p->flags & HP_ITER_HPWL) != 0;
    auto iteration = [&]() -> int {
        HP_TRY(ctx->precision == 32 ? eval_resolved<float>(ctx, NL, chunks, ss, &ep)
                                    : eval_resolved<double>(ctx, NL, chunks, ss, &ep));
        HP_TRY(step_resolved(ctx, NL, chunks, ss));
        if (with_hpwl) HP_TRY(hpwl_resolved(ctx, NL, chunks, ss));
        return HP_OK;
    };
    int done = 0;
    // graph replay of steady blocks of twice the scatter's rebuild interval (the optimiser-state
    // banks and the rebuild phase then come back to where they were)
    if (graph && !hp::g_prof_on) {
        const std::vector<double> key = {0.0, p->gamma, (double)p->flags, (double)NL->regroup_every,
                                         (double)NL->deferred, (double)NL->fused_parts,
                                         (double)NL->nd.spec_threads,
                                         (double)NL->nd.sweep_interleave,
                                         (double)NL->charge_records,
                                         (double)NL->nd.sweep_nt};
        HP_TRY(run_graph_blocks(ctx, std::vector<int32_t>(slots, slots + n), ss, key,
                                2 * NL->regroup_every, iters, done, iteration));
    }
    for (; done < iters; ++done) HP_TRY(iteration());
    if (iters > 0 && !with_hpwl && (p->flags & HP_ITER_HPWL_LAST))
        HP_TRY(hpwl_resolved(ctx, NL, chunks, ss));
    return HP_OK;
}

int hp_graph_stats(hp_ctx *ctx, int64_t *captures, int64_t *replays) {
    HP_GUARD(ctx);
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (captures) *captures = ctx->graph_captures;
    if (replays) *replays = ctx->graph_replays;
    return HP_OK;
}

int hp_iterate_multi(hp_ctx *ctx, const int32_t *slots, int32_t n, const double *gammas,
                     int32_t flags, int32_t iters) {
    HP_GUARD(ctx);
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    if (!slots || n <= 0) return fail(HP_EINVAL, "empty slot list");
    if (n > kMaxSlots) return fail(HP_EINVAL, "at most " + std::to_string(kMaxSlots) + " slots per call");
    if (!gammas) return fail(HP_EINVAL, "gammas is NULL");
    if (iters < 0) return fail(HP_EINVAL, "iters must be >= 0");
    if (flags & ~(HP_ITER_HPWL | HP_ITER_HPWL_LAST | HP_ITER_GRAPH)) return fail(HP_EINVAL, "unknown flags");
    if ((flags & HP_ITER_GRAPH) && ctx->stream == nullptr)
        return fail(HP_EINVAL, "HP_ITER_GRAPH needs a context stream other than the null stream "
                               "(the legacy default stream cannot be captured)");
    std::vector<Slot *> ss;
    std::vector<Netlist *> nls;
    SlotGammas g{};
    for (int i = 0; i < n; ++i) {
        Slot *s;
        Netlist *nl;
        HP_TRY(get_slot(ctx, slots[i], &s, &nl));
        for (const Slot *o : ss)
            if (o == s) return fail(HP_EINVAL, "slot " + std::to_string(slots[i]) + " listed twice");
        if (!(gammas[i] > 0) || !std::isfinite(gammas[i]))
            return fail(HP_EINVAL, "gamma must be > 0 (slot " + std::to_string(slots[i]) + ")");
        // steady state: lambda derived (a first evaluation ran), a scatter grouping, no kept map
        if (!s->lambda_valid || s->since_group < 0 || s->rho_dirty)
            return fail(HP_ESTATE, "slot " + std::to_string(slots[i]) +
                                       " is not in steady state (run one hp_iterate on it first)");
        ss.push_back(s);
        nls.push_back(nl);
        g.inv[i] = 1.0 / gammas[i];
    }
    const std::vector<int32_t> sl(slots, slots + n);
    return ctx->precision == 32 ? iterate_multi<float>(ctx, sl, ss, nls, g, flags, iters)
                                : iterate_multi<double>(ctx, sl, ss, nls, g, flags, iters);
}

int hp_netlist_free(hp_ctx *ctx, int32_t netlist) {
    if (!ctx) return fail(HP_EINVAL, "ctx is NULL");
    std::unique_lock<std::recursive_mutex> lk(ctx->mu);
    if (netlist < 0 || netlist >= (int)ctx->nets.size() || !ctx->nets[netlist].alive)
        return fail(HP_ESTATE, "unknown netlist");
    for (const Slot &s : ctx->slots)
        if (s.alive && s.netlist == netlist)
            return fail(HP_ESTATE, "netlist " + std::to_string(netlist) + " still has live slots");
    ctx->nets[netlist] = Netlist{};  // alive = false; host arrays released
    ++ctx->stream_users;
    lk.unlock();
    const hipError_t e = hipStreamSynchronize(ctx->stream);  // as hp_slot_free
    --ctx->stream_users;
    if (e != hipSuccess) return fail(HP_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    return HP_OK;
}

// Shared by hp_perturb (pool == NULL: every movable cell) and hp_perturb_among.
static int perturb_impl(hp_ctx *ctx, int32_t slot, int mode, double fraction, double sigma_bins,
                        uint64_t seed, const int32_t *pool, int32_t n_pool, int32_t *out_idx,
                        int32_t *out_count) {
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    if (mode < 0 || mode > 2) return fail(HP_EINVAL, "unknown perturbation mode");
    if (mode != 2 && !(fraction >= 0 && fraction <= 1)) return fail(HP_EINVAL, "fraction must be in [0, 1]");
    if (mode == 0 && !(sigma_bins >= 0 && std::isfinite(sigma_bins)))
        return fail(HP_EINVAL, "sigma must be finite and >= 0");
    const int Nm = n->nd.n_mov;
    if (pool) {
        if (mode == 2) return fail(HP_EINVAL, "a uniform restart redraws every cell: no pool");
        if (n_pool < 0 || n_pool > Nm) return fail(HP_EINVAL, "pool size out of range");
        std::vector<char> seen(Nm, 0);
        for (int32_t j = 0; j < n_pool; ++j) {
            const int32_t c = pool[j];
            if (c < 0 || c >= Nm) return fail(HP_EINVAL, "pool cell is not a movable cell");
            if (seen[c]) return fail(HP_EINVAL, "pool cells must be distinct");
            seen[c] = 1;
        }
    }
    const int64_t P = pool ? n_pool : Nm;
    int64_t m = mode == 2 ? Nm : (int64_t)std::floor(fraction * P + 0.5);
    if (m > P) m = P;
    HP_TRY(launch_requested_hpwl(ctx, n, std::vector<Slot *>{s}));  // before u changes
    if (pool && n_pool)
        HP_CHECK(hipMemcpyAsync(s->base + n->L.work, pool, 4 * (size_t)n_pool,
                                hipMemcpyHostToDevice, ctx->stream));
    const int np = pool ? n_pool : -1;
    if (ctx->precision == 32)
        HP_CHECK(launch_perturb<float>(n->nd, s->base, n->L, mode, m, sigma_bins * n->nd.wb,
                                       sigma_bins * n->nd.hb, seed, np, ctx->stream));
    else
        HP_CHECK(launch_perturb<double>(n->nd, s->base, n->L, mode, m, sigma_bins * n->nd.wb,
                                        sigma_bins * n->nd.hb, seed, np, ctx->stream));
    s->lambda_valid = false;
    s->step_proposed = false;
    s->step_fused = false;
    s->since_group = -1;
    s->hpwl_pending = false;  // the device cleared hpwl_valid
    if (out_idx && m)
        HP_CHECK(hipMemcpyAsync(out_idx, s->base + n->L.sel, 4 * (size_t)m, hipMemcpyDeviceToHost,
                                ctx->stream));
    if (out_count) *out_count = (int32_t)m;
    // (a pool was read from caller memory that is only guaranteed until return)
    if (out_idx || out_count || (pool && n_pool)) HP_CHECK(hipStreamSynchronize(ctx->stream));
    return HP_OK;
}

int hp_perturb_wiremask(hp_ctx *ctx, int32_t slot, const int32_t *macros, int32_t n_macros,
                        int32_t *out_moved) {
    HP_GUARD(ctx);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    const int Nm = n->nd.n_mov;
    if (n_macros < 0 || n_macros > Nm) return fail(HP_EINVAL, "macro count out of range");
    if (n_macros > 0 && !macros) return fail(HP_EINVAL, "macros is NULL");
    std::vector<char> seen(Nm, 0);
    for (int32_t j = 0; j < n_macros; ++j) {
        const int32_t c = macros[j];
        if (c < 0 || c >= Nm) return fail(HP_EINVAL, "a listed macro is not a movable cell");
        if (seen[c]) return fail(HP_EINVAL, "listed macros must be distinct");
        seen[c] = 1;
    }
    HP_TRY(launch_requested_hpwl(ctx, n, std::vector<Slot *>{s}));  // before u changes
    hipStream_t st = ctx->stream;
    if (n_macros)
        HP_CHECK(hipMemcpyAsync(s->base + n->L.work + wiremask_pool_offset(n->nd), macros,
                                4 * (size_t)n_macros, hipMemcpyHostToDevice, st));
    if (ctx->precision == 32)
        HP_CHECK(launch_wiremask<float>(n->nd, s->base, n->L, macros, n_macros, st));
    else
        HP_CHECK(launch_wiremask<double>(n->nd, s->base, n->L, macros, n_macros, st));
    s->lambda_valid = false;
    s->step_proposed = false;
    s->step_fused = false;
    s->since_group = -1;
    s->hpwl_pending = false;  // the device cleared hpwl_valid
    int64_t moved = 0;
    HP_CHECK(hipMemcpyAsync(&moved, s->base + n->L.scal + offsetof(Scalars, sel_count), sizeof(moved),
                            hipMemcpyDeviceToHost, st));
    HP_CHECK(hipStreamSynchronize(st));
    if (out_moved) *out_moved = (int32_t)moved;
    return HP_OK;
}

int hp_perturb(hp_ctx *ctx, int32_t slot, int mode, double fraction, double sigma_bins, uint64_t seed,
               int32_t *out_idx, int32_t *out_count) {
    HP_GUARD(ctx);
    return perturb_impl(ctx, slot, mode, fraction, sigma_bins, seed, nullptr, 0, out_idx, out_count);
}

int hp_perturb_among(hp_ctx *ctx, int32_t slot, int mode, double fraction, double sigma_bins,
                     uint64_t seed, const int32_t *cells, int32_t n_pool, int32_t *out_idx,
                     int32_t *out_count) {
    HP_GUARD(ctx);
    if (!cells && n_pool) return fail(HP_EINVAL, "cells is NULL");
    static const int32_t none = 0;
    return perturb_impl(ctx, slot, mode, fraction, sigma_bins, seed, cells ? cells : &none, n_pool,
                        out_idx, out_count);
}

int hp_select_best(hp_ctx *ctx, const int32_t *slots, int32_t n, int32_t incumbent, int32_t *out_best) {
    HP_GUARD(ctx);
    Netlist *NL;
    std::vector<SlotArgs> chunks;
    std::vector<Slot *> ss;
    int rc = resolve(ctx, slots, n, &NL, chunks, ss);
    if (rc) return rc;
    if (n > kMaxSlots) return fail(HP_EINVAL, "at most 32 candidates per selection");
    Slot *inc;
    Netlist *ni;
    rc = get_slot(ctx, incumbent, &inc, &ni);
    if (rc) return rc;
    if (ni != NL) return fail(HP_ESTATE, "incumbent is on another netlist");
    for (Slot *s : ss)
        if (s == inc) return fail(HP_EINVAL, "the incumbent cannot be a candidate");
    std::vector<Slot *> all(ss);
    all.push_back(inc);
    rc = finish_hpwl(ctx, NL, all);
    if (rc) return rc;
    if (ctx->precision == 32)
        HP_CHECK(launch_select_best<float>(NL->nd, chunks[0], inc->base, NL->L, ctx->stream));
    else
        HP_CHECK(launch_select_best<double>(NL->nd, chunks[0], inc->base, NL->L, ctx->stream));
    inc->lambda_valid = false;  // conservatively: the device resets it when a candidate wins
    inc->step_proposed = false;
    inc->step_fused = false;
    inc->since_group = -1;
    if (out_best) {
        int64_t b = -1;
        HP_CHECK(hipMemcpyAsync(&b, inc->base + NL->L.scal + offsetof(Scalars, best), 8,
                                hipMemcpyDeviceToHost, ctx->stream));
        HP_CHECK(hipStreamSynchronize(ctx->stream));
        *out_best = (int32_t)b;
    }
    return HP_OK;
}

int hp_get_map(hp_ctx *ctx, int32_t slot, int which, void *dst) {
    HP_GUARD(ctx);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    if (!dst) return fail(HP_EINVAL, "dst is NULL");
    const size_t nb = (size_t)n->nd.mx * n->nd.my, rs = rsize(ctx);
    const char *src = nullptr;
    size_t bytes = 0;
    if (which == HP_MAP_RHO_FIXED) {
        src = (const char *)n->nd.rho_fixed;
        bytes = 8 * nb;
    } else {
        if (!s->maps_valid) return fail(HP_ESTATE, "no maps kept: evaluate with keep_maps = 1");
        switch (which) {
            case HP_MAP_RHO_MOV: src = s->base + n->L.rho; bytes = 8 * nb; break;
            case HP_MAP_PSI: src = s->base + n->L.psi; bytes = rs * nb; break;
            case HP_MAP_EX:
            case HP_MAP_EY: {  // one component of the interleaved (xi_x, xi_y) map
                std::vector<char> h(2 * nb * rs);  // one contiguous copy, split on the host
                HP_CHECK(hipMemcpyAsync(h.data(), s->base + n->L.exy, h.size(), hipMemcpyDeviceToHost,
                                        ctx->stream));
                HP_CHECK(hipStreamSynchronize(ctx->stream));
                const size_t c = which == HP_MAP_EY ? 1 : 0;
                for (size_t b = 0; b < nb; ++b)
                    std::memcpy((char *)dst + b * rs, &h[(2 * b + c) * rs], rs);
                return HP_OK;
            }
            default: return fail(HP_EINVAL, "unknown map");
        }
    }
    HP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HP_CHECK(hipStreamSynchronize(ctx->stream));
    return HP_OK;
}

int hp_get_state(hp_ctx *ctx, int32_t slot, hp_slot_state *out) {
    HP_GUARD(ctx);
    Slot *s;
    Netlist *n;
    int rc = get_slot(ctx, slot, &s, &n);
    if (rc) return rc;
    if (!out) return fail(HP_EINVAL, "out is NULL");
    rc = finish_hpwl(ctx, n, std::vector<Slot *>{s});
    if (rc) return rc;
    HP_TRY(finish_totals(ctx, n, std::vector<Slot *>{s}));
    Scalars h;
    HP_CHECK(hipMemcpyAsync(&h, s->base + n->L.scal, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HP_CHECK(hipStreamSynchronize(ctx->stream));
    out->k = h.kb[s->bank];
    out->hpwl_q = h.hpwl_valid ? h.hpwl_q : -1;
    out->overflow_num = h.overflow_num;
    out->a = h.ab[s->bank];
    out->alpha = h.alphab[s->bank];
    out->lambda = h.lambda;
    out->wl = h.wl;
    out->energy = h.energy;
    out->overflow = h.overflow;
    out->rejects = h.rejects;
    return HP_OK;
}

}  // extern "C"
