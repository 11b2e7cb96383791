// Internal structures shared by the host code and the kernels of libhybro (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace hp {

constexpr int kBlock = 256;      // threads per block of the sweep, scatter, gradient and
                                 // perturbation kernels (the spectral passes, the Nesterov
                                 // update and the closing reductions choose their own)
constexpr int kMaxSlots = 32;    // slots per launch (longer lists are chunked)
constexpr int kMaxBuckets = 12;
constexpr int kXcds = 8;         // MI355X: 8 XCDs, blocks are dealt round-robin
// cells per accumulation block of the binned scatter (at most): a full chunk is 3 cells a
// thread.  On 2.2 M cells, 1-2 k-cell chunks of the dense tiles made the accumulation's last
// blocks run alone for ~15 us; 768 to 1536 all cut the iteration by 1.4%, and 768 is the best
// of them on 210 k cells (512 costs the placement pass more than it saves)
constexpr int kChunk = 768;
// counting blocks of a grouping at most (rows of the column scan, which covers this many)
constexpr int kMaxSortBlocks = 512;
constexpr int kRegroupEvery = 4; // evaluations between rebuilds of the scatter's tile order
constexpr int kPairNets = 2;     // two-pin nets each lane sweeps (their loads issued together)
constexpr int kBigHalo = 8;      // movable cells whose charge can span more than kBigHalo + 1
constexpr int kBigArea = 8;      // bins on an axis, or covers kBigArea bin areas or more, are
                                 // "big" (the macros): scattered and gathered one block per
                                 // cell, outside the tile grouping

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };
template <typename T> using vec2 = typename V2<T>::type;

// Degree buckets of the net sweep: two-pin nets take a lane each (kPairNets per lane); nets
// with 3..256 pins own G = next power of two >= degree slots (at least 4) and span G / 4 lanes,
// four slots per lane; larger nets take a whole block.
struct Buckets {
    int32_t n;
    int32_t G[kMaxBuckets];      // pin slots per net (2 .. 256), 0: block-per-net
    int32_t net0[kMaxBuckets];   // first (sorted) net of the bucket; entries are in grid order
    int32_t net1[kMaxBuckets];
    int32_t blk0[kMaxBuckets];   // first block; every bucket has a multiple of 8 blocks
    int32_t nblk[kMaxBuckets];
    int32_t pin0[kMaxBuckets];   // padded buckets: first pin slot (G slots per net)
    int32_t total_blocks;
};

// Device view of a loaded netlist (pointers into the caller's netlist buffer).
struct NetDev {
    const int32_t *net_start;      // [ns + 1] sweep order (nets with >= 2 pins)
    const int32_t *pin_cell;       // [ps]
    const void *pin_off;           // vec2<T> [ps] pin offsets
    const int2 *pin_offq;          // [ps] offsets quantized to 2^-16
    const void *net_w;             // T [ns] or nullptr (all weights 1)
    const int32_t *cell_pin_start; // [n_mov + 1]
    const int32_t *cell_pins;      // sweep-order pins of each movable cell
    const int32_t *cell_pin_net;   // the sweep-order net of each of those pins
    const int4 *cq;                // [n_mov] (w'q, h'q, dxq, dyq) in 2^-12
    const int2 *cq16;              // [n_mov] the same as four int16 (w'q | h'q << 16, dxq |
    int32_t cq_compact;            // dyq << 16) when every value fits (1), else 0: read by cell_cq
    const int32_t *rq;             // [n_mov] charge scale in 2^-16
    const void *cstep;             // T [4][n_mov]: pins, area, x max, y max
    const int64_t *rho_fixed;      // [my][mx]
    const void *tw_x, *tw_y;       // vec2<T> [M/2] exp(-2 pi i k / M)
    const void *ph_x, *ph_y;       // vec2<T> [M] (cos, sin)(pi u / (2 M))
    const double *omega;           // [mx + my] pi u / W, then pi v / H
    const double *den1;            // [mx + my] per-axis Laplacian symbol (den = dx[u] + dy[v])
    const void *fixed_pos;         // T [2][n_fixed]
    const double *fixed_xy;        // [2][n_fixed] lower-left x..., y... of the fixed cells
    const double *fixed_wh;        // [2][n_fixed] their widths..., heights...
    const void *cell_wh;           // T [2][n_mov] movable cell sizes
    int32_t n_cells, n_mov, n_fixed, ns, ps;
    int32_t lds_budget;            // dynamic LDS bytes a block may use on this device
    int32_t n_cu;                  // compute units of the device
    const int32_t *sweep_map;      // interleaved order of the padded buckets' blocks (see
                                   // sweep_block)
    int32_t sweep_lead;            // blocks of the block-per-net bucket, which lead the sweep
    int32_t sweep_interleave;      // 1: padded buckets' blocks in sweep_map order
    int32_t sweep_nt;              // 1: the sweep's read-once pin loads and its pin-gradient
                                   // stores carry non-temporal hints
    int32_t spec_threads;          // threads per block of the spectral column and inverse-row
                                   // passes: 512, 1024, or 0 (1024 while a launch has at most
                                   // one block per compute unit)
    // tile-binned charge scatter: ts x ts bin tiles (ts = 1 << log_ts), ntx x nty of them;
    // halo = widest charge footprint in bins - 1; windows of win_side = ts + halo bins
    int32_t log_ts, ntx, nty, ntiles, halo, win_side;
    int32_t sort_cells, sort_blocks, max_chunks;  // cells per counting block; chunk bound
    int32_t mx, my, logmx, logmy;
    int32_t bq, hq, wq_die, hq_die; // bin size and die size in 2^-12 units
    double W, H, wb, hb;
    double density_unit;           // 2^-40 / (wb hb): integer charge -> normalized density
    int64_t area_q;                // bin area in 2^-40 units
    double target_density;
    int64_t total_charge;
    int32_t stretch;               // small cells' charge spread over >= sqrt(2) bins per side
    int32_t offq_exact;            // every pin_off (in T) is a multiple of 2^-16: pin_offq is
                                   // pin_off * 2^16 exactly, and the sweeps form it from pin_off
    const int32_t *pin_off16;      // [ps] the offsets as two int16 (x low, y high) in units of
    int32_t off16_shift;           // 2^-off16_shift, when every offset is such a multiple that
                                   // fits (-1 otherwise): the sweeps read 4 bytes a slot, not 8
    // big cells: w'q >= big_wq or h'q >= big_hq (their footprint can span more than
    // kBigHalo + 1 bins) or w'q h'q >= big_aq; the halo above covers the other cells only
    const int32_t *big_ids;        // [n_big] ascending movable ids
    int32_t n_big, big_wq, big_hq;
    int64_t big_aq;
};

// Cell i's charge constants (w'q, h'q, dxq, dyq), from their compact form when the netlist has
// one (8 bytes instead of 16; the same integers).
__device__ __forceinline__ int4 cell_cq(const NetDev &nd, int i) {
    if (nd.cq_compact) {
        const int2 w = nd.cq16[i];
        return make_int4((int)(int16_t)(w.x & 0xffff), w.x >> 16, (int)(int16_t)(w.y & 0xffff),
                         w.y >> 16);
    }
    return nd.cq[i];
}

__host__ __device__ inline bool is_big(const NetDev &nd, int4 c) {
    return c.x >= nd.big_wq || c.y >= nd.big_hq || (int64_t)c.x * c.y >= nd.big_aq;
}

// Byte offsets of a slot's arrays inside its buffer (identical for all slots of a netlist).
struct SlotLayout {
    size_t u, v;          // vec2<T> [n_cells] (x, y) pairs (fixed cells in the tail, unchanged)
    size_t vprev;         // vec2<T> [n_mov]
    size_t uprev;         // vec2<T> [n_mov] u at the start of the last accepted step
    size_t gprev;         // T [2][n_mov]
    size_t g, gd;         // T [2][n_mov] raw gradient; density part (first evaluation)
    size_t pin_grad;      // vec2<T> [ps]
    size_t rho;           // int64 [my][mx] movable charge
    size_t t1, bx, by, bp;// T [my][mx] spectral intermediates
    size_t psi;           // T [my][mx] potential
    size_t exy;           // vec2<T> [my][mx] field (xi_x, xi_y)
    size_t scal;          // Scalars
    size_t part;          // double partial sums, kPartStride per reduction
    size_t keys, sel, work; // perturbation scratch
    size_t tile, sorted;  // int32 [n_mov]: each cell's tile, cells in tile order
    size_t crec;          // int4 [n_mov]: each cell's charge record from the counting pass
    size_t scnt, soff;    // int32 [sort_blocks][ntiles] histograms; their column offsets
    size_t tstart, cstart;// int32 [ntiles + 1]: tile cell ranges, tile chunk ranges
    size_t chunk;         // int4 [max_chunks]: each chunk's (tile, first, end) in the order
    size_t wins;          // int64 [ntiles][win_side^2] per-tile charge windows (zero between
                          // evaluations: the row pass clears what it reads)
    size_t pstride;       // doubles per reduction in `part` (max blocks of any reduction)
    size_t total;
};

// Per-block partials of every per-slot reduction (doubles; HPWL and overflow are int64 stored
// in the same 8-byte cells).
enum { PART_WL = 0, PART_E = 1, PART_N1 = 2, PART_N2 = 3, PART_DV = 4, PART_DG = 5,
       PART_GMAX = 6, PART_HPWL = 7, PART_OVF = 8, PART_COUNT = 9 };

// Per-slot scalars in device memory.
// The optimiser's own state (Nesterov a, the last step size alpha, the iteration count k) is
// held in two banks: a step reads bank b and writes bank 1 - b, and the host tracks b per slot
// (passed to kernels as one bit per slot of the launch).  So every block of a step may read
// the state it proposes from while one of them commits the next, with no ordering between
// them.  Resets write both banks.
struct Scalars {
    double ab[2], alphab[2];
    double aprevb[2];       // a at the start of the last accepted step (for a redo)
    double lambda, lambda_step, lambda0_scale, lambda_ratio;
    double wl, energy, overflow;
    double step_alpha, step_coef, step_a, step_aprev;  // proposal of the next step
    int64_t step_k, step_reject;                       // (see step_propose)
    int64_t kb[2];
    int64_t readyb[2];      // the last accepted step saved its start (u_prev, a_prev)
    int64_t backtrack;      // 1: steps are checked and redone (ePlace backtracking)
    int64_t rejects;        // steps redone since backtracking was last set
    int64_t ovf_tmp;        // overflow numerator of hp_overflow_of_cells
    int64_t lambda_valid;   // 0 until lambda_0 is derived at the first evaluation
    int64_t init_this_eval; // the last evaluation derived lambda_0
    int64_t hpwl_q, hpwl_valid;
    int64_t overflow_num;
    // perturbation
    uint64_t sel_prefix, sel_mask;
    int64_t sel_remaining, sel_count;
    uint32_t hist[256];
    int64_t best;
};

struct SlotArgs {
    char *base[kMaxSlots];
    int32_t n;
};

// Descriptor at the head of every slot buffer: the device view of the slot's netlist, its
// sweep buckets and the slot's layout, so that a launch over slots of different netlists
// (hp_iterate_multi) finds each slot's netlist in the slot's own buffer.  Kernels of such
// launches take RAG = true and read it per block; the slot's arrays start after it.  Written
// when the slot is allocated and when a launch setting of its netlist changes.
struct SlotDesc {
    NetDev nd;
    Buckets bk;
    SlotLayout L;
};
// 1 / smoothing of each slot of such a launch (kernel argument)
struct SlotGammas {
    double inv[kMaxSlots];
};
constexpr size_t kDescBytes = 4096;
static_assert(sizeof(SlotDesc) <= kDescBytes, "slot descriptor exceeds its reserved bytes");
__host__ __device__ inline const SlotDesc *slot_desc(const char *base) {
    return reinterpret_cast<const SlotDesc *>(base);
}
// The netlist view / layout of a block's slot: the kernel arguments, or (RAG) the slot's
// descriptor.
template <bool RAG>
__device__ __forceinline__ const NetDev &view_nd(const NetDev &arg, const char *base) {
    if constexpr (RAG) return slot_desc(base)->nd;
    else return arg;
}
template <bool RAG>
__device__ __forceinline__ const SlotLayout &view_L(const SlotLayout &arg, const char *base) {
    if constexpr (RAG) return slot_desc(base)->L;
    else return arg;
}
template <bool RAG>
__device__ __forceinline__ const Buckets &view_bk(const Buckets &arg, const char *base) {
    if constexpr (RAG) return slot_desc(base)->bk;
    else return arg;
}
__host__ __device__ inline int round8(int v) { return (v + kXcds - 1) / kXcds * kXcds; }

__host__ __device__ inline Scalars *scalars(char *base, const SlotLayout &L) {
    return reinterpret_cast<Scalars *>(base + L.scal);
}

// ---- optional per-kernel timing --------------------------------------------------------------
// When enabled, every selected launch carries a start and a stop HIP event; the elapsed times
// are collected by hp_profile_read.
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
bool prof_want(const char *name);
hipEvent_t prof_event();
void prof_push(const char *name, hipEvent_t a, hipEvent_t b);

// The events are handed to the dispatch itself (hipExtLaunchKernelGGL), so they time the
// kernel's execution, not the gap before it starts.
#define HP_LAUNCH(NAME, K, GRID, BLOCK, SHMEM, STREAM, ...)                              \
    do {                                                                                \
        if (::hp::prof_want(NAME)) {                                                    \
            hipEvent_t ea_ = ::hp::prof_event(), eb_ = ::hp::prof_event();              \
            hipExtLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, ea_, eb_, 0, __VA_ARGS__); \
            ::hp::prof_push(NAME, ea_, eb_);                                            \
        } else {                                                                        \
            hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);              \
        }                                                                               \
    } while (0)

// ---- launchers (each returns hipError_t of the launch) -----------------------------------
// First launch of an evaluation (WA sweep of v, charge accumulation or the counting pass of a
// regroup, and the HPWL sweep of u for the slots in hpwl_mask, bit i = slot i of the launch).
// sweep = false leaves the net sweep out (a density-only evaluation; hpwl_mask must be 0).
// records: the counting pass also writes the cells' charge records (the new order accumulates
// in the same evaluation).
template <typename T>
hipError_t launch_eval_front(const NetDev &nd, const Buckets &bk, const SlotArgs &sa,
                             const SlotLayout &L, double inv_gamma, uint32_t hpwl_mask,
                             bool accum, bool count, bool records, bool sweep, hipStream_t st);
template <typename T>
hipError_t launch_sweep_hpwl(const NetDev &nd, const Buckets &bk, const SlotArgs &sa,
                             const SlotLayout &L, hipStream_t st);
// Exact HPWL of caller-held positions `pos` (real pairs over all cells): per-block partials
// into part[bk.total_blocks], their sum into out[0].
template <typename T>
hipError_t launch_hpwl_positions(const NetDev &nd, const Buckets &bk, const void *pos,
                                 long long *part, long long *out, hipStream_t st);
// Scan, place and accumulate of a regroup whose counting pass the first launch ran; records:
// that pass wrote the cells' charge records for the accumulation to read.
template <typename T>
hipError_t launch_regroup_tail(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                               bool accum, bool records, hipStream_t st);
size_t scatter_count_lds(const NetDev &nd);
size_t scatter_place_lds(const NetDev &nd);  // the placement pass: ranks and tile starts
size_t scatter_accum_lds(const NetDev &nd);
// Big cells (one block per cell and slot; their charge is scattered in the first launch):
// the wirelength and density parts of their gradient written to g and gd (read back by the
// cell gradient pass).  No-op without any.
template <typename T>
hipError_t launch_big_grad(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                           int grad_mode, hipStream_t st);
// Overflow numerator of the charge of movable cells [0, n_counted) at v, into ovf_tmp of the
// slot's scalars; rho must be zero before and is zero after.
template <typename T>
hipError_t launch_overflow_of_cells(const NetDev &nd, char *base, const SlotLayout &L,
                                    int n_counted, hipStream_t st);
hipError_t launch_clear_rho(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                            hipStream_t st);
// Device-to-device (x, y) pair splitting / joining, rs = element bytes (4 or 8).
hipError_t launch_split_pairs(const void *pairs, void *x, void *y, int n, size_t rs, hipStream_t st);
hipError_t launch_join_pairs(const void *x, const void *y, void *pairs, int n, size_t rs, hipStream_t st);
template <typename T>
hipError_t launch_spectral(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                           bool keep_maps, bool want_psi, hipStream_t st);
// The evaluation's closing reduction: FIN_TOTALS, the totals of nwl sweep, ne energy and nov
// overflow partials; FIN_STEP, the step's lambda and, in steady state, its proposal from the
// optimiser state in bank (banks >> slot) & 1; FIN_FULL, both and lambda_0 on a first
// evaluation.
enum { FIN_TOTALS = 0, FIN_FULL = 1, FIN_STEP = 2 };
hipError_t launch_eval_finish(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L, int nwl,
                              int ne, int nov, int ncell, bool use_fixed, double lam_fixed,
                              int mode, uint32_t banks, hipStream_t st);
// At most this many cell-gradient partials let every block of the step reduce them itself
// (the fused step: no closing reduction launch in steady state).
constexpr int kFusedStepParts = 1024;
hipError_t launch_hpwl_finish(const SlotArgs &sa, const SlotLayout &L, int nparts, hipStream_t st);
// grad_mode bits: GRAD_EXACT, the exact adjoint sum psi dq/dx (needs the psi map) instead of
// the field force -sum q xi; GRAD_DENSITY_ONLY, no wirelength part (the sweep did not run).
enum { GRAD_EXACT = 1, GRAD_DENSITY_ONLY = 2 };
// finish: the closing reduction's mode after it (FIN_*), or -1 for none (the totals are then
// left to a later totals-only reduction and the proposal to the fused step).
template <typename T>
hipError_t launch_cell_grad(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                            double lambda_fixed, bool use_fixed, int grad_mode, int nwl, int ne,
                            int nov, int finish, uint32_t banks, hipStream_t st);
template <typename T>
hipError_t launch_combine(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L,
                          hipStream_t st);
template <typename T> int spectral_energy_parts(const NetDev &nd);
int spectral_overflow_parts(const NetDev &nd);
template <typename T> size_t spectral_max_lds(const NetDev &nd);
template <typename T> hipError_t spectral_prepare(int bytes);
// One Nesterov step; `proposed`: every slot's evaluation already formed the step's
// reductions and proposal (steady state), so only the update runs; `fused`: every slot's
// evaluation formed the reductions' partials but no proposal, which each block of the update
// then derives itself.  banks: the optimiser-state bank of each slot (bit s).
template <typename T>
hipError_t launch_step(const NetDev &nd, const SlotArgs &sa, const SlotLayout &L, bool proposed,
                       bool fused, uint32_t banks, hipStream_t st);
template <typename T>
hipError_t launch_fixed_map(const NetDev &nd, const double *fxy, const double *fwh,
                            int64_t *rho_fixed, hipStream_t st);
template <typename T>
// n_pool >= 0: select among the n_pool distinct cells whose ids the caller put in L.work
hipError_t launch_perturb(const NetDev &nd, char *slot, const SlotLayout &L, int mode,
                          int64_t m, double sigma_x, double sigma_y, uint64_t seed, int n_pool,
                          hipStream_t st);
size_t perturb_work_bytes(int n_mov, int mx, int my);
// WireMask perturbation of the n_pool macros `pool` (host ids, in that order), whose device
// copy the caller put at wiremask_pool_offset of L.work (the optimiser restarts first); the
// moved count goes to sel_count.
template <typename T>
hipError_t launch_wiremask(const NetDev &nd, char *base, const SlotLayout &L, const int32_t *pool,
                           int n_pool, hipStream_t st);
size_t wiremask_pool_offset(const NetDev &nd);
template <typename T>
hipError_t launch_select_best(const NetDev &nd, const SlotArgs &sa, char *incumbent,
                              const SlotLayout &L, hipStream_t st);

int sweep_parts(const Buckets &bk);
__host__ __device__ inline int cell_parts(const NetDev &nd) { return (nd.n_mov + kBlock - 1) / kBlock; }

// ---- launches over steady-state slots of different netlists (hp_iterate_multi) -------------
// Each slot's netlist, layout and smoothing come from its descriptor; grid.x is the largest
// need over the slots (blocks past a slot's own count return); dynamic LDS the largest need.
// Bit s of a mask is slot s of the launch.  accm / cntm: the first launch accumulates the
// charge in the slot's existing grouping / counts for a new one; hmask: its HPWL sweep rides
// along; banks: optimiser-state banks.
template <typename T>
hipError_t rag_front(const SlotArgs &sa, const SlotGammas &g, uint32_t accm, uint32_t cntm,
                     uint32_t hmask, int grid_x, size_t lds, hipStream_t st);
int front_blocks(const NetDev &nd, const Buckets &bk, bool accum, bool count);
template <typename T> size_t front_lds(const NetDev &nd, const Buckets &bk, bool accum, bool count);
// The rest of a rebuild of the scatter's grouping for every slot of sa (scans, placement and
// the accumulation in the new order); grids from the largest slot.
template <typename T>
hipError_t rag_regroup_tail(const SlotArgs &sa, int colscan_x, int place_x, int accum_x,
                            size_t place_lds, size_t accum_lds, hipStream_t st);
int colscan_blocks(const NetDev &nd);
template <typename T>
hipError_t rag_spectral(const SlotArgs &sa, int rows_x, int cols_x, int inv_x, size_t lds_rows,
                        size_t lds_cols, size_t lds_inv, hipStream_t st);
template <typename T>
hipError_t rag_big_grad(const SlotArgs &sa, int grid_x, hipStream_t st);
template <typename T>
hipError_t rag_cell_grad(const SlotArgs &sa, int grid_x, hipStream_t st);
// The closing reduction in steady state (FIN_STEP) of every slot, then the update (fused:
// every block reduces its slot's step partials itself and no closing reduction ran).
hipError_t rag_eval_finish(const SlotArgs &sa, uint32_t banks, hipStream_t st);
template <typename T>
hipError_t rag_step(const SlotArgs &sa, int grid_x, bool fused, uint32_t banks, hipStream_t st);
// host-side sizes the launches above need for one netlist
int rows_fwd_blocks(const NetDev &nd);
template <typename T> size_t rows_fwd_lds_of(const NetDev &nd);
template <typename T> size_t cols_lds_of(const NetDev &nd);
template <typename T> size_t rows_inv_lds_of(const NetDev &nd);
int step_blocks(const NetDev &nd);

}  // namespace hp
