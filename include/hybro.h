/*
 * libhybro -- the data-parallel hot path of the Hybro hybrid global placer on one AMD
 * Instinct MI355X (gfx950), as a C ABI.
 *
 * Paper: "Escaping Local Optima in Global Placement" (Hybro).  The placer minimises the
 * penalised objective of Eq. 2, sum_e WL_e(s) + lambda * D(s), with WL_e the weighted-average
 * wirelength of Eq. 3 and D the density term, by repeated gradient steps (Sec. 3.1); Hybro
 * (Alg. 1) perturbs the result (Sec. 4.2) and re-runs the placer, keeping the solution with
 * the smallest HPWL (Eq. 1).  D, the optimiser and the lambda schedule are only named by the
 * paper; this library uses the ePlace electrostatic system the paper builds on: an integer
 * charge map on a bin grid, a cosine-basis Poisson solve, field forces, and a preconditioned
 * Nesterov method with a Barzilai-Borwein step.
 *
 * Conventions
 *   - Cells [0, n_movable) are movable, [n_movable, n_cells) fixed.  Positions are lower-left
 *     corners on the die [0, W] x [0, H] (xl = yl = 0).  Pin p of net e sits at the cell's
 *     position plus (pin_ox[p], pin_oy[p]).
 *   - A context computes in FP32 or FP64 ("precision").  Position/gradient arrays are of
 *     that type ("real" below).  Reductions are accumulated in FP64; HPWL, the density map
 *     and perturbation indices are integers and therefore exact and run-to-run identical.
 *   - The library never allocates device memory: the caller allocates the byte sizes that
 *     hp_netlist_bytes / hp_slot_bytes return (e.g. as torch uint8 tensors) and lends them
 *     until hp_slot_free / hp_destroy.  Buffers must be 256-byte aligned.
 *   - Every call enqueues on the context's HIP stream.  Calls that return values to host
 *     memory synchronise that stream; calls whose outputs stay on the device do not.
 *   - Errors: a negative return code; hp_last_error gives a message (per thread, valid until
 *     that thread's next call).  On error nothing has been written to outputs.
 *   - A "slot" is one placement instance (its positions, optimiser state and scratch) on a
 *     loaded netlist.  Calls taking a slot list process all of them in one set of launches;
 *     all slots of one call must belong to the same netlist.
 */
#ifndef HYBRO_H
#define HYBRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hp_ctx hp_ctx;

enum {
    HP_OK = 0,
    HP_EINVAL = -1,   /* bad argument or netlist */
    HP_ENOMEM = -2,   /* a lent buffer is too small */
    HP_EDEVICE = -3,  /* a HIP call failed */
    HP_ESTATE = -4,   /* unknown slot / netlist, or slots of different netlists */
    HP_ENOTIMPL = -5
};

/* Die and bin grid.  W, H: at most 16384 (the exact HPWL works on 32-bit pin coordinates in
 * 2^-16 units, so pin coordinates must stay within (-2^15, 2^15); positions the library
 * produces stay inside the die).  mx, my: number of bins, powers of two in [8, 2048] in FP32
 * and [8, 1024] in FP64 (the spectral passes hold rows and columns in LDS); the bin
 * width W/mx and height H/my must be multiples of 2^-12 (so bin edges are exact in the 2^-12
 * integer coordinates of the density map).  target_density: the rho_t of the overflow measure.
 * stretch: 1 spreads a small cell's charge over at least sqrt(2) bins per side (ePlace local
 * smoothing), 0 uses the cell's own rectangle.  fd5: 1 uses the 5-point Laplacian's
 * eigenvalues in the Poisson solve instead of the continuous ones. */
typedef struct {
    double W, H;
    int32_t mx, my;
    double target_density;
    int32_t stretch;
    int32_t fd5;
} hp_die;

typedef struct {
    int32_t n_cells, n_movable, n_nets, n_pins;
} hp_shape;

/* precision: 32 or 64.  hip_stream: a hipStream_t (NULL = the null stream).  Threads may
 * share a context: each call holds the context's lock while it runs (a netlist load only
 * while it registers the netlist; hp_slot_free and hp_netlist_free not while they wait for
 * the stream), so e.g. one thread can load arriving jobs while another iterates the resident
 * ones.  hp_destroy must not overlap any other call on the context. */
int hp_create(hp_ctx **out, int device, void *hip_stream, int precision);
int hp_destroy(hp_ctx *ctx);
const char *hp_last_error(void);

/* Sizes of the device buffers the caller lends (bytes, upper bounds from the shape). */
size_t hp_netlist_bytes(const hp_ctx *ctx, const hp_shape *shape, const hp_die *die);
size_t hp_slot_bytes(const hp_ctx *ctx, const hp_shape *shape, const hp_die *die);

/* Netlist N = (V, E) of Sec. 3 as a net -> pin CSR.  Host arrays are read during the call
 * and not kept.  At least one movable cell (n_movable >= 1; a netlist with nothing to place
 * is HP_EINVAL, and hp_netlist_bytes / hp_slot_bytes return 0 for its shape).
 * cell_w/cell_h [n_cells] (> 0 for movable cells, >= 0 for fixed; zero-area
 * fixed cells are pads); fixed_x/fixed_y [n_cells - n_movable] lower-left of fixed cells;
 * net_start [n_nets + 1] non-decreasing, net_start[0] = 0, net_start[n_nets] = n_pins;
 * pin_cell [n_pins] in [0, n_cells); pin_ox/pin_oy [n_pins]; net_weight [n_nets] or NULL
 * (all 1).  Nets with fewer than two pins add nothing to Eq. 1 or Eq. 3.  Movable cells may
 * be of any size up to the die, macros included: a movable cell whose charge can span more
 * than 9 bins on an axis or covers 8 bin areas or more is scattered and gathered by a block of
 * its own (mixed-size placement; the results are those of any other cell).  Validates everything above
 * (HP_EINVAL) and dev_bytes (HP_ENOMEM).  Synchronises the stream. */
int hp_load_netlist_csr(hp_ctx *ctx, const hp_shape *shape, const hp_die *die,
                        const double *cell_w, const double *cell_h,
                        const double *fixed_x, const double *fixed_y,
                        const int32_t *net_start, const int32_t *pin_cell,
                        const double *pin_ox, const double *pin_oy,
                        const double *net_weight, void *dev_buf, size_t dev_bytes,
                        int32_t *out_netlist);

/* A placement instance on a netlist, in a lent buffer of hp_slot_bytes bytes. */
int hp_slot_alloc(hp_ctx *ctx, int32_t netlist, void *dev_buf, size_t dev_bytes,
                  int32_t *out_slot);
int hp_slot_free(hp_ctx *ctx, int32_t slot);
/* Release a netlist whose slots are all freed (HP_ESTATE while one is alive, or for an unknown
 * id): the context forgets it and waits for its stream, after which the caller may free the
 * netlist's device buffer.  Its id is not reused. */
int hp_netlist_free(hp_ctx *ctx, int32_t netlist);

/* Set the movable cells' positions (real [n_movable] each; host or device memory) and
 * restart the optimiser there: u = v = v_prev = (x, y), k = 0, a = 1, lambda re-derived at
 * the next evaluation.  hp_get_positions copies out the major solution u;
 * hp_get_eval_positions copies out the look-ahead point v of the Nesterov method, where the
 * next hp_eval_objective_grad is taken.  x or y may be NULL to skip that axis. */
int hp_set_positions(hp_ctx *ctx, int32_t slot, const void *x, const void *y, int on_device);
int hp_get_positions(hp_ctx *ctx, int32_t slot, void *x, void *y, int on_device);
int hp_get_eval_positions(hp_ctx *ctx, int32_t slot, void *x, void *y, int on_device);

/* lambda schedule of Eq. 2 (it starts small, Sec. 3): at the first evaluation after
 * hp_set_positions / hp_perturb, lambda_0 = lambda0_scale * |grad WL|_1 / |grad N|_1; every
 * Nesterov step multiplies it by 10^(decades / total_iters).  Defaults: 1e-4, 4, 1000. */
int hp_set_schedule(hp_ctx *ctx, int32_t slot, double lambda0_scale, double decades,
                    int32_t total_iters);
/* Set the factor lambda is multiplied by at every following Nesterov step (ratio > 0, finite):
 * for drivers that adapt the penalty of Eq. 2 as the placement evolves.  Synchronises. */
int hp_set_lambda_ratio(hp_ctx *ctx, int32_t slot, double ratio);

/* Grouping policy of the integer charge scatter (the density term of Eqs. 1-2) for every slot
 * of a netlist; it changes speed only, never results (the charge map is an integer sum and is
 * bit-identical under any grouping).  Cells are grouped by bin tile so that each group's charge
 * is summed in on-chip memory; the grouping is rebuilt every `regroup_every` evaluations
 * (1..64; cells that left their group's window in between take a slower path), and with
 * `deferred` = 1 the rebuilding evaluation still accumulates in the previous grouping and the
 * rebuild finishes after it (fewer launches; better when cells move little), with 0 it
 * accumulates in the new one.  Defaults: 4 and 1.  Returns HP_EINVAL on values out of range,
 * HP_ESTATE on an unknown netlist.  Takes effect at the next evaluation; no device work. */
int hp_set_scatter_policy(hp_ctx *ctx, int32_t netlist, int32_t regroup_every, int32_t deferred);
int hp_get_scatter_policy(hp_ctx *ctx, int32_t netlist, int32_t *regroup_every, int32_t *deferred);

/* Launch-shape settings of a loaded netlist, for tuners and tests; they change speed only.
 *   HP_TUNE_FUSED_STEP_PARTS: the largest number of cell-gradient block partials (one per 256
 *     movable cells) for which every block of the Nesterov update reduces the step's norms
 *     itself; above it a one-block closing reduction forms the step before the update.  Both
 *     forms reduce the partials in the same order, so positions are bit-identical.  [0, 1024],
 *     default 1024 (0: always the closing reduction).
 *   HP_TUNE_SPECTRAL_THREADS: threads per block of the Poisson solve's column and inverse-row
 *     passes, 512 or 1024, or 0 (default: 1024 while a launch has at most one block per
 *     compute unit, else 512).  The field maps are the same; the energy total may differ in
 *     its last bits (its per-block reduction tree changes).
 *   HP_TUNE_SWEEP_INTERLEAVE: order of the net sweep's blocks.  0 (default): degree bucket
 *     after degree bucket; 1: the buckets' blocks interleaved by their progress through the
 *     cell range, so that every bucket gathers the same cells at the same time.  The exact
 *     HPWL is the same; the wirelength total may differ in its last bits.
 *   HP_TUNE_CHARGE_RECORDS: 1 (default): when the charge scatter's grouping is rebuilt and
 *     accumulated in the same evaluation, the counting pass also writes each cell's charge
 *     rectangle and weight, which the accumulation then reads with one gather per cell instead
 *     of three (it pays while cells are spread with no relation to their ids, e.g. from random
 *     positions); 0: no records.  Results are bit-identical.
 *   HP_TUNE_NONTEMPORAL: 1: the net sweep of a launch over this netlist alone reads the pin
 *     lists and writes the pin gradients with non-temporal hints (streamed data that is used
 *     once per evaluation then competes less with the gathered positions for the caches;
 *     it pays on netlists far larger than the last-level cache); 0 (default): plain loads
 *     and stores.  Launches that mix netlists (hp_iterate_multi over several) use plain ones.
 *     Results are bit-identical.
 * Takes effect at the next launch.  HP_EINVAL for an unknown setting or a value out of range
 * (nothing changed), HP_ESTATE for an unknown netlist.  The spectral width and the sweep
 * order also rewrite the descriptors of the netlist's slots (a small copy on the context's
 * stream, waited for); the other settings do no device work. */
enum { HP_TUNE_FUSED_STEP_PARTS = 0, HP_TUNE_SPECTRAL_THREADS = 1, HP_TUNE_SWEEP_INTERLEAVE = 2,
       HP_TUNE_CHARGE_RECORDS = 3, HP_TUNE_NONTEMPORAL = 4 };
int hp_set_tunable(hp_ctx *ctx, int32_t netlist, int32_t which, int32_t value);
int hp_get_tunable(hp_ctx *ctx, int32_t netlist, int32_t which, int32_t *value);

/* Objective of Eq. 2 and its gradient at the slots' reference points v:
 *   wl = sum_e w_e WL_e (Eq. 3, both axes), energy = electrostatic energy N of the charge
 *   map, overflow = sum_b max(0, movable charge - target * free area) / total movable charge
 *   (the D(s) <= eps measure of Eq. 1), gradient = grad WL + lambda * grad N over movable
 *   cells.  gamma: the smoothing length of Eq. 3 (same units as positions).  lambda >= 0 is
 *   used as given; lambda < 0 uses each slot's scheduled lambda.  grad_mode bit 0: 0 the field
 *   force -sum_b q_ib xi_b (ePlace), 1 the exact adjoint sum_b psi_b dq_ib/dx_i of the
 *   continuous charge rectangle (also computes the potential map); bit 1 (HP_GRAD_DENSITY_ONLY):
 *   the density term alone -- the net sweep does not run, wl is 0 and the gradient is
 *   lambda * grad N, for callers that need the density adjoint by itself (needs lambda >= 0,
 *   HP_EINVAL otherwise).  keep_maps 1 keeps the charge,
 *   potential and field maps for hp_get_map.  wl/energy/overflow: host double [n_slots] or
 *   NULL (then nothing is synchronised, and in steady state the totals are reduced only when
 *   first read, by hp_get_state).  grad_x/grad_y: device real [n_slots][n_movable] or
 *   NULL (the gradient always stays in the slot for hp_nesterov_step). */
enum { HP_GRAD_FIELD = 0, HP_GRAD_EXACT = 1, HP_GRAD_DENSITY_ONLY = 2 };
typedef struct {
    double gamma;
    double lambda;
    int32_t grad_mode;
    int32_t keep_maps;
} hp_eval_params;
int hp_eval_objective_grad(hp_ctx *ctx, const int32_t *slots, int32_t n_slots,
                           const hp_eval_params *p, double *wl, double *energy,
                           double *overflow, void *grad_x, void *grad_y);

/* Overflow (the D(s) <= eps measure of Eq. 1, as hp_eval_objective_grad reports it) of the
 * charge of movable cells [0, n_counted) alone, at the slot's evaluation point v: out_num the
 * exact numerator (2^-40 area units), out the numerator over those cells' total charge (either
 * may be NULL).  For netlists whose last movable cells are ePlace filler cells (pinless cells
 * that fill the free area to a target density below 1), the overflow of the real cells; with
 * n_counted = n_movable it is the evaluation's own.  Off the iteration path (two launches, the
 * map is rebuilt with atomics); a map kept by the last evaluation is dropped.  HP_EINVAL if
 * n_counted is outside [0, n_movable].  Synchronises. */
int hp_overflow_of_cells(hp_ctx *ctx, int32_t slot, int32_t n_counted, int64_t *out_num,
                         double *out);

/* Backtracking of the Nesterov step for one slot (ePlace's Nesterov method with Lipschitz
 * prediction, the accelerated form of the descent of Sec. 3.1): on = 1 checks every step
 * after the first following a restart: when the step length predicted at the point the last
 * step reached, |v - v_prev| / |g~ - g~_prev|, is below 0.95 of that step's length, that step
 * is redone from its start with the new length (the gradient just taken is dropped; k, a and
 * lambda do not advance), else the step proceeds as usual.  Checks begin after the first
 * step taken with on = 1.  on = 0 (the default) is the plain method.  Resets the slot's count
 * of redone steps.  HP_EINVAL unless on is 0 or 1.  Synchronises. */
int hp_set_backtracking(hp_ctx *ctx, int32_t slot, int32_t on);

/* One preconditioned Nesterov step per slot from the gradient of the last evaluation:
 * P_i = max(1, pins_i + lambda area_i), g~ = g / P, step alpha_0 = 0.1 bin / max|g~| then
 * Barzilai-Borwein |v - v_prev| / |g~ - g~_prev|, u' = clamp(v - alpha g~),
 * a' = (1 + sqrt(4 a^2 + 1)) / 2, v' = clamp(u' + (a - 1)/a' (u' - u)).  Device only. */
int hp_nesterov_step(hp_ctx *ctx, const int32_t *slots, int32_t n_slots);

/* `iters` iterations of the placer (Sec. 3.1) on every listed slot, all on the device: each is
 * hp_eval_objective_grad with the slots' scheduled lambda and the given gamma (nothing returned
 * to the host) and hp_nesterov_step; with HP_ITER_HPWL every iteration is followed by hp_hpwl
 * without outputs, with HP_ITER_HPWL_LAST only the last one (the exact HPWL of Eq. 1 as a
 * driver reads it, e.g. every 10 iterations).  Does not synchronise.
 * HP_ITER_GRAPH replays steady-state blocks of 2 x (the scatter's rebuild interval)
 * iterations from a captured HIP graph: a block is captured once the slots are in steady
 * state and is replayed whenever the slots' state is the one it was captured from, which
 * every block returns to; leftover iterations run as usual, and results are bit-identical to
 * eager iterations.  No block is captured while another thread uses the context's stream
 * outside the context's lock (a netlist load, or a call waiting for the stream): those
 * iterations run eagerly.  The graph is kept with the context until another block replaces
 * it, a slot of it is freed or the context is destroyed.  It needs a context stream other than the
 * null stream (HP_EINVAL); while per-kernel timing is enabled nothing is captured.  Unknown
 * flags or iters < 0: HP_EINVAL. */
enum { HP_ITER_HPWL = 1, HP_ITER_GRAPH = 2, HP_ITER_HPWL_LAST = 4 };
typedef struct {
    double gamma;
    int32_t flags;
} hp_iter_params;
int hp_iterate(hp_ctx *ctx, const int32_t *slots, int32_t n_slots, const hp_iter_params *p,
               int32_t iters);
/* Graph blocks captured and replayed by hp_iterate and hp_iterate_multi on this context so far
 * (inspection; either
 * output may be NULL).  No device work. */
int hp_graph_stats(hp_ctx *ctx, int64_t *captures, int64_t *replays);

/* `iters` iterations of the placer (Sec. 3.1) on slots of different netlists of this context,
 * each with its own smoothing gammas[i] (> 0, host array [n_slots]), in shared launches: one
 * launch per pass of an iteration covers every listed slot (the batched evaluation of several
 * placement jobs at once).  Each iteration is, per slot, what hp_iterate does with that gamma;
 * results are bit-identical to running each slot alone with hp_iterate.  Every slot must be
 * in steady state: its lambda derived and its charge grouping built by an earlier iteration
 * (one hp_iterate call), and no map kept by an evaluation since (HP_ESTATE otherwise).
 * flags: HP_ITER_HPWL, HP_ITER_HPWL_LAST and HP_ITER_GRAPH as for hp_iterate (a block is the
 * least common multiple of twice the slots' rebuild intervals, at most 64 iterations; longer
 * cycles iterate eagerly; the context's one cached block is shared with hp_iterate).  At most
 * 32 slots, each listed once (HP_EINVAL); iters < 0, an unknown flag, or HP_ITER_GRAPH on a
 * context of the null stream: HP_EINVAL.  Does not synchronise. */
int hp_iterate_multi(hp_ctx *ctx, const int32_t *slots, int32_t n_slots, const double *gammas,
                     int32_t flags, int32_t iters);

/* Perturbation of Alg. 1 / Sec. 4.2 on slot's major solution u, which also restarts the
 * optimiser there.  mode HP_PERTURB_GAUSS: the round(fraction * n_movable) cells with the
 * smallest SplitMix64 keys move by a Gaussian of sigma_bins bins per axis; SHUFFLE: those
 * cells exchange centres by a keyed permutation ("Shuffle (all)"); UNIFORM: every movable
 * cell is redrawn uniformly (random restart).  Moved cells are clamped into the die.
 * out_idx: host int32 [count] of moved cells in ascending order, or NULL; out_count: host or
 * NULL.  Either output synchronises. */
enum { HP_PERTURB_GAUSS = 0, HP_PERTURB_SHUFFLE = 1, HP_PERTURB_UNIFORM = 2 };
int hp_perturb(hp_ctx *ctx, int32_t slot, int mode, double fraction, double sigma_bins,
               uint64_t seed, int32_t *out_idx, int32_t *out_count);

/* hp_perturb restricted to a pool of movable cells, as in "Shuffle" of Sec. 4.2 (p% of the
 * macros are selected and shuffled): cells (host int32 [n_pool], distinct ids in
 * [0, n_movable), any order; read during the call) is the pool, round(fraction * n_pool) of
 * them move, the ones with the smallest (key, id) where a pooled cell's key is its SplitMix64
 * draw shifted right by one bit.  GAUSS and SHUFFLE as in hp_perturb; UNIFORM, an id out of
 * range or repeated, or cells NULL with n_pool > 0: HP_EINVAL with nothing changed.
 * Synchronises when n_pool > 0 or an output is requested. */
int hp_perturb_among(hp_ctx *ctx, int32_t slot, int mode, double fraction, double sigma_bins,
                     uint64_t seed, const int32_t *cells, int32_t n_pool, int32_t *out_idx,
                     int32_t *out_count);

/* WireMask perturbation (Sec. 4.2): the optimiser restarts at u, then the listed macros
 * (host int32 [n_macros], distinct movable ids; the order is the order of the pass, read during
 * the call) each move in turn to the bin-corner position with the least increment of the exact
 * HPWL of Eq. 1 (2^-16 grid) given every other cell where it is, among the positions inside the
 * die where the macro overlaps neither another listed macro nor a fixed cell of nonzero area;
 * ties to the smaller displacement |dx| + |dy|, then the lower candidate index (row-major over
 * the candidates); a macro with no free position stays.  out_moved: host, how many macros
 * changed position, or NULL.  Three launches per macro.  An id out of range or repeated, or
 * macros NULL with n_macros > 0: HP_EINVAL with nothing changed.  Synchronises. */
int hp_perturb_wiremask(hp_ctx *ctx, int32_t slot, const int32_t *macros, int32_t n_macros,
                        int32_t *out_moved);

/* Exact HPWL (Eq. 1) of the slots' major solutions u on pin coordinates quantized to 2^-16:
 * out_q (host int64 [n_slots], units of 2^-16) and/or out (host double) or both NULL (the
 * value stays in the slot for hp_select_best). */
int hp_hpwl(hp_ctx *ctx, const int32_t *slots, int32_t n_slots, int64_t *out_q, double *out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the exact HPWL of Eq. 1, as hp_hpwl computes it, of
 * positions the caller holds, with no slot and no allocation of any kind.
 *   xy: device real pairs [n_cells] (x, y) of every cell of the netlist, movable cells then
 *       fixed ones (the fixed cells at their fixed positions), lower-left corners; aligned to
 *       a pair.
 *   out_q: device int64 [1], the HPWL in 2^-16 units.
 * The sweep's per-block partial sums live in a static device array of the library, 1 MiB
 * (131072 partials) per GPU, held until the process ends: a netlist whose sweep has more
 * blocks than that gets HP_ENOMEM (about 40 M pins in nets of two).  Every call on a GPU
 * uses that GPU's one array, so calls that overlap on one GPU (from different streams or
 * threads) race and must be ordered by the caller.  Enqueued on the context's stream, does
 * not synchronise.  NULL pointers or misalignment: HP_EINVAL; unknown netlist: HP_ESTATE. */
int hp_hpwl_noalloc(hp_ctx *ctx, int32_t netlist, const void *xy, int64_t *out_q);

/* Best solution of Alg. 1: among the slots' last hp_hpwl values (and the incumbent's, if
 * incumbent >= 0 and it has one), the smallest wins, ties to the lowest list position and
 * then to the incumbent; the winner's u is copied into the incumbent's u and v (incumbent
 * restarts there).  out_best: host, list position of the winner or -1 if the incumbent
 * stayed; NULL keeps everything on the device. */
int hp_select_best(hp_ctx *ctx, const int32_t *slots, int32_t n_slots, int32_t incumbent,
                   int32_t *out_best);

/* Inspection (synchronises).  hp_get_map copies a bin map of the last evaluation that ran
 * with keep_maps: HP_MAP_RHO_MOV (int64 charge, 2^-40 area units), HP_MAP_RHO_FIXED (int64),
 * HP_MAP_PSI / HP_MAP_EX / HP_MAP_EY (real; potential and field).  Layout [my][mx]. */
enum { HP_MAP_RHO_MOV = 0, HP_MAP_RHO_FIXED = 1, HP_MAP_PSI = 2, HP_MAP_EX = 3, HP_MAP_EY = 4 };
int hp_get_map(hp_ctx *ctx, int32_t slot, int which, void *host_dst);

/* A slot's device state: iterations taken k (accepted steps), the last exact HPWL (2^-16
 * units; -1 if none since the last restart), the overflow numerator (2^-40 area units) and, in
 * the same order as hp_eval_objective_grad reports them, Nesterov's a, the last step alpha,
 * lambda and the last evaluation's totals; then the steps redone under backtracking since
 * hp_set_backtracking.  Reduces any pending HPWL or totals first (small launches) and
 * synchronises. */
typedef struct {
    int64_t k, hpwl_q, overflow_num;
    double a, alpha, lambda, wl, energy, overflow;
    int64_t rejects;
} hp_slot_state;
int hp_get_state(hp_ctx *ctx, int32_t slot, hp_slot_state *out);

/* Per-kernel timing.  While enabled, every launch of the kernel named only_kernel (or of every
 * kernel if it is NULL) is bracketed by two HIP events on the context's stream (a small host
 * cost per bracketed launch).  hp_profile_read synchronises, adds the elapsed times of all
 * bracketed launches since the last read to per-kernel totals, copies up to `max` totals to
 * `out` (host), sets *n_out to the number of kernels seen, and clears the totals if `reset`.
 * The profiler state is process-wide (guarded: threads may launch while it is on, and their
 * launches are all timed together; launches are not captured into graphs while it is on). */
typedef struct {
    char name[48];
    int64_t count;
    double total_ms;
} hp_kernel_time;
int hp_profile_enable(hp_ctx *ctx, int on, const char *only_kernel);
int hp_profile_read(hp_ctx *ctx, hp_kernel_time *out, int32_t max, int32_t *n_out, int reset);

#ifdef __cplusplus
}
#endif
#endif /* HYBRO_H */
