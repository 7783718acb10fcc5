/*
 * lbm.h - C ABI of the MI355X (gfx950) D2Q9 lattice-Boltzmann library.
 *
 * The library advances the D2Q9 BGK lattice-Boltzmann method of Tomczak,
 * "Data-Oriented Language Implementation of Lattice-Boltzmann Method for Dense
 * and Sparse Geometries" (arXiv 2108.13241): the fused stream-and-collide time
 * step of Algorithm 1 (pull scheme, Sec. 3) with the moments of Eq. 2, the BGK
 * operator of Eqs. 3-5, the equilibrium of Eq. 6 and bounce-back walls marked
 * by a node-type field (Sec. 3), on dense meshes and on sparse geometries
 * (Sec. 4.3: tiles of 16 x 16 nodes, and a per-fluid-node indirect list).
 * Beyond the paper it adds a body force (Guo forcing), a per-node Brinkman drag
 * coefficient, 16-bit shifted population storage and a hand-written adjoint.
 *
 * Conventions shared by every entry point
 *  - Every call returns an lbm_status (0 = LBM_OK).  Nothing aborts or throws
 *    across the ABI.  On LBM_ERR_INVALID / LBM_ERR_UNSUPPORTED nothing changed.
 *    A device failure returns LBM_ERR_DEVICE and marks the context broken: later
 *    calls on it return LBM_ERR_STATE.  lbm_last_error() explains the failure.
 *  - Host arrays are owned by the caller and only read (or written) during the
 *    call.  "Device" pointers are HIP device addresses on the context's device,
 *    owned by the caller; the library only reads / writes them on its stream.
 *  - 2-D host and device fields are row-major [ny][nx] (x fastest), no padding.
 *  - Node types (mask): 0 = fluid, 1 = solid.  Both axes are periodic; walls come
 *    only from solid nodes.  Bounce-back is the halfway, link-wise rule: a
 *    population that would stream into a solid node returns to its origin node
 *    with the opposite direction in the same step.
 *  - Populations are numbered as in the paper's Fig. 1: 0 rest, 1 (+x), 2 (+y),
 *    3 (-x), 4 (-y), 5 (+x+y), 6 (-x+y), 7 (-x-y), 8 (+x-y).
 *  - "Canonical" populations f_i(x, t) are the pre-collision (post-streaming)
 *    values, the left-hand side of Eq. 3, as FP64 [9][ny][nx]; solid slots = 0.
 *    Whatever the layout stores internally, the canonical view is the same.
 *  - One context is not thread-safe; separate contexts are independent.
 *    All work is enqueued on the context's stream (lbm_set_stream); calls that
 *    return host data synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque; owned by the library until lbm_destroy */

/* Population storage type.  F64 stores f_i and computes in FP64.  F32,
 * F16_SHIFTED and BF16_SHIFTED store the deviation f_i - w_i (rho0 = 1), in 32 or
 * 16 bits (round to nearest even), and compute in FP32 on the deviations, which
 * keeps FP32 within 1e-5 relative of FP64 where storing f_i itself does not. */
typedef enum {
    LBM_F64 = 0,
    LBM_F32 = 1,
    LBM_F16_SHIFTED = 2,
    LBM_BF16_SHIFTED = 3
} lbm_dtype;

/* Memory layout of the populations.
 *  DENSE_AB : two full lattices, pull scheme, swapped every step (Algorithm 1,
 *             Sec. 3).  Structure of arrays within chunks of 64 nodes along a
 *             row: each chunk stores its 9 populations as 9 runs of 64.
 *  DENSE_AA : one full lattice updated in place with the AA access pattern
 *             (the single-copy scheme Sec. 3 mentions): even steps read and
 *             write each node's own slots, odd steps read from and write to the
 *             neighbours.
 *  TILED16  : two lattices holding only the non-empty 16 x 16 tiles, compacted
 *             in row-major tile order (each tile stores its 9 populations as 9
 *             runs of 256), with a tile-neighbour table ("pointer tile" of
 *             Sec. 4.3).  Requires nx and ny to be multiples of 16.
 *  INDIRECT : two lattices holding only fluid nodes (row-major compaction) and
 *             a per-node neighbour table (the fluid-index-array approach of
 *             Sec. 1).
 *  TILED16_ALL: the "tile" layout of Sec. 4.3: a dense array of all 16 x 16
 *             tiles, empty ones included, in row-major tile order, run by the
 *             TILED16 kernels (memory and launch cover every tile).  Reported
 *             as TILED16_ALL by lbm_get_info.  Requires nx and ny to be
 *             multiples of 16.
 * The D3Q19 interface (lbm3d.h) takes TILED16 / TILED16_ALL as its tiled
 * layout in 4 x 4 x 4-node blocks (nx, ny, nz multiples of 4). */
typedef enum {
    LBM_DENSE_AB = 0,
    LBM_DENSE_AA = 1,
    LBM_TILED16 = 2,
    LBM_INDIRECT = 3,
    LBM_TILED16_ALL = 4
} lbm_layout;

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID = -1,     /* bad argument; nothing changed */
    LBM_ERR_NOMEM = -2,       /* device or host allocation failed */
    LBM_ERR_DEVICE = -3,      /* HIP runtime error; the context is now broken */
    LBM_ERR_UNSUPPORTED = -4, /* valid request the library does not implement */
    LBM_ERR_STATE = -5        /* context broken by an earlier device error */
} lbm_status;

/* Geometry and size summary of a context. */
typedef struct {
    int32_t nx, ny;
    int32_t dtype, layout;
    int64_t n_nodes;         /* nx * ny */
    int64_t n_fluid;         /* fluid nodes: the ones counted for LUPS (Eq. 8) */
    int64_t n_tiles;         /* TILED16: non-empty tiles; else 0 */
    int64_t time_step;       /* steps taken since the last (re)initialisation */
    int32_t pop_bytes;       /* bytes per stored population: 8, 4 or 2 */
    int32_t has_porosity;    /* 1 once lbm_set_porosity gave a non-NULL field */
    double bytes_per_fluid_node; /* algorithmic bytes per fluid node per step:
                                    18 * pop_bytes + 1 (node type) [+4 with drag] */
    double bytes_moved_per_step; /* bytes the step kernel touches in DRAM per step
                                    under ideal caching (tiles count whole tiles,
                                    INDIRECT adds 32 B/node of neighbour table) */
    size_t device_bytes;     /* device memory held by the context */
} lbm_info_t;

/* Device allocator hook (process-wide).  Every device buffer a context owns is
 * taken from alloc(bytes, user) and returned with free(ptr, user).  Passing
 * NULL, NULL restores hipMalloc / hipFree.  Contexts keep the hook they were
 * created with. */
typedef void *(*lbm_alloc_fn)(size_t bytes, void *user);
typedef void (*lbm_free_fn)(void *ptr, void *user);
int lbm_set_allocator(lbm_alloc_fn alloc, lbm_free_fn free_fn, void *user);

/* Create a lattice (Sec. 3: node-type field; Eq. 5: omega = 1 / tau).
 *  out       receives the context (NULL on failure).
 *  nx, ny    mesh size, >= 1 each (TILED16: multiples of 16).
 *  node_type host uint8 [ny][nx], values 0 (fluid) / 1 (solid); copied.
 *  tau       relaxation time, > 1/2 (viscosity nu = (tau - 1/2) / 3).
 *  force     host double[2] = body-force acceleration (g_x, g_y); NULL = 0.
 *            It enters through Guo's forcing term with force density
 *            F = rho (g - alpha u).
 * The lattice starts at rest (rho = 1, u = 0; Algorithm 1 initialisation) on
 * the current HIP device, using the default stream until lbm_set_stream.
 * Size limits (pitch = nx rounded up to 64): DENSE_AB / DENSE_AA take
 * ny * pitch < 2^31 nodes and 9 * pitch < 2^28, i.e. lattices up to the
 * device's memory (FP64 A-B: 144 B per node, about 2 G nodes in 288 GB; the
 * rest state is written in place, while initialisation from fields and
 * population transfers stage 72 B per node of FP64 for their duration);
 * TILED16 / TILED16_ALL / INDIRECT use 32-bit offsets and take
 * 9 * ny * pitch < 2^32 (about 477 M mesh nodes).
 * Errors: INVALID (sizes, tau, non-finite force, mask value), UNSUPPORTED
 * (layout constraint, size limit), NOMEM, DEVICE. */
int lbm_create(lbm_ctx **out, int32_t nx, int32_t ny, const uint8_t *node_type, double tau,
               const double *force, lbm_dtype dtype, lbm_layout layout);

/* Enqueue all later work on `hip_stream` (a hipStream_t; NULL = default stream).
 * Work already enqueued on the previous stream is waited for first. */
int lbm_set_stream(lbm_ctx *ctx, void *hip_stream);

/* Algorithm 1 initialisation: f_i = f^eq_i(rho0, u0) (Eq. 6) at every fluid
 * node, as the canonical state at time 0.  Host FP64 [ny][nx] fields; NULL
 * means rho0 = 1 / u0 = 0 (all three NULL: the rest state f_i = w_i, written
 * in place without a staging buffer).  Resets the step counter to 0. */
int lbm_init_equilibrium(lbm_ctx *ctx, const double *rho, const double *ux, const double *uy);

/* Per-node Brinkman drag coefficient alpha (host FP32 [ny][nx], each in [0, 1];
 * NULL removes the drag).  The collision uses u = (m / rho + g / 2) / (1 + alpha / 2)
 * and F = rho (g - alpha u).  Errors: INVALID for values outside [0, 1]. */
int lbm_set_porosity(lbm_ctx *ctx, const float *alpha);

/* Open boundaries: constant velocity and constant pressure (Sec. 3, after Zou
 * and He).  bc: host uint8 [ny][nx], per node 0 = none, 1..4 = constant
 * velocity with inward normal +x, -x, +y, -y, 5..8 = constant pressure with
 * the same normals; codes only at fluid nodes.  value: host FP64 [2][ny][nx]:
 * (u_x, u_y) at velocity nodes (|u_x|, |u_y| < 1), (rho, unused) at pressure
 * nodes (rho > 0).  Both are copied.  At an open node the three populations
 * entering across the boundary (c_i . n > 0) are rebuilt, before every
 * collision and in every view of the state, so that the node's density and
 * momentum (Eq. 2, without the force and drag corrections) take the
 * prescribed values (pressure nodes: no tangential velocity) and the normal
 * population pair has equal non-equilibrium parts; whatever streamed into
 * those slots across the periodic seam is discarded.  The canonical state is
 * kept across the call (gathered under the old conditions, stored back under
 * the new ones, which then apply to it).  bc = NULL removes all open
 * boundaries.  Invalid codes
 * or values: LBM_ERR_INVALID, nothing changed.  Contexts with open boundaries
 * have no adjoint (LBM_ERR_UNSUPPORTED).  Synchronises the context's stream. */
int lbm_set_boundaries(lbm_ctx *ctx, const uint8_t *bc, const double *value);

/* Collision model.  magic = 0: BGK (Eqs. 3-6, the default).  magic > 0: the
 * two-relaxation-time collision (a collision model beyond the paper's BGK,
 * which the paper names as future work): each population pair (i, opp(i)) is
 * split into its symmetric and antisymmetric parts; the symmetric parts relax
 * with omega = 1 / tau (so tau sets the viscosity, Eq. 5), the antisymmetric
 * parts with omega_m = 1 / tau_m, tau_m = 1/2 + magic / (tau - 1/2), i.e.
 * magic = (tau - 1/2)(tau_m - 1/2); the forcing term is split the same way.
 * With halfway bounce-back walls, magic = 3/16 puts the walls of a steady
 * channel flow exactly halfway between nodes.  Invalid (negative or not
 * finite): LBM_ERR_INVALID.  Contexts using TRT have no adjoint
 * (LBM_ERR_UNSUPPORTED).  Discards captured step graphs. */
int lbm_set_trt(lbm_ctx *ctx, double magic);

/* Multiple-relaxation-time collision (another collision model beyond the
 * paper's BGK; the moment basis of Lallemand and Luo, 2000).  The populations
 * are mapped to nine orthogonal moments: rho, energy e, energy square eps,
 * momentum j_x, j_y, energy flux q_x, q_y, and the shear moments p_xx, p_xy.
 * Each relaxes towards the moment of f^eq (Eq. 6) at its own rate, with Guo's
 * forcing applied in moment space with the factor (1 - s / 2):
 *   rates  host double[3] = (s_e, s_eps, s_q), each in (0, 2); the shear
 *          moments relax with omega = 1 / tau (the viscosity of Eq. 5), rho
 *          and j are conserved (j gains the force).  NULL switches MRT off
 *          (back to BGK).
 * All rates equal to omega is BGK; s_e = s_eps = omega and
 * s_q = 1 / (1/2 + magic / (tau - 1/2)) is the TRT collision of lbm_set_trt.
 * Selecting MRT switches TRT off and vice versa.  Invalid rates:
 * LBM_ERR_INVALID, nothing changed.  Contexts using MRT have no adjoint
 * (LBM_ERR_UNSUPPORTED).  Discards captured step graphs. */
int lbm_set_mrt(lbm_ctx *ctx, const double *rates);

/* Wall rule.  mode 0: halfway bounce-back (the default; see the conventions
 * above).  mode 1: full-way bounce-back, the boundary nodes of Sec. 4.3 that
 * hold and move populations without computing: a solid node with a fluid
 * neighbour (a "wall node") receives the populations streamed into it,
 * reverses them in the next step instead of colliding, and streams them back,
 * so a population returns to its node two steps after leaving it instead of
 * one (same steady states, different transients).  Under mode 1:
 *  - the canonical state also holds the wall slots: population j of wall node
 *    w, for every j whose source w - c_j is fluid (other solid slots stay 0);
 *    lbm_get_populations returns them, lbm_set_populations reads them (they
 *    must be finite), lbm_mass counts them;
 *  - lbm_init_equilibrium, and switching from mode 0, set wall slot j of w to
 *    population j of the fluid node w - c_j (its value had that node been at
 *    equilibrium in the step before); switching back drops them;
 *  - no extra memory: both lattices of the A-B pair hold state, so DENSE_AA,
 *    raw state checkpoints (lbm_save_state / lbm_load_state and the
 *    checkpointed drivers) and the adjoint return LBM_ERR_UNSUPPORTED.
 * The fluid populations are kept across a switch.  Invalid mode:
 * LBM_ERR_INVALID.  Discards captured step graphs; synchronises the stream. */
int lbm_set_bounce_back(lbm_ctx *ctx, int32_t mode);

/* Replace the body force (host double[2], finite). */
int lbm_set_force(lbm_ctx *ctx, const double *force);

/* Enqueue n >= 0 time steps (Algorithm 1, one fused stream-collide kernel per
 * step).  Asynchronous: returns once enqueued. */
int lbm_step(lbm_ctx *ctx, int64_t n);

/* Replay steps through HIP graphs: lbm_step then enqueues runs of `steps`
 * consecutive steps as one captured graph (captured once, on a private stream,
 * and replayed on the context's stream; bitwise-identical results).  -1 = auto
 * (32 steps for lattices that move less than 128 MB per step, where host launch
 * overhead is a visible share of a step; else off), 0 = off, or an even count in
 * [2, 4096].  The first replay from each parity captures and instantiates its
 * graph (a one-time cost of a few ms).  Changing the force, the drag field or
 * the open boundaries discards captured graphs. */
int lbm_set_graph_steps(lbm_ctx *ctx, int32_t steps);

/* Macroscopic fields (Eq. 2, with the half-force / drag velocity) of the
 * current canonical state into host FP64 [ny][nx] arrays; solid nodes get 0.
 * Any pointer may be NULL.  Synchronises the stream. */
int lbm_macroscopic(lbm_ctx *ctx, double *rho, double *ux, double *uy);

/* Same as lbm_macroscopic into caller-owned device FP64 [ny][nx] buffers
 * (any may be NULL).  Asynchronous. */
int lbm_macroscopic_device(lbm_ctx *ctx, void *rho, void *ux, void *uy);

/* Canonical populations (see the conventions) to / from host FP64 [9][ny][nx].
 * Set ignores solid slots and converts to the storage type (16-bit storage
 * rounds to nearest even).  Both synchronise the stream. */
int lbm_get_populations(lbm_ctx *ctx, double *f);
int lbm_set_populations(lbm_ctx *ctx, const double *f);

/* Total mass sum of rho over fluid nodes (FP64 reduction on the device, fixed
 * summation order, so repeatable).  Synchronises the stream. */
int lbm_mass(lbm_ctx *ctx, double *mass);

/* Raw state checkpoints: bytes of the stored lattice (one lattice for every
 * layout; the step parity of the context is not part of it), and device-to-
 * device copies of it on the context's stream.  A state saved at step t and
 * loaded later reproduces the run from t bitwise (DENSE_AA: load only at a
 * step with the same parity as at save time). */
int lbm_state_bytes(const lbm_ctx *ctx, size_t *bytes);
int lbm_save_state(lbm_ctx *ctx, void *dev_dst);
int lbm_load_state(lbm_ctx *ctx, const void *dev_src);

/* J = mean of u_x over the fluid nodes of column x_col (0 <= x_col < nx),
 * computed in FP64 on the device from the canonical state.  Synchronises.
 * Errors: INVALID if the column has no fluid node. */
int lbm_objective_outlet_ux(lbm_ctx *ctx, int32_t x_col, double *J);

/* ---- Adjoint (reverse mode of the step; DENSE_AB, F64 and F32 only) ------
 * An adjoint field lambda holds 9 values per node of the padded [ny][pitch]
 * mesh in the compute type (FP64 for F64, FP32 for F32), in the library's
 * internal chunked layout: callers treat it as an opaque device buffer of
 * lbm_adjoint_bytes bytes (which also reports the row pitch).
 * lambda_t = dJ / df(t) with f the canonical populations.  Gradients are FP64
 * device buffers owned by the caller and ACCUMULATED into (+=):
 *   grad_alpha_dev [ny][nx], grad_g_dev [2].
 * Every adjoint entry point returns LBM_ERR_UNSUPPORTED for other layouts and
 * types, open boundaries, the TRT collision and the full-way wall rule. */
int lbm_adjoint_bytes(const lbm_ctx *ctx, size_t *bytes, int32_t *pitch);

/* Copy an adjoint field to / from host FP64 [9][ny][nx] (the same indexing as the
 * canonical populations; lambda_t(x)_i = dJ / df_i(x, t)).  Solid entries read as 0
 * and are ignored on input.  Synchronises the stream. */
int lbm_adjoint_get(lbm_ctx *ctx, const void *mu_dev, double *host);
int lbm_adjoint_set(lbm_ctx *ctx, void *mu_dev, const double *host);

/* lambda_T for J = dJ * mean outlet u_x over column x_col, from the current
 * canonical state, written to mu_dev; the direct dJ/dalpha and dJ/dg terms of
 * the objective are added to the gradients. */
int lbm_adjoint_seed_outlet_ux(lbm_ctx *ctx, int32_t x_col, double dJ, void *mu_dev,
                               double *grad_alpha_dev, double *grad_g_dev);

/* One adjoint step: given the raw state saved (lbm_save_state) at step t and
 * lambda_{t+1} in mu_in_dev, write lambda_t to mu_out_dev and add this step's
 * parameter sensitivities to the gradients.  mu_in and mu_out must differ. */
int lbm_adjoint_step(lbm_ctx *ctx, const void *state_t_dev, const void *mu_in_dev,
                     void *mu_out_dev, double *grad_alpha_dev, double *grad_g_dev);

/* lbm_adjoint_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and arguments and bitwise the same results, but the per-block
 * dJ/dg partials and their reduction stage live in a fixed array of 2^17 doubles
 * (1 MiB) that each GPU the library runs on holds until the process ends, so
 * the call allocates nothing (lbm_adjoint_step allocates its partials on first
 * use).  The array fits lattices of up to 16376 row segments of 256 nodes
 * (ceil(nx / 256) * ny <= 16376, e.g. 1024 x 4094 or 2048 x 2047); larger
 * lattices get LBM_ERR_UNSUPPORTED and nothing is launched.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from different host threads) race on it; calls queued on one
 * stream do not.  The first call on a device looks the array up
 * (hipGetSymbolAddress) and may synchronise with that device. */
int lbm_adjoint_step_noalloc(lbm_ctx *ctx, const void *state_t_dev, const void *mu_in_dev,
                             void *mu_out_dev, double *grad_alpha_dev, double *grad_g_dev);

/* Checkpointed forward run: advance T steps from the current state, saving the
 * raw state before steps 0, K, 2K, ... into ckpt_dev (ceil(T / K) slots of
 * lbm_state_bytes each, caller-owned). */
int lbm_run_checkpointed(lbm_ctx *ctx, int64_t T, int64_t K, void *ckpt_dev);

/* Checkpointed adjoint of J = dJ * mean outlet u_x (column x_col) after the T
 * steps of lbm_run_checkpointed: the current state must be the state at T.
 * Segments are replayed from the last to the first: each reloads its
 * checkpoint, recomputes its K states into seg_dev (K slots of state bytes,
 * caller-owned), then runs its adjoint steps backwards.  Gradients accumulate
 * into grad_alpha_dev / grad_g_dev.  The context's state is left at step T. */
int lbm_adjoint_checkpointed(lbm_ctx *ctx, int64_t T, int64_t K, const void *ckpt_dev,
                             void *seg_dev, int32_t x_col, double dJ, double *grad_alpha_dev,
                             double *grad_g_dev);

/* Summary of the context (sizes, fluid count, bytes per step, device memory). */
int lbm_get_info(const lbm_ctx *ctx, lbm_info_t *info);

/* ---- Host-only geometry planning (no device needed) ----------------------
 * Compacted tile list for TILED16: tiles are 16 x 16 nodes; a tile is kept if
 * it holds at least one fluid node; tiles are numbered in row-major tile order.
 *  n_tiles        out: number of kept tiles.
 *  tile_xy        out (may be NULL): int32 [n_tiles][2] tile coordinates (tx, ty).
 *  tile_nbr       out (may be NULL): int32 [n_tiles][9]: entry d is the index of
 *                 the kept tile at (tx + c_d.x, ty + c_d.y) (periodic), -1 if
 *                 that tile is empty; entry 0 is the tile itself.
 * Call with NULL outputs to learn n_tiles first.  Errors: INVALID, UNSUPPORTED
 * (nx or ny not a multiple of 16). */
int lbm_plan_tiles(int32_t nx, int32_t ny, const uint8_t *node_type, int64_t *n_tiles,
                   int32_t *tile_xy, int32_t *tile_nbr);

/* Compacted fluid list for INDIRECT: fluid nodes in row-major order.
 *  n_fluid   out: number of fluid nodes.
 *  fluid_xy  out (may be NULL): int32 [n_fluid][2] node coordinates.
 *  nbr       out (may be NULL): int32 [8][n_fluid]: nbr[i-1][n] is the index of
 *            the fluid node at x_n - c_i (periodic) for i = 1..8, or -1 when that
 *            node is solid (the population bounces back).
 * Call with NULL outputs to learn n_fluid first. */
int lbm_plan_indirect(int32_t nx, int32_t ny, const uint8_t *node_type, int64_t *n_fluid,
                      int32_t *fluid_xy, int32_t *nbr);

/* ---- Measurement aid ---------------------------------------------------------
 * Device copy kernel with the same access width as the step kernels, used to
 * calibrate the achievable DRAM bandwidth (the copy experiment of Sec. 4.2).
 * Copies `bytes` (a multiple of 16) from src to dst on `hip_stream`. */
int lbm_copy_kernel(const void *src, void *dst, size_t bytes, void *hip_stream);

/* Static description of a status code; never NULL. */
const char *lbm_error_string(int status);
/* Message of the last failure on ctx; with ctx == NULL, the calling thread's
 * last failure outside a context (e.g. lbm_create).  Never NULL. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Release the context and every device buffer it holds (NULL is a no-op). */
void lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
