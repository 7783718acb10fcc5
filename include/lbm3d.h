/*
 * lbm3d.h - C ABI of the D3Q19 lattice of the MI355X (gfx950) lattice-Boltzmann
 * library.
 *
 * The paper (Tomczak, arXiv 2108.13241) names the three-dimensional lattice as
 * its future work (Sec. 6).  This interface runs the same update as lbm.h in 3D:
 * the fused pull stream-and-collide step of Algorithm 1 with halfway bounce-back
 * walls (Sec. 3), the BGK operator of Eqs. 3-5 and the equilibrium of Eq. 6 with
 * the D3Q19 weights, plus a body force through Guo's forcing term and, as
 * options, the two- and multiple-relaxation-time collisions and the full-way
 * wall rule.  Four layouts, as lbm.h's: DENSE_AB, two dense lattices swapped
 * every step, and DENSE_AA, one dense lattice updated in place with the AA
 * access pattern (even steps read and write each node's own slots, odd steps
 * read from and write to the neighbours; half the memory); INDIRECT, a sparse
 * layout: two lattices holding the fluid nodes only (row-major order) with a
 * per-node table of the 18 pull sources (the fluid-index-array approach of
 * lbm.h's INDIRECT, Sec. 1); and TILED16, the tiled sparse layout of Sec. 4.3
 * cut for three dimensions: the mesh in 4 x 4 x 4-node blocks (64 nodes, one
 * wavefront), only the blocks that hold a fluid node stored (TILED16_ALL: all
 * blocks), each block's 19 directions as contiguous runs of 64, with an
 * 18-entry block-neighbour table per block.
 *
 * Conventions (as in lbm.h, whose status codes, dtype enum and allocator hook
 * this interface shares)
 *  - Every call returns an lbm_status (0 = LBM_OK); nothing aborts or throws.
 *    On LBM_ERR_INVALID / LBM_ERR_UNSUPPORTED nothing changed.  A device
 *    failure returns LBM_ERR_DEVICE and marks the context broken (later calls
 *    return LBM_ERR_STATE).  lbm3d_last_error() explains the failure.
 *  - Host arrays are owned by the caller and only read (or written) during the
 *    call.  3-D fields are row-major [nz][ny][nx] (x fastest), no padding.
 *  - Node types: 0 = fluid, 1 = solid.  All three axes are periodic; walls come
 *    only from solid nodes.  A population that would stream into a solid node
 *    returns to its origin node reversed in the same step (halfway bounce-back).
 *  - Velocities: 0 rest; 1..6 the axis directions +x, -x, +y, -y, +z, -z;
 *    7..18 the edge directions in opposite pairs (+x+y, -x-y), (+x-y, -x+y),
 *    (+x+z, -x-z), (+x-z, -x+z), (+y+z, -y-z), (+y-z, -y+z).  Weights 1/3 (rest),
 *    1/18 (axes), 1/36 (edges).
 *  - "Canonical" populations are the pre-collision values f_i(x, t) as FP64
 *    [19][nz][ny][nx]; solid slots = 0 (full-way rule: see
 *    lbm3d_set_bounce_back).
 *  - dtype: LBM_F64 stores and computes in FP64; LBM_F32, LBM_F16_SHIFTED and
 *    LBM_BF16_SHIFTED store the deviation f_i - w_i in 32 or 16 bits and compute
 *    in FP32 on the deviations.
 *  - A context is not thread-safe; work is enqueued on its stream, and calls
 *    that return host data synchronise that stream.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d_ctx lbm3d_ctx; /* opaque; owned by the library until lbm3d_destroy */

typedef struct {
    int32_t nx, ny, nz;
    int32_t dtype;
    int32_t layout;              /* LBM_DENSE_AB, LBM_DENSE_AA, LBM_INDIRECT,
                                    LBM_TILED16 or LBM_TILED16_ALL */
    int64_t n_nodes;             /* nx * ny * nz */
    int64_t n_fluid;             /* fluid nodes: the ones counted for LUPS (Eq. 8) */
    int64_t time_step;           /* steps since the last (re)initialisation */
    int32_t pop_bytes;           /* bytes per stored population: 8, 4 or 2 */
    double bytes_per_fluid_node; /* algorithmic bytes per fluid node per step:
                                    38 * pop_bytes + 1 (node type; INDIRECT:
                                    + 36 instead, the source table: eight
                                    row ranks and the solid bits; TILED16:
                                    + 88 / 64, the block table and fluid
                                    bits per stored node) */
    size_t device_bytes;         /* device memory held by the context */
} lbm3d_info_t;

/* Create a D3Q19 lattice (Eq. 5: omega = 1 / tau), at rest (rho = 1, u = 0),
 * on the current HIP device and its default stream.
 *  nx, ny, nz  mesh size, >= 1 each; with pitch = nx rounded up to 64,
 *              nz * ny * pitch must stay below 2^31 nodes and 19 * pitch below
 *              2^28.  Population offsets are 64-bit, so the bound is the
 *              device's memory: an A-B pair takes 38 * pop_bytes per node
 *              (FP32: about 1.8 G nodes in 288 GB).  Creation writes the rest
 *              state in place; initialisation from fields and population
 *              transfers stage 152 B per node of FP64 for their duration.
 *  node_type   host uint8 [nz][ny][nx], 0 fluid / 1 solid; copied.
 *  tau         relaxation time > 1/2 (nu = (tau - 1/2) / 3).
 *  force       host double[3] body-force acceleration (g_x, g_y, g_z); NULL = 0.
 *              Force density F = rho g through Guo's forcing term.
 *  dtype       storage type (see above).
 *  layout      LBM_DENSE_AB, LBM_DENSE_AA (one lattice: 19 * pop_bytes per
 *              node, half of DENSE_AB) or LBM_INDIRECT (fluid nodes only:
 *              38 * pop_bytes + 48 bytes per fluid node: two lattices, the
 *              compact source table (eight row ranks, the solid bits) and the
 *              coordinates, plus 72 bytes per fluid node at x = 0 or nx - 1,
 *              whose 18 sources are listed in full), LBM_TILED16 (4 x 4 x 4
 *              blocks holding a fluid node, nx, ny and nz multiples of 4:
 *              38 * pop_bytes * 64 bytes per stored block for the two
 *              lattices, plus 100 bytes of block table, fluid bits and
 *              coordinates) or LBM_TILED16_ALL (the same with every block).
 * Errors: INVALID (sizes, tau, force, mask values, dtype, layout), UNSUPPORTED
 * (size limit, block layout on sizes that are not multiples of 4), NOMEM,
 * DEVICE. */
int lbm3d_create(lbm3d_ctx **out, int32_t nx, int32_t ny, int32_t nz, const uint8_t *node_type,
                 double tau, const double *force, lbm_dtype dtype, lbm_layout layout);

/* Enqueue later work on `hip_stream` (NULL = default stream), after waiting for
 * the work already enqueued. */
int lbm3d_set_stream(lbm3d_ctx *ctx, void *hip_stream);

/* Reset to the equilibrium (Eq. 6) of host FP64 [nz][ny][nx] fields; any field
 * may be NULL (rho = 1, u = 0; all four NULL: the rest state f_i = w_i, written
 * in place without a staging buffer).  rho > 0 and finite values at fluid
 * nodes. */
int lbm3d_init_equilibrium(lbm3d_ctx *ctx, const double *rho, const double *ux,
                           const double *uy, const double *uz);

/* Change the body-force acceleration (host double[3], finite). */
int lbm3d_set_force(lbm3d_ctx *ctx, const double *force);

/* Collision model, as lbm_set_trt: magic = 0 BGK (the default); magic > 0 the
 * two-relaxation-time collision, whose pair-wise symmetric parts relax with
 * omega = 1 / tau and antisymmetric parts with omega_m = 1 / tau_m,
 * tau_m = 1/2 + magic / (tau - 1/2) (forcing split alike).  Invalid (negative
 * or not finite): LBM_ERR_INVALID. */
int lbm3d_set_trt(lbm3d_ctx *ctx, double magic);

/* Multiple-relaxation-time collision in the D3Q19 moment basis of d'Humieres,
 * Ginzburg, Krafczyk, Lallemand and Luo (2002): nineteen orthogonal moments
 * (rho; energy e; energy square eps; momentum j; energy flux q; the shear
 * moments 3p_xx, p_ww, p_xy, p_yz, p_xz; the fourth-order pi_xx, pi_ww; the
 * third-order m), each relaxing towards the moment of f^eq (Eq. 6) at its own
 * rate, with Guo's forcing in moment space (factor 1 - s / 2):
 *   rates  host double[5] = (s_e, s_eps, s_q, s_pi, s_m), each in (0, 2); the
 *          shear moments relax with omega = 1 / tau (Eq. 5), rho and j are
 *          conserved (j gains the force).  NULL switches MRT off (BGK).
 * All rates omega is BGK; s_e = s_eps = s_pi = omega and s_q = s_m =
 * 1 / (1/2 + magic / (tau - 1/2)) is the TRT collision.  MRT and TRT exclude
 * each other (the last call wins).  Invalid rates: LBM_ERR_INVALID. */
int lbm3d_set_mrt(lbm3d_ctx *ctx, const double *rates);

/* Wall rule, as lbm_set_bounce_back: 0 halfway (the default), 1 full-way (solid
 * nodes next to fluid hold the populations streamed into them, reverse them in
 * the next step and stream them back).  Under mode 1 the canonical state also
 * holds the wall slots (population j of wall node w for every j whose source
 * w - c_j is fluid): lbm3d_get_populations returns them, lbm3d_set_populations
 * reads them (finite), lbm3d_mass counts them; lbm3d_init_equilibrium and a
 * switch from mode 0 set slot j of w to population j of the fluid node
 * w - c_j.  The fluid populations are kept across a switch.  No extra memory
 * (the A-B pair holds the state).  Invalid mode: LBM_ERR_INVALID; mode 1 on a
 * DENSE_AA lattice: LBM_ERR_UNSUPPORTED (in place, no lattice holds the values
 * of two steps back).  Synchronises the stream. */
int lbm3d_set_bounce_back(lbm3d_ctx *ctx, int32_t mode);

/* Enqueue n >= 0 time steps (one kernel launch each). */
int lbm3d_step(lbm3d_ctx *ctx, int64_t n);

/* rho and u = m / rho + g / 2 (Eq. 2 with the half-force correction) into host
 * FP64 [nz][ny][nx] arrays (any may be NULL); solid nodes get 0.  Synchronises. */
int lbm3d_macroscopic(lbm3d_ctx *ctx, double *rho, double *ux, double *uy, double *uz);

/* Same fields into caller-owned device FP64 [nz][ny][nx] buffers (all four
 * required; solid nodes get 0), on the context's stream.  Asynchronous. */
int lbm3d_macroscopic_device(lbm3d_ctx *ctx, void *rho, void *ux, void *uy, void *uz);

/* Raw device checkpoints of the stored state: lbm3d_state_bytes bytes
 * (19 * nz * ny * pitch * pop_bytes), copied on the context's stream to / from a
 * caller-owned device buffer.  A state saved at step t and loaded later
 * reproduces the run from t bitwise (DENSE_AA: load only at a step count of the
 * same parity as at save time).  Under the full-way rule the state spans both
 * lattices: LBM_ERR_UNSUPPORTED. */
int lbm3d_state_bytes(const lbm3d_ctx *ctx, size_t *bytes);
int lbm3d_save_state(lbm3d_ctx *ctx, void *dev_dst);
int lbm3d_load_state(lbm3d_ctx *ctx, const void *dev_src);

/* Canonical populations to / from host FP64 [19][nz][ny][nx].  set requires
 * finite values at fluid nodes (solid slots are ignored) and rounds to the
 * storage type.  Both synchronise. */
int lbm3d_get_populations(lbm3d_ctx *ctx, double *f);
int lbm3d_set_populations(lbm3d_ctx *ctx, const double *f);

/* Total mass (sum of rho over fluid nodes) in a fixed summation order on the
 * device.  Synchronises. */
int lbm3d_mass(lbm3d_ctx *ctx, double *mass);

int lbm3d_get_info(const lbm3d_ctx *ctx, lbm3d_info_t *info);

/* Message of the last failure on ctx; with ctx == NULL, the calling thread's
 * last failure outside a context (e.g. lbm3d_create).  Never NULL. */
const char *lbm3d_last_error(const lbm3d_ctx *ctx);

/* Release the context and its device buffers (NULL is a no-op). */
void lbm3d_destroy(lbm3d_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */
