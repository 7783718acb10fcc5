// Internal interface between the host runtime (lbm_runtime.cpp) and the HIP
// kernels (lbm_kernels.hip, lbm_adjoint.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

enum Dtype : int { kF64 = 0, kF32 = 1, kF16S = 2, kBF16S = 3 };
enum Layout : int { kDenseAB = 0, kDenseAA = 1, kTiled16 = 2, kIndirect = 3 };

constexpr int kTile = 16;
constexpr int kTileNodes = kTile * kTile;

// Per-tile scalars of the tiled step, one 128-byte row per kept tile: the
// tile-neighbour row (as tile_nbr; entry 0 = the tile itself) and, per 64-slot
// wavefront w, its fluid lanes (bit l of fluid[w] <=> slot 64 w + l is fluid).
struct alignas(128) TileMeta {
    int32_t nbr[9];
    int32_t pad[7];
    uint64_t fluid[4];
    uint64_t pad2[4];
};
static_assert(sizeof(TileMeta) == 128, "one 128-byte row per tile");

// Everything a kernel launch needs to know about a context's device state.
struct DevState {
    int dtype = 0, layout = 0;
    int nx = 0, ny = 0;
    int pitch = 0;        // dense: row pitch in elements (multiple of 64)
    size_t plane = 0;     // elements per population plane of one lattice
    void *f[2] = {nullptr, nullptr};  // lattices (f[1] unused by DENSE_AA)
    const uint8_t *type = nullptr;    // node-type codes (dense / tiled)
    const uint8_t *nmask = nullptr;   // solid-neighbour bits (dense / tiled)
    const uint32_t *seg_interior = nullptr;  // dense: per 256-node row segment, 1 = all interior
    double interior_frac = 0.0;       // dense: fraction of the segments that are all interior
    const float *alpha = nullptr;     // drag coefficient, same indexing as type
                                      // (INDIRECT: per compacted node); may be null
    const int32_t *tile_xy = nullptr, *tile_nbr = nullptr;  // TILED16
    const TileMeta *tile_meta = nullptr;  // TILED16: [n_tiles], the step's per-tile scalars
    const int32_t *fluid_xy = nullptr;                      // INDIRECT: [n][2]
    const uint32_t *ind_pk = nullptr;                       // INDIRECT: packed row offsets
    const uint16_t *ind_info = nullptr;                     // INDIRECT: solid bits + edge flag
    const int32_t *ind_edge = nullptr;                      // INDIRECT: edge-node table [][8]
    const double *bc_val = nullptr;   // open-boundary values [node][2], same indexing as
                                      // alpha; read only at open-boundary nodes
    int open = 0;                     // 1 when the node types hold open-boundary codes
    int trt = 0;                      // 1: two-relaxation-time collision (omega_m below)
    int fullway = 0;                  // 1: full-way bounce-back (A-B layouts)
    double omega_m = 1.0;             // antisymmetric relaxation rate (TRT)
    int mrt = 0;                      // 1: multiple-relaxation-time collision
    double s_e = 1.0, s_eps = 1.0, s_q = 1.0;  // its energy, energy-square, flux rates
    int64_t n_tiles = 0, n_fluid = 0;
    double omega = 1.0, gx = 0.0, gy = 0.0;
    hipStream_t stream = nullptr;
    double *red_partials = nullptr;   // reduction scratch (>= red_capacity doubles)
    int64_t red_capacity = 0;
};

// Number of thread blocks the visit / reduction kernels use for this layout.
int64_t visit_blocks(const DevState &s);
// Doubles of reduction scratch (red_partials) a reduction needs: one partial per
// visit block plus the first-stage sums.
int64_t reduction_capacity(const DevState &s);

// One time step from lattice `cur` (A-B layouts write lattice 1 - cur).  For
// DENSE_AA, t is the number of steps already taken (its parity picks the
// even or odd kernel).
hipError_t launch_step(const DevState &s, int64_t t, int cur);

// Canonical populations fc (device FP64 [9][ny][pitch]) -> stored state at step t.
// Full-way rule: fc's wall slots become the populations in flight; with
// fill_walls they are taken instead from the fluid node each slot is fed by
// (slot j of wall node w <- f_j(w - c_j)).
hipError_t launch_scatter_canonical(const DevState &s, int64_t t, int cur, const double *fc,
                                    int fill_walls);
// Rest state (rho = 1, u = 0) straight into one stored lattice (all 9 * plane
// slots), without a canonical staging buffer.
hipError_t launch_rest(const DevState &s, void *lattice);
// Equilibrium (Eq. 6) from device FP64 [ny][nx] fields (null = rest) -> fc.
hipError_t launch_equilibrium(const DevState &s, const double *rho, const double *ux,
                              const double *uy, double *fc);
// Stored state -> canonical fc (solid slots untouched: clear them first).
hipError_t launch_gather_canonical(const DevState &s, int64_t t, int cur, double *fc);
// Macroscopic fields of fluid nodes (solid entries untouched).
hipError_t launch_macroscopic(const DevState &s, int64_t t, int cur, double *rho, double *ux,
                              double *uy);
// Deterministic FP64 sums over fluid nodes into *out (device): total mass, or
// the sum of u_x over the fluid nodes of column x_col.
hipError_t launch_mass(const DevState &s, int64_t t, int cur, double *out);
hipError_t launch_column_ux(const DevState &s, int64_t t, int cur, int x_col, double *out);

hipError_t launch_fill(double *p, size_t n, double v, hipStream_t stream);
hipError_t launch_copy16(const void *src, void *dst, size_t bytes, hipStream_t stream);

// ---- adjoint (DENSE_AB, F64 / F32) --------------------------------------
// Adjoint fields are dense [9][ny][pitch] in the compute type.  dJ/dg block
// partials are pairs (x, y) per block.
int64_t adjoint_blocks(const DevState &s);       // blocks of one adjoint step
int64_t adjoint_step_partials(const DevState &s);  // dJ/dg partial pairs of one adjoint step
// Pairs of adjoint scratch needed: the partials of a step or seed plus the
// first-stage sums of launch_partials_into (written right after the partials).
int64_t adjoint_scratch_pairs(const DevState &s);
int64_t adjoint_seed_blocks(const DevState &s);  // blocks of the seed kernel
// lambda_T of J = scale * sum of u_x over the fluid nodes of column x_col, read
// from the stored lattice `state`; direct dJ/dalpha terms into grad_alpha (if
// a drag field is set) and dJ/dg partials (one pair per seed block).
hipError_t launch_adjoint_seed_raw(const DevState &s, const void *state, int x_col, double scale,
                                   void *mu, double *grad_alpha, double *partials);
// One reverse step: state = stored lattice at step t, mu_in = lambda_{t+1};
// writes lambda_t, adds to grad_alpha, writes (accumulate = 0) or adds
// (accumulate = 1) the per-block dJ/dg partials.
hipError_t launch_adjoint_step_raw(const DevState &s, const void *state, const void *mu_in,
                                   void *mu_out, double *grad_alpha, double *partials,
                                   int accumulate);
// Adjoint field <-> device FP64 planes [9][ny][nx] (to_plain = 1: field -> planes).
hipError_t launch_adjoint_convert(const DevState &s, void *mu, double *plain, int to_plain);
// grad_g[0..1] += fixed-order sum of n partial pairs.
hipError_t launch_partials_into(double *partials, int64_t n, double *grad_g,
                                hipStream_t stream);
hipError_t launch_zero(double *p, int64_t n, hipStream_t stream);
// Allocation-free adjoint step: its dJ/dg partials live in a fixed per-device
// array of kNoAllocScratchDoubles doubles (1 MiB).  adjoint_step_scratch_doubles
// = the doubles one step needs there (partials plus reduction stage);
// noalloc_scratch = that array's device address on `device` (looked up once
// per device with hipGetSymbolAddress, then cached).
constexpr int64_t kNoAllocScratchDoubles = int64_t(1) << 17;
int64_t adjoint_step_scratch_doubles(const DevState &s);
hipError_t noalloc_scratch(int device, double **ptr);

}  // namespace lbm
