// Internal interface between the D3Q19 host runtime (lbm3d_runtime.cpp) and
// its HIP kernels (lbm3d_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {
// The process-wide device allocator registered with lbm_set_allocator (both
// NULL: hipMalloc / hipFree).
void current_allocator(lbm_alloc_fn *alloc, lbm_free_fn *free_fn, void **user);
}  // namespace lbm

namespace lbm3 {

// Device state of a D3Q19 context.  Populations: [nz][ny][pitch/64][19][64]
// (chunks of 64 nodes along x, 19 runs of 64 each); types, neighbour bits and
// canonical planes use the padded node index (z * ny + y) * pitch + x.
struct State3 {
    int dtype = 0;
    int nx = 0, ny = 0, nz = 0;
    int pitch = 0;                           // nx rounded up to a multiple of 64
    void *f[2] = {nullptr, nullptr};         // the two lattices (A-B); DENSE_AA: f[0] only
    int aa = 0;                              // 1: DENSE_AA, one lattice updated in place
    // INDIRECT (list = 1): fluid nodes only, in row-major order; populations
    // [np/64][19][64] (np = n_fluid rounded up to 64); the compact source table
    // (rank8 [8][np], info [np], edge [18][ne] for the border nodes; see
    // pull_list); fxyz[3 n + {0, 1, 2}] = the node's coordinates.
    int list = 0;
    int64_t n_fluid = 0, np = 0, ne = 1;
    const int32_t *rank8 = nullptr;
    const uint32_t *info = nullptr;
    const int32_t *edge = nullptr;
    const int32_t *fxyz = nullptr;
    // TILED16 (blocks = 1): 4 x 4 x 4-node blocks holding a fluid node (all
    // blocks with TILED16_ALL); populations [n_blocks][19][64], slot l = lx +
    // 4 ly + 16 lz; bmeta [n_blocks][20] (the 18 neighbour block indices,
    // n_blocks for a dropped block, and the all-fluid flag), bfluid [n_blocks + 1]
    // (fluid bits per slot; entry n_blocks = 0), bxyz [n_blocks][3] (block
    // coordinates).  See lbm::plan::blocks4.
    int blocks = 0;
    int64_t n_blocks = 0;
    const uint32_t *bmeta = nullptr;
    const uint64_t *bfluid = nullptr;
    const int32_t *bxyz = nullptr;
    const uint8_t *type = nullptr;           // 0 fluid, 1 solid, 2 fluid next to a solid
    const uint32_t *nmask = nullptr;         // bit i-1 set <=> node x - c_i is solid
    const uint32_t *seg_interior = nullptr;  // per 256-node row segment: 1 = all type 0
    double interior_frac = 0.0;              // fraction of all-interior segments (blocks)
    double omega = 1.0, gx = 0.0, gy = 0.0, gz = 0.0;
    int trt = 0;                             // 1: two-relaxation-time collision
    double omega_m = 1.0;                    // its antisymmetric relaxation rate
    int mrt = 0;                             // 1: multiple-relaxation-time collision
    double s_e = 1.0, s_eps = 1.0, s_q = 1.0, s_pi = 1.0, s_m = 1.0;  // its rates
    int fullway = 0;                         // 1: full-way bounce-back
    hipStream_t stream = nullptr;
    double *red = nullptr;                   // reduction scratch (reduction_capacity3 doubles)
};

// One step from lattice cur into lattice 1 - cur.  DENSE_AA (s.aa): one lattice,
// and cur is the parity of the steps taken so far (0: even, the canonical state
// is local; the runtime flips it after every step as for A-B).  The view,
// scatter and macro launches read cur the same way.
hipError_t launch_step3(const State3 &s, int cur);
// Equilibrium of device FP64 [nz][ny][nx] fields (NULL: rho = 1, u = 0) into the
// canonical buffer fc (FP64 [19][nz][ny][pitch]).
hipError_t launch_equilibrium3(const State3 &s, const double *rho, const double *ux,
                               const double *uy, const double *uz, double *fc);
// Rest state (rho = 1, u = 0) straight into one stored lattice, without a
// canonical staging buffer.
hipError_t launch_rest3(const State3 &s, void *lattice);
// Canonical fc -> stored lattice cur (full-way rule: also the other lattice's
// bounce-back slots; with fill_walls the wall slots come from the fluid nodes
// that feed them instead of from fc).
hipError_t launch_scatter3(const State3 &s, int cur, const double *fc, int fill_walls);
// Stored lattice cur -> canonical fc at fluid nodes and (full-way rule) wall
// slots; other slots untouched.
hipError_t launch_gather3(const State3 &s, int cur, double *fc);
// Macroscopic fields of fluid nodes into FP64 [nz][ny][nx] buffers (rho may be
// NULL to skip them; other entries untouched) and, when mass is non-NULL, the
// total mass (full-way rule: wall slots included) into *mass (device) through
// fixed-order sums in s.red.
hipError_t launch_macro3(const State3 &s, int cur, double *rho, double *ux, double *uy, double *uz,
                         double *mass);
int64_t reduction_capacity3(const State3 &s);

}  // namespace lbm3
