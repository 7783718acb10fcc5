// HIP kernels of the D3Q19 lattice (the three-dimensional lattice the paper
// names as future work): the fused pull stream-and-collide step of
// Algorithm 1 with halfway or full-way bounce-back walls, the BGK collision
// (Eqs. 3-6 with the D3Q19 weights) or its TRT / MRT variants, and Guo body
// forcing, on the dense two-lattice (A-B) layout (per node, or staged through
// LDS per row segment), the in-place AA layout, the sparse fluid-node list and
// the sparse 4 x 4 x 4-block tiled layout; plus initialisation, canonical views
// and FP64 reductions.
//
// Dense layout: [nz][ny][pitch/64][19][64] (chunks of 64 nodes along x, each
// holding its 19 populations as runs of 64); node types and solid-neighbour
// bits per node [nz][ny][pitch]; one "all interior" flag per 256-node row
// segment.
#include "lbm3d_launch.h"
#include "lbm_device.h"

namespace lbm3 {
namespace {

using lbm::kChunk;
using lbm::store_nt;
using lbm::xcd_remap;
using lbm::wrap_dec;
using lbm::wrap_inc;
constexpr int kBlock = 256;
constexpr int Q = 19;

// Velocities: rest; axes +x, -x, +y, -y, +z, -z; edges as opposite pairs
// (+x+y, -x-y), (+x-y, -x+y), (+x+z, -x-z), (+x-z, -x+z), (+y+z, -y-z),
// (+y-z, -y+z).  opp(i) = i + 1 for odd i, i - 1 for even i > 0.
__device__ constexpr int kCx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int kCy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int kCz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__device__ constexpr int kOpp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// Weights of Eq. 6 for D3Q19: 1/3 at rest, 1/18 on the axes, 1/36 on the edges.
__device__ constexpr double kW[Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                     1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

enum : uint8_t { kFluid = 0, kSolid = 1, kBoundary = 2 };

// Storage codecs: FP64 stores f_i; the narrow formats store the deviation
// h_i = f_i - w_i (rho0 = 1) and the collision works on h_i (FP32 arithmetic).
struct F64 {
    using mem = double;
    using real = double;
    static constexpr bool kShift = false;
    static __device__ __forceinline__ real ld(mem v, int) { return v; }
    static __device__ __forceinline__ mem st(real v, int) { return v; }
    static __device__ __forceinline__ double canon(real v, int) { return v; }
    static __device__ __forceinline__ mem from_canon(double f, int) { return f; }
};
template <class M>
struct Shifted {
    using mem = M;
    using real = float;
    static constexpr bool kShift = true;
    static __device__ __forceinline__ real ld(mem v, int) { return (float)v; }
    static __device__ __forceinline__ mem st(real v, int)
    {
        if constexpr (sizeof(M) == 2)
            asm volatile("" : "+v"(v));  // round to FP32 first, identically everywhere
        return (mem)v;
    }
    static __device__ __forceinline__ double canon(real v, int i) { return (double)v + kW[i]; }
    static __device__ __forceinline__ mem from_canon(double f, int i)
    {
        return (mem)(float)(f - kW[i]);
    }
};

__device__ __forceinline__ double recip(double v) { return 1.0 / v; }
__device__ __forceinline__ float recip(float v)
{
    const float r = __builtin_amdgcn_rcpf(v);
    return __builtin_fmaf(__builtin_fmaf(-v, r, 1.0f), r, r);
}

// c . v for the first direction of pair k: (1,0,0), (0,1,0), (0,0,1), (1,1,0),
// (1,-1,0), (1,0,1), (1,0,-1), (0,1,1), (0,1,-1), without multiplications.
template <class R>
__device__ __forceinline__ R pair_dot(int k, R vx, R vy, R vz)
{
    switch (k) {
    case 0: return vx;
    case 1: return vy;
    case 2: return vz;
    case 3: return vx + vy;
    case 4: return vx - vy;
    case 5: return vx + vz;
    case 6: return vx - vz;
    case 7: return vy + vz;
    default: return vy - vz;
    }
}

// BGK collision with Guo forcing (F = rho g) at one node, in place:
//   f_i <- f_i - omega (f_i - f^eq_i) + (1 - omega/2) S_i,
// u = m / rho + g / 2, f^eq of Eq. 6 with the D3Q19 weights,
// S_i = w_i [3 (c_i - u) . F + 9 (c_i . u)(c_i . F)].  Opposite directions
// share everything but the terms odd in c, so they are updated as a pair; with
// SHIFT, f holds deviations and rho = 1 + sum is never rounded (rho v = v + sum v).
// TRT: the pair's symmetric part P = (f_i + f_opp)/2 relaxes with omega and its
// antisymmetric part M = (f_i - f_opp)/2 with omega_m (forcing split alike);
// f_i = P + M, f_opp = P - M.
// MRT: multiple-relaxation-time collision in the D3Q19 moment basis of
// d'Humieres et al. (rows, as polynomials of c: rho 1; e 19|c|^2 - 30;
// eps (21|c|^4 - 53|c|^2 + 24)/2; j c; q (5|c|^2 - 9) c; 3p_xx 3c_x^2 - |c|^2;
// 3pi_xx (3|c|^2 - 5)(3c_x^2 - |c|^2); p_ww c_y^2 - c_z^2; pi_ww (3|c|^2 - 5)
// (c_y^2 - c_z^2); p_xy, p_yz, p_xz; m_x (c_y^2 - c_z^2) c_x, m_y (c_z^2 - c_x^2)
// c_y, m_z (c_x^2 - c_y^2) c_z; orthogonal, squared norms kMrt3Norm).  The
// moments of d = f - f^eq and of the forcing term relax as
//   Delta_k = s_k d_k - (1 - s_k / 2) S_k,  f_i <- f_i - sum_k M_ki Delta_k / |M_k|^2,
// with s_e, s_eps, s_q, s_pi, s_m and omega on the shear moments (3p_xx, p_ww,
// p_xy, p_yz, p_xz); Delta_rho = 0 and Delta_j = -F (the conserved moments).
template <class R>
struct Rates3 {
    R omega_m;                         // TRT: antisymmetric rate
    R s_e, s_eps, s_q, s_pi, s_m;      // MRT
};

// Row k of the D3Q19 MRT matrix at direction i (small integers); with the
// loops unrolled every coefficient folds to a constant.
__device__ __forceinline__ constexpr int mrt3_coef(int k, int i)
{
    const int cx = kCx[i], cy = kCy[i], cz = kCz[i], c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return cx;
    case 4: return (5 * c2 - 9) * cx;
    case 5: return cy;
    case 6: return (5 * c2 - 9) * cy;
    case 7: return cz;
    case 8: return (5 * c2 - 9) * cz;
    case 9: return 3 * cx * cx - c2;
    case 10: return (3 * c2 - 5) * (3 * cx * cx - c2);
    case 11: return cy * cy - cz * cz;
    case 12: return (3 * c2 - 5) * (cy * cy - cz * cz);
    case 13: return cx * cy;
    case 14: return cy * cz;
    case 15: return cx * cz;
    case 16: return (cy * cy - cz * cz) * cx;
    case 17: return (cz * cz - cx * cx) * cy;
    default: return (cx * cx - cy * cy) * cz;
    }
}
__device__ constexpr int kMrt3Norm[Q] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36,
                                         72, 12,   24,  4,  4,  4,  8,  8,  8};

template <class R, bool SHIFT, bool FORCE, bool TRT = false, bool MRT = false>
__device__ __forceinline__ void collide3(R (&f)[Q], R omega, R gx, R gy, R gz,
                                         const Rates3<R> &rt = Rates3<R>{})
{
    const R omega_m = rt.omega_m;
    R sum = f[0];
#pragma unroll
    for (int i = 1; i < Q; ++i)
        sum += f[i];
    R mx = R(0), my = R(0), mz = R(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const R d = f[i] - f[i + 1];
        if (kCx[i] > 0) mx += d; else if (kCx[i] < 0) mx -= d;
        if (kCy[i] > 0) my += d; else if (kCy[i] < 0) my -= d;
        if (kCz[i] > 0) mz += d; else if (kCz[i] < 0) mz -= d;
    }
    auto rho_times = [&](R v) -> R {
        if constexpr (SHIFT)
            return v + sum * v;
        else
            return sum * v;
    };
    R ux, uy, uz;
    if constexpr (SHIFT) {
        const R q = sum * recip(R(1) + sum);
        ux = mx - mx * q;
        uy = my - my * q;
        uz = mz - mz * q;
    } else {
        const R inv = recip(sum);
        ux = mx * inv;
        uy = my * inv;
        uz = mz * inv;
    }
    R Fx = R(0), Fy = R(0), Fz = R(0);
    if constexpr (FORCE) {
        ux += R(0.5) * gx;
        uy += R(0.5) * gy;
        uz += R(0.5) * gz;
        Fx = rho_times(gx);
        Fy = rho_times(gy);
        Fz = rho_times(gz);
    }
    const R usq = R(1.5) * (ux * ux + uy * uy + uz * uz);
    const R C0 = SHIFT ? sum - rho_times(usq) : rho_times(R(1) - usq);
    const R keep = R(1) - omega, guo = R(1) - R(0.5) * omega;
    const R uF = ux * Fx + uy * Fy + uz * Fz;
    if constexpr (MRT) {
        R d[Q], sg[Q];
        d[0] = f[0] - R(kW[0]) * C0;
        sg[0] = FORCE ? R(kW[0]) * (R(-3) * uF) : R(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int i = 2 * k + 1, j = i + 1;
            const R w = R(kW[i]);
            const R cu = pair_dot(k, ux, uy, uz);
            const R even = w * (C0 + rho_times(R(4.5) * (cu * cu)));
            const R odd = w * rho_times(R(3) * cu);
            d[i] = f[i] - (even + odd);
            d[j] = f[j] - (even - odd);
            if constexpr (FORCE) {
                const R cF = pair_dot(k, Fx, Fy, Fz);
                const R se = w * (R(9) * cu * cF - R(3) * uF);
                const R so = R(3) * w * cF;
                sg[i] = se + so;
                sg[j] = se - so;
            } else {
                sg[i] = sg[j] = R(0);
            }
        }
        // Delta_k / |M_k|^2 for every row (conserved rows set directly)
        R del[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            if (k == 0) {
                del[k] = R(0);
                continue;
            }
            if (k == 3 || k == 5 || k == 7) {
                const R Fk = k == 3 ? Fx : k == 5 ? Fy : Fz;
                del[k] = FORCE ? -Fk * R(1.0 / kMrt3Norm[k]) : R(0);
                continue;
            }
            R dk = R(0), sk = R(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int c = mrt3_coef(k, i);
                if (c == 1) {
                    dk += d[i];
                    if constexpr (FORCE) sk += sg[i];
                } else if (c == -1) {
                    dk -= d[i];
                    if constexpr (FORCE) sk -= sg[i];
                } else if (c != 0) {
                    dk += R(c) * d[i];
                    if constexpr (FORCE) sk += R(c) * sg[i];
                }
            }
            const R sr = k == 1 ? rt.s_e : k == 2 ? rt.s_eps
                       : (k == 4 || k == 6 || k == 8) ? rt.s_q
                       : (k == 10 || k == 12) ? rt.s_pi
                       : (k >= 16) ? rt.s_m : omega;
            R dl = sr * dk;
            if constexpr (FORCE)
                dl -= (R(1) - R(0.5) * sr) * sk;
            del[k] = dl * R(1.0 / kMrt3Norm[k]);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            R acc = R(0);
#pragma unroll
            for (int k = 1; k < Q; ++k) {
                const int c = mrt3_coef(k, i);
                if (c == 1)
                    acc += del[k];
                else if (c == -1)
                    acc -= del[k];
                else if (c != 0)
                    acc += R(c) * del[k];
            }
            f[i] -= acc;
        }
        return;
    }
    {
        R s = keep * f[0] + omega * (R(kW[0]) * C0);
        if constexpr (FORCE)
            s += guo * (R(kW[0]) * (R(-3) * uF));
        f[0] = s;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1, j = i + 1;
        const R w = R(kW[i]);
        const R cu = pair_dot(k, ux, uy, uz);
        const R even = w * (C0 + rho_times(R(4.5) * (cu * cu)));
        const R odd = w * rho_times(R(3) * cu);
        if constexpr (TRT) {
            R P = keep * (R(0.5) * (f[i] + f[j])) + omega * even;
            R M = (R(1) - omega_m) * (R(0.5) * (f[i] - f[j])) + omega_m * odd;
            if constexpr (FORCE) {
                const R cF = pair_dot(k, Fx, Fy, Fz);
                P += guo * (w * (R(9) * cu * cF - R(3) * uF));
                M += (R(1) - R(0.5) * omega_m) * (R(3) * w * cF);
            }
            f[i] = P + M;
            f[j] = P - M;
        } else {
            R a = keep * f[i] + omega * (even + odd);
            R b = keep * f[j] + omega * (even - odd);
            if constexpr (FORCE) {
                const R cF = pair_dot(k, Fx, Fy, Fz);
                const R se = w * (R(9) * cu * cF - R(3) * uF);
                const R so = R(3) * w * cF;
                a += guo * (se + so);
                b += guo * (se - so);
            }
            f[i] = a;
            f[j] = b;
        }
    }
}

// Row offsets of rows (y + dy, z + dz), dy, dz in {-1, 0, 1} (periodic), and
// column offsets of columns x - 1, x, x + 1: node (x, y, z), direction i has
// element i * 64 + row[dz + 1][dy + 1] + col[dx + 1].  In a step the rows are
// wave-uniform (one row segment per workgroup), so an element is addressed as a
// uniform pointer (64-bit row offsets: a lattice may exceed 2^32 elements) plus
// a 32-bit lane offset; column offsets stay below 2^28 (the runtime bounds
// 19 * pitch).
struct Addr {
    uint64_t row[3][3];
    uint32_t col[3];
};

__device__ __forceinline__ uint32_t col_off(int x)
{
    return ((((uint32_t)x >> 6) * (uint32_t)(Q * kChunk)) | ((uint32_t)x & 63u)) & 0x0FFFFFFFu;
}

// Element of direction i at row slot (dz, dy) and column slot dx.
template <class M>
__device__ __forceinline__ M &elem(M *s, const Addr &a, int i, int dz, int dy, int dx)
{
    M *p = s + ((uint64_t)i * kChunk + a.row[dz][dy]);
    return p[a.col[dx]];
}

__device__ __forceinline__ Addr addr_of(int x, int y, int z, int nx, int ny, int nz, uint32_t cpr)
{
    Addr a;
    const int ys[3] = {wrap_dec(y, ny), y, wrap_inc(y, ny)};
    const int zs[3] = {wrap_dec(z, nz), z, wrap_inc(z, nz)};
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
            a.row[dz][dy] = ((uint64_t)zs[dz] * (uint32_t)ny + (uint32_t)ys[dy]) * cpr *
                            (uint64_t)(Q * kChunk);
    a.col[0] = col_off(wrap_dec(x, nx));
    a.col[1] = col_off(x);
    a.col[2] = col_off(wrap_inc(x, nx));
    return a;
}

// Pull gather: f_i(x) = s_i(x - c_i), or bb_opp(i)(x) when x - c_i is solid
// (bit i of sm): bb = s for halfway bounce-back; for the full-way rule bb is
// the other lattice of the A-B pair, which still holds the node's
// post-collision values of two steps back (the time a population sent into a
// wall node takes to return).
template <class ST>
__device__ __forceinline__ void pull3(const typename ST::mem *__restrict__ s,
                                      const typename ST::mem *bb, const Addr &a, uint32_t sm,
                                      typename ST::real (&f)[Q])
{
    using M = typename ST::mem;
    M *sp = const_cast<M *>(s);
    M *bp = const_cast<M *>(bb);
    if (sm == 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[i] = ST::ld(elem(sp, a, i, 1 - kCz[i], 1 - kCy[i], 1 - kCx[i]), i);
        return;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[i] = ST::ld(((sm >> i) & 1u) ? elem(bp, a, kOpp[i], 1, 1, 1)
                                       : elem(sp, a, i, 1 - kCz[i], 1 - kCy[i], 1 - kCx[i]),
                      i);
}

__device__ __forceinline__ uint32_t solid_bits3(uint8_t t, const uint32_t *__restrict__ nmask,
                                                uint32_t n)
{
    return t == kBoundary ? nmask[n] << 1 : 0u;
}

// One node (x, y, z) of row r = z * ny + y of the dense A-B step; interior:
// its 256-node row segment holds interior fluid nodes only.
template <class ST, bool FORCE, bool TRT, bool MRT>
__device__ __forceinline__ void step3_node(
    const typename ST::mem *__restrict__ src, typename ST::mem *__restrict__ dst,
    const uint8_t *__restrict__ type, const uint32_t *__restrict__ nmask, bool interior, int x,
    int y, int z, uint32_t r, int nx, int ny, int nz, int pitch, typename ST::real omega,
    typename ST::real gx, typename ST::real gy, typename ST::real gz,
    const Rates3<typename ST::real> &rt, int fullway)
{
    using R = typename ST::real;
    const uint32_t n = r * (uint32_t)pitch + (uint32_t)x;
    uint32_t sm = 0;
    if (!interior) {
        const uint8_t t = type[n];
        if (t == kSolid)
            return;
        sm = solid_bits3(t, nmask, n);
    }
    const Addr a = addr_of(x, y, z, nx, ny, nz, (uint32_t)pitch / kChunk);
    R f[Q];
    pull3<ST>(src, fullway ? dst : src, a, sm, f);
    collide3<R, ST::kShift, FORCE, TRT, MRT>(f, omega, gx, gy, gz, rt);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        store_nt(&elem(dst, a, i, 1, 1, 1), ST::st(f[i], i));
}

// Per-node A-B step (one node per lane, shifted loads straight from the
// lattice): the kernel for lattices small enough that a step is bound by
// latency rather than bandwidth.
template <class ST, bool FORCE, bool TRT, bool MRT>
__global__ __launch_bounds__(kBlock) void k_step3(
    const typename ST::mem *__restrict__ src, typename ST::mem *__restrict__ dst,
    const uint8_t *__restrict__ type, const uint32_t *__restrict__ nmask,
    const uint32_t *__restrict__ seg_interior, int nx, int ny, int nz, int pitch, uint32_t bpr,
    uint32_t nblocks, typename ST::real omega, typename ST::real gx, typename ST::real gy,
    typename ST::real gz, Rates3<typename ST::real> rt, int fullway)
{
    const uint32_t L = xcd_remap(blockIdx.x, nblocks);
    const uint32_t r = L / bpr;  // row index z * ny + y
    const int x = (int)(L - r * bpr) * kBlock + (int)threadIdx.x;
    if (x >= nx)
        return;
    const int y = (int)(r % (uint32_t)ny), z = (int)(r / (uint32_t)ny);
    step3_node<ST, FORCE, TRT, MRT>(src, dst, type, nmask, seg_interior[L] != 0, x, y, z, r, nx,
                                    ny, nz, pitch, omega, gx, gy, gz, rt, fullway);
}

// Bit masks of the directions with c_i.x (.y, .z) = +1 and -1: the velocity
// components of a direction index held in a register, without a table.
__device__ constexpr uint32_t dir_bits(const int (&c)[Q], int v)
{
    uint32_t b = 0;
    for (int i = 0; i < Q; ++i)
        if (c[i] == v)
            b |= 1u << i;
    return b;
}
__device__ __forceinline__ int comp_of(uint32_t plus, uint32_t minus, uint32_t i)
{
    return (int)((plus >> i) & 1u) - (int)((minus >> i) & 1u);
}

// A-B step through LDS: a workgroup updates one 256-node row segment of row
// r = z * ny + y.  When the segment is all-interior and whole (x0 + 256 <=
// nx), it first copies, for each direction i, the 256 source values of row
// (y - c_i.y, z - c_i.z), columns x0 - c_i.x .., into LDS with aligned
// 16-byte loads (each 64-node chunk run is contiguous), all in flight
// together, plus the one column beyond the segment's end that the x-shifted
// directions need; after a barrier every lane reads its 19 shifted sources
// from LDS.  Other segments (solid or boundary nodes, or the row's partial last
// segment) run the per-node path.
template <class ST, bool FORCE, bool TRT, bool MRT>
__global__ __launch_bounds__(kBlock) void k_step3_lds(
    const typename ST::mem *__restrict__ src, typename ST::mem *__restrict__ dst,
    const uint8_t *__restrict__ type, const uint32_t *__restrict__ nmask,
    const uint32_t *__restrict__ seg_interior, int nx, int ny, int nz, int pitch, uint32_t bpr,
    uint32_t nblocks, typename ST::real omega, typename ST::real gx, typename ST::real gy,
    typename ST::real gz, Rates3<typename ST::real> rt, int fullway)
{
    using R = typename ST::real;
    using M = typename ST::mem;
    constexpr uint32_t kE = 16u / (uint32_t)sizeof(M);  // elements per 16-byte vector
    constexpr uint32_t kVpc = kChunk / kE;             // vectors per 64-node chunk run
    constexpr uint32_t kV = Q * 4u * kVpc;             // vectors per segment
    constexpr uint32_t kRow = kBlock + 2u * kE;
    // row i: [kE - 1] = column x0 - 1, [kE .. kE + 255] = the segment (16-byte
    // aligned), [kE + 256] = column x0 + 256
    __shared__ __align__(16) M stage[Q][kRow];
    const uint32_t L = xcd_remap(blockIdx.x, nblocks);
    const uint32_t r = L / bpr;  // row index z * ny + y
    const int x0 = (int)(L - r * bpr) * kBlock;
    const int x = x0 + (int)threadIdx.x;
    const int y = (int)(r % (uint32_t)ny), z = (int)(r / (uint32_t)ny);
    const bool inner = seg_interior[L] != 0;
    if (!inner || x0 + kBlock > nx) {
        if (x < nx)
            step3_node<ST, FORCE, TRT, MRT>(src, dst, type, nmask, inner, x, y, z, r, nx, ny, nz,
                                            pitch, omega, gx, gy, gz, rt, fullway);
        return;
    }
    constexpr uint32_t PX = dir_bits(kCx, 1), NX = dir_bits(kCx, -1);
    constexpr uint32_t PY = dir_bits(kCy, 1), NY = dir_bits(kCy, -1);
    constexpr uint32_t PZ = dir_bits(kCz, 1), NZ = dir_bits(kCz, -1);
    const uint32_t cpr = (uint32_t)pitch / kChunk;
    const uint64_t rowel = (uint64_t)cpr * (Q * kChunk);  // elements per row
    // first element of the source row of direction i: row (y - c_i.y, z - c_i.z)
    auto src_row = [=](uint32_t i) -> uint64_t {
        int ys = y - comp_of(PY, NY, i), zs = z - comp_of(PZ, NZ, i);
        ys += ys < 0 ? ny : (ys >= ny ? -ny : 0);
        zs += zs < 0 ? nz : (zs >= nz ? -nz : 0);
        return ((uint64_t)(uint32_t)zs * (uint32_t)ny + (uint32_t)ys) * rowel;
    };
    const uint32_t c0 = (uint32_t)x0 >> 6;
    // halo: lane i (i = 1..18 with c_i.x != 0) fetches the column beyond the
    // segment on the side direction i pulls from
    M hv = M(0);
    const uint32_t hi = threadIdx.x;
    const int hcx = hi < (uint32_t)Q ? comp_of(PX, NX, hi) : 0;
    if (hcx != 0) {
        const int xs = hcx > 0 ? wrap_dec(x0, nx) : wrap_inc(x0 + kBlock - 1, nx);
        hv = src[src_row(hi) + (uint64_t)hi * kChunk + col_off(xs)];
    }
    // the segment's runs: all loads in flight before any LDS write, no branch
    // in between (indices past the last vector repeat the last one: the same
    // value to the same place)
    constexpr uint32_t kIter = (kV + kBlock - 1) / kBlock;
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    v4u vv[kIter];
    uint32_t dst_el[kIter];
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m) {
        const uint32_t q = min(threadIdx.x + m * kBlock, kV - 1u);
        const uint32_t i = q / (4u * kVpc), rr = q - i * (4u * kVpc);
        const uint32_t cc = rr / kVpc, pc = rr - cc * kVpc;
        const uint64_t off = src_row(i) + (uint64_t)(c0 + cc) * (Q * kChunk) +
                             (uint64_t)i * kChunk + (uint64_t)pc * kE;
        vv[m] = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(src + off));
        dst_el[m] = i * kRow + kE + cc * kChunk + pc * kE;
    }
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m)
        *reinterpret_cast<v4u *>(&stage[0][0] + dst_el[m]) = vv[m];
    if (hcx != 0)
        stage[hi][hcx > 0 ? kE - 1 : kE + kBlock] = hv;
    __syncthreads();
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[i] = ST::ld(stage[i][(int)kE + (int)threadIdx.x - kCx[i]], i);
    collide3<R, ST::kShift, FORCE, TRT, MRT>(f, omega, gx, gy, gz, rt);
    M *out = dst + (uint64_t)r * rowel + col_off(x);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        store_nt(out + (uint32_t)i * kChunk, ST::st(f[i], i));
}

// k_step3_lds with two y rows (y0 = 2 p and y0 + 1, one z plane) per workgroup:
// twice the loads in flight per wavefront and two collisions per lane.  Used
// for 16-bit storage with the MRT collision on mostly interior lattices (256^3:
// 278.0 against 292.2 us per step; with BGK it measured 1-2 % slower).  A pair
// whose two segments are not both all-interior and whole, and the single last
// row when ny is odd, take the per-node step.
template <class ST, bool FORCE, bool TRT, bool MRT>
__global__ __launch_bounds__(kBlock) void k_step3_lds2(
    const typename ST::mem *__restrict__ src, typename ST::mem *__restrict__ dst,
    const uint8_t *__restrict__ type, const uint32_t *__restrict__ nmask,
    const uint32_t *__restrict__ seg_interior, int nx, int ny, int nz, int pitch, uint32_t bpr,
    uint32_t nblocks, typename ST::real omega, typename ST::real gx, typename ST::real gy,
    typename ST::real gz, Rates3<typename ST::real> rt, int fullway)
{
    using R = typename ST::real;
    using M = typename ST::mem;
    static_assert(sizeof(M) == 2, "16-bit storage only");
    constexpr uint32_t NR = 2;
    constexpr uint32_t kE = 16u / (uint32_t)sizeof(M);
    constexpr uint32_t kVpc = kChunk / kE;
    constexpr uint32_t kVr = Q * 4u * kVpc;
    constexpr uint32_t kV = NR * kVr;
    constexpr uint32_t kRow = kBlock + 2u * kE;
    __shared__ __align__(16) M stage[NR][Q][kRow];
    const uint32_t L = xcd_remap(blockIdx.x, nblocks);
    const uint32_t npy = (uint32_t)(ny + 1) / 2u;
    const uint32_t rp = L / bpr, sx = L - rp * bpr;
    const int z = (int)(rp / npy);
    const int y0 = (int)(rp - (uint32_t)z * npy) * 2;
    const int x0 = (int)sx * kBlock;
    const int x = x0 + (int)threadIdx.x;
    const uint32_t r0 = (uint32_t)z * (uint32_t)ny + (uint32_t)y0;
    const bool in0 = seg_interior[r0 * bpr + sx] != 0;
    const bool has1 = y0 + 1 < ny;
    const bool in1 = has1 && seg_interior[(r0 + 1u) * bpr + sx] != 0;
    if (!(in0 && in1) || x0 + kBlock > nx) {
        if (x < nx) {
            step3_node<ST, FORCE, TRT, MRT>(src, dst, type, nmask, in0, x, y0, z, r0, nx, ny, nz,
                                            pitch, omega, gx, gy, gz, rt, fullway);
            if (has1)
                step3_node<ST, FORCE, TRT, MRT>(src, dst, type, nmask, in1, x, y0 + 1, z, r0 + 1u,
                                                nx, ny, nz, pitch, omega, gx, gy, gz, rt, fullway);
        }
        return;
    }
    constexpr uint32_t PX = dir_bits(kCx, 1), NX = dir_bits(kCx, -1);
    constexpr uint32_t PY = dir_bits(kCy, 1), NY = dir_bits(kCy, -1);
    constexpr uint32_t PZ = dir_bits(kCz, 1), NZ = dir_bits(kCz, -1);
    const uint32_t cpr = (uint32_t)pitch / kChunk;
    const uint64_t rowel = (uint64_t)cpr * (Q * kChunk);
    auto src_row = [=](uint32_t i, int y) -> uint64_t {
        int ys = y - comp_of(PY, NY, i), zs = z - comp_of(PZ, NZ, i);
        ys += ys < 0 ? ny : (ys >= ny ? -ny : 0);
        zs += zs < 0 ? nz : (zs >= nz ? -nz : 0);
        return ((uint64_t)(uint32_t)zs * (uint32_t)ny + (uint32_t)ys) * rowel;
    };
    const uint32_t c0 = (uint32_t)x0 >> 6;
    M hv = M(0);
    const uint32_t hr = threadIdx.x >> 5, hi = threadIdx.x & 31u;
    const int hcx = hr < NR && hi < (uint32_t)Q ? comp_of(PX, NX, hi) : 0;
    if (hcx != 0) {
        const int xs = hcx > 0 ? wrap_dec(x0, nx) : wrap_inc(x0 + kBlock - 1, nx);
        hv = src[src_row(hi, y0 + (int)hr) + (uint64_t)hi * kChunk + col_off(xs)];
    }
    constexpr uint32_t kIter = (kV + kBlock - 1) / kBlock;
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    v4u vv[kIter];
    uint32_t dst_el[kIter];
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m) {
        const uint32_t q = min(threadIdx.x + m * kBlock, kV - 1u);
        const uint32_t r = q / kVr, qr = q - r * kVr;
        const uint32_t i = qr / (4u * kVpc), rr = qr - i * (4u * kVpc);
        const uint32_t cc = rr / kVpc, pc = rr - cc * kVpc;
        const uint64_t off = src_row(i, y0 + (int)r) + (uint64_t)(c0 + cc) * (Q * kChunk) +
                             (uint64_t)i * kChunk + (uint64_t)pc * kE;
        vv[m] = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(src + off));
        dst_el[m] = (r * Q + i) * kRow + kE + cc * kChunk + pc * kE;
    }
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m)
        *reinterpret_cast<v4u *>(&stage[0][0][0] + dst_el[m]) = vv[m];
    if (hcx != 0)
        stage[hr][hi][hcx > 0 ? kE - 1 : kE + kBlock] = hv;
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < NR; ++r) {
        R f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[i] = ST::ld(stage[r][i][(int)kE + (int)threadIdx.x - kCx[i]], i);
        collide3<R, ST::kShift, FORCE, TRT, MRT>(f, omega, gx, gy, gz, rt);
        M *out = dst + (uint64_t)(r0 + r) * rowel + col_off(x);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            store_nt(out + (uint32_t)i * kChunk, ST::st(f[i], i));
    }
}

// AA pattern (DENSE_AA: one lattice updated in place).  Even steps read node
// x's own slots and write f*_i to its slot opp(i); odd steps read
// f_i = A_opp(i)(x - c_i) (A_i(x) when x - c_i is solid) and write f*_i to
// A_i(x + c_i) (A_opp(i)(x) when x + c_i is solid).  Slot j of node y is read
// and written only by node y in even steps and only by node y - c_j in odd
// steps, so the update is race-free.  After an even number of steps the
// canonical state is local (f_i = A_i(x)); after an odd number it is the odd
// read above.
template <class ST>
__device__ __forceinline__ void aa_odd3(const typename ST::mem *s, const Addr &a, uint32_t sm,
                                        typename ST::real (&f)[Q])
{
    using M = typename ST::mem;
    M *sp = const_cast<M *>(s);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[i] = ST::ld(((sm >> i) & 1u) ? elem(sp, a, i, 1, 1, 1)
                                       : elem(sp, a, kOpp[i], 1 - kCz[i], 1 - kCy[i], 1 - kCx[i]),
                      i);
}

template <class ST>
__device__ __forceinline__ void local3(const typename ST::mem *s, const Addr &a,
                                       typename ST::real (&f)[Q])
{
    using M = typename ST::mem;
    M *sp = const_cast<M *>(s);
    // Nontemporal loads: each slot is read once per even step (measured at
    // 256^3: 3 % shorter AA step pairs in FP64 and FP32; the same hint made the
    // D2Q9 gathers slower, so they keep plain loads).
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[i] = ST::ld(lbm::load_nt(&elem(sp, a, i, 1, 1, 1)), i);
}

// One node of the AA step (row r = z * ny + y); interior: its 256-node row
// segment holds interior fluid nodes only.
template <class ST, bool FORCE, bool TRT, bool MRT, bool ODD>
__device__ __forceinline__ void step3_aa_node(
    typename ST::mem *__restrict__ A, const uint8_t *__restrict__ type,
    const uint32_t *__restrict__ nmask, bool interior, int x, int y, int z, uint32_t r, int nx,
    int ny, int nz, int pitch, typename ST::real omega, typename ST::real gx,
    typename ST::real gy, typename ST::real gz, const Rates3<typename ST::real> &rt)
{
    using R = typename ST::real;
    const uint32_t n = r * (uint32_t)pitch + (uint32_t)x;
    uint32_t sm = 0;
    if (!interior) {
        const uint8_t t = type[n];
        if (t == kSolid)
            return;
        sm = solid_bits3(t, nmask, n);
    }
    const Addr a = addr_of(x, y, z, nx, ny, nz, (uint32_t)pitch / kChunk);
    R f[Q];
    if constexpr (ODD)
        aa_odd3<ST>(A, a, sm, f);
    else
        local3<ST>(A, a, f);
    collide3<R, ST::kShift, FORCE, TRT, MRT>(f, omega, gx, gy, gz, rt);
    if constexpr (ODD) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            store_nt(((sm >> kOpp[i]) & 1u) ? &elem(A, a, kOpp[i], 1, 1, 1)
                                            : &elem(A, a, i, 1 + kCz[i], 1 + kCy[i], 1 + kCx[i]),
                     ST::st(f[i], i));
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            store_nt(&elem(A, a, kOpp[i], 1, 1, 1), ST::st(f[i], i));
    }
}

template <class ST, bool FORCE, bool TRT, bool MRT, bool ODD>
__global__ __launch_bounds__(kBlock) void k_step3_aa(
    typename ST::mem *__restrict__ A, const uint8_t *__restrict__ type,
    const uint32_t *__restrict__ nmask, const uint32_t *__restrict__ seg_interior, int nx, int ny,
    int nz, int pitch, uint32_t bpr, uint32_t nblocks, typename ST::real omega,
    typename ST::real gx, typename ST::real gy, typename ST::real gz, Rates3<typename ST::real> rt)
{
    const uint32_t L = xcd_remap(blockIdx.x, nblocks);
    const uint32_t r = L / bpr;  // row index z * ny + y
    const int x = (int)(L - r * bpr) * kBlock + (int)threadIdx.x;
    if (x >= nx)
        return;
    const int y = (int)(r % (uint32_t)ny), z = (int)(r / (uint32_t)ny);
    step3_aa_node<ST, FORCE, TRT, MRT, ODD>(A, type, nmask, seg_interior[L] != 0, x, y, z, r, nx,
                                            ny, nz, pitch, omega, gx, gy, gz, rt);
}

// Odd AA step through LDS (the staging of k_step3_lds applied to the AA read
// pattern): for each direction i the segment's values A_opp(i) of row
// (y - c_i.y, z - c_i.z), columns x0 - c_i.x .., go into LDS with aligned
// 16-byte loads; after one barrier every lane reads its 19 sources and writes
// f_i to A_i(x + c_i) directly.  Loaded elements that this segment does not use
// may be rewritten meanwhile by the neighbouring segment (their only reader and
// writer is a node there); every element it uses is read and written by its
// own node only.  Other segments run the per-node AA step.
template <class ST, bool FORCE, bool TRT, bool MRT>
__global__ __launch_bounds__(kBlock) void k_step3_aa_odd(
    typename ST::mem *__restrict__ A, const uint8_t *__restrict__ type,
    const uint32_t *__restrict__ nmask, const uint32_t *__restrict__ seg_interior, int nx, int ny,
    int nz, int pitch, uint32_t bpr, uint32_t nblocks, typename ST::real omega,
    typename ST::real gx, typename ST::real gy, typename ST::real gz, Rates3<typename ST::real> rt)
{
    using R = typename ST::real;
    using M = typename ST::mem;
    constexpr uint32_t kE = 16u / (uint32_t)sizeof(M);
    constexpr uint32_t kVpc = kChunk / kE;
    constexpr uint32_t kV = Q * 4u * kVpc;
    constexpr uint32_t kRow = kBlock + 2u * kE;
    __shared__ __align__(16) M stage[Q][kRow];
    const uint32_t L = xcd_remap(blockIdx.x, nblocks);
    const uint32_t r = L / bpr;  // row index z * ny + y
    const int x0 = (int)(L - r * bpr) * kBlock;
    const int x = x0 + (int)threadIdx.x;
    const int y = (int)(r % (uint32_t)ny), z = (int)(r / (uint32_t)ny);
    const bool inner = seg_interior[L] != 0;
    if (!inner || x0 + kBlock > nx) {
        if (x < nx)
            step3_aa_node<ST, FORCE, TRT, MRT, true>(A, type, nmask, inner, x, y, z, r, nx, ny,
                                                     nz, pitch, omega, gx, gy, gz, rt);
        return;
    }
    constexpr uint32_t PX = dir_bits(kCx, 1), NX = dir_bits(kCx, -1);
    constexpr uint32_t PY = dir_bits(kCy, 1), NY = dir_bits(kCy, -1);
    constexpr uint32_t PZ = dir_bits(kCz, 1), NZ = dir_bits(kCz, -1);
    const uint32_t cpr = (uint32_t)pitch / kChunk;
    const uint64_t rowel = (uint64_t)cpr * (Q * kChunk);
    auto src_row = [=](uint32_t i) -> uint64_t {
        int ys = y - comp_of(PY, NY, i), zs = z - comp_of(PZ, NZ, i);
        ys += ys < 0 ? ny : (ys >= ny ? -ny : 0);
        zs += zs < 0 ? nz : (zs >= nz ? -nz : 0);
        return ((uint64_t)(uint32_t)zs * (uint32_t)ny + (uint32_t)ys) * rowel;
    };
    // opp(i) of a runtime index: the pairs (1, 2), (3, 4), .., (17, 18)
    auto dopp = [](uint32_t i) { return i == 0 ? 0u : ((i - 1u) ^ 1u) + 1u; };
    const uint32_t c0 = (uint32_t)x0 >> 6;
    M hv = M(0);
    const uint32_t hi = threadIdx.x;
    const int hcx = hi < (uint32_t)Q ? comp_of(PX, NX, hi) : 0;
    if (hcx != 0) {
        const int xs = hcx > 0 ? wrap_dec(x0, nx) : wrap_inc(x0 + kBlock - 1, nx);
        hv = A[src_row(hi) + (uint64_t)dopp(hi) * kChunk + col_off(xs)];
    }
    constexpr uint32_t kIter = (kV + kBlock - 1) / kBlock;
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    v4u vv[kIter];
    uint32_t dst_el[kIter];
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m) {
        const uint32_t q = min(threadIdx.x + m * kBlock, kV - 1u);
        const uint32_t i = q / (4u * kVpc), rr = q - i * (4u * kVpc);
        const uint32_t cc = rr / kVpc, pc = rr - cc * kVpc;
        const uint64_t off = src_row(i) + (uint64_t)(c0 + cc) * (Q * kChunk) +
                             (uint64_t)dopp(i) * kChunk + (uint64_t)pc * kE;
        vv[m] = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(A + off));
        dst_el[m] = i * kRow + kE + cc * kChunk + pc * kE;
    }
#pragma unroll
    for (uint32_t m = 0; m < kIter; ++m)
        *reinterpret_cast<v4u *>(&stage[0][0] + dst_el[m]) = vv[m];
    if (hcx != 0)
        stage[hi][hcx > 0 ? kE - 1 : kE + kBlock] = hv;
    __syncthreads();
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[i] = ST::ld(stage[i][(int)kE + (int)threadIdx.x - kCx[i]], i);
    collide3<R, ST::kShift, FORCE, TRT, MRT>(f, omega, gx, gy, gz, rt);
    const Addr a = addr_of(x, y, z, nx, ny, nz, cpr);
    // The ten directions with c_x != 0 store runs shifted by one element, so two
    // wavefronts share each 64-element run.  With 16- and 32-bit storage these
    // stores go through the cache without the streaming hint, which lets the
    // halves meet there (256^3 AA step pairs: FP32 436.0 -> 425.3 us, FP16 233.3
    // -> 228.4 us); FP64 keeps the hint (889.1 against 891.5 us).  The D2Q9 odd
    // step measured slower without it at every storage type.
    // (Two separate store expressions: one shared pointer let the compiler
    // merge the branches' stores and drop the hint from all of them.)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (sizeof(M) == 8 || kCx[i] == 0)
            store_nt(&elem(A, a, i, 1 + kCz[i], 1 + kCy[i], 1 + kCx[i]), ST::st(f[i], i));
        else
            elem(A, a, i, 1 + kCz[i], 1 + kCy[i], 1 + kCx[i]) = ST::st(f[i], i);
    }
}

// INDIRECT (node list): element of direction i of list node n in the chunked
// list layout [np/64][19][64].
__device__ __forceinline__ uint64_t lelem(uint32_t n, int i)
{
    return (uint64_t)(n >> 6) * (Q * kChunk) + (uint64_t)i * kChunk + (n & 63u);
}

// Compact source table of the node list (36 B per node instead of 72): info[n]
// holds the solid bits (bit i-1 <=> x - c_i solid) and kListBorder for nodes at
// x = 0 or nx - 1; rank8[r np + n] is the number of fluid nodes before position
// (x, y + dy_r, z + dz_r) in row-major order, rows r in the order of
// list_row().  Since the list is row-major, the source of direction i is
//   n -+ 1 in the node's own row (x -+ 1),
//   q_r, q_r - 1 or q_r + [(x, row r) fluid] in row r for x, x - 1, x + 1,
// except across the periodic seam in x: a border node's rank8[n] holds its slot
// in the full table edge[(i - 1) ne + slot], from which it takes the sources the
// seam or the slot breaks (c_x != 0, and the row-0 source with c_x = 0); the
// other rows' ranks stay valid.
constexpr uint32_t kListBorder = 1u << 31;

__device__ constexpr int list_row(int dy, int dz)
{
    return dz == 0 ? (dy < 0 ? 0 : 1)
         : dy == 0 ? (dz < 0 ? 2 : 3)
         : dz < 0  ? (dy < 0 ? 4 : 5)
                   : (dy < 0 ? 6 : 7);
}

// Direction with velocity (0, cy, cz).
__device__ constexpr int axis_dir(int cy, int cz)
{
    for (int j = 1; j < Q; ++j)
        if (kCx[j] == 0 && kCy[j] == cy && kCz[j] == cz)
            return j;
    return 0;
}

struct ListTable {
    const int32_t *rank8;
    const uint32_t *info;
    const int32_t *edge;
    uint64_t np, ne;
};

__host__ __device__ inline ListTable list_table(const State3 &s)
{
    return ListTable{s.rank8, s.info, s.edge, (uint64_t)s.np, (uint64_t)s.ne};
}

// Pull gather of list node n: f_i = s_i(source), or, when the source is solid,
// slot opp(i) of the node in bb (bb = s: halfway bounce-back; the other lattice
// of the pair: full-way, the value of two steps back).
template <class ST>
__device__ __forceinline__ void pull_list(const typename ST::mem *__restrict__ s,
                                          const typename ST::mem *bb, const ListTable &t,
                                          uint32_t n, typename ST::real (&f)[Q])
{
    const uint32_t bits = t.info[n];
    int32_t q[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
        q[r] = t.rank8[(uint64_t)r * t.np + n];
    uint32_t src[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int dx = -kCx[i], dy = -kCy[i], dz = -kCz[i];
        if (dy == 0 && dz == 0) {
            src[i] = n + dx;
        } else {
            const int32_t qr = q[list_row(dy, dz)];
            if (dx == 0)
                src[i] = (uint32_t)qr;
            else if (dx < 0)
                src[i] = (uint32_t)(qr - 1);
            else
                src[i] = (uint32_t)qr + (((bits >> (axis_dir(-dy, -dz) - 1)) & 1u) ^ 1u);
        }
    }
    if (bits & kListBorder) {
        const uint64_t slot = (uint32_t)q[0];
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if (kCx[i] != 0 || (kCz[i] == 0 && kCy[i] > 0))
                src[i] = (uint32_t)t.edge[(uint64_t)(i - 1) * t.ne + slot];
    }
    f[0] = ST::ld(s[lelem(n, 0)], 0);
#pragma unroll
    for (int i = 1; i < Q; ++i)
        f[i] = ST::ld((bits >> (i - 1)) & 1u ? bb[lelem(n, kOpp[i])] : s[lelem(src[i], i)], i);
}

template <class ST, bool FORCE, bool TRT, bool MRT>
__global__ __launch_bounds__(kBlock) void k_step3_list(
    const typename ST::mem *__restrict__ src, typename ST::mem *__restrict__ dst, ListTable tab,
    uint32_t n_fluid, uint32_t nblocks, typename ST::real omega, typename ST::real gx,
    typename ST::real gy, typename ST::real gz, Rates3<typename ST::real> rt, int fullway)
{
    using R = typename ST::real;
    const uint32_t n = xcd_remap(blockIdx.x, nblocks) * kBlock + threadIdx.x;
    if (n >= n_fluid)
        return;
    R f[Q];
    pull_list<ST>(src, fullway ? dst : src, tab, n, f);
    collide3<R, ST::kShift, FORCE, TRT, MRT>(f, omega, gx, gy, gz, rt);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        store_nt(&dst[lelem(n, i)], ST::st(f[i], i));
}

// ------------------------------------------------------- TILED16: 4x4x4 blocks --
// The tiled layout of the paper's sparse study (Sec. 4.3: only tiles that hold
// fluid nodes are stored, with a table of neighbour tiles) cut for D3Q19: blocks
// of 4 x 4 x 4 nodes, one wavefront each, populations [n_blocks][19][64] with
// node (lx, ly, lz) of a block in slot lx + 4 ly + 16 lz, so that every
// direction's 64 values of a block are one contiguous run.  The pull source
// x - c_i of a node lies in its own block or, on the faces the step crosses, in
// the neighbour block whose offset has the components of -c_i on the crossed
// axes; that offset is itself a D3Q19 velocity (no D3Q19 velocity has three
// non-zero components), so the 18-entry neighbour table covers every source.
constexpr uint32_t kBlockElems = Q * kChunk;
constexpr uint32_t kBlockMeta = 20;  // words per block of the block table

__device__ __forceinline__ uint64_t belem(uint32_t k, int i, uint32_t l)
{
    return (uint64_t)k * kBlockElems + (uint32_t)i * kChunk + l;
}

// Direction with velocity (cx, cy, cz); 0 when there is none (with constant
// arguments the search folds away).
__device__ __forceinline__ constexpr int dir3(int cx, int cy, int cz)
{
    for (int j = 1; j < Q; ++j)
        if (kCx[j] == cx && kCy[j] == cy && kCz[j] == cz)
            return j;
    return 0;
}

struct BlockTable {
    const uint32_t *meta;   // [n_blocks][20]: neighbours in directions 1..18, all-fluid flag
    const uint64_t *fluid;  // [n_blocks + 1]: fluid bits per slot (entry n_blocks = 0)
};

// Block k's neighbourhood: nb[j] = the block at offset c_j (nb[0] = k; a
// dropped block reads as index n_blocks, whose fluid bits are 0), fm[j] its
// fluid bits, interior = every node of the 19 blocks is fluid.
struct BlockNbrs {
    uint32_t nb[Q];
    uint64_t fm[Q];
    bool interior;
};

__device__ __forceinline__ void load_block_nbrs(const BlockTable &t, uint32_t k, BlockNbrs &n)
{
    const uint32_t *m = t.meta + (uint64_t)k * kBlockMeta;
    n.nb[0] = k;
#pragma unroll
    for (int j = 1; j < Q; ++j)
        n.nb[j] = m[j - 1];
    n.interior = m[18] != 0;
    n.fm[0] = t.fluid[k];
#pragma unroll
    for (int j = 1; j < Q; ++j)
        n.fm[j] = n.interior ? ~uint64_t(0) : t.fluid[n.nb[j]];
}

// v[d] of the block holding x - c_i, for the crossed faces X, Y, Z (each only
// possible on an axis where c_i is non-zero, and never all three).
template <class T>
__device__ __forceinline__ T pick_cross(int i, bool X, bool Y, bool Z, const T (&v)[Q])
{
    T r = v[0];
    if (X)
        r = v[dir3(-kCx[i], 0, 0)];
    if (Y)
        r = X ? v[dir3(-kCx[i], -kCy[i], 0)] : v[dir3(0, -kCy[i], 0)];
    if (Z)
        r = X ? v[dir3(-kCx[i], 0, -kCz[i])]
              : (Y ? v[dir3(0, -kCy[i], -kCz[i])] : v[dir3(0, 0, -kCz[i])]);
    return r;
}

// Pull source of direction i for slot l of block k: its block b and slot, and
// whether it is solid.  INTERIOR: the caller knows that every source is fluid.
template <bool INTERIOR>
__device__ __forceinline__ void block_link(const BlockNbrs &n, uint32_t l, int i, uint32_t &b,
                                           uint32_t &slot, bool &solid)
{
    const int lx = (int)(l & 3u), ly = (int)((l >> 2) & 3u), lz = (int)(l >> 4);
    const bool X = kCx[i] > 0 ? lx == 0 : (kCx[i] < 0 ? lx == 3 : false);
    const bool Y = kCy[i] > 0 ? ly == 0 : (kCy[i] < 0 ? ly == 3 : false);
    const bool Z = kCz[i] > 0 ? lz == 0 : (kCz[i] < 0 ? lz == 3 : false);
    b = pick_cross(i, X, Y, Z, n.nb);
    slot = (uint32_t)((lx - kCx[i]) & 3) | ((uint32_t)((ly - kCy[i]) & 3) << 2) |
           ((uint32_t)((lz - kCz[i]) & 3) << 4);
    solid = false;
    if constexpr (!INTERIOR)
        solid = ((pick_cross(i, X, Y, Z, n.fm) >> slot) & 1u) == 0;
}

// Pull gather of slot l of block k (pull3 for the block layout): f_i = the
// source's slot i, or slot opp(i) of the node in bb when the source is solid
// (bb = s: halfway bounce-back; the other lattice: full-way).  sm: bit i set
// <=> x - c_i is solid.
template <class ST, bool INTERIOR>
__device__ __forceinline__ void pull_block(const typename ST::mem *__restrict__ s,
                                           const typename ST::mem *bb, const BlockNbrs &n,
                                           uint32_t l, uint32_t &sm, typename ST::real (&f)[Q])
{
    const uint32_t k = n.nb[0];
    sm = 0;
    f[0] = ST::ld(s[belem(k, 0, l)], 0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        uint32_t b, slot;
        bool solid;
        block_link<INTERIOR>(n, l, i, b, slot, solid);
        sm |= (uint32_t)solid << i;
        const typename ST::mem *p = solid ? &bb[belem(k, kOpp[i], l)] : &s[belem(b, i, slot)];
        f[i] = ST::ld(*p, i);
    }
}

// TILED16 step: a wavefront updates one block (four per workgroup).  Solid
// lanes load nothing, so a 128-byte line of a run that holds only solid slots
// is neither read nor written; in a line that holds a fluid slot every lane
// stores (solid slots receive zero, which nothing reads), so that lines are
// written whole.
template <class ST, bool FORCE, bool TRT, bool MRT, bool INTERIOR>
__device__ __forceinline__ void block_update(const typename ST::mem *__restrict__ src,
                                             typename ST::mem *__restrict__ dst,
                                             const BlockNbrs &n, uint32_t l,
                                             typename ST::real omega, typename ST::real gx,
                                             typename ST::real gy, typename ST::real gz,
                                             const Rates3<typename ST::real> &rt, int fullway)
{
    using R = typename ST::real;
    constexpr uint32_t G = 128u / (uint32_t)sizeof(typename ST::mem);  // slots per line
    constexpr uint64_t kLine = G >= 64 ? ~uint64_t(0) : (uint64_t(1) << G) - 1u;
    const bool fluid = INTERIOR || ((n.fm[0] >> l) & 1u) != 0;
    const bool fill = INTERIOR || ((n.fm[0] >> (l & ~(G - 1u))) & kLine) != 0;
    R f[Q];
    if (fluid) {
        uint32_t sm;
        pull_block<ST, INTERIOR>(src, fullway ? dst : src, n, l, sm, f);
        collide3<R, ST::kShift, FORCE, TRT, MRT>(f, omega, gx, gy, gz, rt);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[i] = R(0);
    }
    if (fill) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            store_nt(&dst[belem(n.nb[0], i, l)], ST::st(f[i], i));
    }
}

template <class ST, bool FORCE, bool TRT, bool MRT>
__global__ __launch_bounds__(kBlock) void k_step3_blocks(
    const typename ST::mem *__restrict__ src, typename ST::mem *__restrict__ dst, BlockTable t,
    uint32_t n_blocks, uint32_t nwg, typename ST::real omega, typename ST::real gx,
    typename ST::real gy, typename ST::real gz, Rates3<typename ST::real> rt, int fullway)
{
    const uint32_t k = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, nwg) * 4u +
                                                      (threadIdx.x >> 6));
    if (k >= n_blocks)
        return;
    const uint32_t l = threadIdx.x & 63u;
    BlockNbrs n;
    load_block_nbrs(t, k, n);
    if (n.interior)
        block_update<ST, FORCE, TRT, MRT, true>(src, dst, n, l, omega, gx, gy, gz, rt, fullway);
    else
        block_update<ST, FORCE, TRT, MRT, false>(src, dst, n, l, omega, gx, gy, gz, rt, fullway);
}

__host__ __device__ inline BlockTable block_table(const State3 &s)
{
    return BlockTable{s.bmeta, s.bfluid};
}

// ------------------------------------------------------------ canonical views --
// Canonical FP64 buffers are [19][nz][ny][pitch].

// Thread gid = node (z * ny + y) * pitch + x: the canonical (pull-gathered)
// populations of a fluid node; false for padding and solid nodes.  bb: the
// bounce-back source of pull3.  Under the full-way rule (bb not st) the node
// also reports its wall slots: bit j of wl set <=> node x + c_j is solid, and
// the population in flight there, f_j(x + c_j), is the node's stored slot j.
// mode: kPull3 (A-B), kAAEven3 / kAAOdd3 (DENSE_AA after an even / odd number
// of steps).
enum Mode3 : int { kPull3 = 0, kAAEven3 = 1, kAAOdd3 = 2 };

template <class ST>
__device__ __forceinline__ bool canonical_at(const State3 &s, const typename ST::mem *st,
                                             const typename ST::mem *bb, int mode, uint32_t gid,
                                             int &x, int &y, int &z, double (&fd)[Q],
                                             uint32_t &wl, double (&wv)[Q])
{
    wl = 0;
    if (s.blocks) {  // gid = 64 * block + slot
        const uint32_t k = gid >> 6, l = gid & 63u;
        if (k >= (uint64_t)s.n_blocks)
            return false;
        BlockNbrs n;
        load_block_nbrs(block_table(s), k, n);
        if (((n.fm[0] >> l) & 1u) == 0)
            return false;
        x = 4 * s.bxyz[3 * (uint64_t)k] + (int)(l & 3u);
        y = 4 * s.bxyz[3 * (uint64_t)k + 1] + (int)((l >> 2) & 3u);
        z = 4 * s.bxyz[3 * (uint64_t)k + 2] + (int)(l >> 4);
        typename ST::real f[Q];
        uint32_t sm;
        pull_block<ST, false>(st, bb, n, l, sm, f);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            fd[i] = ST::canon(f[i], i);
        if (bb != st)  // full-way: the wall slots this node feeds
            for (int j = 1; j < Q; ++j)
                if ((sm >> kOpp[j]) & 1u) {
                    wl |= 1u << j;
                    wv[j] = ST::canon(ST::ld(st[belem(k, j, l)], j), j);
                }
        return true;
    }
    if (s.list) {  // gid = list index
        if (gid >= (uint64_t)s.n_fluid)
            return false;
        x = s.fxyz[3 * (uint64_t)gid];
        y = s.fxyz[3 * (uint64_t)gid + 1];
        z = s.fxyz[3 * (uint64_t)gid + 2];
        typename ST::real f[Q];
        pull_list<ST>(st, bb, list_table(s), gid, f);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            fd[i] = ST::canon(f[i], i);
        if (bb != st) {  // full-way: the wall slots this node feeds
            const uint32_t sm = s.info[gid] << 1;
            for (int j = 1; j < Q; ++j)
                if ((sm >> kOpp[j]) & 1u) {
                    wl |= 1u << j;
                    wv[j] = ST::canon(ST::ld(st[lelem(gid, j)], j), j);
                }
        }
        return true;
    }
    const uint32_t r = gid / (uint32_t)s.pitch;
    x = (int)(gid - r * (uint32_t)s.pitch);
    if (x >= s.nx || r >= (uint32_t)(s.ny * s.nz))
        return false;
    y = (int)(r % (uint32_t)s.ny);
    z = (int)(r / (uint32_t)s.ny);
    const uint8_t t = s.type[gid];
    if (t == kSolid)
        return false;
    const Addr a = addr_of(x, y, z, s.nx, s.ny, s.nz, (uint32_t)s.pitch / kChunk);
    const uint32_t sm = solid_bits3(t, s.nmask, gid);
    typename ST::real f[Q];
    if (mode == kAAEven3)
        local3<ST>(st, a, f);
    else if (mode == kAAOdd3)
        aa_odd3<ST>(st, a, sm, f);
    else
        pull3<ST>(st, bb, a, sm, f);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        fd[i] = ST::canon(f[i], i);
    if (bb != st)
        for (int j = 1; j < Q; ++j)
            if ((sm >> kOpp[j]) & 1u) {  // x + c_j is x - c_opp(j)
                wl |= 1u << j;
                wv[j] = ST::canon(ST::ld(elem(const_cast<typename ST::mem *>(st), a, j, 1, 1, 1),
                                         j),
                                  j);
            }
    return true;
}

// Padded node index of x + c_j (periodic).
__device__ __forceinline__ uint32_t node_plus(const State3 &s, int x, int y, int z, int j)
{
    const int xs = x + kCx[j] < 0 ? s.nx - 1 : (x + kCx[j] >= s.nx ? 0 : x + kCx[j]);
    const int ys = y + kCy[j] < 0 ? s.ny - 1 : (y + kCy[j] >= s.ny ? 0 : y + kCy[j]);
    const int zs = z + kCz[j] < 0 ? s.nz - 1 : (z + kCz[j] >= s.nz ? 0 : z + kCz[j]);
    return ((uint32_t)zs * s.ny + ys) * (uint32_t)s.pitch + xs;
}

template <class ST>
__global__ __launch_bounds__(kBlock) void k_gather3(State3 s, const typename ST::mem *st,
                                                    const typename ST::mem *bb, int mode,
                                                    double *__restrict__ fc)
{
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    int x, y, z;
    double f[Q], wv[Q];
    uint32_t wl;
    if (!canonical_at<ST>(s, st, bb, mode, gid, x, y, z, f, wl, wv))
        return;
    const uint64_t plane = (uint64_t)(s.nz * s.ny) * (uint32_t)s.pitch;
    const uint64_t o = ((uint64_t)z * s.ny + y) * (uint32_t)s.pitch + x;  // gid unless a list
#pragma unroll
    for (int i = 0; i < Q; ++i)
        fc[(uint64_t)i * plane + o] = f[i];
    // wall slots (full-way rule): each has exactly one fluid source node
    for (int j = 1; j < Q; ++j)
        if ((wl >> j) & 1u)
            fc[(uint64_t)j * plane + node_plus(s, x, y, z, j)] = wv[j];
}

// Macroscopic fields (Eq. 2 with the half-force velocity) into [nz][ny][nx]
// buffers, and per-block partial sums of the mass: rho, plus (full-way rule)
// the populations in flight in the wall slots the node feeds.
template <class ST>
__global__ __launch_bounds__(kBlock) void k_macro3(State3 s, const typename ST::mem *st,
                                                   const typename ST::mem *bb, int mode,
                                                   double *rho,
                                                   double *ux, double *uy, double *uz,
                                                   double *partials)
{
    __shared__ double ws[kBlock / 64];
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    int x, y, z;
    double f[Q], wv[Q];
    uint32_t wl;
    double r = 0.0, mass = 0.0;
    if (canonical_at<ST>(s, st, bb, mode, gid, x, y, z, f, wl, wv)) {
        double mx = 0.0, my = 0.0, mz = 0.0;
        for (int i = 0; i < Q; ++i) {
            r += f[i];
            mx += kCx[i] * f[i];
            my += kCy[i] * f[i];
            mz += kCz[i] * f[i];
        }
        if (rho) {
            const size_t o = ((size_t)z * s.ny + y) * s.nx + x;
            rho[o] = r;
            ux[o] = mx / r + 0.5 * s.gx;
            uy[o] = my / r + 0.5 * s.gy;
            uz[o] = mz / r + 0.5 * s.gz;
        }
        mass = r;
        for (int j = 1; j < Q; ++j)
            if ((wl >> j) & 1u)
                mass += wv[j];
    }
    if (partials) {
        for (int o = 32; o > 0; o >>= 1)
            mass += __shfl_down(mass, o, 64);
        if ((threadIdx.x & 63) == 0)
            ws[threadIdx.x >> 6] = mass;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < kBlock / 64; ++i)
                t += ws[i];
            partials[blockIdx.x] = t;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_sum3(const double *__restrict__ in, uint32_t n,
                                                 uint32_t per, double *__restrict__ out)
{
    __shared__ double ws[kBlock / 64];
    const uint32_t lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    double t = 0.0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock)
        t += in[i];
    for (int o = 32; o > 0; o >>= 1)
        t += __shfl_down(t, o, 64);
    if ((threadIdx.x & 63) == 0)
        ws[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double u = 0.0;
        for (int i = 0; i < kBlock / 64; ++i)
            u += ws[i];
        out[blockIdx.x] = u;
    }
}

// Equilibrium (Eq. 6, D3Q19 weights) into a canonical buffer; NULL fields:
// rho = 1, u = 0.
__global__ __launch_bounds__(kBlock) void k_equilibrium3(State3 s, const double *__restrict__ rho,
                                                         const double *__restrict__ ux,
                                                         const double *__restrict__ uy,
                                                         const double *__restrict__ uz,
                                                         double *__restrict__ fc)
{
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t r = gid / (uint32_t)s.pitch;
    const int x = (int)(gid - r * (uint32_t)s.pitch);
    if (x >= s.nx || r >= (uint32_t)(s.ny * s.nz))
        return;
    const size_t o = (size_t)r * s.nx + x;
    const double d = rho ? rho[o] : 1.0, u = ux ? ux[o] : 0.0, v = uy ? uy[o] : 0.0,
                 w = uz ? uz[o] : 0.0;
    const double usq = u * u + v * v + w * w;
    const uint64_t plane = (uint64_t)(s.nz * s.ny) * (uint32_t)s.pitch;
    for (int i = 0; i < Q; ++i) {
        const double cu = kCx[i] * u + kCy[i] * v + kCz[i] * w;
        fc[(uint64_t)i * plane + gid] = kW[i] * d * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    }
}

// Canonical -> stored A-B state: slot s_j(q) streams into f_j(q + c_j), or,
// when q + c_j is solid, into f_opp(j)(q) (the inverse of the pull gather).
// Full-way rule (walls = 1 or 2): s_j(q) = f_j(q + c_j) also when q + c_j is a
// wall node (its wall slot; walls = 2: the node's own f_j, the initial
// wall-slot rule), and the other lattice's slot opp(i) of q holds f_i(q) for
// every bounce-back link i (it returns from the wall at this step).
// DENSE_AA (mode kAAEven3 / kAAOdd3, the inverse of the AA reads): even,
// s_j(q) = f_j(q); odd, s_j(q) = f_opp(j)(q - c_j), or f_j(q) when q - c_j is
// solid.
template <class ST>
__global__ __launch_bounds__(kBlock) void k_scatter3(State3 s, typename ST::mem *st,
                                                     typename ST::mem *other, int walls, int mode,
                                                     const double *__restrict__ fc)
{
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    if (s.blocks) {  // TILED16: gid = 64 * block + slot; as the node list below
        const uint32_t k = gid >> 6, l = gid & 63u;
        if (k >= (uint64_t)s.n_blocks)
            return;
        BlockNbrs n;
        load_block_nbrs(block_table(s), k, n);
        if (((n.fm[0] >> l) & 1u) == 0)
            return;
        const int x = 4 * s.bxyz[3 * (uint64_t)k] + (int)(l & 3u),
                  y = 4 * s.bxyz[3 * (uint64_t)k + 1] + (int)((l >> 2) & 3u),
                  z = 4 * s.bxyz[3 * (uint64_t)k + 2] + (int)(l >> 4);
        const uint64_t plane = (uint64_t)(s.nz * s.ny) * (uint32_t)s.pitch;
        const uint64_t own = ((uint64_t)z * s.ny + y) * (uint32_t)s.pitch + x;
        uint32_t sm = 0;  // bit i <=> x - c_i solid
        for (int i = 1; i < Q; ++i) {
            uint32_t b, slot;
            bool solid;
            block_link<false>(n, l, i, b, slot, solid);
            sm |= (uint32_t)solid << i;
        }
        for (int j = 0; j < Q; ++j) {
            double v;
            if (((sm >> kOpp[j]) & 1u) == 0 || walls == 1)
                v = fc[(uint64_t)j * plane + node_plus(s, x, y, z, j)];
            else
                v = fc[(uint64_t)(walls == 2 ? j : kOpp[j]) * plane + own];
            st[belem(k, j, l)] = ST::from_canon(v, j);
        }
        if (walls != 0)
            for (int i = 1; i < Q; ++i)
                if ((sm >> i) & 1u)
                    other[belem(k, kOpp[i], l)] =
                        ST::from_canon(fc[(uint64_t)i * plane + own], kOpp[i]);
        return;
    }
    if (s.list) {  // INDIRECT: gid = list index; s_j(q) = f_j(q + c_j), or f_opp(j)(q)
        if (gid >= (uint64_t)s.n_fluid)
            return;
        const int x = s.fxyz[3 * (uint64_t)gid], y = s.fxyz[3 * (uint64_t)gid + 1],
                  z = s.fxyz[3 * (uint64_t)gid + 2];
        const uint64_t plane = (uint64_t)(s.nz * s.ny) * (uint32_t)s.pitch;
        const uint64_t own = ((uint64_t)z * s.ny + y) * (uint32_t)s.pitch + x;
        const uint32_t sm = s.info[gid] << 1;  // bit i <=> x - c_i solid
        for (int j = 0; j < Q; ++j) {
            // q + c_j is the pull source of direction opp(j); full-way walls as the
            // dense scatter below
            double v;
            if (((sm >> kOpp[j]) & 1u) == 0 || walls == 1)
                v = fc[(uint64_t)j * plane + node_plus(s, x, y, z, j)];
            else
                v = fc[(uint64_t)(walls == 2 ? j : kOpp[j]) * plane + own];
            st[lelem(gid, j)] = ST::from_canon(v, j);
        }
        if (walls != 0)
            for (int i = 1; i < Q; ++i)
                if ((sm >> i) & 1u)
                    other[lelem(gid, kOpp[i])] =
                        ST::from_canon(fc[(uint64_t)i * plane + own], kOpp[i]);
        return;
    }
    const uint32_t r = gid / (uint32_t)s.pitch;
    const int x = (int)(gid - r * (uint32_t)s.pitch);
    if (x >= s.nx || r >= (uint32_t)(s.ny * s.nz))
        return;
    const uint8_t t = s.type[gid];
    if (t == kSolid)
        return;
    const int y = (int)(r % (uint32_t)s.ny), z = (int)(r / (uint32_t)s.ny);
    const uint32_t sm = solid_bits3(t, s.nmask, gid);
    const uint64_t plane = (uint64_t)(s.nz * s.ny) * (uint32_t)s.pitch;
    const Addr a = addr_of(x, y, z, s.nx, s.ny, s.nz, (uint32_t)s.pitch / kChunk);
    if (mode != kPull3) {
        for (int j = 0; j < Q; ++j) {
            const double v = mode == kAAEven3 || ((sm >> j) & 1u)
                                 ? fc[(uint64_t)j * plane + gid]
                                 : fc[(uint64_t)kOpp[j] * plane + node_plus(s, x, y, z, kOpp[j])];
            elem(st, a, j, 1, 1, 1) = ST::from_canon(v, j);
        }
        return;
    }
    for (int j = 0; j < Q; ++j) {
        double v;
        // q + c_j is node q - c_opp(j): solid iff bit opp(j) is set
        if (((sm >> kOpp[j]) & 1u) == 0 || walls == 1)
            v = fc[(uint64_t)j * plane + node_plus(s, x, y, z, j)];
        else
            v = fc[(uint64_t)(walls == 2 ? j : kOpp[j]) * plane + gid];
        elem(st, a, j, 1, 1, 1) = ST::from_canon(v, j);
    }
    if (walls != 0)
        for (int i = 1; i < Q; ++i)
            if ((sm >> i) & 1u)
                elem(other, a, kOpp[i], 1, 1, 1) = ST::from_canon(fc[(uint64_t)i * plane + gid],
                                                                  kOpp[i]);
}

// Rest state (rho = 1, u = 0) written straight into a stored lattice: every
// slot of direction i holds w_i in storage form.  At rest the canonical ->
// stored map (k_scatter3) sends each slot an equilibrium of its own direction
// or of the opposite one, and w_opp(i) = w_i, so this is what the scatter of a
// rest state stores (it also fills solid and padding slots, which nothing reads).
template <class ST>
__global__ __launch_bounds__(kBlock) void k_rest3(typename ST::mem *p, uint64_t n)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * kBlock) {
        const int i = (int)((e / kChunk) % (uint64_t)Q);
        p[e] = ST::from_canon(kW[i], i);
    }
}

// Resident workgroups per CU (0: as many as registers allow), measured at
// 256^3: the per-node dense and AA steps on mostly interior lattices run faster with
// fewer workgroups in flight (FP32 A-B 433 us at 3 per CU against 453 us
// uncapped, AA 462 against 476 us; FP64 893 against 904 us, AA 943 against
// 950 us); the block step on a sphere packing at fluid fraction 0.4 likewise
// (FP64 482 against 495 us at 3, FP32 271 against 274 us at 5), and the
// node-list step there (FP64 406.2 against 410.5 us at 3, FP32 227.7 against
// 230.9 us at 5; 4: 408.8, 228.4).  16-bit storage gains nothing.
inline int step3_cap(const State3 &s, size_t esize)
{
    if (esize == 2)
        return 0;
    if (s.blocks)
        return esize == 8 ? 3 : 5;
    if (s.list)
        return esize == 8 ? 3 : 5;
    if (s.interior_frac < 0.9)
        return 0;
    return 3;
}

// Resident workgroups per CU of the LDS-staged dense step (0: as many as
// registers and LDS allow), measured at 256^3: FP64 Taylor-Green 839 us at 2
// per CU against 874 us at the 4 its LDS allows (sphere packing at fluid
// fraction 0.4: 846 against 867 us), the MRT collision 865 us at 3 against 872
// at 2; FP32 424 us at 4 against 440 us at 8 (sphere packing: 534 us at 3
// against 575 us; MRT no gain); 16-bit storage gains nothing.
inline int step3_lds_cap(const State3 &s, size_t esize)
{
    if (esize == 8)
        return s.mrt ? 3 : 2;
    if (esize == 4 && !s.mrt)
        return s.interior_frac >= 0.9 ? 4 : 3;
    return 0;
}

// The even AA step (local reads with nontemporal loads, local writes) on
// mostly interior lattices, measured at 256^3 (AA step pairs with the odd step
// through LDS): 2 workgroups per CU FP64 891 us per step, FP32 436 us (3: 898,
// 440; 4: 899, 444; uncapped 899, 452).
inline int step3_aa_even_cap(const State3 &s, size_t esize)
{
    if (esize == 2 || s.interior_frac < 0.9)
        return 0;
    return 2;
}

// The odd AA step through LDS, measured at 256^3 (AA step pairs): FP64 at 2
// workgroups per CU 923 us per step (933 uncapped, 943 with the per-node odd
// kernel), FP32 at 4 454 us (457, 464); 16-bit uncapped 238 us (247).
inline int step3_aa_odd_cap(const State3 &s, size_t esize)
{
    if (esize == 2 || s.interior_frac < 0.9)
        return 0;
    return esize == 8 ? 2 : 4;
}

template <class ST, bool TRT, bool MRT>
void step_launch3(const State3 &s, int cur)
{
    using M = typename ST::mem;
    using R = typename ST::real;
    const uint32_t bpr = (uint32_t)((s.nx + kBlock - 1) / kBlock);
    const uint32_t nb = bpr * (uint32_t)s.ny * (uint32_t)s.nz;
    const bool force = s.gx != 0.0 || s.gy != 0.0 || s.gz != 0.0;
    const R g[3] = {force ? (R)s.gx : R(0), force ? (R)s.gy : R(0), force ? (R)s.gz : R(0)};
    const Rates3<R> rt{(R)s.omega_m, (R)s.s_e, (R)s.s_eps, (R)s.s_q, (R)s.s_pi, (R)s.s_m};
    const uint32_t dyn = lbm::occupancy_cap_lds(step3_cap(s, sizeof(M)), 0u);
    if (s.blocks) {
        const uint32_t nwg = (uint32_t)((s.n_blocks + 3) / 4);
        if (nwg == 0)
            return;
        const M *src = (const M *)s.f[cur];
        M *dst = (M *)s.f[1 - cur];
        auto go = [&](auto kernel) {
            kernel<<<nwg, kBlock, dyn, s.stream>>>(src, dst, block_table(s), (uint32_t)s.n_blocks,
                                                 nwg, (R)s.omega, g[0], g[1], g[2], rt,
                                                 s.fullway);
        };
        if (force)
            go(k_step3_blocks<ST, true, TRT, MRT>);
        else
            go(k_step3_blocks<ST, false, TRT, MRT>);
        return;
    }
    if (s.list) {
        const uint32_t nbl = (uint32_t)((s.n_fluid + kBlock - 1) / kBlock);
        if (nbl == 0)
            return;
        const M *src = (const M *)s.f[cur];
        M *dst = (M *)s.f[1 - cur];
        auto go = [&](auto kernel) {
            kernel<<<nbl, kBlock, dyn, s.stream>>>(src, dst, list_table(s), (uint32_t)s.n_fluid,
                                                 nbl, (R)s.omega, g[0], g[1], g[2], rt,
                                                 s.fullway);
        };
        if (force)
            go(k_step3_list<ST, true, TRT, MRT>);
        else
            go(k_step3_list<ST, false, TRT, MRT>);
        return;
    }
    if (s.aa) {
        M *A = (M *)s.f[0];
        auto go = [&](auto kernel, uint32_t dl) {
            kernel<<<nb, kBlock, dl, s.stream>>>(A, s.type, s.nmask, s.seg_interior, s.nx, s.ny,
                                               s.nz, s.pitch, bpr, nb, (R)s.omega, g[0], g[1],
                                               g[2], rt);
        };
        // odd steps of large lattices through LDS (as for the A-B step)
        const bool lds = 38.0 * (double)s.nz * s.ny * s.pitch * sizeof(M) >= 128.0 * (1 << 20);
        if (cur && lds) {
            const uint32_t st =
                Q * (kBlock + 2u * (16u / (uint32_t)sizeof(M))) * (uint32_t)sizeof(M);
            const uint32_t dl = lbm::occupancy_cap_lds(step3_aa_odd_cap(s, sizeof(M)), st);
            force ? go(k_step3_aa_odd<ST, true, TRT, MRT>, dl)
                  : go(k_step3_aa_odd<ST, false, TRT, MRT>, dl);
        } else {
            const uint32_t de = lbm::occupancy_cap_lds(step3_aa_even_cap(s, sizeof(M)), 0u);
            if (force)
                cur ? go(k_step3_aa<ST, true, TRT, MRT, true>, dyn)
                    : go(k_step3_aa<ST, true, TRT, MRT, false>, de);
            else
                cur ? go(k_step3_aa<ST, false, TRT, MRT, true>, dyn)
                    : go(k_step3_aa<ST, false, TRT, MRT, false>, de);
        }
        return;
    }
    const M *src = (const M *)s.f[cur];
    M *dst = (M *)s.f[1 - cur];
    // the LDS-staged kernel once a step moves 128 MiB or more (as for D2Q9)
    const bool lds = 38.0 * (double)s.nz * s.ny * s.pitch * sizeof(M) >= 128.0 * (1 << 20);
    auto go = [&](auto kernel, uint32_t dl) {
        kernel<<<nb, kBlock, dl, s.stream>>>(src, dst, s.type, s.nmask, s.seg_interior, s.nx, s.ny,
                                           s.nz, s.pitch, bpr, nb, (R)s.omega, g[0], g[1], g[2],
                                           rt, s.fullway);
    };
    if (lds) {
        const uint32_t st = Q * (kBlock + 2u * (16u / (uint32_t)sizeof(M))) * (uint32_t)sizeof(M);
        const uint32_t dl = lbm::occupancy_cap_lds(step3_lds_cap(s, sizeof(M)), st);
        if constexpr (sizeof(M) == 2 && MRT) {
            if (s.interior_frac >= 0.9) {
                const uint32_t nb2 = bpr * (uint32_t)((s.ny + 1) / 2) * (uint32_t)s.nz;
                auto go2 = [&](auto kernel) {
                    kernel<<<nb2, kBlock, 0, s.stream>>>(src, dst, s.type, s.nmask, s.seg_interior,
                                                       s.nx, s.ny, s.nz, s.pitch, bpr, nb2,
                                                       (R)s.omega, g[0], g[1], g[2], rt, s.fullway);
                };
                if (force)
                    go2(k_step3_lds2<ST, true, TRT, MRT>);
                else
                    go2(k_step3_lds2<ST, false, TRT, MRT>);
                return;
            }
        }
        if (force)
            go(k_step3_lds<ST, true, TRT, MRT>, dl);
        else
            go(k_step3_lds<ST, false, TRT, MRT>, dl);
    } else if (force) {
        go(k_step3<ST, true, TRT, MRT>, dyn);
    } else {
        go(k_step3<ST, false, TRT, MRT>, dyn);
    }
}

template <class ST>
hipError_t step_typed(const State3 &s, int cur)
{
    if (s.mrt)
        step_launch3<ST, false, true>(s, cur);
    else if (s.trt)
        step_launch3<ST, true, false>(s, cur);
    else
        step_launch3<ST, false, false>(s, cur);
    return hipGetLastError();
}

int view_mode(const State3 &s, int cur)
{
    return s.aa ? (cur ? kAAOdd3 : kAAEven3) : kPull3;
}

uint32_t dense_blocks(const State3 &s)
{
    return (uint32_t)(((int64_t)s.nz * s.ny * s.pitch + kBlock - 1) / kBlock);
}

// Blocks of a per-node view kernel: every padded node (dense layouts) or every
// list node (INDIRECT); 0 for an empty list.
uint32_t node_blocks(const State3 &s)
{
    if (s.blocks)
        return (uint32_t)((s.n_blocks * kChunk + kBlock - 1) / kBlock);
    if (s.list)
        return (uint32_t)((s.n_fluid + kBlock - 1) / kBlock);
    return dense_blocks(s);
}

}  // namespace

hipError_t launch_step3(const State3 &s, int cur)
{
    switch (s.dtype) {
    case 0: return step_typed<F64>(s, cur);
    case 1: return step_typed<Shifted<float>>(s, cur);
    case 2: return step_typed<Shifted<_Float16>>(s, cur);
    case 3: return step_typed<Shifted<__bf16>>(s, cur);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_equilibrium3(const State3 &s, const double *rho, const double *ux,
                               const double *uy, const double *uz, double *fc)
{
    k_equilibrium3<<<dense_blocks(s), kBlock, 0, s.stream>>>(s, rho, ux, uy, uz, fc);
    return hipGetLastError();
}

// Calls fn with a value of the storage codec of the context.
template <class Fn>
hipError_t by_dtype(int dtype, Fn fn)
{
    switch (dtype) {
    case 0: fn(F64{}); break;
    case 1: fn(Shifted<float>{}); break;
    case 2: fn(Shifted<_Float16>{}); break;
    case 3: fn(Shifted<__bf16>{}); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scatter3(const State3 &s, int cur, const double *fc, int fill_walls)
{
    const uint32_t nb = node_blocks(s);
    if (nb == 0)
        return hipSuccess;
    const int walls = s.fullway ? (fill_walls ? 2 : 1) : 0;
    return by_dtype(s.dtype, [&](auto st) {
        using M = typename decltype(st)::mem;
        if (s.aa)
            k_scatter3<decltype(st)><<<nb, kBlock, 0, s.stream>>>(
                s, (M *)s.f[0], nullptr, 0, cur ? kAAOdd3 : kAAEven3, fc);
        else
            k_scatter3<decltype(st)><<<nb, kBlock, 0, s.stream>>>(
                s, (M *)s.f[cur], (M *)s.f[1 - cur], walls, kPull3, fc);
    });
}

hipError_t launch_rest3(const State3 &s, void *lattice)
{
    // (an empty block layout still holds one block of storage)
    const uint64_t stored = s.blocks ? (uint64_t)(s.n_blocks > 0 ? s.n_blocks : 1) * kChunk
                          : s.list   ? (uint64_t)s.np
                                     : (uint64_t)s.nz * s.ny * s.pitch;
    const uint64_t n = (uint64_t)Q * stored;
    uint64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 65536)
        blocks = 65536;
    return by_dtype(s.dtype, [&](auto st) {
        using M = typename decltype(st)::mem;
        k_rest3<decltype(st)><<<(uint32_t)blocks, kBlock, 0, s.stream>>>((M *)lattice, n);
    });
}

hipError_t launch_gather3(const State3 &s, int cur, double *fc)
{
    const uint32_t nb = node_blocks(s);
    if (nb == 0)
        return hipSuccess;
    return by_dtype(s.dtype, [&](auto st) {
        using M = typename decltype(st)::mem;
        const M *src = (const M *)s.f[s.aa ? 0 : cur];
        const M *bb = s.fullway ? (const M *)s.f[1 - cur] : src;
        k_gather3<decltype(st)><<<nb, kBlock, 0, s.stream>>>(s, src, bb, view_mode(s, cur), fc);
    });
}

int64_t reduction_capacity3(const State3 &s)
{
    const int64_t nb = node_blocks(s);
    return nb + (nb + 2047) / 2048 + 1;
}

hipError_t launch_macro3(const State3 &s, int cur, double *rho, double *ux, double *uy, double *uz,
                         double *mass)
{
    const uint32_t nb = node_blocks(s);
    if (nb == 0) {  // no fluid node: zero mass
        if (mass)
            k_sum3<<<1, kBlock, 0, s.stream>>>(s.red, 0, 1, mass);
        return hipGetLastError();
    }
    double *part = mass ? s.red : nullptr;
    hipError_t e = by_dtype(s.dtype, [&](auto st) {
        using M = typename decltype(st)::mem;
        const M *src = (const M *)s.f[s.aa ? 0 : cur];
        const M *bb = s.fullway ? (const M *)s.f[1 - cur] : src;
        k_macro3<decltype(st)><<<nb, kBlock, 0, s.stream>>>(s, src, bb, view_mode(s, cur), rho,
                                                            ux, uy, uz, part);
    });
    if (e != hipSuccess || !mass)
        return e;
    // fixed-order sums: blocks of 2048 partials, then one block
    const uint32_t nst = (nb + 2047) / 2048;
    k_sum3<<<nst, kBlock, 0, s.stream>>>(s.red, nb, 2048, s.red + nb);
    k_sum3<<<1, kBlock, 0, s.stream>>>(s.red + nb, nst, nst, mass);
    return hipGetLastError();
}

}  // namespace lbm3
