// Device-side building blocks of the D2Q9 step: lattice constants, storage
// codecs, the collision (one function shared by every layout, so that all
// layouts produce bitwise-identical populations), and small launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// D2Q9 lattice velocities in the paper's Fig. 1 numbering (Sec. 2.2):
// 0 rest, 1 +x, 2 +y, 3 -x, 4 -y, 5 (+x,+y), 6 (-x,+y), 7 (-x,-y), 8 (+x,-y).
__device__ constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// Equilibrium weights of Eq. 6.
__device__ constexpr double kW[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Node-type codes held in the type array (one byte per node).
enum : uint8_t {
    kFluid = 0,     // fluid node whose 8 neighbours are all fluid
    kSolid = 1,     // solid node: no populations, never updated
    kBoundary = 2,  // fluid node with at least one solid neighbour; its
                    // solid-neighbour bits are in the nmask array:
                    // bit i-1 set <=> node x - c_i is solid (i = 1..8)
    kOpen = 3,      // codes 3..10: open-boundary node with boundary code
                    // 1..8 (= code - 2, see apply_open); nmask as for kBoundary
};

// Solid-neighbour set of a node as a 9-bit mask: bit i set <=> node x - c_i is
// solid (bit 0 never set).  Interior fluid nodes need no nmask read.
__device__ __forceinline__ unsigned solid_bits(uint8_t code, const uint8_t *__restrict__ nmask,
                                               uint32_t idx)
{
    return code >= kBoundary ? (unsigned)nmask[idx] << 1 : 0u;
}

// Boundary code (0 = none, 1..8) of a dense or tiled node-type code.
__device__ __forceinline__ unsigned open_code(uint8_t code)
{
    return code >= kOpen ? (unsigned)(code - kOpen + 1) : 0u;
}

// ---------------------------------------------------------------- storage --
// A codec maps a stored population (mem) to the compute type (real) and back.
// kShift = false: the stored value is f_i itself (FP64).
// kShift = true : the stored value is the deviation h_i = f_i - w_i * rho0 with
//                 rho0 = 1 (FP32, FP16, BF16), and the collision works on h_i
//                 directly.  Near rest |h_i| << w_i, so rounding a deviation to
//                 the storage type costs far less absolute accuracy than rounding
//                 f_i itself.
// ld / st convert between storage and compute representation; canon / from_canon
// convert between storage and the canonical FP64 populations f_i.
// kExact: FP32 reciprocals are Newton-refined; the 16-bit codecs, whose storage
// rounding (2^-11 or 2^-8 of a deviation) dwarfs a 1-ulp FP32 reciprocal error,
// use the raw hardware reciprocal and save the refinement's instructions.
// kAligned: in the per-node path of the dense step (interior wavefronts of a
// row's partial last segment; whole interior segments are staged in LDS), full
// interior wavefronts gather with aligned loads and lane shifts
// (dense_pull_aligned).  It pays off for the 2-byte formats, whose shifted
// 128-byte wavefront loads would touch two cache lines instead of one; for FP32
// and FP64 the plain shifted loads are as fast and move slightly fewer bytes.
struct F64 {
    using mem = double;
    using real = double;
    static constexpr bool kShift = false;
    static constexpr bool kExact = true;
    static constexpr bool kAligned = false;
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
    static constexpr bool kExact = sizeof(M) == 4;
    static constexpr bool kAligned = sizeof(M) == 2;
    static __device__ __forceinline__ real ld(mem v, int) { return (float)v; }
    static __device__ __forceinline__ mem st(real v, int)
    {
        // Round to FP32 first, then to the 16-bit format: the empty asm keeps
        // the compiler from fusing the last FP32 FMA with the conversion (a
        // mixed-precision FMA rounds once), which it might do in some kernels
        // and not in others; every layout must round the same way.
        if constexpr (sizeof(M) == 2)
            asm volatile("" : "+v"(v));
        return (mem)v;
    }
    static __device__ __forceinline__ double canon(real v, int i) { return (double)v + kW[i]; }
    static __device__ __forceinline__ mem from_canon(double f, int i)
    {
        return (mem)(float)(f - kW[i]);
    }
};
using F32 = Shifted<float>;
using F16S = Shifted<_Float16>;
using BF16S = Shifted<__bf16>;

// -------------------------------------------------------------- collision --
// 1 / v: correctly rounded in FP64; in FP32 the hardware reciprocal refined by
// one Newton step, r + r (1 - v r) (two FMAs instead of a full division).  The
// raw reciprocal alone is 1 ulp off with a bias that accumulates over steps.
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }
__device__ __forceinline__ float recip(float v)
{
    const float r = __builtin_amdgcn_rcpf(v);
    return __builtin_fmaf(__builtin_fmaf(-v, r, 1.0f), r, r);
}
// EXACT = false: the raw FP32 hardware reciprocal (FP64 stays exact).
template <bool EXACT>
__device__ __forceinline__ double recip_p(double v) { return 1.0 / v; }
template <bool EXACT>
__device__ __forceinline__ float recip_p(float v)
{
    if constexpr (EXACT)
        return recip(v);
    else
        return __builtin_amdgcn_rcpf(v);
}

// c . v for the first direction of the k-th opposite pair (c = (1,0), (0,1),
// (1,1), (-1,1)), written out so no multiplication by a zero component is left.
template <class R>
__device__ __forceinline__ R pair_dot(int k, R vx, R vy)
{
    return k == 0 ? vx : k == 1 ? vy : k == 2 ? vx + vy : vy - vx;
}

// Collision at one fluid node, in place on f (right-hand side of Eq. 3):
//   rho = sum f_i, m = sum c_i f_i                        (Eq. 2)
//   u   = (m / rho + g / 2) / (1 + alpha / 2)             (half-force, drag)
//   F   = rho (g - alpha u)
//   f_i <- f_i - omega (f_i - f^eq_i) + (1 - omega / 2) S_i
// with f^eq of Eq. 6, omega = 1 / tau (Eq. 5) and Guo's forcing term
//   S_i = w_i [3 (c_i - u) . F + 9 (c_i . u)(c_i . F)].
// With g = 0 and alpha = 0 it is exactly the BGK update of Eqs. 3-6.
// SHIFT: f holds deviations h_i = f_i - w_i.  Since sum w_i = 1 and
// sum w_i c_i = 0, rho = 1 + sum h_i and m = sum c_i h_i, and the update keeps
// its form with f^eq_i - w_i = w_i (sum h + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)).
// FORCE = false (g = 0, no drag) drops the forcing terms, which are then
// exactly zero.  Opposite directions i, opp(i) share everything but the sign
// of the terms odd in c_i, so they are updated as a pair:
//   f^eq_{i, opp} = w (C0 + 4.5 rho (c.u)^2) +- 3 w rho (c.u),
//   S_{i, opp}    = w (9 (c.u)(c.F) - 3 u.F) +- 3 w (c.F),
// with C0 = rho (1 - 1.5 u.u), or sum h - 1.5 rho u.u for deviations.
// EXACT = false (16-bit storage): raw hardware reciprocals and u = m / rho
// taken directly (see kExact of the codecs).
// TRT: two-relaxation-time collision (a collision model beyond the paper's
// BGK): the symmetric part of each pair, fp = (f_i + f_opp(i)) / 2, relaxes
// with omega (and sets the viscosity), the antisymmetric part fm with
// omega_m; the forcing term is split the same way.  Per pair
//   P = (1 - omega) fp + omega even  [+ (1 - omega/2) S_even],
//   M = (1 - omega_m) fm + omega_m odd  [+ (1 - omega_m/2) S_odd],
//   f_i <- P + M,  f_opp(i) <- P - M,
// with even / odd the parts of f^eq; omega_m = omega is BGK.
// MRT: multiple-relaxation-time collision (moment basis of Lallemand and Luo:
// rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy, orthogonal rows with squared
// norms 9, 36, 36, 6, 12, 6, 12, 4, 4).  The moments of d = f - f^eq and of
// the forcing term S relax as
//   Delta_k = s_k d_k - (1 - s_k / 2) S_k,   f_i <- f_i - sum_k M_ki Delta_k / |M_k|^2,
// with s = s_e, s_eps on the energy moments, s_q on the energy fluxes and omega
// on the shear moments (viscosity of Eq. 5).  The conserved moments are set
// directly: Delta_rho = 0 and Delta_j = -F (whatever their rates, since
// j - j^eq = -F / 2 and S_j = F).
template <class R>
struct Rates {
    R omega_m;        // TRT: antisymmetric rate
    R s_e, s_eps, s_q;  // MRT: energy, energy square, energy flux
};

// The nine MRT moments of v in the row order above.
template <class R>
struct MrtMoments {
    R e, eps, qx, qy, pxx, pxy;
};
template <class R>
__device__ __forceinline__ MrtMoments<R> mrt_moments(const R (&v)[9])
{
    const R ax = v[1] + v[3], ay = v[2] + v[4];
    const R dg = (v[5] + v[6]) + (v[7] + v[8]);
    const R sx = v[1] - v[3], sy = v[2] - v[4];
    const R dx = (v[5] - v[6]) + (v[8] - v[7]);
    const R dy = (v[5] + v[6]) - (v[7] + v[8]);
    MrtMoments<R> m;
    m.e = R(-4) * v[0] - (ax + ay) + R(2) * dg;
    m.eps = R(4) * v[0] - R(2) * (ax + ay) + dg;
    m.qx = R(-2) * sx + dx;
    m.qy = R(-2) * sy + dy;
    m.pxx = ax - ay;
    m.pxy = (v[5] + v[7]) - (v[6] + v[8]);
    return m;
}

template <class R, bool DRAG, bool SHIFT, bool FORCE = true, bool EXACT = true, bool TRT = false,
          bool MRT = false>
__device__ __forceinline__ void collide(R (&f)[9], const R omega, const R gx, const R gy,
                                        const R alpha, const Rates<R> &rt = Rates<R>{})
{
    const R omega_m = rt.omega_m;
    const R sum = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const R mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const R my = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    // rho * v.  With deviations, rho = 1 + sum is never formed: near rho = 1 that
    // sum would round to half an FP32 ulp of 1 (6e-8), a bias that depends on the
    // local density and accumulates over steps; v + sum v keeps full precision.
    auto rho_times = [&](R v) -> R {
        if constexpr (SHIFT)
            return v + sum * v;
        else
            return sum * v;
    };
    R ux, uy;
    if constexpr (SHIFT && !EXACT) {
        const R inv_rho = recip_p<false>(R(1) + sum);
        ux = mx * inv_rho;
        uy = my * inv_rho;
    } else if constexpr (SHIFT) {
        const R q = sum * recip(R(1) + sum);  // (rho - 1) / rho
        ux = mx - mx * q;
        uy = my - my * q;
    } else {
        const R inv_rho = recip(sum);
        ux = mx * inv_rho;
        uy = my * inv_rho;
    }
    R Fx = R(0), Fy = R(0);
    if constexpr (FORCE) {
        ux += R(0.5) * gx;
        uy += R(0.5) * gy;
        if constexpr (DRAG) {
            const R invD = recip_p<EXACT>(R(1) + R(0.5) * alpha);
            ux *= invD;
            uy *= invD;
            Fx = rho_times(gx - alpha * ux);
            Fy = rho_times(gy - alpha * uy);
        } else {
            Fx = rho_times(gx);
            Fy = rho_times(gy);
        }
    }
    const R usq = R(1.5) * (ux * ux + uy * uy);
    // C0 = rho (1 - 1.5 u.u) - (1 if SHIFT): the isotropic part of f^eq / w
    const R C0 = SHIFT ? sum - rho_times(usq) : rho_times(R(1) - usq);
    const R keep = R(1) - omega;
    const R guo = R(1) - R(0.5) * omega;
    const R uF = ux * Fx + uy * Fy;
    if constexpr (MRT) {
        R d[9], sg[9];
        {
            const R w = R(kW[0]);
            d[0] = f[0] - w * C0;
            sg[0] = FORCE ? w * (R(-3) * uF) : R(0);
        }
        constexpr int PM[4] = {1, 2, 5, 6};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = PM[k], j = kOpp[i];
            const R w = R(kW[i]);
            const R cu = pair_dot(k, ux, uy);
            const R even = w * (C0 + rho_times(R(4.5) * (cu * cu)));
            const R odd = w * rho_times(R(3) * cu);
            d[i] = f[i] - (even + odd);
            d[j] = f[j] - (even - odd);
            if constexpr (FORCE) {
                const R cF = pair_dot(k, Fx, Fy);
                const R se = w * (R(9) * cu * cF - R(3) * uF);
                const R so = R(3) * w * cF;
                sg[i] = se + so;
                sg[j] = se - so;
            } else {
                sg[i] = sg[j] = R(0);
            }
        }
        const MrtMoments<R> md = mrt_moments(d);
        MrtMoments<R> ms{};
        if constexpr (FORCE)
            ms = mrt_moments(sg);
        auto relax = [](R s, R dk, R sk) {
            if constexpr (FORCE)
                return s * dk - (R(1) - R(0.5) * s) * sk;
            else
                return s * dk;
        };
        const R b = relax(rt.s_e, md.e, ms.e) * R(1.0 / 36.0);
        const R c = relax(rt.s_eps, md.eps, ms.eps) * R(1.0 / 36.0);
        const R qx = relax(rt.s_q, md.qx, ms.qx) * R(1.0 / 12.0);
        const R qy = relax(rt.s_q, md.qy, ms.qy) * R(1.0 / 12.0);
        const R p = relax(omega, md.pxx, ms.pxx) * R(0.25);
        const R r = relax(omega, md.pxy, ms.pxy) * R(0.25);
        const R jx = FORCE ? Fx * R(-1.0 / 6.0) : R(0);
        const R jy = FORCE ? Fy * R(-1.0 / 6.0) : R(0);
        // f_i -= sum_k M_ki Delta_k / |M_k|^2 (rows written out per direction)
        f[0] -= R(4) * (c - b);
        const R A = -(b + R(2) * c), D = R(2) * b + c;
        const R X = jx + qx, Y = jy + qy;
        f[1] -= A + (jx - R(2) * qx) + p;
        f[3] -= A - (jx - R(2) * qx) + p;
        f[2] -= A + (jy - R(2) * qy) - p;
        f[4] -= A - (jy - R(2) * qy) - p;
        f[5] -= D + X + Y + r;
        f[6] -= D - X + Y - r;
        f[7] -= D - X - Y + r;
        f[8] -= D + X - Y - r;
        return;
    }
    // rest population
    {
        const R w = R(kW[0]);
        R s = keep * f[0] + omega * (w * C0);
        if constexpr (FORCE)
            s += guo * (w * (R(-3) * uF));
        f[0] = s;
    }
    // pairs (i, opp(i)) with c_i = (1,0), (0,1), (1,1), (-1,1)
    constexpr int P[4] = {1, 2, 5, 6};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = P[k], j = kOpp[i];
        const R w = R(kW[i]);
        const R cu = pair_dot(k, ux, uy);
        const R even = w * (C0 + rho_times(R(4.5) * (cu * cu)));
        const R odd = w * rho_times(R(3) * cu);
        if constexpr (TRT) {
            const R fp = R(0.5) * (f[i] + f[j]), fm = R(0.5) * (f[i] - f[j]);
            R P = keep * fp + omega * even;
            R M = (R(1) - omega_m) * fm + omega_m * odd;
            if constexpr (FORCE) {
                const R cF = pair_dot(k, Fx, Fy);
                P += guo * (w * (R(9) * cu * cF - R(3) * uF));
                M += (R(1) - R(0.5) * omega_m) * (R(3) * w * cF);
            }
            f[i] = P + M;
            f[j] = P - M;
            continue;
        }
        R a = keep * f[i] + omega * (even + odd);
        R b = keep * f[j] + omega * (even - odd);
        if constexpr (FORCE) {
            const R cF = pair_dot(k, Fx, Fy);
            const R se = w * (R(9) * cu * cF - R(3) * uF);
            const R so = R(3) * w * cF;
            a += guo * (se + so);
            b += guo * (se - so);
        }
        f[i] = a;
        f[j] = b;
    }
}

// Macroscopic moments of the canonical populations (Eq. 2 with the same
// corrected velocity the collision uses), in FP64.
// ---------------------------------------------------- open boundaries --
// Constant-velocity / constant-pressure node (Sec. 3, after Zou and He).
// Boundary code b = 1..8: 1..4 constant velocity with inward normal n = +x,
// -x, +y, -y; 5..8 constant pressure with the same normals; unit tangent
// t = (-n_y, n_x).  v = the node's two FP64 boundary values: (u_x, u_y), or
// (rho, unused).
// The three populations entering across the boundary (c_i . n > 0) are
// rebuilt from the other six so that the node's density and momentum (Eq. 2)
// take the prescribed values and the normal pair has equal non-equilibrium
// parts.  With S = sum_{c.n=0} f + 2 sum_{c.n<0} f and T = sum_{c.n=0} (c.t) f:
//   velocity (u prescribed): rho = S / (1 - u.n);
//   pressure (rho prescribed, u.t = 0): rho u.n = rho - S;
//   normal direction: f_i = f_opp(i) + (2/3) rho u.n;
//   diagonals, s_i = c_i . t = +-1:
//     f_i = f_opp(i) + rho u.n / 6 + (s_i / 2) (rho u.t - T).
// Shifted storage holds h = f - w: opposite populations have equal weights and
// the weights in S sum to 1, so in deviations S_h = S - 1, T is unchanged and
// the rebuilt h_i use the same relations, with rho = 1 + drho carried as drho:
//   velocity: drho = (S_h + u.n) / (1 - u.n); pressure: rho u.n = (rho - 1) - S_h.
// Written with the normal as a runtime value and every population index a
// compile-time constant (the roles of the directions become predicates), so
// that the populations stay in registers.
template <class R, bool SHIFT>
__device__ __forceinline__ void apply_open(R (&f)[9], unsigned b, const double *__restrict__ v)
{
    const unsigned k = (b - 1u) & 3u;  // normal +x, -x, +y, -y
    const int nxn = k == 0 ? 1 : (k == 1 ? -1 : 0);
    const int nyn = k == 2 ? 1 : (k == 3 ? -1 : 0);
    const int tx = -nyn, ty = nxn;
    const bool velocity = b <= 4u;
    const double v0 = v[0], v1 = v[1];
    R par = R(0), outg = R(0), tsum = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int d = kCx[i] * nxn + kCy[i] * nyn;
        const int si = kCx[i] * tx + kCy[i] * ty;
        par += d == 0 ? f[i] : R(0);
        outg += d < 0 ? f[i] : R(0);
        tsum += d == 0 ? (si > 0 ? f[i] : (si < 0 ? -f[i] : R(0))) : R(0);
    }
    const R S = par + R(2) * outg;
    R run, rut;  // rho u.n, rho u.t
    if (velocity) {
        const R un = (R)(v0 * nxn + v1 * nyn), ut = (R)(v0 * tx + v1 * ty);
        if constexpr (SHIFT) {
            const R drho = (S + un) / (R(1) - un);
            run = un + drho * un;
            rut = ut + drho * ut;
        } else {
            const R rho = S / (R(1) - un);
            run = rho * un;
            rut = rho * ut;
        }
    } else {
        run = SHIFT ? (R)(v0 - 1.0) - S : (R)v0 - S;
        rut = R(0);
    }
    const R tang = R(0.5) * (rut - tsum);
    const R diag = run * R(1.0 / 6.0);
    const R axis = run * R(2.0 / 3.0);
    R g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int d = kCx[i] * nxn + kCy[i] * nyn;
        const int si = kCx[i] * tx + kCy[i] * ty;
        const R inc = si == 0 ? axis : (si > 0 ? diag + tang : diag - tang);
        g[i] = d > 0 ? f[kOpp[i]] + inc : f[i];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i] = g[i];
}

__device__ __forceinline__ void moments(const double (&f)[9], double gx, double gy, double alpha,
                                        double &rho, double &ux, double &uy)
{
    rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const double mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const double my = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const double invD = 1.0 / (1.0 + 0.5 * alpha);
    ux = (mx / rho + 0.5 * gx) * invD;
    uy = (my / rho + 0.5 * gy) * invD;
}

// ------------------------------------------------------------- launching --
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap the hardware block index so that XCD j processes one contiguous
// range of logical blocks: neighbouring blocks, which share cache lines at
// their edges, then run on the same XCD.  A bijection on [0, n).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n)
{
    const uint32_t q = n >> 3, r = n & 7u, j = b & 7u, k = b >> 3;
    return j * q + (j < r ? j : r) + k;
}

// Dynamic LDS bytes that cap a launch at `wg` resident workgroups per CU
// (0: no cap), for a kernel with `static_lds` bytes of its own: each workgroup
// then holds just over 1 / (wg + 1) of the CU's 160 KB of LDS.
inline uint32_t occupancy_cap_lds(int wg, uint32_t static_lds)
{
    if (wg <= 0)
        return 0u;
    const uint32_t want = 163840u * 2u / (2u * (uint32_t)wg + 1u);
    return want > static_lds ? want - static_lds : 0u;
}

// Periodic neighbour coordinates.
__device__ __forceinline__ int wrap_dec(int a, int n) { return a == 0 ? n - 1 : a - 1; }
__device__ __forceinline__ int wrap_inc(int a, int n) { return a == n - 1 ? 0 : a + 1; }

// ---------------------------------------------------------- population layouts --
// Populations are stored array-of-structures-of-arrays: the nodes are cut into
// chunks, and a chunk holds its 9 populations one after another, each as a run
// of consecutive nodes.  Population i of the node with base offset b sits at
// b + i * stride.  A 64-lane wavefront then reads or writes 9 contiguous runs
// inside one chunk instead of 9 far-apart planes, which keeps the DRAM access
// stream close to a copy's.
//  dense rows : chunks of 64 nodes along x; node (x, y) -> chunk y * cpr + x / 64
//               (cpr = pitch / 64 chunks per row), stride 64
//  node lists : chunks of 64 consecutive list entries, stride 64
//  tiles      : one chunk per 16 x 16 tile (256 nodes), stride 256; inside a
//               tile the nodes run in 4 x 4 blocks (tile_slot), so that a
//               128-byte line holds a compact block of nodes, not a strip of a
//               row: on sparse geometries fewer lines then mix fluid and solid
//               nodes (4 tile rows, one wavefront, stay one contiguous run)
constexpr uint32_t kChunk = 64;
constexpr uint32_t kTileStride = 256;

__device__ __forceinline__ uint64_t dense_base(int x, int y, uint32_t cpr)
{
    return ((uint64_t)y * cpr + ((uint32_t)x >> 6)) * (9u * kChunk) + ((uint32_t)x & 63u);
}
__device__ __forceinline__ uint32_t list_base(uint32_t n)
{
    return (n >> 6) * (9u * kChunk) + (n & 63u);
}
__device__ __forceinline__ uint32_t tile_base(uint32_t k, uint32_t t)
{
    return k * (9u * kTileStride) + t;
}
// In-tile slot of node (lx, ly), 0 <= lx, ly < 16: bits ly3 ly2 | lx3 lx2 |
// ly1 ly0 | lx1 lx0 (4 x 4 blocks, blocks row-major, nodes row-major inside).
__device__ __forceinline__ uint32_t tile_slot(uint32_t lx, uint32_t ly)
{
    return ((ly & 12u) << 4) | ((lx & 12u) << 2) | ((ly & 3u) << 2) | (lx & 3u);
}

// nb[i] = base offset of node x - c_i (periodic) in the dense layout;
// nb[0] = the node itself.  Dense offsets are 64-bit (a lattice may exceed 2^32
// elements); tile and node-list offsets stay 32-bit.
__device__ __forceinline__ void dense_bases(int x, int y, int nx, int ny, uint32_t cpr,
                                            uint64_t (&nb)[9])
{
    const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
    const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
    nb[0] = dense_base(x, y, cpr);
    nb[1] = dense_base(xm, y, cpr);   // c1 = (+1, 0)
    nb[2] = dense_base(x, ym, cpr);   // c2 = (0, +1)
    nb[3] = dense_base(xp, y, cpr);   // c3 = (-1, 0)
    nb[4] = dense_base(x, yp, cpr);   // c4 = (0, -1)
    nb[5] = dense_base(xm, ym, cpr);  // c5 = (+1, +1)
    nb[6] = dense_base(xp, ym, cpr);  // c6 = (-1, +1)
    nb[7] = dense_base(xp, yp, cpr);  // c7 = (-1, -1)
    nb[8] = dense_base(xm, yp, cpr);  // c8 = (+1, -1)
}

// Streaming stores: the lattice written by a step is not read again until the
// next step, so the stores bypass the caches' retention (nontemporal).
// Dense addressing split into row and column parts: node (x, y) has base
// offset row_off(y) + col_off(x).  A step workgroup is one row segment, so the
// three row offsets (rows y-1, y, y+1) are uniform (64-bit, scalar registers)
// and each lane keeps three column offsets (columns x-1, x, x+1), which stay
// below 2^28 (the runtime bounds 9 * pitch), so that a load address is a
// scalar base plus a 32-bit lane offset.
struct DenseRC {
    uint64_t r[3];  // rows y-1, y, y+1
    uint32_t c[3];  // columns x-1, x, x+1
};

__device__ __forceinline__ uint32_t col_off(int x)
{
    return ((((uint32_t)x >> 6) * (9u * kChunk)) | ((uint32_t)x & 63u)) & 0x0FFFFFFFu;
}

__device__ __forceinline__ DenseRC dense_rc(int x, int y, int nx, int ny, uint32_t cpr)
{
    DenseRC a;
    const uint64_t row = (uint64_t)cpr * (9u * kChunk);
    a.r[0] = (uint64_t)wrap_dec(y, ny) * row;
    a.r[1] = (uint64_t)y * row;
    a.r[2] = (uint64_t)wrap_inc(y, ny) * row;
    a.c[0] = col_off(wrap_dec(x, nx));
    a.c[1] = col_off(x);
    a.c[2] = col_off(wrap_inc(x, nx));
    return a;
}

// Element of population plane `i` at row slot `ri`, column slot `ci` of a
// dense lattice: scalar part i * 64 + r[ri], lane part c[ci].
template <class M>
__device__ __forceinline__ M &dense_at(M *__restrict__ s, const DenseRC &a, int i, int ri, int ci)
{
    M *p = s + ((uint64_t)i * kChunk + a.r[ri]);
    return p[a.c[ci]];
}

template <class T>
__device__ __forceinline__ void store_nt(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}
template <>
__device__ __forceinline__ void store_nt<__bf16>(__bf16 *p, __bf16 v)
{
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), (unsigned short *)p);
}

// Streaming load (nontemporal hint), for populations that a kernel reads once
// and nothing reuses from the cache.
template <class T>
__device__ __forceinline__ T load_nt(const T *p)
{
    return __builtin_nontemporal_load(p);
}
template <>
__device__ __forceinline__ __bf16 load_nt<__bf16>(const __bf16 *p)
{
    return __builtin_bit_cast(__bf16, __builtin_nontemporal_load((const unsigned short *)p));
}

}  // namespace lbm
