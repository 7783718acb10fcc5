// Hand-written adjoint of the fused D2Q9 step (dense A-B layout, F64 / F32).
//
// Forward map on canonical populations: f(t+1) = Stream(C(f(t); alpha, g)),
// with C the collision of the step kernel and Stream the pull streaming with
// halfway bounce-back (a permutation of fluid slots).  With lambda_t = dJ/df(t):
//   nu(x)_i      = lambda_{t+1,i}(x + c_i), or lambda_{t+1,opp(i)}(x) when
//                  x + c_i is solid             (transposed streaming: reverse pull)
//   lambda_t(x)  = (dC/df)^T nu(x)              (transposed collision Jacobian)
//   dJ/dalpha(x) += nu(x) . dC/dalpha,   dJ/dg += sum_x nu(x) . dC/dg
// f(t)(x) is recomputed from the stored lattice at step t by the same pull
// gather as the forward kernel.  The vector-Jacobian product below runs the
// collision's statements backwards (reverse-mode differentiation by hand).
// Gradients accumulate in FP64; the per-block dJ/dg partials are summed in a
// fixed order, so results are repeatable.
#include <mutex>

#include "lbm_device.h"
#include "lbm_launch.h"

namespace lbm {
namespace {

constexpr int kBlock = 256;

// Reverse of collide<R, DRAG, SHIFT>: given the pre-collision f and the adjoint nu of
// the post-collision populations, return fb = (dC/df)^T nu, ab = nu . dC/dalpha
// and (gbx, gby) = nu . dC/dg.  Opposite directions i, j = opp(i) are taken as a
// pair, as in the forward collision: c_j = -c_i flips the sign of c.u and c.F,
// so with e = omega w nu and s = (1 - omega/2) w nu the pair contributes
//   to rho:    (e_i + e_j)(1 + 4.5 (c.u)^2 - 1.5 u.u) + 3 (c.u)(e_i - e_j),
//   to u:      c_i [rho (3 (e_i - e_j) + 9 (c.u)(e_i + e_j)) + 9 (c.F)(s_i + s_j)],
//   to F:      c_i [3 (s_i - s_j) + 9 (c.u)(s_i + s_j)],
// and -rho e, -3 s to the adjoints of 1.5 u.u and u.F for every direction.
template <class R, bool DRAG, bool SHIFT>
__device__ __forceinline__ void collide_vjp(const R (&f)[9], const R (&nu)[9], const R omega,
                                            const R gx, const R gy, const R alpha, R (&fb)[9],
                                            R &ab, R &gbx, R &gby)
{
    // forward recomputation (same statements as collide; with SHIFT, f holds the
    // deviations h_i = f_i - w_i and d/dh_i = d/df_i)
    const R sum = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const R rho = SHIFT ? R(1) + sum : sum;
    const R mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const R my = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const R inv_rho = recip(rho);
    const R ux0 = mx * inv_rho + R(0.5) * gx;
    const R uy0 = my * inv_rho + R(0.5) * gy;
    R ux = ux0, uy = uy0, invD = R(1);
    if constexpr (DRAG) {
        invD = recip(R(1) + R(0.5) * alpha);
        ux = ux0 * invD;
        uy = uy0 * invD;
    }
    const R a = DRAG ? alpha : R(0);
    const R Fx = rho * (gx - a * ux), Fy = rho * (gy - a * uy);
    const R usq = R(1.5) * (ux * ux + uy * uy);
    const R guo = R(1) - R(0.5) * omega;

    // reverse sweep: rest population, then the four opposite pairs
    R rhob, esum, ssum, ubx = R(0), uby = R(0), Fbx = R(0), Fby = R(0);
    {
        const R t = nu[0] * R(kW[0]);
        const R e = omega * t;
        rhob = e * (R(1) - usq);
        esum = e;
        ssum = guo * t;
    }
    constexpr int P[4] = {1, 2, 5, 6};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = P[k], j = kOpp[i];
        const R w = R(kW[i]);
        const R tp = (nu[i] + nu[j]) * w, tm = (nu[i] - nu[j]) * w;
        const R ep = omega * tp, em = omega * tm, sp = guo * tp, sm = guo * tm;
        const R cu = pair_dot(k, ux, uy), cF = pair_dot(k, Fx, Fy);
        rhob += ep * (R(1) + R(4.5) * cu * cu - usq) + R(3) * cu * em;
        esum += ep;
        ssum += sp;
        const R du = rho * (R(3) * em + R(9) * cu * ep) + R(9) * cF * sp;
        const R dF = R(3) * sm + R(9) * cu * sp;
        // along c_i = (1,0), (0,1), (1,1), (-1,1)
        if (k != 1) {
            ubx += k == 3 ? -du : du;
            Fbx += k == 3 ? -dF : dF;
        }
        if (k != 0) {
            uby += du;
            Fby += dF;
        }
    }
    const R usqb = -rho * esum, uFb = R(-3) * ssum;
    // uF = u . F and usq = 1.5 u . u
    ubx += uFb * Fx + R(3) * usqb * ux;
    uby += uFb * Fy + R(3) * usqb * uy;
    Fbx += uFb * ux;
    Fby += uFb * uy;
    // F = rho (g - alpha u)
    rhob += Fbx * (gx - a * ux) + Fby * (gy - a * uy);
    if constexpr (DRAG) {
        ubx -= rho * a * Fbx;
        uby -= rho * a * Fby;
    }
    gbx = rho * Fbx;
    gby = rho * Fby;
    ab = -rho * (Fbx * ux + Fby * uy);
    // u = u0 / (1 + alpha / 2)
    R u0bx = ubx, u0by = uby;
    if constexpr (DRAG) {
        u0bx = ubx * invD;
        u0by = uby * invD;
        const R invDb = ubx * ux0 + uby * uy0;
        ab -= R(0.5) * invDb * invD * invD;
    }
    // u0 = m / rho + g / 2
    const R mbx = u0bx * inv_rho, mby = u0by * inv_rho;
    const R inv_rhob = u0bx * mx + u0by * my;
    gbx += R(0.5) * u0bx;
    gby += R(0.5) * u0by;
    rhob -= inv_rhob * inv_rho * inv_rho;
    // rho = sum f, m = sum c f; plus the direct (1 - omega) f_i term
    const R keep = R(1) - omega;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        R acc = keep * nu[j] + rhob;
        if (kCx[j] > 0)
            acc += mbx;
        else if (kCx[j] < 0)
            acc -= mbx;
        if (kCy[j] > 0)
            acc += mby;
        else if (kCy[j] < 0)
            acc -= mby;
        fb[j] = acc;
    }
}

// Sum of two values over one wavefront (valid in lane 0); no barrier.
__device__ __forceinline__ void wave_sum2(double &a, double &b)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
}

__device__ __forceinline__ void block_sum2(double &a, double &b)
{
    __shared__ double ws[2][kBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        ws[0][w] = a;
        ws[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0;
        for (int i = 0; i < kBlock / 64; ++i) {
            s0 += ws[0][i];
            s1 += ws[1][i];
        }
        a = s0;
        b = s1;
    }
}

template <class ST, bool DRAG>
__global__ __launch_bounds__(kBlock) void k_adjoint_step(
    const typename ST::mem *__restrict__ state, const typename ST::real *__restrict__ mu_in,
    typename ST::real *__restrict__ mu_out, const uint8_t *__restrict__ type,
    const uint8_t *__restrict__ nmask, const uint32_t *__restrict__ seg_interior,
    const float *__restrict__ alpha, double *__restrict__ grad_alpha,
    double *__restrict__ partials, int accumulate, int nx, int ny, int pitch, uint32_t bpr,
    uint32_t nblocks, typename ST::real omega, typename ST::real gx, typename ST::real gy)
{
    using R = typename ST::real;
    using M = typename ST::mem;
    const uint32_t L = xcd_remap(blockIdx.x, nblocks);
    const int y = (int)(L / bpr);
    const int x = (int)(L - (uint32_t)y * bpr) * kBlock + (int)threadIdx.x;
    double gxs = 0.0, gys = 0.0;
    if (x < nx) {
        const uint32_t own = (uint32_t)y * pitch + x;
        // all-interior row segments read neither the node type nor the neighbour bits
        unsigned sm = 0;
        bool fluid = true;
        if (!seg_interior[L]) {
            const uint8_t t = type[own];
            fluid = t != kSolid;
            sm = solid_bits(t, nmask, own);
        }
        if (fluid) {
            const DenseRC a = dense_rc(x, y, nx, ny, (uint32_t)pitch / kChunk);
            M *sp = const_cast<M *>(state);
            R *mp = const_cast<R *>(mu_in);
            R f[9], nu[9];
            if (sm == 0) {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    // forward pull f_i(x) = s_i(x - c_i); reverse pull nu_i = mu_i(x + c_i)
                    f[i] = ST::ld(dense_at(sp, a, i, 1 - kCy[i], 1 - kCx[i]), i);
                    nu[i] = dense_at(mp, a, i, 1 + kCy[i], 1 + kCx[i]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    // x - c_i solid: bounce-back slot s_opp(i)(x); x + c_i is node
                    // x - c_opp(i), solid: the adjoint of that bounce-back, mu_opp(i)(x)
                    f[i] = ST::ld(((sm >> i) & 1u) ? dense_at(sp, a, kOpp[i], 1, 1)
                                                   : dense_at(sp, a, i, 1 - kCy[i], 1 - kCx[i]),
                                  i);
                    nu[i] = ((sm >> kOpp[i]) & 1u) ? dense_at(mp, a, kOpp[i], 1, 1)
                                                   : dense_at(mp, a, i, 1 + kCy[i], 1 + kCx[i]);
                }
            }
            const R al = DRAG ? (R)alpha[own] : R(0);
            R fb[9], ab, gbx, gby;
            collide_vjp<R, DRAG, ST::kShift>(f, nu, omega, gx, gy, al, fb, ab, gbx, gby);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                store_nt(&dense_at(mu_out, a, i, 1, 1), fb[i]);
            if (DRAG)
                grad_alpha[(size_t)y * nx + x] += (double)ab;
            gxs = (double)gbx;
            gys = (double)gby;
        }
    }
    // one dJ/dg partial pair per wavefront (no workgroup barrier)
    wave_sum2(gxs, gys);
    if ((threadIdx.x & 63u) == 0) {
        const uint32_t p = 2u * (blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
        if (accumulate) {
            partials[p] += gxs;
            partials[p + 1] += gys;
        } else {
            partials[p] = gxs;
            partials[p + 1] = gys;
        }
    }
}

// lambda_T = scale * d(sum over column x_col of u_x)/df at the canonical state
// pulled from the stored lattice, zero elsewhere; direct alpha / g terms too.
template <class ST>
__global__ __launch_bounds__(kBlock) void k_adjoint_seed(
    const typename ST::mem *__restrict__ state, typename ST::real *__restrict__ mu,
    const uint8_t *__restrict__ type, const uint8_t *__restrict__ nmask,
    const float *__restrict__ alpha, double *__restrict__ grad_alpha, double *__restrict__ partials,
    int x_col, double scale, int nx, int ny, int pitch, double gx, double gy)
{
    using R = typename ST::real;
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    const int y = (int)(gid / (uint32_t)pitch), x = (int)(gid - (uint32_t)y * pitch);
    double gxs = 0.0;
    if (y < ny) {
        R lam[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (x == x_col && type[gid] != kSolid) {
            const unsigned sm = solid_bits(type[gid], nmask, gid);
            uint64_t nb[9];
            dense_bases(x, y, nx, ny, (uint32_t)pitch / kChunk, nb);
            double f[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint64_t o = ((sm >> i) & 1u) ? (uint64_t)kOpp[i] * kChunk + nb[0]
                                                    : (uint64_t)i * kChunk + nb[i];
                f[i] = ST::canon(ST::ld(state[o], i), i);
            }
            const double al = alpha ? (double)alpha[gid] : 0.0;
            const double rho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
            const double mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
            const double invD = 1.0 / (1.0 + 0.5 * al);
            const double ux = (mx / rho + 0.5 * gx) * invD;
            // u_x = (m_x / rho + g_x / 2) / D:  du_x/df_j = (c_jx - m_x / rho) / (rho D)
#pragma unroll
            for (int j = 0; j < 9; ++j)
                lam[j] = (R)(scale * (kCx[j] - mx / rho) * invD / rho);
            if (alpha)
                grad_alpha[(size_t)y * nx + x] += scale * (-0.5 * ux * invD);
            gxs = scale * 0.5 * invD;
        }
        const uint64_t base = dense_base(x, y, (uint32_t)pitch / kChunk);
#pragma unroll
        for (int j = 0; j < 9; ++j)
            mu[(uint64_t)j * kChunk + base] = lam[j];
    }
    double gys = 0.0;
    block_sum2(gxs, gys);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = gxs;
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

// grad_g += fixed-order sum of n partial pairs (one block).
// Two-stage fixed-order sum of n interleaved (dJ/dg_x, dJ/dg_y) partial pairs:
// block b of the first stage adds pairs [b * kSumPer, (b + 1) * kSumPer).
constexpr uint32_t kSumPer = 2048;

__global__ __launch_bounds__(kBlock) void k_pairs_stage(const double *__restrict__ in, uint32_t n,
                                                        double *__restrict__ out)
{
    const uint32_t lo = blockIdx.x * kSumPer;
    const uint32_t hi = lo + kSumPer < n ? lo + kSumPer : n;
    double a = 0.0, b = 0.0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        a += in[2 * i];
        b += in[2 * i + 1];
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = a;
        out[2 * blockIdx.x + 1] = b;
    }
}

__global__ __launch_bounds__(kBlock) void k_partials_into(const double *__restrict__ partials,
                                                          uint32_t n, double *grad_g)
{
    double a = 0.0, b = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        grad_g[0] += a;
        grad_g[1] += b;
    }
}

__global__ __launch_bounds__(kBlock) void k_zero(double *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        p[i] = 0.0;
}

// Adjoint field (chunked, compute type) <-> plain FP64 planes [9][ny][nx];
// solid and padding entries read as / are written from zero.
template <class R>
__global__ __launch_bounds__(kBlock) void k_adjoint_convert(R *__restrict__ mu,
                                                            double *__restrict__ plain,
                                                            const uint8_t *__restrict__ type,
                                                            int nx, int ny, int pitch,
                                                            int to_plain)
{
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    const int y = (int)(gid / (uint32_t)pitch), x = (int)(gid - (uint32_t)y * pitch);
    if (y >= ny)
        return;
    const uint64_t base = dense_base(x, y, (uint32_t)pitch / kChunk);
    const bool fluid = x < nx && type[gid] != kSolid;
    for (int i = 0; i < 9; ++i) {
        if (to_plain) {
            if (x < nx)
                plain[((size_t)i * ny + y) * nx + x] = fluid ? (double)mu[(uint64_t)i * kChunk + base] : 0.0;
        } else {
            mu[(uint64_t)i * kChunk + base] =
                fluid ? (R)plain[((size_t)i * ny + y) * nx + x] : R(0);
        }
    }
}

// Resident workgroups per CU of the adjoint step on mostly interior lattices
// (0: as many as registers allow), measured on a 4096^2 channel with a drag
// field: FP32 372.8 us at 4 per CU against 390.2 us uncapped (3: 385.0, 6:
// 385.1), FP64 681.8 us at 3 against 699.5 us (4: 692.9, 6: 698.5).
inline int adjoint_cap(const DevState &s, size_t esize)
{
    if (s.interior_frac < 0.9)
        return 0;
    return esize == 8 ? 3 : 4;
}

template <class ST>
hipError_t step_typed(const DevState &s, const void *state, const void *mu_in, void *mu_out,
                      double *grad_alpha, double *partials, int accumulate)
{
    using R = typename ST::real;
    const uint32_t bpr = (uint32_t)((s.nx + kBlock - 1) / kBlock);
    const uint32_t nblocks = bpr * (uint32_t)s.ny;
    const R om = (R)s.omega, gx = (R)s.gx, gy = (R)s.gy;
    const uint32_t dyn = occupancy_cap_lds(adjoint_cap(s, sizeof(typename ST::mem)), 0u);
    if (s.alpha)
        k_adjoint_step<ST, true><<<nblocks, kBlock, dyn, s.stream>>>(
            (const typename ST::mem *)state, (const R *)mu_in, (R *)mu_out, s.type, s.nmask,
            s.seg_interior, s.alpha, grad_alpha, partials, accumulate, s.nx, s.ny, s.pitch, bpr,
            nblocks, om, gx, gy);
    else
        k_adjoint_step<ST, false><<<nblocks, kBlock, dyn, s.stream>>>(
            (const typename ST::mem *)state, (const R *)mu_in, (R *)mu_out, s.type, s.nmask,
            s.seg_interior, s.alpha, grad_alpha, partials, accumulate, s.nx, s.ny, s.pitch, bpr,
            nblocks, om, gx, gy);
    return hipGetLastError();
}

}  // namespace

int64_t adjoint_blocks(const DevState &s)
{
    return (int64_t)((s.nx + kBlock - 1) / kBlock) * s.ny;
}

int64_t adjoint_step_partials(const DevState &s) { return adjoint_blocks(s) * (kBlock / 64); }

int64_t adjoint_scratch_pairs(const DevState &s)
{
    const int64_t n = std::max(adjoint_step_partials(s), adjoint_seed_blocks(s));
    return n + (n + kSumPer - 1) / kSumPer + 1;
}

int64_t adjoint_seed_blocks(const DevState &s) { return ((int64_t)s.ny * s.pitch + kBlock - 1) / kBlock; }

hipError_t launch_adjoint_step_raw(const DevState &s, const void *state, const void *mu_in,
                                   void *mu_out, double *grad_alpha, double *partials,
                                   int accumulate)
{
    if (s.dtype == kF64)
        return step_typed<F64>(s, state, mu_in, mu_out, grad_alpha, partials, accumulate);
    if (s.dtype == kF32)
        return step_typed<F32>(s, state, mu_in, mu_out, grad_alpha, partials, accumulate);
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_seed_raw(const DevState &s, const void *state, int x_col, double scale,
                                   void *mu, double *grad_alpha, double *partials)
{
    const uint32_t blocks = (uint32_t)adjoint_seed_blocks(s);
    if (s.dtype == kF64)
        k_adjoint_seed<F64><<<blocks, kBlock, 0, s.stream>>>(
            (const double *)state, (double *)mu, s.type, s.nmask, s.alpha, grad_alpha, partials,
            x_col, scale, s.nx, s.ny, s.pitch, s.gx, s.gy);
    else if (s.dtype == kF32)
        k_adjoint_seed<F32><<<blocks, kBlock, 0, s.stream>>>(
            (const float *)state, (float *)mu, s.type, s.nmask, s.alpha, grad_alpha, partials,
            x_col, scale, s.nx, s.ny, s.pitch, s.gx, s.gy);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_adjoint_convert(const DevState &s, void *mu, double *plain, int to_plain)
{
    const uint32_t blocks = (uint32_t)adjoint_seed_blocks(s);
    if (s.dtype == kF64)
        k_adjoint_convert<double><<<blocks, kBlock, 0, s.stream>>>(
            (double *)mu, plain, s.type, s.nx, s.ny, s.pitch, to_plain);
    else if (s.dtype == kF32)
        k_adjoint_convert<float><<<blocks, kBlock, 0, s.stream>>>(
            (float *)mu, plain, s.type, s.nx, s.ny, s.pitch, to_plain);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_partials_into(double *partials, int64_t n, double *grad_g,
                                hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    if (n <= 4 * (int64_t)kSumPer) {  // few partials: one block, one launch
        k_partials_into<<<1, kBlock, 0, stream>>>(partials, (uint32_t)n, grad_g);
        return hipGetLastError();
    }
    // stage results go right after the n pairs (see adjoint_scratch_pairs)
    const int64_t nst = (n + kSumPer - 1) / kSumPer;
    double *stage = partials + 2 * n;
    k_pairs_stage<<<(uint32_t)nst, kBlock, 0, stream>>>(partials, (uint32_t)n, stage);
    k_partials_into<<<1, kBlock, 0, stream>>>(stage, (uint32_t)nst, grad_g);
    return hipGetLastError();
}

// ------------------------------------------------ allocation-free scratch --
// dJ/dg partial pairs (and their reduction stage) of lbm_adjoint_step_noalloc,
// in a fixed array that each GPU the library runs on holds until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host it
// names a stand-in, not device memory): it takes the device address from
// hipGetSymbolAddress, once per device with that device current, and passes
// that.  Every call on one GPU shares its array.
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[kMaxDevices] = {};
}  // namespace

int64_t adjoint_step_scratch_doubles(const DevState &s)
{
    const int64_t n = adjoint_step_partials(s);
    // the partial pairs, then (above 4 * kSumPer pairs) one stage pair per kSumPer
    return 2 * (n + (n > 4 * (int64_t)kSumPer ? (n + kSumPer - 1) / kSumPer : 0));
}

hipError_t noalloc_scratch(int device, double **ptr)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess)
            return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess)
            return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess)
                e = e2;
        }
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_addr[device] = (double *)p;
    }
    *ptr = g_scratch_addr[device];
    return hipSuccess;
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    uint32_t blocks = (uint32_t)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    k_zero<<<blocks, kBlock, 0, stream>>>(p, (uint32_t)n);
    return hipGetLastError();
}

}  // namespace lbm
