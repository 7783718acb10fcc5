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
#include "lbm_device.h"
#include "lbm_launch.h"

namespace lbm {
namespace {

constexpr int kBlock = 256;

// Reverse of collide<R, DRAG, SHIFT>: given the pre-collision f and the adjoint nu of
// the post-collision populations, return fb = (dC/df)^T nu, ab = nu . dC/dalpha
// and (gbx, gby) = nu . dC/dg.
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
    const R inv_rho = R(1) / rho;
    const R ux0 = mx * inv_rho + R(0.5) * gx;
    const R uy0 = my * inv_rho + R(0.5) * gy;
    R ux = ux0, uy = uy0, invD = R(1);
    if constexpr (DRAG) {
        invD = R(1) / (R(1) + R(0.5) * alpha);
        ux = ux0 * invD;
        uy = uy0 * invD;
    }
    const R a = DRAG ? alpha : R(0);
    const R Fx = rho * (gx - a * ux), Fy = rho * (gy - a * uy);
    const R usq = R(1.5) * (ux * ux + uy * uy);
    const R guo = R(1) - R(0.5) * omega;

    // reverse sweep
    R rhob = 0, ubx = 0, uby = 0, Fbx = 0, Fby = 0, usqb = 0, uFb = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R cx = R(kCx[i]), cy = R(kCy[i]), w = R(kW[i]);
        const R cu = cx * ux + cy * uy;
        const R cF = cx * Fx + cy * Fy;
        const R e = omega * nu[i] * w;  // (adjoint of f^eq_i) * w_i
        const R sb = guo * nu[i] * w;   // (adjoint of S_i) * w_i
        rhob += e * (R(1) + R(3) * cu + R(4.5) * cu * cu - usq);
        usqb -= e * rho;
        const R cub = e * rho * (R(3) + R(9) * cu) + sb * R(9) * cF;
        const R cFb = sb * (R(3) + R(9) * cu);
        uFb -= R(3) * sb;
        ubx += cub * cx;
        uby += cub * cy;
        Fbx += cFb * cx;
        Fby += cFb * cy;
    }
    // uF = u . F and usq = 1.5 u . u
    ubx += uFb * Fx + R(3) * usqb * ux;
    uby += uFb * Fy + R(3) * usqb * uy;
    Fbx += uFb * ux;
    Fby += uFb * uy;
    // F = rho (g - alpha u)
    rhob += Fbx * (gx - a * ux) + Fby * (gy - a * uy);
    ubx -= rho * a * Fbx;
    uby -= rho * a * Fby;
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
#pragma unroll
    for (int j = 0; j < 9; ++j)
        fb[j] = (R(1) - omega) * nu[j] + rhob + R(kCx[j]) * mbx + R(kCy[j]) * mby;
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
    const uint8_t *__restrict__ nmask, const float *__restrict__ alpha,
    double *__restrict__ grad_alpha, double *__restrict__ partials, int accumulate, int nx, int ny,
    int pitch, uint32_t bpr, uint32_t nblocks, typename ST::real omega, typename ST::real gx,
    typename ST::real gy)
{
    using R = typename ST::real;
    const uint32_t L = xcd_remap(blockIdx.x, nblocks);
    const int y = (int)(L / bpr);
    const int x = (int)(L - (uint32_t)y * bpr) * kBlock + (int)threadIdx.x;
    double gxs = 0.0, gys = 0.0;
    if (x < nx) {
        const uint32_t own = (uint32_t)y * pitch + x;
        const uint8_t t = type[own];
        if (t != kSolid) {
            const unsigned sm = solid_bits(t, nmask, own);
            uint32_t nb[9];
            dense_bases(x, y, nx, ny, (uint32_t)pitch / kChunk, nb);
            R f[9], nu[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                // forward pull: f_i(x) = s_i(x - c_i) or s_opp(i)(x)
                const uint32_t o = ((sm >> i) & 1u) ? (uint32_t)kOpp[i] * kChunk + nb[0]
                                                    : (uint32_t)i * kChunk + nb[i];
                f[i] = ST::ld(state[o], i);
                // reverse pull: x + c_i is node x - c_opp(i)
                const uint32_t q = ((sm >> kOpp[i]) & 1u) ? (uint32_t)kOpp[i] * kChunk + nb[0]
                                                          : (uint32_t)i * kChunk + nb[kOpp[i]];
                nu[i] = mu_in[q];
            }
            const R al = DRAG ? (R)alpha[own] : R(0);
            R fb[9], ab, gbx, gby;
            collide_vjp<R, DRAG, ST::kShift>(f, nu, omega, gx, gy, al, fb, ab, gbx, gby);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                store_nt(&mu_out[(uint32_t)i * kChunk + nb[0]], fb[i]);
            if (DRAG)
                grad_alpha[(size_t)y * nx + x] += (double)ab;
            gxs = (double)gbx;
            gys = (double)gby;
        }
    }
    block_sum2(gxs, gys);
    if (threadIdx.x == 0) {
        if (accumulate) {
            partials[2 * blockIdx.x] += gxs;
            partials[2 * blockIdx.x + 1] += gys;
        } else {
            partials[2 * blockIdx.x] = gxs;
            partials[2 * blockIdx.x + 1] = gys;
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
            uint32_t nb[9];
            dense_bases(x, y, nx, ny, (uint32_t)pitch / kChunk, nb);
            double f[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint32_t o = ((sm >> i) & 1u) ? (uint32_t)kOpp[i] * kChunk + nb[0]
                                                    : (uint32_t)i * kChunk + nb[i];
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
        const uint32_t base = dense_base(x, y, (uint32_t)pitch / kChunk);
#pragma unroll
        for (int j = 0; j < 9; ++j)
            mu[(uint32_t)j * kChunk + base] = lam[j];
    }
    double gys = 0.0;
    block_sum2(gxs, gys);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = gxs;
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

// grad_g += fixed-order sum of n partial pairs (one block).
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
    const uint32_t base = dense_base(x, y, (uint32_t)pitch / kChunk);
    const bool fluid = x < nx && type[gid] != kSolid;
    for (int i = 0; i < 9; ++i) {
        if (to_plain) {
            if (x < nx)
                plain[((size_t)i * ny + y) * nx + x] = fluid ? (double)mu[(uint32_t)i * kChunk + base] : 0.0;
        } else {
            mu[(uint32_t)i * kChunk + base] =
                fluid ? (R)plain[((size_t)i * ny + y) * nx + x] : R(0);
        }
    }
}

template <class ST>
hipError_t step_typed(const DevState &s, const void *state, const void *mu_in, void *mu_out,
                      double *grad_alpha, double *partials, int accumulate)
{
    using R = typename ST::real;
    const uint32_t bpr = (uint32_t)((s.nx + kBlock - 1) / kBlock);
    const uint32_t nblocks = bpr * (uint32_t)s.ny;
    const R om = (R)s.omega, gx = (R)s.gx, gy = (R)s.gy;
    if (s.alpha)
        k_adjoint_step<ST, true><<<nblocks, kBlock, 0, s.stream>>>(
            (const typename ST::mem *)state, (const R *)mu_in, (R *)mu_out, s.type, s.nmask,
            s.alpha, grad_alpha, partials, accumulate, s.nx, s.ny, s.pitch, bpr, nblocks, om, gx,
            gy);
    else
        k_adjoint_step<ST, false><<<nblocks, kBlock, 0, s.stream>>>(
            (const typename ST::mem *)state, (const R *)mu_in, (R *)mu_out, s.type, s.nmask,
            s.alpha, grad_alpha, partials, accumulate, s.nx, s.ny, s.pitch, bpr, nblocks, om, gx,
            gy);
    return hipGetLastError();
}

}  // namespace

int64_t adjoint_blocks(const DevState &s)
{
    return (int64_t)((s.nx + kBlock - 1) / kBlock) * s.ny;
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

hipError_t launch_partials_into(const double *partials, int64_t n, double *grad_g,
                                hipStream_t stream)
{
    k_partials_into<<<1, kBlock, 0, stream>>>(partials, (uint32_t)n, grad_g);
    return hipGetLastError();
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
