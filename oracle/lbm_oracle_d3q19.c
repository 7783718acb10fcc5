/*
 * Plain FP64 CPU oracle of the D3Q19 BGK lattice-Boltzmann time step with
 * halfway bounce-back walls and Guo body forcing: the three-dimensional
 * lattice that the paper names as its future work, with the same update as
 * the two-dimensional oracle (Sec. 2.2, Eq. 3 as collision then streaming;
 * Eq. 4 BGK; Eq. 6 equilibrium, which holds unchanged in 3D with the D3Q19
 * weights; Eq. 5 viscosity), and the two-relaxation-time collision of the
 * two-dimensional oracle (each population pair split into its symmetric and
 * antisymmetric parts, relaxed at omega_p and omega_m), the multiple-relaxation-
 * time collision in the D3Q19 moment basis of d'Humieres et al. (oracle3_collide_mrt),
 * and its full-way wall
 * rule (solid nodes next to fluid hold populations, reverse them instead of
 * colliding and stream them back; the state then includes those wall slots,
 * and slots not fed by a fluid node hold 0).
 *
 * TEST INFRASTRUCTURE ONLY.  The GPU library never links, calls, includes or
 * shares anything with this file; only the test-suite and the benchmark's
 * CPU-baseline leg load it.
 *
 * State: f[((i*nz + z)*ny + y)*nx + x] holds the canonical pre-collision
 * populations at fluid nodes; solid slots hold 0.  mask[(z*ny + y)*nx + x]:
 * 0 fluid, 1 solid.  All three axes wrap periodically; walls come only from
 * the mask.  Build with -O2 -ffp-contract=off, no fast-math.
 *
 * Velocities (the paper numbers only D2Q9): 0 rest; 1..6 the axis directions
 * +x, -x, +y, -y, +z, -z; 7..18 the twelve edge directions as opposite pairs
 * (+x+y, -x-y), (+x-y, -x+y), (+x+z, -x-z), (+x-z, -x+z), (+y+z, -y-z),
 * (+y-z, -y+z).  Weights: 1/3 at rest, 1/18 on the axes, 1/36 on the edges.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q3 19

static const int CX3[Q3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY3[Q3] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ3[Q3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double weight3(int i)
{
    int s = abs(CX3[i]) + abs(CY3[i]) + abs(CZ3[i]);
    return s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

static int opposite3(int i)
{
    for (int j = 0; j < Q3; ++j)
        if (CX3[j] == -CX3[i] && CY3[j] == -CY3[i] && CZ3[j] == -CZ3[i])
            return j;
    return -1;
}

static int wrap3(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

static size_t slot3(int i, int x, int y, int z, int nx, int ny, int nz)
{
    return (((size_t)i * nz + z) * ny + y) * nx + x;
}

void oracle3_constants(int *cx, int *cy, int *cz, double *w, int *opp)
{
    for (int i = 0; i < Q3; ++i) {
        cx[i] = CX3[i];
        cy[i] = CY3[i];
        cz[i] = CZ3[i];
        w[i] = weight3(i);
        opp[i] = opposite3(i);
    }
}

/* Eq. 6 with the D3Q19 weights. */
void oracle3_equilibrium(double rho, double ux, double uy, double uz, double *feq)
{
    double usq = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < Q3; ++i) {
        double cu = CX3[i] * ux + CY3[i] * uy + CZ3[i] * uz;
        feq[i] = weight3(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    }
}

/* Guo forcing term: S_i = w_i [3 (c_i - u) . F + 9 (c_i . u)(c_i . F)]. */
void oracle3_guo_source(double ux, double uy, double uz, double Fx, double Fy, double Fz,
                        double *S)
{
    for (int i = 0; i < Q3; ++i) {
        double cu = CX3[i] * ux + CY3[i] * uy + CZ3[i] * uz;
        double cF = CX3[i] * Fx + CY3[i] * Fy + CZ3[i] * Fz;
        double uF = ux * Fx + uy * Fy + uz * Fz;
        S[i] = weight3(i) * (3.0 * (cF - uF) + 9.0 * cu * cF);
    }
}

/* rho, and the velocity with the half-force correction u = m/rho + g/2. */
void oracle3_node_velocity(const double *f, double gx, double gy, double gz, double *out)
{
    double rho = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    for (int i = 0; i < Q3; ++i) {
        rho += f[i];
        mx += CX3[i] * f[i];
        my += CY3[i] * f[i];
        mz += CZ3[i] * f[i];
    }
    out[0] = rho;
    out[1] = mx / rho + 0.5 * gx;
    out[2] = my / rho + 0.5 * gy;
    out[3] = mz / rho + 0.5 * gz;
}

/* BGK collision with forcing F = rho g:
 *   fstar_i = f_i - omega (f_i - f^eq_i) + (1 - omega/2) S_i. */
void oracle3_collide(const double *f, double gx, double gy, double gz, double omega,
                     double *fstar)
{
    double m[4];
    oracle3_node_velocity(f, gx, gy, gz, m);
    double feq[Q3], S[Q3];
    oracle3_equilibrium(m[0], m[1], m[2], m[3], feq);
    oracle3_guo_source(m[1], m[2], m[3], m[0] * gx, m[0] * gy, m[0] * gz, S);
    for (int i = 0; i < Q3; ++i)
        fstar[i] = f[i] - omega * (f[i] - feq[i]) + (1.0 - 0.5 * omega) * S[i];
}

/* Two-relaxation-time collision with forcing F = rho g: for each pair
 * (i, opp(i)) the symmetric parts (f_i + f_opp)/2 relax with omega_p and the
 * antisymmetric parts (f_i - f_opp)/2 with omega_m, towards the same parts of
 * f^eq; the forcing term is split alike, with factors (1 - omega/2) of its own
 * rate.  omega_m = omega_p is the BGK collision. */
void oracle3_collide_trt(const double *f, double gx, double gy, double gz, double omega_p,
                         double omega_m, double *fstar)
{
    double m[4];
    oracle3_node_velocity(f, gx, gy, gz, m);
    double feq[Q3], S[Q3];
    oracle3_equilibrium(m[0], m[1], m[2], m[3], feq);
    oracle3_guo_source(m[1], m[2], m[3], m[0] * gx, m[0] * gy, m[0] * gz, S);
    for (int i = 0; i < Q3; ++i) {
        int j = opposite3(i);
        double fp = 0.5 * (f[i] + f[j]), fm = 0.5 * (f[i] - f[j]);
        double ep = 0.5 * (feq[i] + feq[j]), em = 0.5 * (feq[i] - feq[j]);
        double sp = 0.5 * (S[i] + S[j]), sm = 0.5 * (S[i] - S[j]);
        fstar[i] = f[i] - omega_p * (fp - ep) - omega_m * (fm - em) + (1.0 - 0.5 * omega_p) * sp +
                   (1.0 - 0.5 * omega_m) * sm;
    }
}

/* Multiple-relaxation-time collision (a richer collision model beyond BGK; the
 * D3Q19 moment basis of d'Humieres, Ginzburg, Krafczyk, Lallemand and Luo,
 * 2002).  Nineteen moments m = M f, each row a polynomial of c = v_i:
 *   0 rho: 1            1 e: 19|c|^2 - 30     2 eps: (21|c|^4 - 53|c|^2 + 24) / 2
 *   3 j_x: c_x          4 q_x: (5|c|^2 - 9) c_x
 *   5 j_y: c_y          6 q_y: (5|c|^2 - 9) c_y
 *   7 j_z: c_z          8 q_z: (5|c|^2 - 9) c_z
 *   9 3p_xx: 3c_x^2 - |c|^2      10 3pi_xx: (3|c|^2 - 5)(3c_x^2 - |c|^2)
 *   11 p_ww: c_y^2 - c_z^2       12 pi_ww: (3|c|^2 - 5)(c_y^2 - c_z^2)
 *   13 p_xy: c_x c_y   14 p_yz: c_y c_z   15 p_xz: c_x c_z
 *   16 m_x: (c_y^2 - c_z^2) c_x  17 m_y: (c_z^2 - c_x^2) c_y  18 m_z: (c_x^2 - c_y^2) c_z
 * The rows are orthogonal, so M^-1 = M^T diag(1 / |row_k|^2); as in the D2Q9
 * oracle, every moment relaxes towards the moment of f^eq (Eq. 6) with its own
 * rate and Guo's term enters with (1 - s_k / 2):
 *   mstar_k = m_k - s_k (m_k - (M f^eq)_k) + (1 - s_k / 2) (M S)_k,  fstar = M^-1 mstar.
 * All rates omega is BGK; omega+ on the even rows (0-2, 9-15) and omega- on the
 * odd ones (3-8, 16-18) is TRT. */
static double mrt3_row(int k, int i)
{
    double cx = CX3[i], cy = CY3[i], cz = CZ3[i], c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return cx;
    case 4: return (5.0 * c2 - 9.0) * cx;
    case 5: return cy;
    case 6: return (5.0 * c2 - 9.0) * cy;
    case 7: return cz;
    case 8: return (5.0 * c2 - 9.0) * cz;
    case 9: return 3.0 * cx * cx - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2);
    case 11: return cy * cy - cz * cz;
    case 12: return (3.0 * c2 - 5.0) * (cy * cy - cz * cz);
    case 13: return cx * cy;
    case 14: return cy * cz;
    case 15: return cx * cz;
    case 16: return (cy * cy - cz * cz) * cx;
    case 17: return (cz * cz - cx * cx) * cy;
    default: return (cx * cx - cy * cy) * cz;
    }
}

void oracle3_mrt_matrix(double *M)
{
    for (int k = 0; k < Q3; ++k)
        for (int i = 0; i < Q3; ++i)
            M[k * Q3 + i] = mrt3_row(k, i);
}

void oracle3_collide_mrt(const double *f, double gx, double gy, double gz, const double *rates,
                         double *fstar)
{
    double mo[4];
    oracle3_node_velocity(f, gx, gy, gz, mo);
    double feq[Q3], S[Q3], mstar[Q3];
    oracle3_equilibrium(mo[0], mo[1], mo[2], mo[3], feq);
    oracle3_guo_source(mo[1], mo[2], mo[3], mo[0] * gx, mo[0] * gy, mo[0] * gz, S);
    for (int k = 0; k < Q3; ++k) {
        double m = 0.0, meq = 0.0, ms = 0.0;
        for (int i = 0; i < Q3; ++i) {
            m += mrt3_row(k, i) * f[i];
            meq += mrt3_row(k, i) * feq[i];
            ms += mrt3_row(k, i) * S[i];
        }
        mstar[k] = m - rates[k] * (m - meq) + (1.0 - 0.5 * rates[k]) * ms;
    }
    for (int i = 0; i < Q3; ++i) {
        double v = 0.0;
        for (int k = 0; k < Q3; ++k) {
            double norm = 0.0;
            for (int l = 0; l < Q3; ++l)
                norm += mrt3_row(k, l) * mrt3_row(k, l);
            v += mrt3_row(k, i) * mstar[k] / norm;
        }
        fstar[i] = v;
    }
}

/* f_i = f^eq_i(rho0, u0) at fluid nodes; NULL fields mean rho0 = 1, u0 = 0. */
int oracle3_init(int nx, int ny, int nz, const uint8_t *mask, const double *rho0,
                 const double *ux0, const double *uy0, const double *uz0, double *f)
{
    if (nx < 1 || ny < 1 || nz < 1)
        return -1;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = ((size_t)z * ny + y) * nx + x;
                double feq[Q3] = {0};
                if (mask[n] == 0)
                    oracle3_equilibrium(rho0 ? rho0[n] : 1.0, ux0 ? ux0[n] : 0.0,
                                        uy0 ? uy0[n] : 0.0, uz0 ? uz0[n] : 0.0, feq);
                for (int i = 0; i < Q3; ++i)
                    f[slot3(i, x, y, z, nx, ny, nz)] = feq[i];
            }
    return 0;
}

/* Collision phase: every fluid node collides into `post`; with `wall`
 * non-NULL (full-way rule) every wall node reverses its populations. */
static void collide_phase3(int nx, int ny, int nz, const uint8_t *mask, const uint8_t *wall,
                           const double *f, double *post, double omega, double omega_m,
                           const double *mrt, double gx, double gy, double gz)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = ((size_t)z * ny + y) * nx + x;
                if (mask[n] != 0) {
                    if (wall && wall[n])
                        for (int i = 0; i < Q3; ++i)
                            post[slot3(i, x, y, z, nx, ny, nz)] =
                                f[slot3(opposite3(i), x, y, z, nx, ny, nz)];
                    continue;
                }
                double fl[Q3], fs[Q3];
                for (int i = 0; i < Q3; ++i)
                    fl[i] = f[slot3(i, x, y, z, nx, ny, nz)];
                if (mrt)
                    oracle3_collide_mrt(fl, gx, gy, gz, mrt, fs);
                else if (omega_m == omega)
                    oracle3_collide(fl, gx, gy, gz, omega, fs);
                else
                    oracle3_collide_trt(fl, gx, gy, gz, omega, omega_m, fs);
                for (int i = 0; i < Q3; ++i)
                    post[slot3(i, x, y, z, nx, ny, nz)] = fs[i];
            }
}

/* Halfway streaming: push every post-collision population of a fluid node to
 * x + c_i, or back to its origin reversed when x + c_i is solid. */
static void stream_halfway3(int nx, int ny, int nz, const uint8_t *mask, double *f,
                            const double *post)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = ((size_t)z * ny + y) * nx + x;
                if (mask[n] != 0)
                    continue;
                for (int i = 0; i < Q3; ++i) {
                    int xn = wrap3(x + CX3[i], nx), yn = wrap3(y + CY3[i], ny),
                        zn = wrap3(z + CZ3[i], nz);
                    double v = post[slot3(i, x, y, z, nx, ny, nz)];
                    if (mask[((size_t)zn * ny + yn) * nx + xn] == 0)
                        f[slot3(i, xn, yn, zn, nx, ny, nz)] = v;
                    else
                        f[slot3(opposite3(i), x, y, z, nx, ny, nz)] = v;
                }
            }
}

/* Full-way streaming: every post-collision population of a fluid or wall node
 * moves to x + c_i; a fluid target takes it from either kind of source, a
 * wall target only from a fluid source (its other slots are cleared). */
static void stream_fullway3(int nx, int ny, int nz, const uint8_t *mask, const uint8_t *wall,
                            double *f, const double *post)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                if (wall[((size_t)z * ny + y) * nx + x])
                    for (int i = 0; i < Q3; ++i)
                        f[slot3(i, x, y, z, nx, ny, nz)] = 0.0;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = ((size_t)z * ny + y) * nx + x;
                if (mask[n] != 0 && !wall[n])
                    continue;
                for (int i = 0; i < Q3; ++i) {
                    int xn = wrap3(x + CX3[i], nx), yn = wrap3(y + CY3[i], ny),
                        zn = wrap3(z + CZ3[i], nz);
                    size_t t = ((size_t)zn * ny + yn) * nx + xn;
                    if (mask[t] == 0 || (wall[t] && mask[n] == 0))
                        f[slot3(i, xn, yn, zn, nx, ny, nz)] = post[slot3(i, x, y, z, nx, ny, nz)];
                }
            }
}

/* Wall nodes: solid nodes with at least one fluid neighbour. */
static void find_walls3(int nx, int ny, int nz, const uint8_t *mask, uint8_t *wall)
{
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = ((size_t)z * ny + y) * nx + x;
                wall[n] = 0;
                if (mask[n] == 0)
                    continue;
                for (int i = 1; i < Q3; ++i)
                    if (mask[((size_t)wrap3(z + CZ3[i], nz) * ny + wrap3(y + CY3[i], ny)) * nx +
                             wrap3(x + CX3[i], nx)] == 0)
                        wall[n] = 1;
            }
}

/* Full-way initial wall slots: slot i of wall node w takes f_i of the fluid
 * node w - c_i, 0 where w - c_i is not fluid; fluid slots unchanged. */
int oracle3_fullway_fill(int nx, int ny, int nz, const uint8_t *mask, double *f)
{
    if (nx < 1 || ny < 1 || nz < 1)
        return -1;
    uint8_t *wall = (uint8_t *)malloc((size_t)nx * ny * nz);
    if (!wall)
        return -2;
    find_walls3(nx, ny, nz, mask, wall);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!wall[((size_t)z * ny + y) * nx + x])
                    continue;
                for (int i = 0; i < Q3; ++i) {
                    int xs = wrap3(x - CX3[i], nx), ys = wrap3(y - CY3[i], ny),
                        zs = wrap3(z - CZ3[i], nz);
                    f[slot3(i, x, y, z, nx, ny, nz)] =
                        mask[((size_t)zs * ny + ys) * nx + xs] == 0
                            ? f[slot3(i, xs, ys, zs, nx, ny, nz)]
                            : 0.0;
                }
            }
    free(wall);
    return 0;
}

/* nsteps steps in place; tau_m is the antisymmetric relaxation time of the
 * two-relaxation-time collision (tau_m = tau: BGK); fullway selects the
 * full-way wall rule. */
static int run_general3(int nx, int ny, int nz, const uint8_t *mask, double *f, double tau,
                        double tau_m, const double *mrt, double gx, double gy, double gz,
                        long nsteps, int nthreads, int fullway)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(tau > 0.5) || !(tau_m > 0.5) || nsteps < 0)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    size_t total = (size_t)Q3 * nx * ny * nz;
    double *post = (double *)calloc(total, sizeof(double));
    uint8_t *wall = fullway ? (uint8_t *)malloc((size_t)nx * ny * nz) : NULL;
    if (!post || (fullway && !wall)) {
        free(post);
        free(wall);
        return -2;
    }
    if (wall)
        find_walls3(nx, ny, nz, mask, wall);
    double omega = 1.0 / tau, omega_m = tau_m == tau ? omega : 1.0 / tau_m;
    for (long s = 0; s < nsteps; ++s) {
        collide_phase3(nx, ny, nz, mask, wall, f, post, omega, omega_m, mrt, gx, gy, gz);
        if (wall)
            stream_fullway3(nx, ny, nz, mask, wall, f, post);
        else
            stream_halfway3(nx, ny, nz, mask, f, post);
    }
    free(post);
    free(wall);
    return 0;
}

int oracle3_run_walls(int nx, int ny, int nz, const uint8_t *mask, double *f, double tau,
                      double tau_m, double gx, double gy, double gz, long nsteps, int nthreads,
                      int fullway)
{
    return run_general3(nx, ny, nz, mask, f, tau, tau_m, NULL, gx, gy, gz, nsteps, nthreads,
                        fullway);
}

/* As oracle3_run_walls with the multiple-relaxation-time collision: the shear
 * moments (3p_xx, p_ww, p_xy, p_yz, p_xz) relax with omega = 1/tau, e with s_e,
 * eps with s_eps, q with s_q, the pi moments with s_pi, the m moments with s_m;
 * rho and j with 1. */
int oracle3_run_mrt(int nx, int ny, int nz, const uint8_t *mask, double *f, double tau,
                    const double *r5, double gx, double gy, double gz, long nsteps, int nthreads,
                    int fullway)
{
    if (!(tau > 0.5) || !r5)
        return -1;
    double w = 1.0 / tau;
    double rates[Q3] = {1.0, r5[0], r5[1], 1.0, r5[2], 1.0, r5[2], 1.0, r5[2], w,
                        r5[3], w,   r5[3], w,   w,     w,   r5[4], r5[4], r5[4]};
    return run_general3(nx, ny, nz, mask, f, tau, tau, rates, gx, gy, gz, nsteps, nthreads,
                        fullway);
}

int oracle3_run_trt(int nx, int ny, int nz, const uint8_t *mask, double *f, double tau,
                    double tau_m, double gx, double gy, double gz, long nsteps, int nthreads)
{
    return oracle3_run_walls(nx, ny, nz, mask, f, tau, tau_m, gx, gy, gz, nsteps, nthreads, 0);
}

int oracle3_run(int nx, int ny, int nz, const uint8_t *mask, double *f, double tau, double gx,
                double gy, double gz, long nsteps, int nthreads)
{
    return oracle3_run_trt(nx, ny, nz, mask, f, tau, tau, gx, gy, gz, nsteps, nthreads);
}

/* rho and the corrected velocity of the canonical state; solid nodes 0. */
int oracle3_macroscopic(int nx, int ny, int nz, const uint8_t *mask, const double *f, double gx,
                        double gy, double gz, double *rho, double *ux, double *uy, double *uz)
{
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = ((size_t)z * ny + y) * nx + x;
                if (mask[n] != 0) {
                    rho[n] = ux[n] = uy[n] = uz[n] = 0.0;
                    continue;
                }
                double fl[Q3], m[4];
                for (int i = 0; i < Q3; ++i)
                    fl[i] = f[slot3(i, x, y, z, nx, ny, nz)];
                oracle3_node_velocity(fl, gx, gy, gz, m);
                rho[n] = m[0];
                ux[n] = m[1];
                uy[n] = m[2];
                uz[n] = m[3];
            }
    return 0;
}
