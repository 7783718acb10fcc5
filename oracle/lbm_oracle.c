/*
 * Plain FP64 CPU oracle of the D2Q9 BGK lattice-Boltzmann time step with
 * halfway bounce-back walls, Guo body forcing and Brinkman drag, plus the
 * exact reverse-mode gradient of an outlet-velocity objective.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously correct reference
 * the GPU library is checked against.  The GPU library never links, calls,
 * includes or shares anything with this file (no common constant tables, no
 * common helpers); only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.
 *
 * Form.  The paper's update (Sec. 2.2, Eq. 3) is written as two alternating
 * phases: collision (right-hand side of Eq. 3, with the BGK operator of
 * Eq. 4 and the equilibrium of Eq. 6) and streaming (the left-hand side).
 * This oracle does exactly that, in that order, over plain dense arrays:
 * every fluid node collides, then every post-collision population is pushed
 * to its neighbour.  It is deliberately the push form; the GPU kernels use the
 * fused pull form of Algorithm 1, and the two must agree.
 *
 * State.  f[(i*ny + y)*nx + x] holds the canonical pre-collision populations
 * f_i(x, t) (left-hand side of Eq. 3) at fluid nodes; solid slots hold 0.
 * Node types: mask[y*nx + x] = 0 fluid, 1 solid.  Both axes wrap
 * periodically; walls come only from the mask.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - bounce-back is the halfway, link-wise variant: a population that would
 *     stream into a solid node returns to its origin with reversed direction;
 *   - a body force g (an acceleration) enters through Guo's forcing scheme,
 *     with force density F = rho*(g - alpha*u) and the half-force velocity;
 *   - a per-node Brinkman coefficient alpha adds the linear drag -rho*alpha*u,
 *     taken implicitly: u = (m/rho + g/2) / (1 + alpha/2);
 *   - with g = 0 and alpha = 0 the collision is exactly Eqs. 2-6;
 *   - open boundaries (Sec. 3: constant velocity and constant pressure after
 *     Zou and He) are boundary nodes with a prescribed inward normal n along
 *     an axis.  After every streaming phase (and on the initial state) the
 *     three populations with v_i . n > 0, which would have come from outside
 *     the domain, are rebuilt so that the node's Eq. 2 moments take the
 *     prescribed values (velocity: m = rho u_b; pressure: rho = rho_b with no
 *     tangential velocity) and the non-equilibrium part of the normal
 *     population equals that of its opposite.  Whatever streamed into those
 *     slots across the periodic seam is discarded;
 *   - the multiple-relaxation-time collision (oracle_collide_mrt) uses the
 *     moment basis of Lallemand and Luo with Guo's forcing in moment space;
 *   - full-way bounce-back (the alternative wall rule, selected per run): the
 *     paper's bounce-back boundary nodes hold and move populations without
 *     computing anything (Sec. 4.3).  Solid nodes with at least one fluid
 *     neighbour ("wall nodes") then store populations: in a step they do not
 *     collide but reverse what they hold (post_i = f_opp(i)), and they take
 *     part in streaming.  Only wall slots fed by a fluid node carry values
 *     (the others hold 0).  A population sent into a wall returns to its
 *     origin two steps later instead of one; steady states equal those of
 *     the halfway rule.
 *
 * Precision: FP64 throughout; build with -O2 -ffp-contract=off, no fast-math;
 * sums over directions run in ascending i.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9

/* D2Q9 lattice velocities v_i, numbered as in the paper's Fig. 1 (Sec. 2.2):
 * 0 rest, 1 east, 2 north, 3 west, 4 south, 5 NE, 6 NW, 7 SW, 8 SE.
 * The paper spells out v_0 = [0,0], v_1 = [1,0], v_4 = [0,-1], v_6 = [-1,1]. */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Weights w_i of Eq. 6: 4/9 at rest, 1/9 on the axes, 1/36 on the diagonals. */
static const double W[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* The direction j with v_j = -v_i (searched, not tabulated). */
static int opposite(int i)
{
    for (int j = 0; j < Q; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i])
            return j;
    return -1;
}

static int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

static size_t slot(int i, int x, int y, int nx, int ny)
{
    return ((size_t)i * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x;
}

void oracle_constants(int *cx, int *cy, double *w, int *opp)
{
    for (int i = 0; i < Q; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        w[i] = W[i];
        opp[i] = opposite(i);
    }
}

/* Eq. 6: f^eq_i = w_i rho (1 + 3 v_i.u + 9/2 (v_i.u)^2 - 3/2 u.u). */
void oracle_equilibrium(double rho, double ux, double uy, double *feq)
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        feq[i] = W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Guo forcing term S_i = w_i [3 (v_i - u) + 9 (v_i.u) v_i] . F. */
void oracle_guo_source(double ux, double uy, double Fx, double Fy, double *S)
{
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        double cF = CX[i] * Fx + CY[i] * Fy;
        S[i] = W[i] * (3.0 * ((CX[i] - ux) * Fx + (CY[i] - uy) * Fy) + 9.0 * cu * cF);
    }
}

/* Moments of Eq. 2 with the half-force and implicit drag correction:
 * out = {rho, ux, uy}, u = (m/rho + g/2) / (1 + alpha/2). */
void oracle_node_velocity(const double *f, double alpha, double gx, double gy, double *out)
{
    double rho = 0.0, mx = 0.0, my = 0.0;
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        mx += CX[i] * f[i];
        my += CY[i] * f[i];
    }
    double D = 1.0 + 0.5 * alpha;
    out[0] = rho;
    out[1] = (mx / rho + 0.5 * gx) / D;
    out[2] = (my / rho + 0.5 * gy) / D;
}

/* Collision at one fluid node (right-hand side of Eq. 3 with the BGK operator
 * of Eq. 4, omega = 1/tau from Eq. 5, plus the forcing term):
 *   fstar_i = f_i - omega (f_i - f^eq_i) + (1 - omega/2) S_i. */
void oracle_collide(const double *f, double alpha, double gx, double gy, double omega,
                    double *fstar)
{
    double m[3];
    oracle_node_velocity(f, alpha, gx, gy, m);
    double rho = m[0], ux = m[1], uy = m[2];
    double Fx = rho * (gx - alpha * ux);
    double Fy = rho * (gy - alpha * uy);
    double feq[Q], S[Q];
    oracle_equilibrium(rho, ux, uy, feq);
    oracle_guo_source(ux, uy, Fx, Fy, S);
    for (int i = 0; i < Q; ++i)
        fstar[i] = f[i] - omega * (f[i] - feq[i]) + (1.0 - 0.5 * omega) * S[i];
}

/* Two-relaxation-time collision (a collision model other than the paper's
 * BGK, named as the paper's future work): every population pair (i, opp(i))
 * is split into its symmetric and antisymmetric parts,
 *   f^+_i = (f_i + f_opp(i)) / 2,  f^-_i = (f_i - f_opp(i)) / 2,
 * and likewise f^eq and the forcing term S; the symmetric parts relax with
 * omega+ (which sets the viscosity as omega does in Eq. 5), the antisymmetric
 * parts with omega-:
 *   fstar_i = f_i - omega+ (f^+_i - f^eq+_i) - omega- (f^-_i - f^eq-_i)
 *             + (1 - omega+/2) S^+_i + (1 - omega-/2) S^-_i.
 * omega- = omega+ is the BGK collision above. */
void oracle_collide_trt(const double *f, double alpha, double gx, double gy, double omega_p,
                        double omega_m, double *fstar)
{
    double m[3];
    oracle_node_velocity(f, alpha, gx, gy, m);
    double rho = m[0], ux = m[1], uy = m[2];
    double Fx = rho * (gx - alpha * ux);
    double Fy = rho * (gy - alpha * uy);
    double feq[Q], S[Q];
    oracle_equilibrium(rho, ux, uy, feq);
    oracle_guo_source(ux, uy, Fx, Fy, S);
    for (int i = 0; i < Q; ++i) {
        int j = opposite(i);
        double fp = 0.5 * (f[i] + f[j]), fm = 0.5 * (f[i] - f[j]);
        double ep = 0.5 * (feq[i] + feq[j]), em = 0.5 * (feq[i] - feq[j]);
        double sp = 0.5 * (S[i] + S[j]), sm = 0.5 * (S[i] - S[j]);
        fstar[i] = f[i] - omega_p * (fp - ep) - omega_m * (fm - em) + (1.0 - 0.5 * omega_p) * sp +
                   (1.0 - 0.5 * omega_m) * sm;
    }
}

/* Multiple-relaxation-time collision (another collision model beyond the
 * paper's BGK; the moment basis of Lallemand and Luo, 2000).  Nine moments
 * m = M f, each row of M a polynomial of the velocity c = v_i:
 *   rho: 1              e: -4 + 3|c|^2     eps: 4 - 21/2 |c|^2 + 9/2 |c|^4
 *   j_x: c_x            q_x: (-5 + 3|c|^2) c_x
 *   j_y: c_y            q_y: (-5 + 3|c|^2) c_y
 *   p_xx: c_x^2 - c_y^2 p_xy: c_x c_y
 * The rows are orthogonal, so M^-1 = M^T diag(1 / |row_k|^2).  Each moment
 * relaxes towards the moment of f^eq (Eq. 6) with its own rate s_k, and the
 * Guo term enters in moment space with the factor (1 - s_k / 2):
 *   mstar_k = m_k - s_k (m_k - (M f^eq)_k) + (1 - s_k / 2) (M S)_k,
 *   fstar   = M^-1 mstar.
 * rates[9] = s_k in the row order above; all s_k = omega is the BGK collision,
 * s_k = omega+ on the even rows (rho, e, eps, p_xx, p_xy) and omega- on the odd
 * ones (j, q) the TRT collision.  The rates of rho and j do not matter (those
 * moments are conserved, j up to the force, whatever s_k). */
static double mrt_row(int k, int i)
{
    double cx = CX[i], cy = CY[i], c2 = cx * cx + cy * cy;
    switch (k) {
    case 0: return 1.0;
    case 1: return -4.0 + 3.0 * c2;
    case 2: return 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
    case 3: return cx;
    case 4: return (-5.0 + 3.0 * c2) * cx;
    case 5: return cy;
    case 6: return (-5.0 + 3.0 * c2) * cy;
    case 7: return cx * cx - cy * cy;
    default: return cx * cy;
    }
}

void oracle_mrt_matrix(double *M)
{
    for (int k = 0; k < Q; ++k)
        for (int i = 0; i < Q; ++i)
            M[k * Q + i] = mrt_row(k, i);
}

void oracle_collide_mrt(const double *f, double alpha, double gx, double gy, const double *rates,
                        double *fstar)
{
    double mo[3];
    oracle_node_velocity(f, alpha, gx, gy, mo);
    double rho = mo[0], ux = mo[1], uy = mo[2];
    double Fx = rho * (gx - alpha * ux);
    double Fy = rho * (gy - alpha * uy);
    double feq[Q], S[Q], mstar[Q];
    oracle_equilibrium(rho, ux, uy, feq);
    oracle_guo_source(ux, uy, Fx, Fy, S);
    for (int k = 0; k < Q; ++k) {
        double m = 0.0, meq = 0.0, ms = 0.0;
        for (int i = 0; i < Q; ++i) {
            m += mrt_row(k, i) * f[i];
            meq += mrt_row(k, i) * feq[i];
            ms += mrt_row(k, i) * S[i];
        }
        mstar[k] = m - rates[k] * (m - meq) + (1.0 - 0.5 * rates[k]) * ms;
    }
    for (int i = 0; i < Q; ++i) {
        double v = 0.0;
        for (int k = 0; k < Q; ++k) {
            double norm = 0.0;
            for (int l = 0; l < Q; ++l)
                norm += mrt_row(k, l) * mrt_row(k, l);
            v += mrt_row(k, i) * mstar[k] / norm;
        }
        fstar[i] = v;
    }
}

/* Initialisation (Algorithm 1, first loop): f_i = f^eq_i(rho0, u0) at every
 * fluid node.  NULL fields mean rho0 = 1, u0 = 0.  Solid slots are zeroed. */
int oracle_init(int nx, int ny, const uint8_t *mask, const double *rho0, const double *ux0,
                const double *uy0, double *f)
{
    if (nx < 1 || ny < 1)
        return -1;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            double feq[Q] = {0};
            if (mask[n] == 0)
                oracle_equilibrium(rho0 ? rho0[n] : 1.0, ux0 ? ux0[n] : 0.0, uy0 ? uy0[n] : 0.0,
                                   feq);
            for (int i = 0; i < Q; ++i)
                f[slot(i, x, y, nx, ny)] = feq[i];
        }
    return 0;
}

/* Zou-He boundary node (Sec. 3, constant velocity / constant pressure).
 * kind 1: prescribed velocity (a, b) = (u_x, u_y); kind 2: prescribed density
 * a (b unused).  (nxn, nyn) is the inward unit normal, along an axis.  Reads
 * the 9 populations of the node after streaming; writes them with the three
 * entering ones (v_i . n > 0) replaced.  Conditions, with t the unit tangent:
 *   sum f = rho,  sum (v.n) f = rho u_n,  sum (v.t) f = rho u_t,
 *   f_n - f_opp(n) = (2/3) rho u_n   (equilibrium difference of the pair),
 * which for a velocity node fix rho and for a pressure node fix u_n
 * (u_t = 0).  Solved in closed form: with S = sum_{v.n=0} f + 2 sum_{v.n<0} f,
 *   velocity: rho = S / (1 - u_n);  pressure: u_n = 1 - S / rho;
 *   normal population: f_i = f_opp(i) + (2/3) rho u_n;
 *   diagonal i, tangential part s_i = v_i . t = +-1:
 *     f_i = f_opp(i) + (1/6) rho u_n + (s_i / 2) (rho u_t - T),
 *   T = sum_{v.n=0} (v.t) f.  Returns 0, or -1 for a bad kind or normal. */
int oracle_zou_he(const double *f, int kind, int nxn, int nyn, double a, double b, double *out)
{
    if ((kind != 1 && kind != 2) || abs(nxn) + abs(nyn) != 1)
        return -1;
    const int tx = -nyn, ty = nxn; /* unit tangent */
    double par = 0.0, outgoing = 0.0, tan_sum = 0.0;
    for (int i = 0; i < Q; ++i) {
        int d = CX[i] * nxn + CY[i] * nyn;
        if (d == 0) {
            par += f[i];
            tan_sum += (double)(CX[i] * tx + CY[i] * ty) * f[i];
        } else if (d < 0) {
            outgoing += f[i];
        }
    }
    const double S = par + 2.0 * outgoing;
    double rho, un, ut;
    if (kind == 1) {
        un = a * nxn + b * nyn;
        ut = a * tx + b * ty;
        rho = S / (1.0 - un);
    } else {
        rho = a;
        un = 1.0 - S / rho;
        ut = 0.0;
    }
    for (int i = 0; i < Q; ++i)
        out[i] = f[i];
    for (int i = 0; i < Q; ++i) {
        if (CX[i] * nxn + CY[i] * nyn <= 0)
            continue;
        const int j = opposite(i);
        const int si = CX[i] * tx + CY[i] * ty;
        if (si == 0)
            out[i] = f[j] + (2.0 / 3.0) * rho * un;
        else
            out[i] = f[j] + rho * un / 6.0 + 0.5 * (double)si * (rho * ut - tan_sum);
    }
    return 0;
}

/* Boundary-node code: 0 none, 1..4 constant velocity with inward normal
 * +x, -x, +y, -y, 5..8 constant pressure with the same normals. */
static int bc_decode(uint8_t code, int *kind, int *nxn, int *nyn)
{
    if (code < 1 || code > 8)
        return -1;
    static const int NX_[4] = {1, -1, 0, 0}, NY_[4] = {0, 0, 1, -1};
    *kind = code <= 4 ? 1 : 2;
    *nxn = NX_[(code - 1) % 4];
    *nyn = NY_[(code - 1) % 4];
    return 0;
}

/* Apply the boundary conditions to the canonical state f in place:
 * value[(k*ny + y)*nx + x], k = 0, 1 = (u_x, u_y) for velocity nodes,
 * (rho, unused) for pressure nodes.  Codes at solid nodes are an error. */
int oracle_apply_boundaries(int nx, int ny, const uint8_t *mask, const uint8_t *bc,
                            const double *value, double *f)
{
    const size_t plane = (size_t)nx * ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            if (bc[n] == 0)
                continue;
            int kind, nxn, nyn;
            if (bc_decode(bc[n], &kind, &nxn, &nyn) || mask[n] != 0)
                return -1;
            double fl[Q], fo[Q];
            for (int i = 0; i < Q; ++i)
                fl[i] = f[slot(i, x, y, nx, ny)];
            oracle_zou_he(fl, kind, nxn, nyn, value[n], value[plane + n], fo);
            for (int i = 0; i < Q; ++i)
                f[slot(i, x, y, nx, ny)] = fo[i];
        }
    return 0;
}

/* Collision phase: every fluid node collides into `post`; with `wall`
 * non-NULL (full-way rule) every wall node reverses its populations into
 * `post`. */
static void collide_phase(int nx, int ny, const uint8_t *mask, const uint8_t *wall,
                          const double *f, double *post, double omega, double omega_m,
                          const double *mrt, double gx, double gy, const double *alpha)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            if (mask[n] != 0) {
                if (wall && wall[n])
                    for (int i = 0; i < Q; ++i)
                        post[slot(i, x, y, nx, ny)] = f[slot(opposite(i), x, y, nx, ny)];
                continue;
            }
            double fl[Q], fs[Q];
            for (int i = 0; i < Q; ++i)
                fl[i] = f[slot(i, x, y, nx, ny)];
            if (mrt)
                oracle_collide_mrt(fl, alpha ? alpha[n] : 0.0, gx, gy, mrt, fs);
            else if (omega_m == omega)
                oracle_collide(fl, alpha ? alpha[n] : 0.0, gx, gy, omega, fs);
            else
                oracle_collide_trt(fl, alpha ? alpha[n] : 0.0, gx, gy, omega, omega_m, fs);
            for (int i = 0; i < Q; ++i)
                post[slot(i, x, y, nx, ny)] = fs[i];
        }
}

/* Halfway streaming: for each fluid x and each i, the neighbour is
 * y = x + v_i (periodic).  If y is fluid, f_i(y, t+1) = fstar_i(x); otherwise
 * the population bounces back halfway: f_opp(i)(x, t+1) = fstar_i(x).  This
 * is a bijection on fluid slots. */
static void stream_halfway(int nx, int ny, const uint8_t *mask, double *f, const double *post)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            if (mask[n] != 0)
                continue;
            for (int i = 0; i < Q; ++i) {
                int xn = wrap(x + CX[i], nx), yn = wrap(y + CY[i], ny);
                if (mask[(size_t)yn * nx + xn] == 0)
                    f[slot(i, xn, yn, nx, ny)] = post[slot(i, x, y, nx, ny)];
                else
                    f[slot(opposite(i), x, y, nx, ny)] = post[slot(i, x, y, nx, ny)];
            }
        }
}

/* Full-way streaming: every post-collision population of a fluid or wall node
 * moves to x + v_i.  A fluid target takes it from either kind of source (a
 * fluid node's neighbours are all fluid or wall); a wall target only from a
 * fluid source, and its other slots are cleared. */
static void stream_fullway(int nx, int ny, const uint8_t *mask, const uint8_t *wall, double *f,
                           const double *post)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            if (wall[(size_t)y * nx + x])
                for (int i = 0; i < Q; ++i)
                    f[slot(i, x, y, nx, ny)] = 0.0;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            if (mask[n] != 0 && !wall[n])
                continue;
            for (int i = 0; i < Q; ++i) {
                int xn = wrap(x + CX[i], nx), yn = wrap(y + CY[i], ny);
                size_t t = (size_t)yn * nx + xn;
                if (mask[t] == 0 || (wall[t] && mask[n] == 0))
                    f[slot(i, xn, yn, nx, ny)] = post[slot(i, x, y, nx, ny)];
            }
        }
}

/* Wall nodes of a mask: solid nodes with at least one fluid neighbour. */
static void find_walls(int nx, int ny, const uint8_t *mask, uint8_t *wall)
{
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            wall[n] = 0;
            if (mask[n] == 0)
                continue;
            for (int i = 1; i < Q; ++i)
                if (mask[(size_t)wrap(y + CY[i], ny) * nx + wrap(x + CX[i], nx)] == 0)
                    wall[n] = 1;
        }
}

/* Full-way initial wall slots: slot i of a wall node w takes f_i of the fluid
 * node w - v_i (its value had that node been at rest in the step before: an
 * equilibrium state maps to itself under a force-free collision), 0 where
 * w - v_i is not fluid.  Fluid slots are unchanged. */
int oracle_fullway_fill(int nx, int ny, const uint8_t *mask, double *f)
{
    if (nx < 1 || ny < 1)
        return -1;
    uint8_t *wall = (uint8_t *)malloc((size_t)nx * ny);
    if (!wall)
        return -2;
    find_walls(nx, ny, mask, wall);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (!wall[(size_t)y * nx + x])
                continue;
            for (int i = 0; i < Q; ++i) {
                int xs = wrap(x - CX[i], nx), ys = wrap(y - CY[i], ny);
                f[slot(i, x, y, nx, ny)] =
                    mask[(size_t)ys * nx + xs] == 0 ? f[slot(i, xs, ys, nx, ny)] : 0.0;
            }
        }
    free(wall);
    return 0;
}

/* Run nsteps steps in place.  tau > 1/2 (Eq. 5: omega = 1/tau); tau_m > 1/2
 * is the antisymmetric relaxation time of the two-relaxation-time collision
 * (tau_m = tau: BGK).  alpha may be NULL (no drag).  bc / value may be NULL
 * (no open boundaries); else the boundary conditions are applied after every
 * streaming phase.  fullway selects the full-way wall rule (the state then
 * includes the wall slots).  nthreads <= 0 keeps the OpenMP default. */
static int run_general(int nx, int ny, const uint8_t *mask, double *f, double tau, double tau_m,
                       const double *mrt, double gx, double gy, const double *alpha,
                       const uint8_t *bc, const double *value, long nsteps, int nthreads,
                       int fullway)
{
    if (nx < 1 || ny < 1 || !(tau > 0.5) || !(tau_m > 0.5) || nsteps < 0)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    double omega = 1.0 / tau, omega_m = tau_m == tau ? omega : 1.0 / tau_m;
    size_t total = (size_t)Q * nx * ny;
    double *post = (double *)calloc(total, sizeof(double));
    uint8_t *wall = fullway ? (uint8_t *)malloc((size_t)nx * ny) : NULL;
    if (!post || (fullway && !wall)) {
        free(post);
        free(wall);
        return -2;
    }
    if (wall)
        find_walls(nx, ny, mask, wall);
    int rc = 0;
    for (long s = 0; s < nsteps && rc == 0; ++s) {
        collide_phase(nx, ny, mask, wall, f, post, omega, omega_m, mrt, gx, gy, alpha);
        if (wall)
            stream_fullway(nx, ny, mask, wall, f, post);
        else
            stream_halfway(nx, ny, mask, f, post);
        if (bc && oracle_apply_boundaries(nx, ny, mask, bc, value, f))
            rc = -1;
    }
    free(post);
    free(wall);
    return rc;
}

int oracle_run_walls(int nx, int ny, const uint8_t *mask, double *f, double tau, double tau_m,
                     double gx, double gy, const double *alpha, const uint8_t *bc,
                     const double *value, long nsteps, int nthreads, int fullway)
{
    return run_general(nx, ny, mask, f, tau, tau_m, NULL, gx, gy, alpha, bc, value, nsteps,
                       nthreads, fullway);
}

/* As oracle_run_walls with the multiple-relaxation-time collision: the shear
 * moments p_xx, p_xy relax with omega = 1/tau (which sets the viscosity as in
 * Eq. 5), e with s_e, eps with s_eps, q_x and q_y with s_q; rho and j with 1. */
int oracle_run_mrt(int nx, int ny, const uint8_t *mask, double *f, double tau, double s_e,
                   double s_eps, double s_q, double gx, double gy, const double *alpha,
                   const uint8_t *bc, const double *value, long nsteps, int nthreads,
                   int fullway)
{
    if (!(tau > 0.5))
        return -1;
    double omega = 1.0 / tau;
    double rates[Q] = {1.0, s_e, s_eps, 1.0, s_q, 1.0, s_q, omega, omega};
    return run_general(nx, ny, mask, f, tau, tau, rates, gx, gy, alpha, bc, value, nsteps,
                       nthreads, fullway);
}

int oracle_run_trt(int nx, int ny, const uint8_t *mask, double *f, double tau, double tau_m,
                   double gx, double gy, const double *alpha, const uint8_t *bc,
                   const double *value, long nsteps, int nthreads)
{
    return oracle_run_walls(nx, ny, mask, f, tau, tau_m, gx, gy, alpha, bc, value, nsteps,
                            nthreads, 0);
}

int oracle_run_bc(int nx, int ny, const uint8_t *mask, double *f, double tau, double gx,
                  double gy, const double *alpha, const uint8_t *bc, const double *value,
                  long nsteps, int nthreads)
{
    return oracle_run_trt(nx, ny, mask, f, tau, tau, gx, gy, alpha, bc, value, nsteps, nthreads);
}

int oracle_run(int nx, int ny, const uint8_t *mask, double *f, double tau, double gx, double gy,
               const double *alpha, long nsteps, int nthreads)
{
    return oracle_run_bc(nx, ny, mask, f, tau, gx, gy, alpha, NULL, NULL, nsteps, nthreads);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Macroscopic fields of the canonical state (Eq. 2 with the corrected
 * velocity); solid nodes report rho = 0, u = 0. */
int oracle_macroscopic(int nx, int ny, const uint8_t *mask, const double *f, double gx, double gy,
                       const double *alpha, double *rho, double *ux, double *uy)
{
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            if (mask[n] != 0) {
                rho[n] = ux[n] = uy[n] = 0.0;
                continue;
            }
            double fl[Q], m[3];
            for (int i = 0; i < Q; ++i)
                fl[i] = f[slot(i, x, y, nx, ny)];
            oracle_node_velocity(fl, alpha ? alpha[n] : 0.0, gx, gy, m);
            rho[n] = m[0];
            ux[n] = m[1];
            uy[n] = m[2];
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gradient of J = mean u_x over the fluid nodes of column x_out at time T.  */
/* ------------------------------------------------------------------------ */

/* Directional derivative (forward mode) of the collision along
 * (df, dalpha, dgx, dgy): each line is the linearisation of the matching line
 * of oracle_collide. */
static void collide_tangent(const double *f, double alpha, double gx, double gy, double omega,
                            const double *df, double dalpha, double dgx, double dgy,
                            double *dfstar)
{
    double rho = 0.0, mx = 0.0, my = 0.0, drho = 0.0, dmx = 0.0, dmy = 0.0;
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        mx += CX[i] * f[i];
        my += CY[i] * f[i];
        drho += df[i];
        dmx += CX[i] * df[i];
        dmy += CY[i] * df[i];
    }
    double D = 1.0 + 0.5 * alpha, dD = 0.5 * dalpha;
    double ux = (mx / rho + 0.5 * gx) / D;
    double uy = (my / rho + 0.5 * gy) / D;
    double dux = ((dmx * rho - mx * drho) / (rho * rho) + 0.5 * dgx) / D - ux * dD / D;
    double duy = ((dmy * rho - my * drho) / (rho * rho) + 0.5 * dgy) / D - uy * dD / D;
    double Fx = rho * (gx - alpha * ux);
    double Fy = rho * (gy - alpha * uy);
    double dFx = drho * (gx - alpha * ux) + rho * (dgx - dalpha * ux - alpha * dux);
    double dFy = drho * (gy - alpha * uy) + rho * (dgy - dalpha * uy - alpha * duy);
    double uu = ux * ux + uy * uy;
    double duu = 2.0 * (ux * dux + uy * duy);
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        double dcu = CX[i] * dux + CY[i] * duy;
        double poly = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
        double dpoly = 3.0 * dcu + 9.0 * cu * dcu - 1.5 * duu;
        double dfeq = W[i] * (drho * poly + rho * dpoly);
        double cF = CX[i] * Fx + CY[i] * Fy;
        double dcF = CX[i] * dFx + CY[i] * dFy;
        double dS = W[i] * (3.0 * (-dux * Fx - duy * Fy + (CX[i] - ux) * dFx + (CY[i] - uy) * dFy) +
                            9.0 * (dcu * cF + cu * dcF));
        dfstar[i] = df[i] - omega * (df[i] - dfeq) + (1.0 - 0.5 * omega) * dS;
    }
}

/* Full local Jacobian of the collision at one node:
 *   dfdf[i*9 + j] = d fstar_i / d f_j,  dfda[i] = d fstar_i / d alpha,
 *   dfdg[i*2 + b] = d fstar_i / d g_b. */
void oracle_collide_jacobian(const double *f, double alpha, double gx, double gy, double omega,
                             double *dfdf, double *dfda, double *dfdg)
{
    double e[Q], col[Q];
    for (int j = 0; j < Q; ++j) {
        for (int k = 0; k < Q; ++k)
            e[k] = (k == j) ? 1.0 : 0.0;
        collide_tangent(f, alpha, gx, gy, omega, e, 0.0, 0.0, 0.0, col);
        for (int i = 0; i < Q; ++i)
            dfdf[i * Q + j] = col[i];
    }
    for (int k = 0; k < Q; ++k)
        e[k] = 0.0;
    collide_tangent(f, alpha, gx, gy, omega, e, 1.0, 0.0, 0.0, col);
    for (int i = 0; i < Q; ++i)
        dfda[i] = col[i];
    collide_tangent(f, alpha, gx, gy, omega, e, 0.0, 1.0, 0.0, col);
    for (int i = 0; i < Q; ++i)
        dfdg[i * 2 + 0] = col[i];
    collide_tangent(f, alpha, gx, gy, omega, e, 0.0, 0.0, 1.0, col);
    for (int i = 0; i < Q; ++i)
        dfdg[i * 2 + 1] = col[i];
}

/* J = (1/n_out) sum over fluid nodes (x_out, y) of u_x. */
int oracle_objective_outlet_ux(int nx, int ny, const uint8_t *mask, const double *f, double gx,
                               double gy, const double *alpha, int x_out, double *J)
{
    if (x_out < 0 || x_out >= nx)
        return -1;
    double sum = 0.0;
    int n_out = 0;
    for (int y = 0; y < ny; ++y) {
        size_t n = (size_t)y * nx + x_out;
        if (mask[n] != 0)
            continue;
        double fl[Q], m[3];
        for (int i = 0; i < Q; ++i)
            fl[i] = f[slot(i, x_out, y, nx, ny)];
        oracle_node_velocity(fl, alpha ? alpha[n] : 0.0, gx, gy, m);
        sum += m[1];
        ++n_out;
    }
    if (n_out == 0)
        return -1;
    *J = sum / n_out;
    return 0;
}

/* Reverse-mode gradient of J after T steps from the initial state f0, with
 * respect to the per-node alpha field and the body force g.  Every state
 * f(0..T) is kept (no checkpointing).  lambda_t = dJ/df(t):
 *   lambda_T      from the objective,
 *   lambda*(x)_i  = lambda_{t+1,i}(x + v_i) if x + v_i is fluid, else
 *                   lambda_{t+1,opp(i)}(x)          (transpose of streaming),
 *   lambda_t(x)_j = sum_i dfstar_i/df_j  lambda*(x)_i  (transpose of collision),
 *   dJ/dalpha(x) += sum_i dfstar_i/dalpha lambda*(x)_i,
 *   dJ/dg        += sum_x sum_i dfstar_i/dg lambda*(x)_i.
 * grad_alpha ([ny][nx]) and grad_g ([2]) are overwritten; J is J(T). */
int oracle_outlet_ux_gradient(int nx, int ny, const uint8_t *mask, const double *f0, double tau,
                              double gx, double gy, const double *alpha, long T, int x_out,
                              double *J, double *grad_alpha, double *grad_g)
{
    if (nx < 1 || ny < 1 || !(tau > 0.5) || T < 0 || x_out < 0 || x_out >= nx)
        return -1;
    double omega = 1.0 / tau;
    size_t nn = (size_t)nx * ny, total = (size_t)Q * nn;
    double *states = (double *)malloc((size_t)(T + 1) * total * sizeof(double));
    double *post = (double *)calloc(total, sizeof(double));
    double *lam = (double *)calloc(total, sizeof(double));
    double *lam_next = (double *)calloc(total, sizeof(double));
    if (!states || !post || !lam || !lam_next) {
        free(states);
        free(post);
        free(lam);
        free(lam_next);
        return -2;
    }
    memcpy(states, f0, total * sizeof(double));
    for (long t = 0; t < T; ++t) {
        memcpy(states + (size_t)(t + 1) * total, states + (size_t)t * total,
               total * sizeof(double));
        double *ft = states + (size_t)(t + 1) * total;
        collide_phase(nx, ny, mask, NULL, ft, post, omega, omega, NULL, gx, gy, alpha);
        stream_halfway(nx, ny, mask, ft, post);
    }
    const double *fT = states + (size_t)T * total;
    if (oracle_objective_outlet_ux(nx, ny, mask, fT, gx, gy, alpha, x_out, J) != 0) {
        free(states);
        free(post);
        free(lam);
        free(lam_next);
        return -1;
    }

    for (size_t k = 0; k < nn; ++k)
        grad_alpha[k] = 0.0;
    grad_g[0] = grad_g[1] = 0.0;

    /* Seed: derivatives of J through u_x = (m_x/rho + g_x/2) / (1 + alpha/2). */
    int n_out = 0;
    for (int y = 0; y < ny; ++y)
        if (mask[(size_t)y * nx + x_out] == 0)
            ++n_out;
    for (int y = 0; y < ny; ++y) {
        size_t n = (size_t)y * nx + x_out;
        if (mask[n] != 0)
            continue;
        double a = alpha ? alpha[n] : 0.0, D = 1.0 + 0.5 * a;
        double rho = 0.0, mx = 0.0;
        for (int i = 0; i < Q; ++i) {
            rho += fT[slot(i, x_out, y, nx, ny)];
            mx += CX[i] * fT[slot(i, x_out, y, nx, ny)];
        }
        double ux = (mx / rho + 0.5 * gx) / D;
        for (int j = 0; j < Q; ++j)
            lam[slot(j, x_out, y, nx, ny)] = (CX[j] - mx / rho) / (rho * D) / n_out;
        grad_alpha[n] += -0.5 * ux / D / n_out;
        grad_g[0] += 0.5 / D / n_out;
    }

    for (long t = T - 1; t >= 0; --t) {
        const double *ft = states + (size_t)t * total;
        double *tmp = lam_next;
        lam_next = lam; /* lambda_{t+1} */
        lam = tmp;
        for (size_t k = 0; k < total; ++k)
            lam[k] = 0.0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = (size_t)y * nx + x;
                if (mask[n] != 0)
                    continue;
                double ls[Q], fl[Q];
                for (int i = 0; i < Q; ++i) {
                    int xn = wrap(x + CX[i], nx), yn = wrap(y + CY[i], ny);
                    if (mask[(size_t)yn * nx + xn] == 0)
                        ls[i] = lam_next[slot(i, xn, yn, nx, ny)];
                    else
                        ls[i] = lam_next[slot(opposite(i), x, y, nx, ny)];
                    fl[i] = ft[slot(i, x, y, nx, ny)];
                }
                double dfdf[Q * Q], dfda[Q], dfdg[Q * 2];
                oracle_collide_jacobian(fl, alpha ? alpha[n] : 0.0, gx, gy, omega, dfdf, dfda,
                                        dfdg);
                for (int j = 0; j < Q; ++j) {
                    double s = 0.0;
                    for (int i = 0; i < Q; ++i)
                        s += dfdf[i * Q + j] * ls[i];
                    lam[slot(j, x, y, nx, ny)] = s;
                }
                double sa = 0.0, sgx = 0.0, sgy = 0.0;
                for (int i = 0; i < Q; ++i) {
                    sa += dfda[i] * ls[i];
                    sgx += dfdg[i * 2 + 0] * ls[i];
                    sgy += dfdg[i * 2 + 1] * ls[i];
                }
                grad_alpha[n] += sa;
                grad_g[0] += sgx;
                grad_g[1] += sgy;
            }
    }
    free(states);
    free(post);
    free(lam);
    free(lam_next);
    return 0;
}
