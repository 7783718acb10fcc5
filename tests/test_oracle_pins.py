"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test states the property it checks and the passage it comes from.  None of them
re-derives a value by retyping the oracle's own formula: they use values printed in
the paper, closed-form moments and conservation laws, lattice symmetry, exact closed
forms of the discrete dynamics, exact-rational brute force and finite differences.
"""
import json
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import synthetic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- constants --
def test_lattice_numbering_matches_paper(oracle_mod):
    """Sec. 2.2: v_0 = [0,0], v_1 = [1,0], v_4 = [0,-1], v_6 = [-1,1]; the rest of the
    numbering from the label positions of Fig. 1; weights of Eq. 6."""
    g = json.load(open(os.path.join(GOLDEN, "paper_lattice.json")))
    cx, cy, w, opp = oracle_mod.constants()
    for k, v in g["velocities_spelled_out"].items():
        assert (cx[int(k)], cy[int(k)]) == tuple(v)
    pos = {int(k): v for k, v in g["fig1_label_positions"].items() if not k.startswith("_")}
    # the centre node sits midway between the labels of opposite axis links 1/3 and 2/4
    centre = ((pos[1][0] + pos[3][0]) / 2, (pos[2][1] + pos[4][1]) / 2)
    for i, (px, py) in pos.items():
        dx, dy = px - centre[0], py - centre[1]
        sx = 0 if abs(dx) < 0.1 else int(math.copysign(1, dx))
        sy = 0 if abs(dy) < 0.1 else int(math.copysign(1, dy))
        assert (cx[i], cy[i]) == (sx, sy), i
    assert w[0] == pytest.approx(4 / 9, abs=1e-17)
    assert np.allclose(w[1:5], 1 / 9, atol=1e-17, rtol=0)
    assert np.allclose(w[5:9], 1 / 36, atol=1e-17, rtol=0)
    for i in range(9):
        assert (cx[opp[i]], cy[opp[i]]) == (-cx[i], -cy[i])


def test_lattice_isotropy(oracle_mod):
    """Weight moments the D2Q9 equilibrium of Eq. 6 relies on: sum w = 1, sum w c = 0,
    sum w c_a c_b = delta_ab / 3, fourth moment = (dd + dd + dd) / 9."""
    cx, cy, w, _ = oracle_mod.constants()
    c = np.stack([cx, cy], 1).astype(float)
    d = np.eye(2)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.abs(w @ c).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(m4, iso, atol=1e-16)


# ----------------------------------------------------- equilibrium / forcing --
@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (1.03, 0.05, -0.02), (0.9, -0.08, 0.07)])
def test_equilibrium_moments(oracle_mod, rho, ux, uy):
    """Eq. 6 has the hydrodynamic moments rho, rho u and rho (u u + I/3)."""
    cx, cy, _, _ = oracle_mod.constants()
    c = np.stack([cx, cy], 1).astype(float)
    feq = oracle_mod.equilibrium(rho, ux, uy)
    u = np.array([ux, uy])
    assert feq.sum() == pytest.approx(rho, abs=1e-15)
    assert np.allclose(c.T @ feq, rho * u, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", feq, c, c), rho * (np.outer(u, u) + np.eye(2) / 3),
                       atol=1e-15)


@pytest.mark.parametrize("u,F", [((0.0, 0.0), (1e-3, 0.0)), ((0.04, -0.03), (2e-4, -5e-4))])
def test_forcing_term_moments(oracle_mod, u, F):
    """Guo's forcing term: zeroth moment 0, first moment F, second moment u F + F u."""
    cx, cy, _, _ = oracle_mod.constants()
    c = np.stack([cx, cy], 1).astype(float)
    S = oracle_mod.guo_source(u[0], u[1], F[0], F[1])
    uu, FF = np.array(u), np.array(F)
    assert abs(S.sum()) < 1e-18
    assert np.allclose(c.T @ S, FF, atol=1e-18)
    assert np.allclose(np.einsum("i,ia,ib->ab", S, c, c), np.outer(uu, FF) + np.outer(FF, uu),
                       atol=1e-18)


def _random_pops(seed):
    rng = np.random.default_rng(seed)
    cx_rho = 1.0 + 0.05 * rng.standard_normal()
    f = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36]) * cx_rho
    return f * (1 + 0.2 * rng.standard_normal(9))


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("alpha,g", [(0.0, (0.0, 0.0)), (0.0, (1e-3, -2e-3)), (0.7, (1e-3, 5e-4))])
def test_collision_conservation(oracle_mod, seed, alpha, g):
    """The collision conserves mass and changes momentum by exactly one force density,
    F = rho (g - alpha u) with u the corrected velocity (forcing and drag readings)."""
    cx, cy, _, _ = oracle_mod.constants()
    f = _random_pops(seed)
    fs = oracle_mod.collide(f, 1 / 0.8, alpha, g)
    rho, ux, uy = oracle_mod.node_velocity(f, alpha, g)
    assert fs.sum() == pytest.approx(f.sum(), abs=1e-15)
    m0 = np.array([cx @ f, cy @ f])
    m1 = np.array([cx @ fs, cy @ fs])
    F = rho * (np.array(g) - alpha * np.array([ux, uy]))
    assert np.allclose(m1, m0 + F, atol=1e-16)


def test_bgk_special_case(oracle_mod):
    """With g = 0 and alpha = 0 the collision is exactly BGK (Eqs. 3-4): the result is
    affine in omega, and omega = 1 lands on the equilibrium with the moments of the
    pre-collision state."""
    cx, cy, _, _ = oracle_mod.constants()
    c = np.stack([cx, cy], 1).astype(float)
    f = _random_pops(7)
    f1 = oracle_mod.collide(f, 1.0)
    rho = f.sum()
    u = (c.T @ f) / rho
    assert np.allclose(c.T @ f1, rho * u, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", f1, c, c), rho * (np.outer(u, u) + np.eye(2) / 3),
                       atol=1e-15)
    for om in (0.6, 1.25, 1.9):
        assert np.allclose(oracle_mod.collide(f, om), (1 - om) * f + om * f1, atol=1e-16)


def test_equilibrium_is_collision_fixed_point(oracle_mod):
    feq = oracle_mod.equilibrium(1.02, 0.03, -0.04)
    assert np.allclose(oracle_mod.collide(feq, 1 / 0.6), feq, atol=2e-16)


# ------------------------------------------------------------------ dynamics --
def test_uniform_flow_fixed_point(oracle_mod):
    """A uniform equilibrium on a periodic lattice stays put (streaming of a uniform
    state is the identity; the collision fixes f^eq)."""
    m = synthetic.all_fluid(12, 10)
    f0 = oracle_mod.init(m, np.full((10, 12), 1.0), np.full((10, 12), 0.05),
                         np.full((10, 12), -0.02))
    f = oracle_mod.run(m, f0, 0.7, 100)
    assert np.abs(f - f0).max() < 1e-13


def test_rest_state_with_walls_fixed_point(oracle_mod):
    m = synthetic.random_mask(16, 16, seed=3, solid_fraction=0.3, walls=True)
    f0 = oracle_mod.init(m)
    f = oracle_mod.run(m, f0, 0.9, 100)
    assert np.abs(f - f0).max() < 1e-15


@pytest.mark.parametrize("case", ["periodic", "walls", "porous"])
def test_mass_conservation(oracle_mod, case):
    """Halfway bounce-back streaming is a bijection on fluid slots and the collision
    conserves mass, so total mass is constant to rounding (with force and drag)."""
    nx, ny = 24, 20
    if case == "periodic":
        m = synthetic.all_fluid(nx, ny)
    elif case == "walls":
        m = synthetic.channel_mask(nx, ny)
    else:
        m = synthetic.random_mask(nx, ny, seed=11, solid_fraction=0.25, walls=True)
    rho, ux, uy = synthetic.random_fields(nx, ny, seed=5)
    alpha = synthetic.brinkman_alpha(nx, ny, seed=3, sigma=2.0)
    f0 = oracle_mod.init(m, rho, ux, uy)
    f = oracle_mod.run(m, f0, 0.75, 300, g=(1e-4, -5e-5), alpha=alpha)
    M0, M1 = f0.sum(), f.sum()
    assert abs(M1 - M0) / M0 < 1e-13
    assert np.all(f[:, m == 1] == 0)


def test_momentum_gain_periodic(oracle_mod):
    """Fully periodic, no drag: total momentum grows by exactly g * M per step."""
    nx, ny = 16, 12
    m = synthetic.all_fluid(nx, ny)
    cx, cy, _, _ = oracle_mod.constants()
    rho, ux, uy = synthetic.random_fields(nx, ny, seed=9)
    f0 = oracle_mod.init(m, rho, ux, uy)
    g = (3e-5, -1e-5)
    steps = 200
    f = oracle_mod.run(m, f0, 0.8, steps, g=g)
    M = f0.sum()
    P0 = np.array([np.tensordot(cx, f0, 1).sum(), np.tensordot(cy, f0, 1).sum()])
    P1 = np.array([np.tensordot(cx, f, 1).sum(), np.tensordot(cy, f, 1).sum()])
    expect = P0 + steps * M * np.array(g)
    assert np.allclose(P1, expect, rtol=1e-12, atol=1e-13)


def test_brinkman_recurrence(oracle_mod):
    """Uniform state, uniform alpha and g on a periodic lattice: the momentum per node
    obeys p' = (p (1 - alpha/2) + g) / (1 + alpha/2), so u -> g / alpha."""
    nx, ny = 6, 5
    m = synthetic.all_fluid(nx, ny)
    a, g = 0.3, 2e-3
    f = oracle_mod.init(m, None, np.full((ny, nx), 0.01), None)
    p = 0.01
    for _ in range(40):
        f = oracle_mod.run(m, f, 0.7, 1, g=(g, 0.0), alpha=np.full((ny, nx), a))
        p = (p * (1 - a / 2) + g) / (1 + a / 2)
        cx, _, _, _ = oracle_mod.constants()
        px = np.tensordot(cx, f, 1)
        assert np.allclose(px, p, rtol=1e-13)
    _, ux, _ = oracle_mod.macroscopic(m, f, g=(g, 0.0), alpha=np.full((ny, nx), a))
    assert abs(ux[0, 0] - g / a) / (g / a) < 0.02


def _rotate(f, m, alpha):
    """Quarter turn of the lattice: node (x, y) -> ((-y) mod N, x), v -> (-v_y, v_x).
    Direction map from Fig. 1's numbering: 1->2->3->4->1 and 5->6->7->8->5."""
    R = [0, 2, 3, 4, 1, 6, 7, 8, 5]
    n = m.shape[0]
    idx_new_y, idx_new_x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    src_x = idx_new_y               # y' = x
    src_y = (-idx_new_x) % n        # x' = -y  ->  y = -x'
    fr = np.zeros_like(f)
    for i in range(9):
        fr[R[i]] = f[i][src_y, src_x]
    return fr, m[src_y, src_x], None if alpha is None else alpha[src_y, src_x]


def _mirror(f, m, alpha):
    """Mirror x -> -x: v -> (-v_x, v_y); directions 1<->3, 5<->6, 7<->8."""
    M = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    n = m.shape[1]
    src_x = (-np.arange(n)) % n
    fr = np.zeros_like(f)
    for i in range(9):
        fr[M[i]] = f[i][:, src_x]
    return fr, m[:, src_x], None if alpha is None else alpha[:, src_x]


@pytest.mark.parametrize("op", ["rotate", "mirror"])
def test_lattice_symmetry(oracle_mod, op):
    """Stepping commutes with the lattice's symmetry operations (with mask, force and
    drag transformed alike): catches a wrong velocity, weight or opposite index."""
    n = 14
    m = synthetic.random_mask(n, n, seed=21, solid_fraction=0.2)
    rho, ux, uy = synthetic.random_fields(n, n, seed=22)
    alpha = synthetic.brinkman_alpha(n, n, seed=4, sigma=1.5)
    f0 = oracle_mod.init(m, rho, ux, uy)
    g = (2e-4, 1e-4)
    f1 = oracle_mod.run(m, f0, 0.65, 25, g=g, alpha=alpha)
    if op == "rotate":
        fr0, mr, ar = _rotate(f0, m, alpha)
        gr = (-g[1], g[0])
        fr1, _, _ = _rotate(f1, m, alpha)
    else:
        fr0, mr, ar = _mirror(f0, m, alpha)
        gr = (-g[0], g[1])
        fr1, _, _ = _mirror(f1, m, alpha)
    got = oracle_mod.run(mr, fr0, 0.65, 25, g=gr, alpha=ar)
    assert np.abs(got - fr1).max() < 1e-14


def test_steady_poiseuille_closed_form(oracle_mod):
    """Steady body-force channel: x-uniform, rho = 1, u_y = 0 and
    u(y) = (g/2nu)(y - 1/2)(H + 1/2 - y) + (g/nu)(16 (tau - 1/2)^2 - 3)/24 for fluid rows
    1..H (walls halfway at y = 1/2 and H + 1/2).  The parabola is Eq. 7's profile with
    R = H/2; the constant is the exact BGK + halfway bounce-back slip, which vanishes at
    tau = 1/2 + sqrt(3/16)."""
    tau, g, ny = 0.8, 1e-6, 64
    nu, H = (tau - 0.5) / 3, ny - 2
    m = synthetic.channel_mask(4, ny)
    f = oracle_mod.run(m, oracle_mod.init(m), tau, 110000, g=(g, 0.0))
    rho, ux, uy = oracle_mod.macroscopic(m, f, g=(g, 0.0))
    y = np.arange(1, ny - 1)
    exact = (g / (2 * nu)) * (y - 0.5) * (H + 0.5 - y) + (g / nu) * (16 * (tau - 0.5) ** 2 - 3) / 24
    assert np.abs(ux[1:-1, 0] - exact).max() / exact.max() < 1e-10
    assert np.abs(uy).max() < 1e-12 * exact.max() * 100
    assert np.abs(rho[1:-1] - 1).max() < 1e-10
    for col in range(1, 4):
        assert np.array_equal(ux[:, 0], ux[:, col])


def _startup_series(eta, t, g, nu, H, terms=400):
    s = (g / (2 * nu)) * eta * (H - eta)
    for k in range(1, 2 * terms, 2):
        s = s - 4 * g * H ** 2 / (nu * math.pi ** 3 * k ** 3) * np.sin(k * math.pi * eta / H) \
            * math.exp(-k * k * math.pi ** 2 * nu * t / H ** 2)
    return s


def test_channel_startup_series(oracle_mod):
    """The 256 x 64 body-force channel after 2000 steps from rest (flow ~40 % developed)
    against the start-up series of plane Poiseuille flow (walls at eta = 0, H)."""
    tau, g, ny = 0.8, 1e-6, 64
    nu, H = (tau - 0.5) / 3, ny - 2
    m = synthetic.channel_mask(256, ny)
    f = oracle_mod.run(m, oracle_mod.init(m), tau, 2000, g=(g, 0.0))
    _, ux, _ = oracle_mod.macroscopic(m, f, g=(g, 0.0))
    eta = np.arange(1, ny - 1) - 0.5
    ref = _startup_series(eta, 2000, g, nu, H)
    centre = ref.max()
    assert np.abs(ux[1:-1, 17] - ref).max() / centre < 2e-3
    assert np.abs(ux[1:-1, :] - ux[1:-1, :1]).max() < 1e-16 * 1e3


@pytest.mark.parametrize("n", [32, 64])
def test_taylor_green_decay_rate(oracle_mod, n):
    """Viscosity from Eq. 5 (nu = (tau - 1/2)/3): a Taylor-Green mode decays at 2 nu k^2."""
    tau = 0.6
    nu, k = (tau - 0.5) / 3, 2 * math.pi / n
    rho0, ux0, uy0 = synthetic.taylor_green(n, 0.01)
    m = synthetic.all_fluid(n, n)
    f = oracle_mod.init(m, rho0, ux0, uy0)
    t0, t1 = int(0.05 * n * n), int(0.3 * n * n)
    f0 = oracle_mod.run(m, f, tau, t0)
    f1 = oracle_mod.run(m, f0, tau, t1 - t0)
    x = np.arange(n)[None, :]
    y = np.arange(n)[:, None]
    shape = -np.cos(k * x) * np.sin(k * y)
    amp = []
    for ff in (f0, f1):
        _, ux, _ = oracle_mod.macroscopic(m, ff)
        amp.append((ux * shape).sum() / (shape * shape).sum())
    rate = -math.log(amp[1] / amp[0]) / (t1 - t0)
    assert abs(rate / (2 * nu * k * k) - 1) < 5e-4


# ------------------------------------------------------- exact-rational pins --
def _exact_case(case):
    rng = np.random.default_rng(100 + case)
    nx = ny = 4
    mask = [[0] * nx for _ in range(ny)]
    g = (Fr(0), Fr(0))
    alpha = None
    if case == 1:
        mask[2][1] = 1
        alpha = [[Fr(int(rng.integers(0, 10)), 10) for _ in range(nx)] for _ in range(ny)]
    if case == 2:
        mask[0] = [1] * nx
        mask[3] = [1] * nx
        g = (Fr(1, 1000), Fr(0))
    rho = [[Fr(90 + int(rng.integers(0, 21)), 100) for _ in range(nx)] for _ in range(ny)]
    ux = [[Fr(int(rng.integers(-5, 6)), 100) for _ in range(nx)] for _ in range(ny)]
    uy = [[Fr(int(rng.integers(-5, 6)), 100) for _ in range(nx)] for _ in range(ny)]
    return mask, rho, ux, uy, g, alpha


@pytest.mark.parametrize("case", [0, 1, 2])
def test_exact_rational_4x4(oracle_mod, case):
    """Three 4x4 lattices, 3 steps, tau = 4/5: fully periodic; one solid node with a
    rational drag field; walls with a body force.  FP64 oracle vs exact rationals."""
    from oracle import exact
    mask, rho, ux, uy, g, alpha = _exact_case(case)
    ex = exact.run(mask, rho, ux, uy, Fr(4, 5), 3, g=g, alpha=alpha)
    m = np.array(mask, dtype=np.uint8)
    tofl = lambda a: np.array([[float(v) for v in row] for row in a])
    f = oracle_mod.init(m, tofl(rho), tofl(ux), tofl(uy))
    f = oracle_mod.run(m, f, 0.8, 3, g=(float(g[0]), float(g[1])),
                       alpha=None if alpha is None else tofl(alpha))
    worst = 0.0
    for (x, y), pops in ex.items():
        for i in range(9):
            worst = max(worst, abs(f[i, y, x] - float(pops[i])))
    assert worst < 1e-15


# ----------------------------------------------------------------- gradient --
def test_collision_jacobian_vs_finite_differences(oracle_mod):
    """The oracle's local Jacobian (forward-mode tangents) against central differences
    of its own collision function (Richardson-extrapolated)."""
    f = _random_pops(5)
    om, a, g = 1 / 0.7, 0.4, (2e-3, -1e-3)
    dfdf, dfda, dfdg = oracle_mod.collide_jacobian(f, om, a, g)

    def cd(fun, h):
        return (fun(h) - fun(-h)) / (2 * h)

    def rich(fun, h=1e-3):
        return (4 * cd(fun, h / 2) - cd(fun, h)) / 3

    for j in range(9):
        e = np.zeros(9)
        e[j] = 1
        num = rich(lambda h: oracle_mod.collide(f + h * e, om, a, g))
        assert np.allclose(dfdf[:, j], num, atol=1e-10)
    num = rich(lambda h: oracle_mod.collide(f, om, a + h, g))
    assert np.allclose(dfda, num, atol=1e-10)
    num = rich(lambda h: oracle_mod.collide(f, om, a, (g[0] + h, g[1])))
    assert np.allclose(dfdg[:, 0], num, atol=1e-10)
    num = rich(lambda h: oracle_mod.collide(f, om, a, (g[0], g[1] + h)))
    assert np.allclose(dfdg[:, 1], num, atol=1e-10)


def test_outlet_gradient_vs_finite_differences(oracle_mod):
    """Reverse-mode dJ/dalpha and dJ/dg against central differences of the forward run
    (J = mean outlet u_x after T steps), on a small porous channel."""
    nx, ny, T, tau = 12, 8, 40, 0.8
    m = synthetic.channel_mask(nx, ny)
    m[3, 5] = 1
    alpha = synthetic.brinkman_alpha(nx, ny, seed=7, sigma=2.0)
    g = (1e-3, 2e-4)
    f0 = oracle_mod.init(m)
    J, ga, gg = oracle_mod.outlet_ux_gradient(m, f0, tau, T, nx - 1, g=g, alpha=alpha)

    def Jof(a, gv):
        f = oracle_mod.run(m, f0, tau, T, g=gv, alpha=a)
        return oracle_mod.objective_outlet_ux(m, f, nx - 1, g=gv, alpha=a)

    assert J == pytest.approx(Jof(alpha, g), rel=1e-14)
    h = 1e-5
    rng = np.random.default_rng(3)
    fluid = np.argwhere(m == 0)
    for (y, x) in fluid[rng.choice(len(fluid), 8, replace=False)]:
        ap, am = alpha.copy(), alpha.copy()
        ap[y, x] += h
        am[y, x] -= h
        fd = (Jof(ap, g) - Jof(am, g)) / (2 * h)
        assert abs(fd - ga[y, x]) <= 1e-6 * np.abs(ga).max() + 1e-5 * abs(fd)
    assert np.all(ga[m == 1] == 0)
    for b in range(2):
        gp, gm = list(g), list(g)
        gp[b] += h
        gm[b] -= h
        fd = (Jof(alpha, tuple(gp)) - Jof(alpha, tuple(gm))) / (2 * h)
        assert fd == pytest.approx(gg[b], rel=1e-6, abs=1e-9)
