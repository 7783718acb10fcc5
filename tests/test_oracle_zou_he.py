"""Pins of the oracle's open boundaries (Sec. 3: constant velocity and constant pressure after
Zou and He), each against something other than the oracle's own closed form:

* the defining conditions, solved as a 4 x 4 linear system here (density, normal and
  tangential momentum of Eq. 2, and equal non-equilibrium parts of the normal pair);
* the 90-degree rotation symmetry of the lattice (all four normals agree);
* uniform flow at equilibrium is an exact fixed point of a domain with open ends;
* the prescribed moments hold at boundary nodes throughout a run;
* the developed channel flows of Sec. 4.1 (chan_v, chan_p): the profile is the parabola of
  Eq. 7 with halfway walls, the inflow mass flux is carried through the channel, and the
  pressure-driven peak velocity matches G H^2 / (8 nu) (Eq. 5 viscosity).
"""
import numpy as np
import pytest

import synthetic

# D2Q9 velocities, the paper's Fig. 1 numbering (pinned against the paper in test_oracle_pins)
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
NORMALS = [(1, 0), (-1, 0), (0, 1), (0, -1)]


def _random_populations(rng):
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return w * (1.0 + 0.2 * (2.0 * rng.random(9) - 1.0))


def _solve_definition(f, kind, n, value):
    """Unknowns: (rho or u_n, then the three entering populations).  Conditions:
    sum f = rho; sum (c.n) f = rho u_n; sum (c.t) f = rho u_t; f_n - f_opp(n) = 2/3 rho u_n."""
    nx_, ny_ = n
    tx, ty = -ny_, nx_
    cn = CX * nx_ + CY * ny_
    ct = CX * tx + CY * ty
    entering = [i for i in range(9) if cn[i] > 0]
    known = [i for i in range(9) if cn[i] <= 0]
    i_n = [i for i in entering if ct[i] == 0][0]
    A = np.zeros((4, 4))
    b = np.zeros(4)
    rows = [np.ones(9), cn.astype(float), ct.astype(float)]
    if kind == "velocity":
        un = value[0] * nx_ + value[1] * ny_
        ut = value[0] * tx + value[1] * ty
        targets = [1.0, un, ut]       # coefficient of rho in each moment condition
        for r, (row, tcoef) in enumerate(zip(rows, targets)):
            A[r, 0] = -tcoef
            for k, i in enumerate(entering):
                A[r, 1 + k] = row[i]
            b[r] = -sum(row[i] * f[i] for i in known)
        A[3, 0] = -2.0 / 3.0 * un
    else:
        rho = value[0]
        # sum f = rho; sum (c.n) f - rho u_n = 0; sum (c.t) f = 0
        for k, i in enumerate(entering):
            A[0, 1 + k] = 1.0
            A[1, 1 + k] = cn[i]
            A[2, 1 + k] = ct[i]
        b[0] = rho - sum(f[i] for i in known)
        A[1, 0] = -rho
        b[1] = -sum(cn[i] * f[i] for i in known)
        b[2] = -sum(ct[i] * f[i] for i in known)
        A[3, 0] = -2.0 / 3.0 * rho
    A[3, 1 + entering.index(i_n)] = 1.0
    b[3] = f[OPP[i_n]]
    sol = np.linalg.solve(A, b)
    out = np.array(f, dtype=np.float64)
    for k, i in enumerate(entering):
        out[i] = sol[1 + k]
    return out


@pytest.mark.parametrize("kind", ["velocity", "pressure"])
@pytest.mark.parametrize("n", NORMALS)
def test_zou_he_solves_defining_conditions(oracle_mod, kind, n):
    rng = np.random.default_rng(11)
    for _ in range(20):
        f = _random_populations(rng)
        value = (0.1 * (2 * rng.random() - 1), 0.1 * (2 * rng.random() - 1)) if kind == "velocity" \
            else (1.0 + 0.05 * (2 * rng.random() - 1), 0.0)
        got = oracle_mod.zou_he(f, kind, n, value)
        ref = _solve_definition(f, kind, n, value)
        assert np.abs(got - ref).max() < 1e-15
        # the known populations are untouched
        cn = CX * n[0] + CY * n[1]
        assert np.array_equal(got[cn <= 0], f[cn <= 0])


def _rotation_permutation():
    """p with c_p(i) = R c_i, R the rotation by +90 degrees: (x, y) -> (-y, x)."""
    p = np.zeros(9, dtype=int)
    for i in range(9):
        rx, ry = -CY[i], CX[i]
        p[i] = [j for j in range(9) if CX[j] == rx and CY[j] == ry][0]
    return p


@pytest.mark.parametrize("kind", ["velocity", "pressure"])
def test_zou_he_rotation_symmetry(oracle_mod, kind):
    rng = np.random.default_rng(12)
    p = _rotation_permutation()
    for n in NORMALS:
        f = _random_populations(rng)
        value = (0.07, -0.03) if kind == "velocity" else (1.02, 0.0)
        out = oracle_mod.zou_he(f, kind, n, value)
        fr = np.zeros(9)
        fr[p] = f
        nr = (-n[1], n[0])
        vr = (-value[1], value[0]) if kind == "velocity" else value
        outr = oracle_mod.zou_he(fr, kind, nr, vr)
        expect = np.zeros(9)
        expect[p] = out
        assert np.abs(outr - expect).max() < 1e-15


@pytest.mark.parametrize("case", ["velocity-velocity-oblique", "velocity-pressure",
                                  "vertical-velocity-pressure"])
def test_uniform_flow_is_fixed_point(oracle_mod, case):
    """f^eq(1, u) everywhere, open ends prescribing that same flow, periodic sides: exact."""
    nx, ny = 24, 10
    vertical = case.startswith("vertical")
    if vertical:
        nx, ny = ny, nx
    m = synthetic.all_fluid(nx, ny)
    bc = np.zeros((ny, nx), np.uint8)
    val = np.zeros((2, ny, nx))
    U, V = (0.06, 0.02) if case == "velocity-velocity-oblique" else (0.06, 0.0)
    if vertical:
        U, V = 0.0, 0.05
        bc[0, :] = synthetic.BC_VELOCITY[(0, 1)]
        val[0, 0, :], val[1, 0, :] = U, V
        bc[ny - 1, :] = synthetic.BC_PRESSURE[(0, -1)]
        val[0, ny - 1, :] = 1.0
    else:
        bc[:, 0] = synthetic.BC_VELOCITY[(1, 0)]
        val[0, :, 0], val[1, :, 0] = U, V
        if case == "velocity-velocity-oblique":
            bc[:, nx - 1] = synthetic.BC_VELOCITY[(-1, 0)]
            val[0, :, nx - 1], val[1, :, nx - 1] = U, V
        else:
            bc[:, nx - 1] = synthetic.BC_PRESSURE[(-1, 0)]
            val[0, :, nx - 1] = 1.0
    f0 = oracle_mod.init(m, None, np.full((ny, nx), U), np.full((ny, nx), V), bc=bc, value=val)
    feq = oracle_mod.equilibrium(1.0, U, V)
    assert np.abs(f0 - feq[:, None, None]).max() < 1e-15
    f = oracle_mod.run(m, f0, 0.7, 50, bc=bc, value=val)
    assert np.abs(f - feq[:, None, None]).max() < 1e-14


@pytest.mark.parametrize("inlet", ["velocity", "pressure"])
def test_boundary_moments_hold_during_run(oracle_mod, inlet):
    nx, ny = 40, 12
    m, bc, val = synthetic.open_channel(nx, ny, inlet, u_in=0.05, rho_in=1.02)
    f = oracle_mod.init(m, bc=bc, value=val)
    for _ in range(3):
        f = oracle_mod.run(m, f, 0.8, 37, bc=bc, value=val)
        rho, ux, uy = oracle_mod.macroscopic(m, f)
        inl = slice(1, ny - 1)
        if inlet == "velocity":
            assert np.abs(ux[inl, 0] - 0.05).max() < 1e-15
        else:
            assert np.abs(rho[inl, 0] - 1.02).max() < 1e-15
        assert np.abs(uy[inl, 0]).max() < 1e-15
        assert np.abs(rho[inl, nx - 1] - 1.0).max() < 1e-15
        assert np.abs(uy[inl, nx - 1]).max() < 1e-15


def _profile_fit(prof, H):
    y = np.arange(1, H + 1)
    par = (y - 0.5) * (H + 0.5 - y)
    c = (prof * par).sum() / (par * par).sum()
    return np.abs(prof - c * par).max() / prof.max()


def test_chan_v_develops_parabola_and_carries_inflow(oracle_mod):
    """Sec. 4.1 chan_v, scaled down: velocity inlet u = 0.05, pressure outlet rho = 1, halfway
    walls (H = 16 fluid rows), tau = 0.8.  After 10000 steps the flow is steady: the middle
    column is the parabola of Eq. 7 (walls halfway between nodes) within 1 %, and its mass flux
    equals the inflow through the inlet column (steady mass conservation) within 1e-6."""
    nx, ny = 160, 18
    m, bc, val = synthetic.open_channel(nx, ny, "velocity", u_in=0.05)
    f = oracle_mod.run(m, oracle_mod.init(m, bc=bc, value=val), 0.8, 10000, bc=bc, value=val)
    rho, ux, _ = oracle_mod.macroscopic(m, f)
    prof = ux[1:ny - 1, nx // 2]
    assert _profile_fit(prof, ny - 2) < 1e-2
    flux = (rho * ux)[1:ny - 1, :].sum(axis=0)
    assert abs(flux[nx // 2] / flux[0] - 1.0) < 1e-6
    assert np.all(ux[1:ny - 1, :] > 0)


def test_chan_p_pressure_driven_peak_velocity(oracle_mod):
    """Sec. 4.1 chan_p, scaled down: inlet rho = 1.016, outlet rho = 1.0 (initial 1.008),
    H = 16, tau = 0.8.  Steady state: density falls linearly (pressure p = rho / 3), and the
    centre velocity is G H^2 / (8 nu) with G = (dp/dx) / rho and nu = (tau - 1/2) / 3 (Eq. 5),
    within 2 % (compressibility and wall slip); profile parabolic within 1 %."""
    nx, ny, tau = 160, 18, 0.8
    m, bc, val = synthetic.open_channel(nx, ny, "pressure", rho_in=1.016, rho_out=1.0)
    f0 = oracle_mod.init(m, np.full((ny, nx), 1.008), bc=bc, value=val)
    f = oracle_mod.run(m, f0, tau, 15000, bc=bc, value=val)
    rho, ux, _ = oracle_mod.macroscopic(m, f)
    H = ny - 2
    grad = -(1.016 - 1.0) / (nx - 1)
    drho = (rho[ny // 2, nx // 2 + 20] - rho[ny // 2, nx // 2 - 20]) / 40.0
    assert abs(drho / grad - 1.0) < 1e-2
    G = -(grad / 3.0) / rho[1:ny - 1, 1:nx - 1].mean()
    nu = (tau - 0.5) / 3.0
    prof = ux[1:ny - 1, nx // 2]
    assert abs(prof.max() / (G * H * H / (8.0 * nu)) - 1.0) < 2e-2
    assert _profile_fit(prof, H) < 1e-2


def test_lid_cavity_moments_and_circulation(oracle_mod):
    """Sec. 4.1 lid-driven cavity (small, Re = 10): the lid nodes keep the lid velocity, and
    the lid drives a clockwise vortex: positive u_x under the lid, negative near the bottom,
    rising along the left wall and sinking along the right one."""
    n = 34
    m, bc, val = synthetic.lid_cavity(n, 0.1)
    nu = 0.1 * (n - 2) / 10.0
    tau = 3.0 * nu + 0.5
    f = oracle_mod.run(m, oracle_mod.init(m, bc=bc, value=val), tau, 3000, bc=bc, value=val)
    rho, ux, uy = oracle_mod.macroscopic(m, f)
    assert np.abs(ux[n - 1, 1:n - 1] - 0.1).max() < 1e-15
    assert np.abs(uy[n - 1, 1:n - 1]).max() < 1e-15
    mid = n // 2
    assert ux[n - 3, mid] > 0.02 and ux[3, mid] < 0.0
    assert uy[mid, 3] > 0.0 > uy[mid, n - 4]  # clockwise: up along the left wall, down on the right


def test_bad_codes_rejected(oracle_mod):
    m = synthetic.channel_mask(8, 6)
    bc = np.zeros((6, 8), np.uint8)
    val = np.zeros((2, 6, 8))
    f = oracle_mod.init(m)
    bc[0, 3] = 1  # at a solid node
    with pytest.raises(ValueError):
        oracle_mod.apply_boundaries(m, f, bc, val)
    bc[0, 3] = 0
    bc[2, 3] = 9
    with pytest.raises(ValueError):
        oracle_mod.apply_boundaries(m, f, bc, val)
