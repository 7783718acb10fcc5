"""Pins of the D3Q19 oracle (the three-dimensional lattice the paper names as future work), each
against something other than its own arithmetic:

* lattice tensors: sum w = 1, sum w c c = I/3, the fourth-order isotropic tensor / 9, odd
  moments zero;
* moments of the equilibrium (Eq. 6) and of the forcing term; collision conserves mass and adds
  exactly the force;
* projection onto D2Q9: the D3Q19 weights summed over c_z are the D2Q9 weights (1/3 + 2/18 = 4/9,
  1/18 + 2/36 = 1/9, 1/36), so a z-invariant D3Q19 run, summed over c_z, is the pinned D2Q9 oracle
  run (walls, force, random fields) to rounding;
* a shear wave along z decays at nu k^2 (Eq. 5), and the update commutes with the cyclic
  rotation x -> y -> z of the lattice (all three axes alike);
* mass conservation with walls; momentum gain t g M under a force.
"""
import itertools
import math

import numpy as np
import pytest

import synthetic


@pytest.fixture(scope="module")
def lat3(oracle_mod):
    cx, cy, cz, w, opp = oracle_mod.constants3()
    return np.stack([cx, cy, cz]), w, opp


def test_lattice_tensors(lat3):
    c, w, opp = lat3
    assert c.shape == (3, 19) and abs(w.sum() - 1.0) < 1e-15
    assert len({tuple(v) for v in c.T}) == 19
    for i in range(19):
        assert np.array_equal(c[:, opp[i]], -c[:, i])
    d = np.eye(3)
    for a in range(3):
        assert abs((w * c[a]).sum()) < 1e-16
        for b in range(3):
            assert abs((w * c[a] * c[b]).sum() - d[a, b] / 3.0) < 1e-15
            for e in range(3):
                assert abs((w * c[a] * c[b] * c[e]).sum()) < 1e-16
                for g in range(3):
                    t4 = (w * c[a] * c[b] * c[e] * c[g]).sum()
                    iso = (d[a, b] * d[e, g] + d[a, e] * d[b, g] + d[a, g] * d[b, e]) / 9.0
                    assert abs(t4 - iso) < 1e-15


def test_equilibrium_and_forcing_moments(oracle_mod, lat3):
    c, w, _ = lat3
    rho, u = 1.03, np.array([0.04, -0.02, 0.03])
    feq = oracle_mod.equilibrium3(rho, *u)
    assert abs(feq.sum() - rho) < 1e-15
    assert np.abs(c @ feq - rho * u).max() < 1e-16
    P = np.einsum("ai,bi,i->ab", c, c, feq)
    assert np.abs(P - rho * (np.outer(u, u) + np.eye(3) / 3.0)).max() < 1e-15
    F = np.array([1e-3, -2e-3, 5e-4])
    S = oracle_mod.guo_source3(u, F)
    assert abs(S.sum()) < 1e-17
    assert np.abs(c @ S - F).max() < 1e-17


def test_collision_conserves_mass_and_adds_force(oracle_mod, lat3):
    c, w, _ = lat3
    rng = np.random.default_rng(3)
    g = (1e-3, -5e-4, 2e-4)
    for _ in range(10):
        f = oracle_mod.equilibrium3(1.0, 0.03, 0.01, -0.02) * (1 + 0.02 * rng.standard_normal(19))
        out = oracle_mod.collide3(f, 1.0 / (0.5 + rng.random()), g)
        rho = f.sum()
        assert abs(out.sum() - rho) < 1e-15
        assert np.abs(c @ out - c @ f - rho * np.array(g)).max() < 1e-16


def test_z_invariant_projection_is_d2q9(oracle_mod, lat3):
    """Walls, a random solid mask, body force, random initial fields; 4 z-layers; 60 steps."""
    c, _, _ = lat3
    nx, ny, nz = 24, 16, 4
    m2 = synthetic.random_mask(nx, ny, seed=8, solid_fraction=0.15)
    m2[0, :] = 1
    m2[ny - 1, :] = 1
    rho, ux, uy = synthetic.random_fields(nx, ny, seed=2, rho_spread=0.03, u_amp=0.03)
    g = (2e-4, -1e-4)
    f2 = oracle_mod.run(m2, oracle_mod.init(m2, rho, ux, uy), 0.7, 60, g=g)
    rep = lambda a: np.repeat(a[None], nz, axis=0)
    m3 = rep(m2)
    f3 = oracle_mod.init3(m3, rep(rho), rep(ux), rep(uy), None)
    f3 = oracle_mod.run3(m3, f3, 0.7, 60, g=(g[0], g[1], 0.0))
    cx2, cy2, _, _ = oracle_mod.constants()
    for k in range(9):
        group = [i for i in range(19) if c[0, i] == cx2[k] and c[1, i] == cy2[k]]
        proj = f3[group].sum(axis=0)
        for z in range(nz):
            assert np.abs(proj[z] - f2[k]).max() < 1e-14


def test_shear_wave_along_z(oracle_mod):
    nx, ny, nz, tau, u0 = 2, 2, 48, 0.75, 1e-4
    k = 2 * math.pi / nz
    m = np.zeros((nz, ny, nx), np.uint8)
    z = np.arange(nz)[:, None, None] * np.ones((1, ny, nx))
    f = oracle_mod.init3(m, None, u0 * np.sin(k * z), None, None)
    amp = []
    for t in (100, 600):
        ft = oracle_mod.run3(m, f, tau, t)
        _, ux, _, _ = oracle_mod.macroscopic3(m, ft)
        amp.append((ux[:, 0, 0] * np.sin(k * np.arange(nz))).sum() * 2 / nz)
    rate = -math.log(amp[1] / amp[0]) / 500.0
    nu = (tau - 0.5) / 3.0
    assert abs(rate / (nu * k * k) - 1.0) < 2e-3


def test_cyclic_rotation_symmetry(oracle_mod, lat3):
    """Rotating the lattice x -> y -> z -> x (arrays [z, y, x] -> [y, x, z], velocity components
    permuted) commutes with 10 steps with walls and a force."""
    c, _, _ = lat3
    rng = np.random.default_rng(5)
    nx, ny, nz = 6, 5, 7
    m = (rng.random((nz, ny, nx)) < 0.15).astype(np.uint8)
    f = oracle_mod.init3(m, 1 + 0.02 * rng.random((nz, ny, nx)), 0.02 * rng.random((nz, ny, nx)),
                         -0.01 * rng.random((nz, ny, nx)), 0.015 * rng.random((nz, ny, nx)))
    g = (1e-3, 2e-4, -3e-4)
    a = oracle_mod.run3(m, f, 0.8, 10, g=g)
    # rotated lattice: new coordinates (x', y', z') = (z, x, y), velocity (c_z, c_x, c_y)
    perm = [int(np.flatnonzero((c[0] == c[2, i]) & (c[1] == c[0, i]) & (c[2] == c[1, i]))[0])
            for i in range(19)]
    rot = lambda arr: np.transpose(arr, (1, 2, 0))  # [z, y, x] -> [y, x, z] = [z', y', x']
    fr = np.zeros((19,) + rot(m).shape)
    for i in range(19):
        fr[perm[i]] = rot(f[i])
    b = oracle_mod.run3(rot(m), fr, 0.8, 10, g=(g[2], g[0], g[1]))
    for i in range(19):
        assert np.abs(b[perm[i]] - rot(a[i])).max() < 1e-15


def test_mass_and_momentum(oracle_mod, lat3):
    c, _, _ = lat3
    rng = np.random.default_rng(6)
    nx, ny, nz = 8, 6, 5
    m = (rng.random((nz, ny, nx)) < 0.2).astype(np.uint8)
    f = oracle_mod.init3(m, 1 + 0.05 * rng.random((nz, ny, nx)))
    M0 = f.sum()
    f1 = oracle_mod.run3(m, f, 0.7, 200, g=(1e-4, 0.0, -1e-4))
    assert abs(f1.sum() - M0) < 1e-12 * M0
    mp = np.zeros((nz, ny, nx), np.uint8)
    fp = oracle_mod.init3(mp, 1 + 0.05 * rng.random((nz, ny, nx)))
    g = np.array([1e-4, -2e-4, 3e-4])
    T = 50
    P0 = np.einsum("ai,izyx->a", c, fp)
    P1 = np.einsum("ai,izyx->a", c, oracle_mod.run3(mp, fp, 0.9, T, g=tuple(g)))
    assert np.abs(P1 - P0 - T * g * fp.sum()).max() < 1e-12 * fp.sum()


# ------------------------------------------------------- two-relaxation-time --
def _random_f3(oracle_mod, rng):
    return oracle_mod.equilibrium3(1.0, 0.03, -0.02, 0.01) * (1 + 0.03 * rng.standard_normal(19))


def test_trt3_reduces_to_bgk(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(10):
        f = _random_f3(oracle_mod, rng)
        om = 1.0 / (0.5 + rng.random())
        g = tuple(1e-3 * rng.standard_normal(3))
        assert np.abs(oracle_mod.collide3_trt(f, om, om, g) - oracle_mod.collide3(f, om, g)).max() < 1e-16


def test_trt3_conservation_and_force(oracle_mod, lat3):
    c, _, _ = lat3
    rng = np.random.default_rng(12)
    g = np.array([2e-3, -1e-3, 5e-4])
    for _ in range(10):
        f = _random_f3(oracle_mod, rng)
        op, om = 1.0 / (0.5 + rng.random()), 1.0 / (0.5 + rng.random())
        out = oracle_mod.collide3_trt(f, op, om, tuple(g))
        rho = f.sum()
        assert abs(out.sum() - rho) < 1e-15
        assert np.abs(c @ out - c @ f - rho * g).max() < 1e-16


@pytest.mark.parametrize("tau_m", [0.55, 0.8, 1.7])
def test_trt3_viscosity_from_tau_plus(oracle_mod, tau_m):
    """Shear wave u_x = u0 sin(k z): decay exp(-nu k^2 t), nu = (tau+ - 1/2)/3, any tau-, up
    to the O(k^2) dispersion term, whose coefficient depends on Lambda (2-D pin: same k)."""
    nx, ny, nz, tau, u0 = 2, 2, 64, 0.8, 1e-4
    k = 2 * math.pi / nz
    m = np.zeros((nz, ny, nx), np.uint8)
    z = np.arange(nz)[:, None, None] * np.ones((1, ny, nx))
    f = oracle_mod.init3(m, None, u0 * np.sin(k * z), None, None)
    amp = []
    for t in (200, 1200):
        ft = oracle_mod.run3(m, f, tau, t, tau_minus=tau_m)
        _, ux, _, _ = oracle_mod.macroscopic3(m, ft)
        amp.append((ux[:, 0, 0] * np.sin(k * np.arange(nz))).sum() * 2 / nz)
    rate = -math.log(amp[1] / amp[0]) / 1000.0
    nu = (tau - 0.5) / 3.0
    assert abs(rate / (nu * k * k) - 1.0) < 2e-3


@pytest.mark.parametrize("magic", [3.0 / 16.0, 0.25, 1.0 / 12.0])
def test_trt3_steady_channel_closed_form(oracle_mod, magic):
    """Walls at z = 0 and nz - 1, force along x: the exact TRT halfway-bounce-back profile
    u(z) = (g/2nu)(z - 1/2)(H + 1/2 - z) + (g/nu)(16 Lambda - 3)/24, H = nz - 2."""
    nx, ny, nz, tau, g = 2, 2, 14, 0.9, 1e-5
    H = nz - 2
    m = np.zeros((nz, ny, nx), np.uint8)
    m[0] = 1
    m[nz - 1] = 1
    tau_m = oracle_mod.trt_tau_minus(tau, magic)
    f = oracle_mod.run3(m, oracle_mod.init3(m), tau, 30000, g=(g, 0.0, 0.0), tau_minus=tau_m)
    _, ux, uy, uz = oracle_mod.macroscopic3(m, f, g=(g, 0.0, 0.0))
    nu = (tau - 0.5) / 3.0
    zz = np.arange(1, nz - 1)
    exact = g / (2 * nu) * (zz - 0.5) * (H + 0.5 - zz) + g / nu * (16 * magic - 3) / 24
    assert np.abs(ux[1:nz - 1, 0, 0] - exact).max() < 1e-10 * exact.max()
    assert max(np.abs(uy[1:nz - 1]).max(), np.abs(uz[1:nz - 1]).max()) < 1e-12 * exact.max()


def test_trt3_z_invariant_projection_is_d2q9(oracle_mod, lat3):
    """As the BGK projection pin, with the two-relaxation-time collision on both sides."""
    c, _, _ = lat3
    nx, ny, nz = 20, 14, 3
    m2 = synthetic.random_mask(nx, ny, seed=9, solid_fraction=0.15)
    m2[0, :] = 1
    m2[ny - 1, :] = 1
    rho, ux, uy = synthetic.random_fields(nx, ny, seed=4, rho_spread=0.03, u_amp=0.03)
    g = (2e-4, -1e-4)
    tm = 1.3
    f2 = oracle_mod.run(m2, oracle_mod.init(m2, rho, ux, uy), 0.7, 40, g=g, tau_minus=tm)
    rep = lambda a: np.repeat(a[None], nz, axis=0)
    m3 = rep(m2)
    f3 = oracle_mod.init3(m3, rep(rho), rep(ux), rep(uy), None)
    f3 = oracle_mod.run3(m3, f3, 0.7, 40, g=(g[0], g[1], 0.0), tau_minus=tm)
    cx2, cy2, _, _ = oracle_mod.constants()
    for k in range(9):
        group = [i for i in range(19) if c[0, i] == cx2[k] and c[1, i] == cy2[k]]
        proj = f3[group].sum(axis=0)
        for z in range(nz):
            assert np.abs(proj[z] - f2[k]).max() < 1e-14
