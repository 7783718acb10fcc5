"""Pins of the D3Q19 oracle's multiple-relaxation-time collision (moment basis of d'Humieres,
Ginzburg, Krafczyk, Lallemand and Luo), against what does not depend on the oracle's own
arithmetic:

* the moment matrix has orthogonal rows with the published squared norms 19, 2394, 252, 10, 40,
  10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8, and maps the (pinned) equilibrium of Eq. 6 to
  the published closed-form equilibrium moments (e = rho(-11 + 19u.u), eps = rho(3 - 11/2 u.u),
  q = -2/3 rho u, 3p_xx = rho(3u_x^2 - u.u), 3pi_xx = -3p_xx / 2, p_ww = rho(u_y^2 - u_z^2),
  pi_ww = -p_ww / 2, p_ab = rho u_a u_b, m = 0);
* all rates omega is the (pinned) D3Q19 BGK collision; omega+ on the even moments and omega- on
  the odd ones is the (pinned) D3Q19 TRT collision;
* mass is conserved and the momentum gain is the force density for any rates; the rates of the
  conserved moments do not matter;
* each non-conserved moment relaxes alone, by the factor 1 - s_k;
* the viscosity depends on the shear rate alone, for an off-diagonal shear wave (along z) and
  for a normal-stress-difference wave (along x + y, the 3p_xx and p_ww moments);
* steady channel flow between walls in z is exactly the TRT closed form with
  Lambda = (1/omega - 1/2)(1/s_q - 1/2) when s_e = omega and s_m = s_q (any s_eps, s_pi); a
  different s_m moves the wall (a first-order change of the slip), a different s_e adds a
  second-order deviation.
"""
import math

import numpy as np
import pytest

NORMS = [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
EVEN = [0, 1, 2, 9, 10, 11, 12, 13, 14, 15]
ODD = [3, 4, 5, 6, 7, 8, 16, 17, 18]


def _random_f(oracle_mod, rng):
    u = 0.05 * rng.random(3) - 0.025
    return oracle_mod.equilibrium3(1.0 + 0.05 * rng.random(), *u) * \
        (1.0 + 0.02 * rng.standard_normal(19))


def _rates(rng):
    return 1.0 / (0.5 + rng.random(19))


def test_matrix_and_equilibrium_moments(oracle_mod):
    cx, cy, cz, _, _ = oracle_mod.constants3()
    M = oracle_mod.mrt_matrix3()
    assert np.array_equal(M @ M.T, np.diag(np.array(NORMS, dtype=float)))
    assert np.array_equal(M[0], np.ones(19))
    assert np.array_equal(M[3], cx) and np.array_equal(M[5], cy) and np.array_equal(M[7], cz)
    assert np.array_equal(M[13], cx * cy) and np.array_equal(M[14], cy * cz)
    assert np.array_equal(M[15], cx * cz)
    rng = np.random.default_rng(7)
    for _ in range(10):
        rho = 1.0 + 0.1 * rng.random()
        ux, uy, uz = 0.1 * rng.random(3) - 0.05
        uu = ux * ux + uy * uy + uz * uz
        p, w = 3 * ux * ux - uu, uy * uy - uz * uz
        closed = [rho, rho * (-11 + 19 * uu), rho * (3 - 5.5 * uu), rho * ux, -2 / 3 * rho * ux,
                  rho * uy, -2 / 3 * rho * uy, rho * uz, -2 / 3 * rho * uz, rho * p,
                  -0.5 * rho * p, rho * w, -0.5 * rho * w, rho * ux * uy, rho * uy * uz,
                  rho * ux * uz, 0.0, 0.0, 0.0]
        got = M @ oracle_mod.equilibrium3(rho, ux, uy, uz)
        assert np.abs(got - closed).max() < 1e-14


@pytest.mark.parametrize("g", [(0.0, 0.0, 0.0), (1e-3, -2e-4, 5e-4)])
def test_reduces_to_bgk_and_trt(oracle_mod, g):
    rng = np.random.default_rng(8)
    for _ in range(10):
        f = _random_f(oracle_mod, rng)
        op, om = 1.0 / (0.5 + rng.random()), 1.0 / (0.5 + rng.random())
        bgk = oracle_mod.collide3_mrt(f, [op] * 19, g)
        assert np.abs(bgk - oracle_mod.collide3(f, op, g)).max() < 1e-15
        r = np.zeros(19)
        r[EVEN], r[ODD] = op, om
        trt = oracle_mod.collide3_mrt(f, r, g)
        assert np.abs(trt - oracle_mod.collide3_trt(f, op, om, g)).max() < 1e-15


def test_conservation_force_and_conserved_rates(oracle_mod):
    cx, cy, cz, _, _ = oracle_mod.constants3()
    rng = np.random.default_rng(9)
    g = (2e-3, -1e-3, 5e-4)
    for _ in range(10):
        f = _random_f(oracle_mod, rng)
        r = _rates(rng)
        out = oracle_mod.collide3_mrt(f, r, g)
        rho = f.sum()
        assert abs(out.sum() - rho) < 1e-15
        for c, gc in zip((cx, cy, cz), g):
            assert abs((c * out).sum() - (c * f).sum() - rho * gc) < 1e-15
        r2 = r.copy()
        r2[[0, 3, 5, 7]] = rng.random(4) * 1.9 + 0.05
        assert np.abs(oracle_mod.collide3_mrt(f, r2, g) - out).max() < 1e-15


@pytest.mark.parametrize("k", [1, 2, 4, 8, 9, 10, 12, 14, 16, 18])
def test_single_moment_relaxes_alone(oracle_mod, k):
    M = oracle_mod.mrt_matrix3()
    Minv = np.linalg.inv(M)
    rng = np.random.default_rng(20 + k)
    feq = oracle_mod.equilibrium3(1.02, 0.02, -0.01, 0.015)
    delta = 1e-3
    f = feq + delta * Minv[:, k]
    r = _rates(rng)
    out = oracle_mod.collide3_mrt(f, r)
    dm = M @ (out - feq)
    expect = np.zeros(19)
    expect[k] = (1 - r[k]) * delta
    assert np.abs(dm - expect).max() < 1e-14


@pytest.mark.parametrize("r5", [(1.2, 1.4, 1.6, 1.3, 1.1), (0.9, 1.8, 1.2, 1.7, 1.5)])
def test_viscosity_from_shear_rate(oracle_mod, r5):
    """Shear wave u_x = u0 sin(k z) on a periodic 2 x 2 x 64 lattice, tau = 0.8: decay at
    nu k^2, nu = (tau - 1/2) / 3, whatever the other rates."""
    nx, ny, nz, tau, u0 = 2, 2, 64, 0.8, 1e-4
    k = 2 * math.pi / nz
    m = np.zeros((nz, ny, nx), np.uint8)
    z = np.arange(nz)[:, None, None] * np.ones((1, ny, nx))
    f = oracle_mod.init3(m, None, u0 * np.sin(k * z), None, None)
    amp = []
    for t in (200, 1200):
        ft = oracle_mod.run3(m, f, tau, t, mrt=r5)
        _, ux, _, _ = oracle_mod.macroscopic3(m, ft)
        amp.append((ux[:, 0, 0] * np.sin(k * np.arange(nz))).sum() * 2 / nz)
    rate = -math.log(amp[1] / amp[0]) / 1000.0
    nu = (tau - 0.5) / 3.0
    assert abs(rate / (nu * k * k) - 1.0) < 2e-3


@pytest.mark.parametrize("r5", [(1.2, 1.4, 1.6, 1.3, 1.1), (1.7, 0.9, 1.3, 1.5, 1.8)])
def test_viscosity_normal_stress_mode(oracle_mod, r5):
    """Shear wave u = u0 (1, -1, 0) sin(k (x + y)) on a periodic 32 x 32 x 2 lattice: its
    strain is a pure normal-stress difference (the 3p_xx and p_ww moments, not p_xy), and it
    decays at nu |k|^2 with the same nu, whatever the other rates."""
    n, tau, u0 = 32, 0.8, 1e-4
    k = 2 * math.pi / n
    m = np.zeros((2, n, n), np.uint8)
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ph = np.sin(k * (x + y))
    ux = np.broadcast_to(u0 * ph, (2, n, n)).copy()
    f = oracle_mod.init3(m, None, ux, -ux, None)
    amp = []
    for t in (100, 600):
        ft = oracle_mod.run3(m, f, tau, t, mrt=r5)
        _, uxt, _, _ = oracle_mod.macroscopic3(m, ft)
        amp.append((uxt[0] * ph).sum() * 2 / (n * n))
    rate = -math.log(amp[1] / amp[0]) / 500.0
    nu = (tau - 0.5) / 3.0
    assert abs(rate / (nu * 2 * k * k) - 1.0) < 3e-3


def _channel(oracle_mod, r5, magic, g=1e-5):
    nx, ny, nz, tau = 2, 2, 14, 0.9
    H = nz - 2
    m = np.zeros((nz, ny, nx), np.uint8)
    m[0] = 1
    m[nz - 1] = 1
    f = oracle_mod.run3(m, oracle_mod.init3(m), tau, 20000, g=(g, 0.0, 0.0), mrt=r5)
    _, ux, _, uz = oracle_mod.macroscopic3(m, f, g=(g, 0.0, 0.0))
    nu = (tau - 0.5) / 3.0
    zz = np.arange(1, nz - 1)
    exact = g / (2 * nu) * (zz - 0.5) * (H + 0.5 - zz) + g / nu * (16 * magic - 3) / 24
    return ux[1:nz - 1, 0, 0], uz, exact


@pytest.mark.parametrize("magic,seps,spi", [(3.0 / 16.0, 1.3, 1.2), (0.25, 1.9, 0.7)])
def test_steady_channel_closed_form(oracle_mod, magic, seps, spi):
    tau = 0.9
    sq = 1.0 / oracle_mod.trt_tau_minus(tau, magic)
    got, uz, exact = _channel(oracle_mod, (1.0 / tau, seps, sq, spi, sq), magic)
    assert np.abs(got - exact).max() < 1e-10 * exact.max()
    assert np.abs(uz).max() < 1e-10 * exact.max()
    # another rate of the m moments moves the wall: a first-order change
    got2, _, _ = _channel(oracle_mod, (1.0 / tau, seps, sq, spi, 1.5), magic)
    assert np.abs(got2 - exact).max() > 1e-3 * exact.max()
