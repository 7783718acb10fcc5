"""Pins of the oracle's multiple-relaxation-time collision (a richer collision model, which
the paper plans as future work; moment basis of Lallemand and Luo), against what does not depend
on the oracle's own arithmetic:

* the moment matrix has orthogonal rows with norms 9, 36, 36, 6, 12, 6, 12, 4, 4, its rows rho,
  j and p are the plain velocity monomials, and it maps the (pinned) equilibrium of Eq. 6 to the
  closed-form equilibrium moments rho, rho(-2 + 3u.u), rho(1 - 3u.u), rho u_x, -rho u_x,
  rho u_y, -rho u_y, rho(u_x^2 - u_y^2), rho u_x u_y;
* all rates equal to omega is the (pinned) BGK collision; omega+ on the even moments and
  omega- on the odd ones is the (pinned) TRT collision;
* mass is conserved and the momentum gain is the force density, for any rates; the rates of
  the conserved moments do not change the result;
* each non-conserved moment relaxes on its own: a state off equilibrium in one moment only
  stays off in that moment alone, by the factor 1 - s_k;
* the viscosity depends on the shear rate alone (a shear wave decays at nu k^2 whatever the
  other rates);
* steady channel flow between halfway bounce-back walls is exactly the TRT closed form with
  Lambda = (1/s_nu - 1/2)(1/s_q - 1/2) when the energy rate s_e equals the shear rate (any
  s_eps); another s_e adds a deviation of second order in the Mach number (relative
  deviation proportional to g^2, with a density variation of the same order).
"""
import math

import numpy as np
import pytest

import synthetic

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
EVEN = [0, 1, 2, 7, 8]   # rho, e, eps, p_xx, p_xy
ODD = [3, 4, 5, 6]       # j_x, q_x, j_y, q_y


def _random_f(oracle_mod, rng):
    return oracle_mod.equilibrium(1.0 + 0.05 * rng.random(), 0.05 * rng.random(),
                                  -0.04 * rng.random()) * (1.0 + 0.02 * rng.standard_normal(9))


def _rates(rng):
    return 1.0 / (0.5 + rng.random(9))


def test_matrix_structure_and_equilibrium_moments(oracle_mod):
    M = oracle_mod.mrt_matrix()
    G = M @ M.T
    assert np.array_equal(G, np.diag([9.0, 36, 36, 6, 12, 6, 12, 4, 4]))
    assert np.array_equal(M[0], np.ones(9))
    assert np.array_equal(M[3], CX) and np.array_equal(M[5], CY)
    assert np.array_equal(M[7], CX * CX - CY * CY) and np.array_equal(M[8], CX * CY)
    rng = np.random.default_rng(3)
    for _ in range(10):
        rho, ux, uy = 1.0 + 0.1 * rng.random(), 0.1 * rng.random() - 0.05, 0.1 * rng.random()
        uu = ux * ux + uy * uy
        closed = [rho, rho * (-2 + 3 * uu), rho * (1 - 3 * uu), rho * ux, -rho * ux, rho * uy,
                  -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy]
        assert np.abs(M @ oracle_mod.equilibrium(rho, ux, uy) - closed).max() < 1e-15


@pytest.mark.parametrize("alpha,g", [(0.0, (0.0, 0.0)), (0.3, (1e-3, -2e-4))])
def test_reduces_to_bgk_and_trt(oracle_mod, alpha, g):
    rng = np.random.default_rng(4)
    for _ in range(10):
        f = _random_f(oracle_mod, rng)
        op, om = 1.0 / (0.5 + rng.random()), 1.0 / (0.5 + rng.random())
        bgk = oracle_mod.collide_mrt(f, [op] * 9, alpha, g)
        assert np.abs(bgk - oracle_mod.collide(f, op, alpha, g)).max() < 1e-15
        r = np.zeros(9)
        r[EVEN], r[ODD] = op, om
        trt = oracle_mod.collide_mrt(f, r, alpha, g)
        assert np.abs(trt - oracle_mod.collide_trt(f, op, om, alpha, g)).max() < 1e-15


@pytest.mark.parametrize("alpha", [0.0, 0.4])
def test_conservation_force_and_conserved_rates(oracle_mod, alpha):
    rng = np.random.default_rng(5)
    g = (2e-3, -1e-3)
    for _ in range(10):
        f = _random_f(oracle_mod, rng)
        r = _rates(rng)
        out = oracle_mod.collide_mrt(f, r, alpha, g)
        rho, ux, uy = oracle_mod.node_velocity(f, alpha, g)
        assert abs(out.sum() - f.sum()) < 1e-15
        Fx, Fy = rho * (g[0] - alpha * ux), rho * (g[1] - alpha * uy)
        assert abs((CX * out).sum() - (CX * f).sum() - Fx) < 1e-15
        assert abs((CY * out).sum() - (CY * f).sum() - Fy) < 1e-15
        r2 = r.copy()
        r2[[0, 3, 5]] = rng.random(3) * 1.9 + 0.05
        assert np.abs(oracle_mod.collide_mrt(f, r2, alpha, g) - out).max() < 1e-15


@pytest.mark.parametrize("k", [1, 2, 4, 6, 7, 8])
def test_single_moment_relaxes_alone(oracle_mod, k):
    """f = f^eq + delta M^-1 e_k (no force): after the collision the moments differ from those
    of f^eq in row k only, by (1 - s_k) delta.  M^-1 from numpy's general inverse."""
    M = oracle_mod.mrt_matrix()
    Minv = np.linalg.inv(M)
    rng = np.random.default_rng(10 + k)
    feq = oracle_mod.equilibrium(1.03, 0.02, -0.01)
    delta = 1e-3
    f = feq + delta * Minv[:, k]
    rho, ux, uy = oracle_mod.node_velocity(f)
    assert abs(rho - 1.03) < 1e-15  # row k is neither rho nor j: same moments of Eq. 2
    r = _rates(rng)
    out = oracle_mod.collide_mrt(f, r)
    dm = M @ (out - feq)
    expect = np.zeros(9)
    expect[k] = (1 - r[k]) * delta
    assert np.abs(dm - expect).max() < 1e-15


@pytest.mark.parametrize("rates", [(1.1, 1.4, 1.7), (0.6, 1.9, 0.9)])
def test_viscosity_from_shear_rate(oracle_mod, rates):
    """Shear wave u_x = u0 sin(k y) on a periodic 4 x 64 lattice, tau = 0.8: the amplitude
    decays as exp(-nu k^2 t) with nu = (tau - 1/2) / 3, whatever s_e, s_eps, s_q."""
    nx, ny, tau, u0 = 4, 64, 0.8, 1e-4
    k = 2 * math.pi / ny
    m = synthetic.all_fluid(nx, ny)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    f = oracle_mod.init(m, None, u0 * np.sin(k * y), None)
    amp = []
    for t in (200, 1200):
        ft = oracle_mod.run(m, f, tau, t, mrt=rates)
        _, ux, _ = oracle_mod.macroscopic(m, ft)
        amp.append((ux[:, 0] * np.sin(k * np.arange(ny))).sum() * 2 / ny)
    rate = -math.log(amp[1] / amp[0]) / 1000.0
    nu = (tau - 0.5) / 3.0
    assert abs(rate / (nu * k * k) - 1.0) < 2e-3


def _channel(oracle_mod, magic, se, seps, g):
    nx, ny, tau = 4, 14, 0.9
    H = ny - 2
    sq = 1.0 / oracle_mod.trt_tau_minus(tau, magic)
    m = synthetic.channel_mask(nx, ny)
    f = oracle_mod.run(m, oracle_mod.init(m), tau, 30000, g=(g, 0.0), mrt=(se, seps, sq))
    _, ux, uy = oracle_mod.macroscopic(m, f, g=(g, 0.0))
    nu = (tau - 0.5) / 3.0
    y = np.arange(1, ny - 1)
    exact = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y) + g / nu * (16 * magic - 3) / 24
    return ux[1:ny - 1, 0], uy[1:ny - 1], exact


@pytest.mark.parametrize("magic,seps", [(3.0 / 16.0, 1.5), (0.25, 1.95), (1.0 / 12.0, 0.6)])
def test_steady_channel_closed_form(oracle_mod, magic, seps):
    got, uy, exact = _channel(oracle_mod, magic, 1.0 / 0.9, seps, 1e-5)
    assert np.abs(got - exact).max() < 1e-10 * exact.max()
    assert np.abs(uy).max() < 1e-10 * exact.max()  # zero up to the rounding of the moment sums


def test_steady_channel_energy_rate_is_second_order(oracle_mod):
    dev = []
    for g in (1e-5, 2e-5):
        got, uy, exact = _channel(oracle_mod, 3.0 / 16.0, 1.3, 1.5, g)
        dev.append(np.abs(got - exact).max() / exact.max())
        assert dev[-1] < 0.01 * exact.max() ** 2
        assert np.abs(uy).max() < 1e-10 * exact.max()
    assert abs(dev[1] / dev[0] - 4.0) < 0.1
