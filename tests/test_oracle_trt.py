"""Pins of the oracle's two-relaxation-time collision (a collision model other than the paper's
BGK; the paper names other collision models as future work), against what does not depend on
the oracle's own arithmetic:

* omega- = omega+ is the BGK collision (Eqs. 3-6 with forcing);
* mass is conserved and the momentum gain is exactly the force density, for any omega+-;
* the viscosity depends on tau+ alone (Eq. 5): a shear wave decays at nu k^2 whatever tau-;
* steady channel flow between halfway bounce-back walls is, exactly,
  u(y) = (g / 2nu)(y - 1/2)(H + 1/2 - y) + (g / nu)(16 Lambda - 3) / 24,
  Lambda = (tau+ - 1/2)(tau- - 1/2): the wall slip vanishes for Lambda = 3/16.  (For BGK,
  Lambda = (tau - 1/2)^2, the exact BGK profile pinned in test_oracle_pins.)
"""
import math

import numpy as np
import pytest

import synthetic

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def _random_f(oracle_mod, rng):
    return oracle_mod.equilibrium(1.0 + 0.05 * rng.random(), 0.05 * rng.random(),
                                  -0.04 * rng.random()) * (1.0 + 0.02 * rng.standard_normal(9))


def test_trt_reduces_to_bgk(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(10):
        f = _random_f(oracle_mod, rng)
        om = 1.0 / (0.5 + rng.random())
        a = oracle_mod.collide_trt(f, om, om, 0.3, (1e-3, -2e-4))
        b = oracle_mod.collide(f, om, 0.3, (1e-3, -2e-4))
        assert np.abs(a - b).max() < 1e-15


@pytest.mark.parametrize("alpha", [0.0, 0.4])
def test_trt_conservation_and_force(oracle_mod, alpha):
    rng = np.random.default_rng(2)
    g = (2e-3, -1e-3)
    for _ in range(10):
        f = _random_f(oracle_mod, rng)
        op, om = 1.0 / (0.5 + rng.random()), 1.0 / (0.5 + rng.random())
        out = oracle_mod.collide_trt(f, op, om, alpha, g)
        rho, ux, uy = oracle_mod.node_velocity(f, alpha, g)
        assert abs(out.sum() - f.sum()) < 1e-15
        Fx, Fy = rho * (g[0] - alpha * ux), rho * (g[1] - alpha * uy)
        assert abs((CX * out).sum() - (CX * f).sum() - Fx) < 1e-15
        assert abs((CY * out).sum() - (CY * f).sum() - Fy) < 1e-15


@pytest.mark.parametrize("tau_m", [0.55, 0.8, 1.7])
def test_trt_viscosity_from_tau_plus(oracle_mod, tau_m):
    """Shear wave u_x = u0 sin(k y) on a periodic 4 x 64 lattice, tau+ = 0.8: the amplitude
    decays as exp(-nu k^2 t) with nu = (tau+ - 1/2) / 3, independent of tau-."""
    nx, ny, tau, u0 = 4, 64, 0.8, 1e-4
    k = 2 * math.pi / ny
    m = synthetic.all_fluid(nx, ny)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    f = oracle_mod.init(m, None, u0 * np.sin(k * y), None)
    amp = []
    for t in (200, 1200):
        ft = oracle_mod.run(m, f, tau, t, tau_minus=tau_m)
        _, ux, _ = oracle_mod.macroscopic(m, ft)
        amp.append((ux[:, 0] * np.sin(k * np.arange(ny))).sum() * 2 / ny)
    rate = -math.log(amp[1] / amp[0]) / 1000.0
    nu = (tau - 0.5) / 3.0
    assert abs(rate / (nu * k * k) - 1.0) < 2e-3


@pytest.mark.parametrize("magic", [3.0 / 16.0, 0.25, 1.0 / 12.0])
def test_trt_steady_channel_closed_form(oracle_mod, magic):
    nx, ny, tau, g = 4, 14, 0.9, 1e-5
    H = ny - 2
    tau_m = oracle_mod.trt_tau_minus(tau, magic)
    m = synthetic.channel_mask(nx, ny)
    f = oracle_mod.run(m, oracle_mod.init(m), tau, 30000, g=(g, 0.0), tau_minus=tau_m)
    _, ux, uy = oracle_mod.macroscopic(m, f, g=(g, 0.0))
    nu = (tau - 0.5) / 3.0
    y = np.arange(1, ny - 1)
    exact = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y) + g / nu * (16 * magic - 3) / 24
    got = ux[1:ny - 1, 0]
    assert np.abs(got - exact).max() < 1e-10 * exact.max()
    assert np.abs(uy[1:ny - 1]).max() < 1e-12 * exact.max()
