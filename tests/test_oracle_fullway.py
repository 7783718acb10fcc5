"""Pins of the oracle's full-way bounce-back rule (wall nodes that hold populations, reverse them
instead of colliding, and stream them back), each against something other than its own code:

* brute force in another formulation: halfway bounce-back with a one-step delay line, i.e.
  f_i(x, t+1) = p_opp(i)(x, t-1) on a wall link (p = post-collision, node by node from the
  pinned collision), seeded from the wall slots; tiny random lattices, force, 8 steps, and
  isolated fluid nodes (all 8 neighbours solid);
* mass, counted over fluid and wall slots, is conserved with random solids, force and drag;
* at steady state the two rules coincide: the body-force channel reaches the closed-form BGK
  profile u(y) = (g/2nu)(y - 1/2)(H + 1/2 - y) + (g/nu)(16 (tau - 1/2)^2 - 3)/24;
* without solids the full-way run is the halfway run;
* the initial wall slots hold f_i of the fluid source node w - c_i and 0 elsewhere.
"""
import numpy as np
import pytest

import synthetic


def _isolated_mask(nx, ny):
    """Fluid at even (x, y), solid elsewhere: every fluid node's 8 neighbours are solid."""
    m = np.ones((ny, nx), np.uint8)
    m[0::2, 0::2] = 0
    return m


def _random_state(oracle_mod, m, seed):
    _, _, w, _ = oracle_mod.constants()
    rng = np.random.default_rng(seed)
    f = w[:, None, None] * (1.0 + 0.2 * (2 * rng.random((9,) + m.shape) - 1))
    return f * (m == 0)


def _delay_line(oracle_mod, m, f0, tau, steps, g):
    """Full-way bounce-back as halfway bounce-back whose bounced value is one step late:
    f_i(x, t+1) = p_i(x - c_i, t) from a fluid source, else p_opp(i)(x, t-1), with
    p_opp(i)(x, -1) = the wall slot opp(i) of the wall node x - c_i at t = 0.  Returns the
    fluid populations and the wall slots f_i(w, t) = p_i(w - c_i, t - 1) after each step."""
    cx, cy, _, opp = oracle_mod.constants()
    ny, nx = m.shape
    fluid = [(x, y) for y in range(ny) for x in range(nx) if m[y, x] == 0]
    cur = {q: f0[:, q[1], q[0]].copy() for q in fluid}
    prev = {}
    for (x, y) in fluid:
        p = np.zeros(9)
        for i in range(9):
            xs, ys = (x - cx[i]) % nx, (y - cy[i]) % ny
            if m[ys, xs]:
                p[opp[i]] = f0[opp[i], ys, xs]
        prev[(x, y)] = p
    out = []
    for _ in range(steps):
        post = {q: oracle_mod.collide(cur[q], 1.0 / tau, 0.0, g) for q in fluid}
        new = {}
        for (x, y) in fluid:
            v = np.zeros(9)
            for i in range(9):
                xs, ys = (x - cx[i]) % nx, (y - cy[i]) % ny
                v[i] = post[(xs, ys)][i] if m[ys, xs] == 0 else prev[(x, y)][opp[i]]
            new[(x, y)] = v
        walls = np.zeros((9, ny, nx))
        for y in range(ny):
            for x in range(nx):
                if m[y, x]:
                    for i in range(9):
                        xs, ys = (x - cx[i]) % nx, (y - cy[i]) % ny
                        if m[ys, xs] == 0:
                            walls[i, y, x] = post[(xs, ys)][i]
        prev, cur = post, new
        fl = np.zeros((9, ny, nx))
        for (x, y), v in cur.items():
            fl[:, y, x] = v
        out.append(fl + walls)
    return out


@pytest.mark.parametrize("case", ["random", "isolated"])
def test_delay_line_brute_force(oracle_mod, case):
    if case == "random":
        m = synthetic.random_mask(7, 6, seed=11, solid_fraction=0.35)
    else:
        m = _isolated_mask(6, 4)
    f0 = _random_state(oracle_mod, m, seed=1)
    rng = np.random.default_rng(2)
    fw = oracle_mod.fullway_fill(m, f0)
    # perturb the wall slots that carry values, so that the seed of the delay line matters
    fw += (fw != 0) * (m == 1) * 0.01 * rng.random(fw.shape)
    g = (2e-3, -1e-3)
    ref = _delay_line(oracle_mod, m, fw, 0.8, 8, g)
    for t in range(1, 9):
        got = oracle_mod.run(m, fw, 0.8, t, g=g, fullway=True)
        assert np.array_equal(got, ref[t - 1]), t


def test_mass_conserved_with_wall_slots(oracle_mod):
    m = synthetic.random_mask(40, 30, seed=5, solid_fraction=0.2, walls=True)
    rho, ux, uy = synthetic.random_fields(40, 30, seed=6, rho_spread=0.03, u_amp=0.03)
    f = oracle_mod.fullway_fill(m, oracle_mod.init(m, rho, ux, uy))
    alpha = synthetic.brinkman_alpha(40, 30, seed=2, sigma=3.0).astype(np.float64)
    M0 = f.sum()
    f1 = oracle_mod.run(m, f, 0.8, 400, g=(1e-4, -5e-5), alpha=alpha, fullway=True)
    assert abs(f1.sum() - M0) < 1e-12 * M0
    # the halfway rule applied to the same state loses the in-flight wall mass at once
    fluid_mass = f[:, m == 0].sum()
    assert f1.sum() > fluid_mass


def test_steady_channel_closed_form(oracle_mod):
    nx, ny, tau, g = 4, 14, 0.9, 1e-5
    H = ny - 2
    m = synthetic.channel_mask(nx, ny)
    f = oracle_mod.fullway_fill(m, oracle_mod.init(m))
    f = oracle_mod.run(m, f, tau, 30000, g=(g, 0.0), fullway=True)
    _, ux, uy = oracle_mod.macroscopic(m, f, g=(g, 0.0))
    nu = (tau - 0.5) / 3.0
    y = np.arange(1, ny - 1)
    exact = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y) + g / nu * (16 * (tau - 0.5) ** 2 - 3) / 24
    assert np.abs(ux[1:ny - 1, 0] - exact).max() < 1e-10 * exact.max()
    assert np.abs(uy[1:ny - 1]).max() < 1e-12 * exact.max()


def test_transient_differs_from_halfway(oracle_mod):
    """Same channel from rest: the two rules give different transients (the wall delay)."""
    m = synthetic.channel_mask(4, 14)
    f0 = oracle_mod.init(m)
    half = oracle_mod.run(m, f0, 0.9, 50, g=(1e-5, 0.0))
    full = oracle_mod.run(m, oracle_mod.fullway_fill(m, f0), 0.9, 50, g=(1e-5, 0.0), fullway=True)
    fl = m == 0
    assert np.abs(full[:, fl] - half[:, fl]).max() > 1e-9


def test_no_solids_is_halfway(oracle_mod):
    m = synthetic.all_fluid(16, 12)
    rho, ux, uy = synthetic.random_fields(16, 12, seed=3)
    f = oracle_mod.init(m, rho, ux, uy)
    a = oracle_mod.run(m, f, 0.7, 30, g=(1e-4, 0.0))
    b = oracle_mod.run(m, f, 0.7, 30, g=(1e-4, 0.0), fullway=True)
    assert np.array_equal(a, b)


def test_fill_rule(oracle_mod):
    m = synthetic.random_mask(9, 7, seed=8, solid_fraction=0.4)
    cx, cy, _, _ = oracle_mod.constants()
    f = _random_state(oracle_mod, m, seed=4)
    g = oracle_mod.fullway_fill(m, f)
    ny, nx = m.shape
    for y in range(ny):
        for x in range(nx):
            if m[y, x] == 0:
                assert np.array_equal(g[:, y, x], f[:, y, x])
                continue
            for i in range(9):
                xs, ys = (x - cx[i]) % nx, (y - cy[i]) % ny
                exp = f[i, ys, xs] if m[ys, xs] == 0 else 0.0
                # a solid node with no fluid neighbour is not a wall node: all slots stay 0
                assert g[i, y, x] == exp
