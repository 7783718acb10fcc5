"""Pins of the D3Q19 oracle's full-way bounce-back rule, each against something other than its
own code:

* brute force in another formulation (halfway bounce-back whose bounced value is one step late,
  node by node from the pinned D3Q19 collision), bit-exact with wall slots, on tiny lattices;
* mass over fluid and wall slots is conserved;
* the steady channel with walls in z reaches the closed-form profile of the halfway rule;
* without solids the full-way run is the halfway run;
* a z-invariant run, summed over c_z, is the pinned D2Q9 full-way run, wall slots included;
* the initial wall-slot rule.
"""
import numpy as np
import pytest

import synthetic


def _random_state3(oracle_mod, m, seed):
    _, _, _, w, _ = oracle_mod.constants3()
    return synthetic.random_populations(w, m.shape, seed=seed, amp=0.2) * (m == 0)


def _delay_line3(oracle_mod, m, f0, tau, steps, g):
    cx, cy, cz, _, opp = oracle_mod.constants3()
    nz, ny, nx = m.shape
    fluid = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx) if m[z, y, x] == 0]
    src = lambda x, y, z, i: ((x - cx[i]) % nx, (y - cy[i]) % ny, (z - cz[i]) % nz)
    cur = {q: f0[:, q[2], q[1], q[0]].copy() for q in fluid}
    prev = {}
    for q in fluid:
        p = np.zeros(19)
        for i in range(19):
            xs, ys, zs = src(*q, i)
            if m[zs, ys, xs]:
                p[opp[i]] = f0[opp[i], zs, ys, xs]
        prev[q] = p
    out = []
    for _ in range(steps):
        post = {q: oracle_mod.collide3(cur[q], 1.0 / tau, g) for q in fluid}
        new = {}
        for q in fluid:
            v = np.zeros(19)
            for i in range(19):
                xs, ys, zs = src(*q, i)
                v[i] = post[(xs, ys, zs)][i] if m[zs, ys, xs] == 0 else prev[q][opp[i]]
            new[q] = v
        state = np.zeros((19, nz, ny, nx))
        for (x, y, z) in np.ndindex(nx, ny, nz):
            if m[z, y, x]:
                for i in range(19):
                    xs, ys, zs = src(x, y, z, i)
                    if m[zs, ys, xs] == 0:
                        state[i, z, y, x] = post[(xs, ys, zs)][i]
        prev, cur = post, new
        for (x, y, z), v in cur.items():
            state[:, z, y, x] = v
        out.append(state)
    return out


@pytest.mark.parametrize("shape,frac", [((4, 3, 3), 0.35), ((3, 4, 2), 0.5)])
def test_delay_line_brute_force3(oracle_mod, shape, frac):
    nx, ny, nz = shape
    m = synthetic.random_mask3(nx, ny, nz, seed=17, solid_fraction=frac)
    f0 = _random_state3(oracle_mod, m, seed=2)
    fw = oracle_mod.fullway_fill3(m, f0)
    rng = np.random.default_rng(3)
    fw += (fw != 0) * (m[None] == 1) * 0.01 * rng.random(fw.shape)
    g = (2e-3, -1e-3, 5e-4)
    ref = _delay_line3(oracle_mod, m, fw, 0.8, 6, g)
    for t in range(1, 7):
        got = oracle_mod.run3(m, fw, 0.8, t, g=g, fullway=True)
        assert np.array_equal(got, ref[t - 1]), t


def test_mass_conserved_with_wall_slots3(oracle_mod):
    m = synthetic.random_mask3(16, 12, 10, seed=5, solid_fraction=0.2, walls=True)
    f = oracle_mod.fullway_fill3(m, oracle_mod.init3(m, *synthetic.random_fields3(16, 12, 10, seed=6)))
    M0 = f.sum()
    f1 = oracle_mod.run3(m, f, 0.8, 200, g=(1e-4, -5e-5, 2e-5), fullway=True)
    assert abs(f1.sum() - M0) < 1e-12 * M0


def test_steady_channel_closed_form3(oracle_mod):
    nx, ny, nz, tau, g = 2, 2, 14, 0.9, 1e-5
    H = nz - 2
    m = np.zeros((nz, ny, nx), np.uint8)
    m[0] = 1
    m[nz - 1] = 1
    f = oracle_mod.fullway_fill3(m, oracle_mod.init3(m))
    f = oracle_mod.run3(m, f, tau, 30000, g=(g, 0.0, 0.0), fullway=True)
    _, ux, _, uz = oracle_mod.macroscopic3(m, f, g=(g, 0.0, 0.0))
    nu = (tau - 0.5) / 3.0
    zz = np.arange(1, nz - 1)
    exact = g / (2 * nu) * (zz - 0.5) * (H + 0.5 - zz) + g / nu * (16 * (tau - 0.5) ** 2 - 3) / 24
    assert np.abs(ux[1:nz - 1, 0, 0] - exact).max() < 1e-10 * exact.max()
    assert np.abs(uz[1:nz - 1]).max() < 1e-12 * exact.max()


def test_no_solids_is_halfway3(oracle_mod):
    m = np.zeros((5, 6, 7), np.uint8)
    f = oracle_mod.init3(m, *synthetic.random_fields3(7, 6, 5, seed=3))
    a = oracle_mod.run3(m, f, 0.7, 20, g=(1e-4, 0.0, 0.0))
    b = oracle_mod.run3(m, f, 0.7, 20, g=(1e-4, 0.0, 0.0), fullway=True)
    assert np.array_equal(a, b)


def test_z_invariant_projection_is_d2q9_fullway(oracle_mod):
    cx, cy, _, _, _ = oracle_mod.constants3()
    nx, ny, nz = 18, 12, 3
    m2 = synthetic.random_mask(nx, ny, seed=13, solid_fraction=0.2)
    m2[0, :] = 1
    m2[ny - 1, :] = 1
    rho, ux, uy = synthetic.random_fields(nx, ny, seed=5, rho_spread=0.03, u_amp=0.03)
    g = (2e-4, -1e-4)
    f2 = oracle_mod.fullway_fill(m2, oracle_mod.init(m2, rho, ux, uy))
    f2 = oracle_mod.run(m2, f2, 0.75, 30, g=g, fullway=True)
    rep = lambda a: np.repeat(a[None], nz, axis=0)
    m3 = rep(m2)
    f3 = oracle_mod.fullway_fill3(m3, oracle_mod.init3(m3, rep(rho), rep(ux), rep(uy), None))
    f3 = oracle_mod.run3(m3, f3, 0.75, 30, g=(g[0], g[1], 0.0), fullway=True)
    cx2, cy2, _, _ = oracle_mod.constants()
    for k in range(9):
        group = [i for i in range(19) if cx[i] == cx2[k] and cy[i] == cy2[k]]
        proj = f3[group].sum(axis=0)
        for z in range(nz):
            assert np.abs(proj[z] - f2[k]).max() < 1e-14  # fluid and wall slots alike


def test_fill_rule3(oracle_mod):
    cx, cy, cz, _, _ = oracle_mod.constants3()
    m = synthetic.random_mask3(5, 4, 3, seed=8, solid_fraction=0.4)
    f = _random_state3(oracle_mod, m, seed=4)
    g = oracle_mod.fullway_fill3(m, f)
    nz, ny, nx = m.shape
    for z, y, x in np.ndindex(nz, ny, nx):
        if m[z, y, x] == 0:
            assert np.array_equal(g[:, z, y, x], f[:, z, y, x])
            continue
        for i in range(19):
            xs, ys, zs = (x - cx[i]) % nx, (y - cy[i]) % ny, (z - cz[i]) % nz
            assert g[i, z, y, x] == (f[i, zs, ys, xs] if m[zs, ys, xs] == 0 else 0.0)
