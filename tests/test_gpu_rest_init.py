"""The rest state (rho = 1, u = 0; the initialisation of Algorithm 1) is written straight into
the stored lattices, without the canonical staging buffer that initialisation from fields
uses.  Checks: for every layout and storage type the canonical populations equal those of a
lattice initialised through explicit uniform fields (bitwise) and the oracle's rest state (FP64:
exactly w_i), and stay bitwise equal after steps; with the full-way rule, a rest
re-initialisation followed by steps matches the oracle (both lattices hold the rest state)."""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce

pytestmark = pytest.mark.gpu

LAYOUTS = ["dense_ab", "dense_aa", "tiled16", "indirect"]
DTYPES = ["f64", "f32", "f16s", "bf16s"]


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("layout", LAYOUTS)
def test_rest_matches_uniform_fields(lbm, oracle_mod, layout, dtype):
    announce(f"rest init {layout} {dtype}")
    nx, ny = 96, 48
    m = synthetic.random_mask(nx, ny, seed=31, solid_fraction=0.2, walls=True)
    g = (1e-4, -2e-5)
    a = lbm.Lattice(m, 0.7, force=g, dtype=dtype, layout=layout)   # created at rest
    b = lbm.Lattice(m, 0.7, force=g, dtype=dtype, layout=layout)
    b.init_equilibrium(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    fa, fb = a.get_populations(), b.get_populations()
    assert np.array_equal(fa, fb)
    if dtype == "f64":
        assert np.array_equal(fa[:, m == 0], oracle_mod.init(m)[:, m == 0])
    a.step(7)
    b.step(7)
    a.step(6)  # AA: odd and even step counts alike
    b.step(6)
    assert np.array_equal(a.get_populations(), b.get_populations())
    a.init_equilibrium()  # rest re-initialisation after steps
    assert np.array_equal(a.get_populations(), fb)
    assert a.info()["time_step"] == 0
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["dense_ab", "tiled16", "indirect"])
def test_rest_fullway(lbm, oracle_mod, layout, dtype):
    announce(f"rest init fullway {layout} {dtype}")
    nx, ny = 64, 32
    m = synthetic.random_mask(nx, ny, seed=33, solid_fraction=0.25, walls=True)
    g = (2e-4, 1e-4)
    lat = lbm.Lattice(m, 0.75, force=g, dtype=dtype, layout=layout)
    lat.step(5)
    lat.set_bounce_back("fullway")
    lat.init_equilibrium()
    f0 = oracle_mod.fullway_fill(m, oracle_mod.init(m))
    got0 = lat.get_populations()
    assert np.array_equal(got0, f0)  # FP32 stores deviations from w_i: exact at rest
    lat.step(23)
    got = lat.get_populations()
    lat.close()
    ref = oracle_mod.run(m, f0, 0.75, 23, g=g, fullway=True)
    sel = (m[None] == 0) | (ref != 0)
    a, b = got[sel], ref[sel]
    err = np.abs(a - b).max() if dtype == "f64" else (np.abs(a - b) / np.abs(b)).max()
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_rest_d3q19(lbm, oracle_mod, dtype):
    announce(f"rest init d3q19 {dtype}")
    nx, ny, nz = 70, 12, 10
    m = synthetic.random_mask3(nx, ny, nz, seed=35, solid_fraction=0.15, walls=True)
    g = (2e-5, -1e-5, 1e-5)
    a = lbm.Lattice3D(m, 0.7, force=g, dtype=dtype)
    b = lbm.Lattice3D(m, 0.7, force=g, dtype=dtype)
    ones, zeros = np.ones((nz, ny, nx)), np.zeros((nz, ny, nx))
    b.init_equilibrium(ones, zeros, zeros, zeros)
    fa, fb = a.get_populations(), b.get_populations()
    assert np.array_equal(fa, fb)
    if dtype == "f64":
        assert np.array_equal(fa[:, m == 0], oracle_mod.init3(m)[:, m == 0])
    a.step(9)
    b.step(9)
    assert np.array_equal(a.get_populations(), b.get_populations())
    if dtype in ("f64", "f32"):
        a.set_bounce_back("fullway")
        a.init_equilibrium()
        a.step(17)
        got = a.get_populations()
        f0 = oracle_mod.fullway_fill3(m, oracle_mod.init3(m))
        ref = oracle_mod.run3(m, f0, 0.7, 17, g=g, fullway=True)
        sel = (m[None] == 0) | (ref != 0)
        x, y = got[sel], ref[sel]
        err = np.abs(x - y).max() if dtype == "f64" else (np.abs(x - y) / np.abs(y)).max()
        assert err <= TOL[dtype]
    a.close()
    b.close()
