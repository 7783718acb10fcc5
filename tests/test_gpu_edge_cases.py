"""Degenerate geometries on every layout: an all-solid mesh (no fluid node: no tiles, an empty
node list) steps, reports zero mass and zero fields, and takes state round trips; a single
fluid node in a periodic 1 x 1 mesh (its own neighbour in every direction) and a fluid row
between walls match the oracle; zero steps change nothing."""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce, fp_error

pytestmark = pytest.mark.gpu

LAYOUTS = ["dense_ab", "dense_aa", "tiled16", "indirect", "tiled16_all"]


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_all_solid(lbm, layout, dtype):
    announce(f"all solid {layout} {dtype}")
    m = np.ones((32, 48), np.uint8)
    lat = lbm.Lattice(m, 0.8, force=(1e-4, 0.0), dtype=dtype, layout=layout)
    info = lat.info()
    assert info["n_fluid"] == 0
    lat.step(5)
    assert lat.mass() == 0.0
    assert not np.any(lat.get_populations())
    for a in lat.macroscopic():
        assert not np.any(a)
    lat.set_populations(np.zeros((9, 32, 48)))
    lat.init_equilibrium()
    if layout != "dense_aa":
        lat.set_bounce_back("fullway")
        lat.step(3)
        assert lat.mass() == 0.0
    lat.close()


@pytest.mark.parametrize("layout", ["dense_ab", "dense_aa"])
def test_all_solid_d3q19(lbm, layout):
    announce(f"all solid d3q19 {layout}")
    m = np.ones((6, 8, 70), np.uint8)
    lat = lbm.Lattice3D(m, 0.8, force=(1e-4, 0.0, 0.0), dtype="f32", layout=layout)
    lat.step(4)
    assert lat.mass() == 0.0
    assert not np.any(lat.get_populations())
    for a in lat.macroscopic():
        assert not np.any(a)
    lat.close()


@pytest.mark.parametrize("layout", ["dense_ab", "dense_aa", "indirect"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_node_and_single_row(lbm, oracle_mod, layout, dtype):
    announce(f"single node / row {layout} {dtype}")
    fields = synthetic.random_fields(1, 1, seed=3, rho_spread=0.02, u_amp=0.05)
    m = np.zeros((1, 1), np.uint8)
    g = (1e-3, -5e-4)
    ref = oracle_mod.run(m, oracle_mod.init(m, *fields), 0.7, 13, g=g)
    lat = lbm.Lattice(m, 0.7, force=g, dtype=dtype, layout=layout)
    lat.init_equilibrium(*fields)
    lat.step(0)
    assert lat.info()["time_step"] == 0
    lat.step(13)
    assert fp_error(lat.get_populations(), ref, m, dtype) <= TOL[dtype]
    lat.close()
    m = np.ones((3, 70), np.uint8)
    m[1] = 0
    fields = synthetic.random_fields(70, 3, seed=4, rho_spread=0.02, u_amp=0.05)
    ref = oracle_mod.run(m, oracle_mod.init(m, *fields), 0.7, 21, g=g)
    lat = lbm.Lattice(m, 0.7, force=g, dtype=dtype, layout=layout)
    lat.init_equilibrium(*fields)
    lat.step(21)
    assert fp_error(lat.get_populations(), ref, m, dtype) <= TOL[dtype]
    lat.close()
