"""GPU parity of the sparse D3Q19 layout (INDIRECT: fluid nodes only, with a per-node table of
the 18 pull sources) against the FP64 D3Q19 oracle and the dense A-B layout.

Tolerances: FP64 max |f_gpu - f_oracle| <= 1e-12; FP32 max relative error <= 1e-5.  The list
step gathers the same values and runs the same collision as the dense step, so the two layouts
agree bitwise for every storage type and collision model.
"""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce, fp_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


def run_gpu(lbm, mask, tau, steps, dtype, layout, g=(0.0, 0.0, 0.0), fields=None, model=None):
    lat = lbm.Lattice3D(mask, tau, force=g, dtype=dtype, layout=layout)
    if model is not None:
        model(lat)
    if fields is not None:
        lat.init_equilibrium(*fields)
    lat.step(steps)
    f = lat.get_populations()
    lat.close()
    return f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape,frac,steps", [((70, 24, 20), 0.3, 40), ((300, 5, 7), 0.5, 33),
                                              ((64, 16, 12), 0.0, 21)])
def test_list_vs_oracle(lbm, oracle_mod, dtype, shape, frac, steps):
    """Random solids (30 % / 50 % / none), walls in z, a body force along all three axes,
    random initial fields."""
    nx, ny, nz = shape
    announce(f"d3q19 list {nx}x{ny}x{nz} phi={1 - frac} {dtype}")
    m = synthetic.random_mask3(nx, ny, nz, seed=71, solid_fraction=frac, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=72)
    g = (2e-5, -1e-5, 1e-5)
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.7, steps, g=g)
    got = run_gpu(lbm, m, 0.7, steps, dtype, "indirect", g=g, fields=fields)
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]
    assert not np.any(got[:, m == 1])


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s", "bf16s"])
def test_list_matches_dense_bitwise(lbm, dtype):
    announce(f"d3q19 list vs dense bitwise {dtype}")
    nx, ny, nz = 80, 16, 12
    m = synthetic.random_mask3(nx, ny, nz, seed=73, solid_fraction=0.35, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=74)
    g = (1e-5, 2e-5, -1e-5)
    models = [None, lambda lat: lat.set_trt(0.25),
              lambda lat: lat.set_mrt((1.19, 1.4, 1.64, 1.3, 1.55))]
    for model in models:
        for steps in (0, 1, 6):
            a = run_gpu(lbm, m, 0.8, steps, dtype, "dense_ab", g=g, fields=fields, model=model)
            b = run_gpu(lbm, m, 0.8, steps, dtype, "indirect", g=g, fields=fields, model=model)
            assert np.array_equal(a, b), steps


def test_list_views_state_and_errors(lbm, oracle_mod):
    """macroscopic fields and mass against the oracle; set / get populations exact; save / load
    replays bitwise; info reports the layout and fewer device bytes than the dense layout on a
    sparse geometry; an all-solid mesh has an empty list."""
    import torch
    announce("d3q19 list views and state")
    nx, ny, nz = 48, 20, 16
    m = synthetic.random_mask3(nx, ny, nz, seed=75, solid_fraction=0.6, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=76)
    g = (3e-5, 1e-5, -2e-5)
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.7, 30, g=g)
    lat = lbm.Lattice3D(m, 0.7, force=g, dtype="f64", layout="indirect")
    dense = lbm.Lattice3D(m, 0.7, force=g, dtype="f64")
    info = lat.info()
    assert info["layout"] == 3 and info["n_fluid"] == int((m == 0).sum())
    assert info["device_bytes"] < dense.info()["device_bytes"]
    dense.close()
    lat.init_equilibrium(*fields)
    M0 = lat.mass()
    lat.step(30)
    for a, b in zip(lat.macroscopic(), oracle_mod.macroscopic3(m, ref, g=g)):
        assert np.abs(a - b).max() <= 1e-12
    assert abs(lat.mass() - M0) <= 1e-12 * M0
    assert abs(lat.mass() - ref.sum()) <= 1e-12 * M0
    _, _, _, w, _ = oracle_mod.constants3()
    f = synthetic.random_populations(w, m.shape, seed=77) * (m == 0)
    lat.set_populations(f)
    assert np.array_equal(lat.get_populations(), f)
    buf = torch.empty(lat.state_bytes(), dtype=torch.uint8, device="cuda")
    lat.save_state(buf)
    lat.step(5)
    a = lat.get_populations()
    lat.load_state(buf)
    lat.step(5)
    assert np.array_equal(lat.get_populations(), a)
    assert fp_error(a, oracle_mod.run3(m, f, 0.7, 5, g=g), m, "f64") <= TOL["f64"]
    lat.close()
    empty = lbm.Lattice3D(np.ones((4, 6, 70), np.uint8), 0.8, force=g, dtype="f32",
                          layout="indirect")
    assert empty.info()["n_fluid"] == 0
    empty.step(3)
    assert empty.mass() == 0.0
    assert not np.any(empty.get_populations())
    empty.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_list_fullway(lbm, oracle_mod, dtype):
    """Full-way walls on the node list: against the oracle (fluid and wall slots), bitwise
    against the dense A-B layout, a switch back to halfway, and the mass with wall slots."""
    announce(f"d3q19 list fullway {dtype}")
    nx, ny, nz = 70, 12, 10
    m = synthetic.random_mask3(nx, ny, nz, seed=78, solid_fraction=0.25, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=79)
    g = (2e-5, -1e-5, 1e-5)
    f0 = oracle_mod.fullway_fill3(m, oracle_mod.init3(m, *fields))
    ref = oracle_mod.run3(m, f0, 0.7, 31, g=g, fullway=True)
    out = {}
    for layout in ("dense_ab", "indirect"):
        lat = lbm.Lattice3D(m, 0.7, force=g, dtype=dtype, layout=layout)
        lat.set_bounce_back("fullway")
        lat.init_equilibrium(*fields)
        M0 = lat.mass()
        lat.step(31)
        out[layout] = lat.get_populations()
        if dtype == "f64":
            assert abs(lat.mass() - M0) <= 1e-12 * M0
        lat.set_bounce_back("halfway")
        lat.step(4)
        out[layout + " halfway"] = lat.get_populations()
        lat.close()
    assert np.array_equal(out["indirect"], out["dense_ab"])
    assert np.array_equal(out["indirect halfway"], out["dense_ab halfway"])
    got = out["indirect"]
    sel = (m[None] == 0) | (ref != 0)
    a, b = got[sel], ref[sel]
    err = np.abs(a - b).max() if dtype == "f64" else (np.abs(a - b) / np.abs(b)).max()
    assert err <= TOL[dtype]
