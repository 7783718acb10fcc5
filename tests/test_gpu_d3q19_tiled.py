"""GPU parity of the sparse tiled D3Q19 layout (TILED16: 4 x 4 x 4-node blocks holding a fluid
node, with an 18-entry block-neighbour table) against the FP64 D3Q19 oracle and the dense A-B
layout.

Tolerances: FP64 max |f_gpu - f_oracle| <= 1e-12; FP32 max relative error <= 1e-5.  The block
step gathers the same values and runs the same collision as the dense step, so the layouts
agree bitwise for every storage type and collision model.  Shapes include meshes one block wide
in an axis (a block is then its own neighbour across that axis) and a single-block mesh.
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
@pytest.mark.parametrize("shape,frac,steps", [((68, 24, 20), 0.3, 40), ((32, 8, 12), 0.5, 33),
                                              ((64, 16, 12), 0.0, 21), ((4, 4, 4), 0.2, 9),
                                              ((8, 4, 12), 0.3, 17)])
def test_tiled_vs_oracle(lbm, oracle_mod, dtype, shape, frac, steps):
    """Random solids (none to 50 %), walls in z, a body force along all three axes, random
    initial fields."""
    nx, ny, nz = shape
    announce(f"d3q19 tiled {nx}x{ny}x{nz} phi={1 - frac} {dtype}")
    m = synthetic.random_mask3(nx, ny, nz, seed=81, solid_fraction=frac, walls=frac > 0)
    fields = synthetic.random_fields3(nx, ny, nz, seed=82)
    g = (2e-5, -1e-5, 1e-5)
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.7, steps, g=g)
    got = run_gpu(lbm, m, 0.7, steps, dtype, "tiled16", g=g, fields=fields)
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]
    assert not np.any(got[:, m == 1])


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s", "bf16s"])
def test_tiled_matches_dense_bitwise(lbm, dtype):
    """BGK, TRT and MRT, after 0, 1 and 6 steps, both block layouts (kept blocks only, and
    every block) against the dense A-B step, on a mesh with solid slabs that drop whole
    blocks."""
    announce(f"d3q19 tiled vs dense bitwise {dtype}")
    nx, ny, nz = 80, 16, 12
    m = synthetic.random_mask3(nx, ny, nz, seed=83, solid_fraction=0.35, walls=True)
    m[:, :, 20:32] = 1
    fields = synthetic.random_fields3(nx, ny, nz, seed=84)
    g = (1e-5, 2e-5, -1e-5)
    models = [None, lambda lat: lat.set_trt(0.25),
              lambda lat: lat.set_mrt((1.19, 1.4, 1.64, 1.3, 1.55))]
    for model in models:
        for steps in (0, 1, 6):
            a = run_gpu(lbm, m, 0.8, steps, dtype, "dense_ab", g=g, fields=fields, model=model)
            for layout in ("tiled16", "tiled16_all"):
                b = run_gpu(lbm, m, 0.8, steps, dtype, layout, g=g, fields=fields, model=model)
                assert np.array_equal(a, b), (layout, steps)


def test_tiled_spheres_bitwise(lbm):
    """A 64^3 sphere packing at fluid fraction 0.4 (walls in z, force along x), FP32, 25 steps:
    bitwise equal to the dense A-B layout; fewer device bytes."""
    announce("d3q19 tiled spheres 64^3 bitwise")
    m = synthetic.random_spheres3(64, 0.4, rmin=3, rmax=8)
    out, dev = {}, {}
    for layout in ("dense_ab", "tiled16"):
        lat = lbm.Lattice3D(m, 0.6, force=(1e-5, 0.0, 0.0), dtype="f32", layout=layout)
        lat.step(25)
        out[layout] = lat.get_populations()
        dev[layout] = lat.info()["device_bytes"]
        lat.close()
    assert np.array_equal(out["dense_ab"], out["tiled16"])
    assert dev["tiled16"] < dev["dense_ab"]


def test_tiled_views_state_and_errors(lbm, oracle_mod):
    """macroscopic fields and mass against the oracle; set / get populations exact; save / load
    replays bitwise; info reports the layout; an all-solid mesh stores no block; sizes that are
    not multiples of 4 are refused."""
    import torch
    announce("d3q19 tiled views and state")
    nx, ny, nz = 48, 20, 16
    m = synthetic.random_mask3(nx, ny, nz, seed=85, solid_fraction=0.6, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=86)
    g = (3e-5, 1e-5, -2e-5)
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.7, 30, g=g)
    lat = lbm.Lattice3D(m, 0.7, force=g, dtype="f64", layout="tiled16")
    info = lat.info()
    assert info["layout"] == 2 and info["n_fluid"] == int((m == 0).sum())
    lat.init_equilibrium(*fields)
    M0 = lat.mass()
    lat.step(30)
    for a, b in zip(lat.macroscopic(), oracle_mod.macroscopic3(m, ref, g=g)):
        assert np.abs(a - b).max() <= 1e-12
    assert abs(lat.mass() - M0) <= 1e-12 * M0
    assert abs(lat.mass() - ref.sum()) <= 1e-12 * M0
    _, _, _, w, _ = oracle_mod.constants3()
    f = synthetic.random_populations(w, m.shape, seed=87) * (m == 0)
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
    allb = lbm.Lattice3D(m, 0.7, force=g, dtype="f64", layout="tiled16_all")
    assert allb.info()["layout"] == 4
    allb.close()
    empty = lbm.Lattice3D(np.ones((4, 8, 12), np.uint8), 0.8, force=g, dtype="f32",
                          layout="tiled16")
    assert empty.info()["n_fluid"] == 0
    empty.step(3)
    assert empty.mass() == 0.0
    assert not np.any(empty.get_populations())
    empty.close()
    with pytest.raises(lbm.LbmError):
        lbm.Lattice3D(np.zeros((4, 4, 6), np.uint8), 0.8, layout="tiled16")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tiled_fullway(lbm, oracle_mod, dtype):
    """Full-way walls on the block layout: against the oracle (fluid and wall slots), bitwise
    against the dense A-B layout, a switch back to halfway, and the mass with wall slots."""
    announce(f"d3q19 tiled fullway {dtype}")
    nx, ny, nz = 68, 12, 8
    m = synthetic.random_mask3(nx, ny, nz, seed=88, solid_fraction=0.25, walls=True)
    m[:, :, 8:12] = 1
    fields = synthetic.random_fields3(nx, ny, nz, seed=89)
    g = (2e-5, -1e-5, 1e-5)
    f0 = oracle_mod.fullway_fill3(m, oracle_mod.init3(m, *fields))
    ref = oracle_mod.run3(m, f0, 0.7, 31, g=g, fullway=True)
    out = {}
    for layout in ("dense_ab", "tiled16"):
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
    assert np.array_equal(out["tiled16"], out["dense_ab"])
    assert np.array_equal(out["tiled16 halfway"], out["dense_ab halfway"])
    got = out["tiled16"]
    sel = (m[None] == 0) | (ref != 0)
    a, b = got[sel], ref[sel]
    err = np.abs(a - b).max() if dtype == "f64" else (np.abs(a - b) / np.abs(b)).max()
    assert err <= TOL[dtype]
