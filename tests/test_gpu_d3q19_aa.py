"""GPU parity of the D3Q19 DENSE_AA layout (one lattice updated in place with the AA access
pattern) against the FP64 D3Q19 oracle and the A-B layout.

Tolerances (as for the A-B layout): FP64 max |f_gpu - f_oracle| <= 1e-12; FP32 max relative
error <= 1e-5.  The AA step computes the same collision from the same values as the A-B step,
so the two layouts agree bitwise for every storage type, after odd and even step counts.
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


def run_gpu(lbm, mask, tau, steps, dtype, layout, g=(0.0, 0.0, 0.0), fields=None, trt=0.0):
    lat = lbm.Lattice3D(mask, tau, force=g, dtype=dtype, layout=layout)
    lat.set_trt(trt)
    if fields is not None:
        lat.init_equilibrium(*fields)
    lat.step(steps)
    f = lat.get_populations()
    lat.close()
    return f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape,steps", [((70, 24, 20), 40), ((70, 24, 20), 41),
                                         ((300, 5, 7), 33)])
def test_aa_vs_oracle(lbm, oracle_mod, dtype, shape, steps):
    """Random solids (12 %), walls at z = 0 and nz - 1, a body force along all three axes,
    random initial fields; even and odd step counts; nx not a multiple of 64 and, for
    nx = 300, a second 256-node row segment."""
    nx, ny, nz = shape
    announce(f"d3q19 aa {nx}x{ny}x{nz} {dtype} {steps} steps")
    m = synthetic.random_mask3(nx, ny, nz, seed=41, solid_fraction=0.12, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=42)
    g = (2e-5, -1e-5, 1e-5)
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.7, steps, g=g)
    got = run_gpu(lbm, m, 0.7, steps, dtype, "dense_aa", g=g, fields=fields)
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]
    assert not np.any(got[:, m == 1])


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s", "bf16s"])
def test_aa_matches_ab_bitwise(lbm, dtype):
    announce(f"d3q19 aa vs ab bitwise {dtype}")
    nx, ny, nz = 80, 16, 12
    m = synthetic.random_mask3(nx, ny, nz, seed=43, solid_fraction=0.15, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=44)
    g = (1e-5, 2e-5, -1e-5)
    for steps in (0, 1, 2, 7):
        a = run_gpu(lbm, m, 0.8, steps, dtype, "dense_ab", g=g, fields=fields)
        b = run_gpu(lbm, m, 0.8, steps, dtype, "dense_aa", g=g, fields=fields)
        assert np.array_equal(a, b), steps


@pytest.mark.parametrize("steps", [30, 31])
def test_aa_trt_and_force_free(lbm, oracle_mod, steps):
    announce(f"d3q19 aa trt / force-free {steps}")
    nx, ny, nz = 64, 12, 10
    m = synthetic.random_mask3(nx, ny, nz, seed=45, solid_fraction=0.1, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=46)
    tm = oracle_mod.trt_tau_minus(0.75, 0.25)
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.75, steps, g=(1e-5, 0.0, 0.0),
                          tau_minus=tm)
    got = run_gpu(lbm, m, 0.75, steps, "f64", "dense_aa", g=(1e-5, 0.0, 0.0), fields=fields,
                  trt=0.25)
    assert fp_error(got, ref, m, "f64") <= TOL["f64"]
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.75, steps)
    got = run_gpu(lbm, m, 0.75, steps, "f64", "dense_aa", fields=fields)
    assert fp_error(got, ref, m, "f64") <= TOL["f64"]


def test_aa_views_roundtrip_mass_and_errors(lbm, oracle_mod):
    """macroscopic fields and mass at an odd step against the oracle; set_populations at odd
    and even steps is read back exactly and continues as the oracle from that state; a rest
    re-initialisation; full-way refused; one lattice (info)."""
    announce("d3q19 aa views and errors")
    nx, ny, nz = 48, 20, 16
    m = synthetic.random_mask3(nx, ny, nz, seed=47, solid_fraction=0.15, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=48)
    g = (3e-5, 1e-5, -2e-5)
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.7, 31, g=g)
    lat = lbm.Lattice3D(m, 0.7, force=g, dtype="f64", layout="dense_aa")
    ab = lbm.Lattice3D(m, 0.7, force=g, dtype="f64")
    info = lat.info()
    assert info["layout"] == 1 and ab.info()["layout"] == 0
    assert info["device_bytes"] < 0.6 * ab.info()["device_bytes"]
    ab.close()
    lat.init_equilibrium(*fields)
    M0 = lat.mass()
    lat.step(31)
    out = lat.macroscopic()
    exp = oracle_mod.macroscopic3(m, ref, g=g)
    for a, b in zip(out, exp):
        assert np.abs(a - b).max() <= 1e-12
    assert abs(lat.mass() - M0) <= 1e-12 * M0
    assert abs(lat.mass() - ref.sum()) <= 1e-12 * M0
    _, _, _, w, _ = oracle_mod.constants3()
    f = synthetic.random_populations(w, m.shape, seed=49) * (m == 0)
    for _ in range(2):  # state set at an odd (31), then an even (40) step count
        lat.set_populations(f)
        assert np.array_equal(lat.get_populations(), f)
        lat.step(9)
        ref2 = oracle_mod.run3(m, f, 0.7, 9, g=g)
        assert fp_error(lat.get_populations(), ref2, m, "f64") <= TOL["f64"]
    with pytest.raises(lbm.LbmError) as e:
        lat.set_bounce_back("fullway")
    assert e.value.status == -4
    lat.init_equilibrium()
    assert np.array_equal(lat.get_populations()[:, m == 0], oracle_mod.init3(m)[:, m == 0])
    assert lat.info()["time_step"] == 0
    lat.close()


@pytest.mark.parametrize("layout", ["dense_ab", "dense_aa"])
def test_state_checkpoints_and_device_fields(lbm, layout):
    """save_state / load_state reproduce a run bitwise (AA: loaded at a step count of the
    same parity); macroscopic_device equals the host fields bitwise; full-way checkpoints
    and missing device fields are refused; undersized buffers raise in the binding."""
    import torch
    announce(f"d3q19 checkpoints and device fields {layout}")
    nx, ny, nz = 40, 12, 10
    m = synthetic.random_mask3(nx, ny, nz, seed=51, solid_fraction=0.1, walls=True)
    lat = lbm.Lattice3D(m, 0.75, force=(2e-5, 0.0, -1e-5), dtype="f32", layout=layout)
    lat.init_equilibrium(*synthetic.random_fields3(nx, ny, nz, seed=52))
    lat.step(5)
    buf = torch.empty(lat.state_bytes(), dtype=torch.uint8, device="cuda")
    lat.save_state(buf)
    lat.step(6)
    a = lat.get_populations()
    lat.load_state(buf)
    lat.step(6)
    assert np.array_equal(lat.get_populations(), a)
    host = lat.macroscopic()
    dev = [torch.full((nz, ny, nx), 7.0, dtype=torch.float64, device="cuda") for _ in range(4)]
    lat.macroscopic_device(*dev)
    torch.cuda.synchronize()
    for h, d in zip(host, dev):
        assert np.array_equal(h, d.cpu().numpy())
    with pytest.raises(ValueError, match="bytes"):
        lat.save_state(buf[:-1])
    with pytest.raises(lbm.LbmError) as e:
        lat._check(lat._lib.lbm3d_macroscopic_device(lat._ctx, dev[0].data_ptr(), None, None,
                                                     None))
    assert e.value.status == -1
    if layout == "dense_ab":
        lat.set_bounce_back("fullway")
        with pytest.raises(lbm.LbmError) as e:
            lat.save_state(buf)
        assert e.value.status == -4
    lat.close()
