"""GPU parity of the full-way bounce-back rule (lbm_set_bounce_back) against the FP64 oracle.

Compared: every fluid slot and every wall slot (population j of a solid node whose source
w - c_j is fluid).  FP64: max abs error <= 1e-12; FP32: max relative error <= 1e-5 (wall
slots relative to the value, fluid slots as in the halfway tests).  Two-lattice layouts only.
"""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce

pytestmark = pytest.mark.gpu

AB_LAYOUTS = ["dense_ab", "tiled16", "indirect", "tiled16_all"]


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


def slots(mask, ref):
    """Boolean [9, ny, nx]: fluid slots and wall slots that carry a population."""
    fl = np.broadcast_to(mask[None] == 0, ref.shape)
    return fl | ((mask[None] == 1) & (ref != 0))


def err(got, ref, mask, dtype):
    sel = slots(mask, ref)
    a, b = got[sel], ref[sel]
    if dtype == "f64":
        return float(np.abs(a - b).max())
    return float((np.abs(a - b) / np.abs(b)).max())


def run_gpu(lbm, mask, tau, steps, dtype, layout, g=(0.0, 0.0), alpha=None, fields=None,
            trt=0.0, bc=None, value=None):
    lat = lbm.Lattice(mask, tau, force=g, dtype=dtype, layout=layout)
    lat.set_bounce_back("fullway")
    if trt:
        lat.set_trt(trt)
    if bc is not None:
        lat.set_boundaries(bc, value)
    if fields is not None:
        lat.init_equilibrium(*fields)
    if alpha is not None:
        lat.set_porosity(alpha)
    lat.step(steps)
    f = lat.get_populations()
    lat.close()
    return f


def run_oracle(oracle_mod, mask, tau, steps, g=(0.0, 0.0), alpha=None, fields=None, trt=0.0,
               bc=None, value=None):
    # the GPU context fills the wall slots from the equilibrium state, and the open-boundary
    # conditions then apply to the fluid nodes in every view
    f0 = oracle_mod.fullway_fill(mask, oracle_mod.init(mask, *(fields or (None, None, None))))
    if bc is not None:
        f0 = oracle_mod.apply_boundaries(mask, f0, bc, value)
    a64 = None if alpha is None else np.asarray(alpha, np.float32).astype(np.float64)
    tm = oracle_mod.trt_tau_minus(tau, trt) if trt else None
    return oracle_mod.run(mask, f0, tau, steps, g=g, alpha=a64, bc=bc, value=value,
                          tau_minus=tm, fullway=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", AB_LAYOUTS)
def test_porous_vs_oracle(lbm, oracle_mod, dtype, layout):
    """128^2 porous discs with walls, body force, drag field, random initial fields, 61 steps."""
    announce(f"fullway porous 128 {dtype} {layout}")
    m, _ = synthetic.porous_discs(128, 0.55, rmin=3, rmax=10)
    alpha = synthetic.brinkman_alpha(128, 128, seed=4, sigma=5.0)
    fields = synthetic.random_fields(128, 128, seed=5, rho_spread=0.02, u_amp=0.02)
    g = (2e-5, -1e-5)
    ref = run_oracle(oracle_mod, m, 0.7, 61, g=g, alpha=alpha, fields=fields)
    got = run_gpu(lbm, m, 0.7, 61, dtype, layout, g=g, alpha=alpha, fields=fields)
    assert err(got, ref, m, dtype) <= TOL[dtype]
    # solid slots that carry nothing stay zero
    assert not np.any(got[~slots(m, ref)])


@pytest.mark.parametrize("layout", ["dense_ab", "indirect"])
def test_open_channel_trt_vs_oracle(lbm, oracle_mod, layout):
    """Pressure-driven channel (Zou-He inlet and outlet) with TRT collision, FP64."""
    announce(f"fullway open channel trt {layout}")
    m, bc, value = synthetic.open_channel(96, 24, inlet="pressure")
    ref = run_oracle(oracle_mod, m, 0.8, 150, trt=0.25, bc=bc, value=value)
    got = run_gpu(lbm, m, 0.8, 150, "f64", layout, trt=0.25, bc=bc, value=value)
    assert err(got, ref, m, "f64") <= TOL["f64"]


@pytest.mark.parametrize("layout", ["dense_ab", "tiled16"])
def test_switch_rules_midway(lbm, oracle_mod, layout):
    """30 halfway steps, switch to full-way (wall slots filled from their sources), 30 steps,
    switch back, 10 steps; the fluid populations carry across both switches."""
    announce(f"fullway switch {layout}")
    m = synthetic.random_mask(64, 48, seed=9, solid_fraction=0.2, walls=True)
    fields = synthetic.random_fields(64, 48, seed=2, rho_spread=0.02, u_amp=0.02)
    g = (1e-4, 0.0)
    f = oracle_mod.run(m, oracle_mod.init(m, *fields), 0.75, 30, g=g)
    f = oracle_mod.run(m, oracle_mod.fullway_fill(m, f), 0.75, 30, g=g, fullway=True)
    f_full = f.copy()
    f = oracle_mod.run(m, f * (m[None] == 0), 0.75, 10, g=g)
    lat = lbm.Lattice(m, 0.75, force=g, dtype="f64", layout=layout)
    lat.init_equilibrium(*fields)
    lat.step(30)
    lat.set_bounce_back("fullway")
    lat.step(30)
    got_full = lat.get_populations()
    lat.set_bounce_back("halfway")
    lat.step(10)
    got = lat.get_populations()
    lat.close()
    assert err(got_full, f_full, m, "f64") <= TOL["f64"]
    fl = m == 0
    assert np.abs(got[:, fl] - f[:, fl]).max() <= TOL["f64"]
    assert not np.any(got[:, m == 1])


@pytest.mark.parametrize("layout", AB_LAYOUTS)
def test_mass_includes_wall_slots(lbm, oracle_mod, layout):
    announce(f"fullway mass {layout}")
    m = synthetic.random_mask(96, 64, seed=3, solid_fraction=0.25, walls=True)
    fields = synthetic.random_fields(96, 64, seed=7, rho_spread=0.03, u_amp=0.03)
    lat = lbm.Lattice(m, 0.8, force=(1e-4, 5e-5), dtype="f64", layout=layout)
    lat.set_bounce_back("fullway")
    lat.init_equilibrium(*fields)
    M0 = lat.mass()
    f0 = lat.get_populations()
    lat.step(200)
    M1 = lat.mass()
    lat.close()
    ref0 = oracle_mod.fullway_fill(m, oracle_mod.init(m, *fields))
    assert abs(M0 - ref0.sum()) <= 1e-12 * M0
    assert abs(f0.sum() - M0) <= 1e-12 * M0
    assert abs(M1 - M0) <= 1e-12 * M0


@pytest.mark.parametrize("layout", AB_LAYOUTS)
def test_populations_roundtrip_with_wall_slots(lbm, oracle_mod, layout):
    announce(f"fullway roundtrip {layout}")
    m = synthetic.random_mask(64, 32, seed=1, solid_fraction=0.3)
    rng = np.random.default_rng(0)
    f = np.where(m[None] == 0, 0.05 + 0.1 * rng.random((9, 32, 64)), 0.0)
    f = oracle_mod.fullway_fill(m, f)
    f += (f != 0) * (m[None] == 1) * 0.01  # wall slots distinct from their sources
    lat = lbm.Lattice(m, 0.8, dtype="f64", layout=layout)
    lat.set_bounce_back("fullway")
    for steps in (0, 3):
        lat.step(steps)
        lat.set_populations(f)
        assert np.array_equal(lat.get_populations(), f)
    lat.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s", "bf16s"])
def test_layouts_bitwise_equal(lbm, dtype):
    announce(f"fullway layouts bitwise {dtype}")
    m, _ = synthetic.porous_discs(128, 0.6, rmin=4, rmax=12)
    fields = synthetic.random_fields(128, 128, seed=12, rho_spread=0.02, u_amp=0.02)
    ref = run_gpu(lbm, m, 0.75, 41, dtype, "dense_ab", g=(1e-5, 0.0), fields=fields)
    for layout in ("tiled16", "indirect", "tiled16_all"):
        got = run_gpu(lbm, m, 0.75, 41, dtype, layout, g=(1e-5, 0.0), fields=fields)
        assert np.array_equal(got, ref), layout


def test_refusals(lbm):
    announce("fullway refusals")
    m = synthetic.channel_mask(64, 16)
    lat = lbm.Lattice(m, 0.8, dtype="f64", layout="dense_aa")
    with pytest.raises(lbm.LbmError) as e:
        lat.set_bounce_back("fullway")
    assert e.value.status == -4
    lat.close()
    lat = lbm.Lattice(m, 0.8, dtype="f64", layout="dense_ab")
    with pytest.raises(lbm.LbmError) as e:
        lat.set_bounce_back(2)
    assert e.value.status == -1
    lat.set_bounce_back("fullway")
    import torch
    buf = torch.empty(lat.state_bytes(), dtype=torch.uint8, device="cuda")
    with pytest.raises(lbm.LbmError) as e:
        lat.save_state(buf)
    assert e.value.status == -4
    with pytest.raises(lbm.LbmError) as e:
        lat.adjoint_bytes()
    assert e.value.status == -4
    # the context stays usable
    lat.step(3)
    assert np.isfinite(lat.mass())
    lat.close()
