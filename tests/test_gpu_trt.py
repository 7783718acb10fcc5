"""Two-relaxation-time collision on the GPU against the FP64 oracle: every layout, FP64 and
FP32 (tolerances as for BGK: FP64 max abs 1e-12, FP32 max relative 1e-5), with body force, drag
field and open boundaries; bitwise layout agreement; switching back to BGK; graph replay; and
the adjoint's refusal of TRT lattices."""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce, fp_error, fp_error_w

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


def _gpu(lbm, m, tau, magic, steps, dtype, layout, g=(0.0, 0.0), alpha=None, fields=None,
         bc=None, val=None, graph=-1):
    lat = lbm.Lattice(m, tau, force=g, dtype=dtype, layout=layout)
    lat.set_graph_steps(graph)
    lat.set_trt(magic)
    if bc is not None:
        lat.set_boundaries(bc, val)
    if fields is not None:
        lat.init_equilibrium(*fields)
    if alpha is not None:
        lat.set_porosity(alpha)
    lat.step(steps)
    f = lat.get_populations()
    lat.close()
    return f


def _oracle(oracle_mod, m, tau, magic, steps, g=(0.0, 0.0), alpha=None, fields=None, bc=None,
            val=None):
    f0 = oracle_mod.init(m, *(fields or (None, None, None)), bc=bc, value=val)
    a64 = None if alpha is None else np.asarray(alpha, np.float32).astype(np.float64)
    tm = oracle_mod.trt_tau_minus(tau, magic)
    return oracle_mod.run(m, f0, tau, steps, g=g, alpha=a64, bc=bc, value=val, tau_minus=tm)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("magic", [3.0 / 16.0, 0.05])
def test_trt_porous_vs_oracle(lbm, oracle_mod, dtype, layout, magic):
    """128^2 porous discs, walls, body force, drag field, random initial fields, 151 steps."""
    announce(f"trt porous {layout} {dtype} magic={magic}")
    m, _ = synthetic.porous_discs(128, 0.6, rmin=4, rmax=12)
    alpha = synthetic.brinkman_alpha(128, 128, seed=3, sigma=5.0)
    fields = synthetic.random_fields(128, 128, seed=9, rho_spread=0.02, u_amp=0.02)
    g = (2e-5, -1e-5)
    ref = _oracle(oracle_mod, m, 0.7, magic, 151, g=g, alpha=alpha, fields=fields)
    got = _gpu(lbm, m, 0.7, magic, 151, dtype, layout, g=g, alpha=alpha, fields=fields)
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]


@pytest.mark.parametrize("layout", ["dense_ab", "indirect"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_trt_open_channel_vs_oracle(lbm, oracle_mod, layout, dtype):
    announce(f"trt open channel {layout} {dtype}")
    m, bc, val = synthetic.open_channel(96, 32, "velocity", u_in=0.05)
    ref = _oracle(oracle_mod, m, 0.9, 0.25, 301, bc=bc, val=val)
    got = _gpu(lbm, m, 0.9, 0.25, 301, dtype, layout, bc=bc, val=val)
    assert fp_error_w(got, ref, m, dtype) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s", "bf16s"])
def test_trt_layouts_bitwise(lbm, dtype):
    announce(f"trt layouts bitwise {dtype}")
    m, _ = synthetic.porous_discs(96, 0.6, rmin=4, rmax=10)
    fields = synthetic.random_fields(96, 96, seed=4, rho_spread=0.02, u_amp=0.02)
    for steps in (30, 31):
        ref = _gpu(lbm, m, 0.75, 0.1, steps, dtype, "dense_ab", g=(1e-5, 0.0), fields=fields)
        for layout in LAYOUTS[1:]:
            got = _gpu(lbm, m, 0.75, 0.1, steps, dtype, layout, g=(1e-5, 0.0), fields=fields)
            assert np.array_equal(got, ref), (layout, steps)


def test_trt_switch_back_to_bgk_and_graphs(lbm):
    """set_trt(0) is BGK bitwise; graph replay with TRT equals single launches bitwise."""
    announce("trt switch and graphs")
    import torch
    m = synthetic.random_mask(64, 48, seed=5, solid_fraction=0.2)
    lat = lbm.Lattice(m, 0.8, force=(1e-4, 0.0), dtype="f64", layout="dense_ab")
    lat.step(40)
    bgk = lat.get_populations()
    lat.close()
    lat = lbm.Lattice(m, 0.8, force=(1e-4, 0.0), dtype="f64", layout="dense_ab")
    lat.set_trt(0.3)
    lat.set_trt(0.0)
    lat.step(40)
    assert np.array_equal(lat.get_populations(), bgk)
    lat.set_trt(0.2)
    with pytest.raises(lbm.LbmError) as e:
        lat.adjoint_bytes()
    assert e.value.status == -4
    with pytest.raises(lbm.LbmError) as e:
        lat.set_trt(-1.0)
    assert e.value.status == -1
    lat.close()
    a = _gpu(lbm, m, 0.8, 0.2, 77, "f64", "dense_aa", g=(1e-4, 0.0), graph=0)
    b = _gpu(lbm, m, 0.8, 0.2, 77, "f64", "dense_aa", g=(1e-4, 0.0), graph=8)
    assert np.array_equal(a, b)
