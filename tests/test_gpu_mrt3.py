"""D3Q19 multiple-relaxation-time collision on the GPU against the FP64 D3Q19 oracle: A-B and
AA layouts, FP64 and FP32 (FP64 max abs 1e-12, FP32 max relative 1e-5), with a body force or
none, and full-way walls; bitwise A-B / AA agreement; equivalence with BGK and TRT rates;
switching between collision models; invalid rates."""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce, fp_error

pytestmark = pytest.mark.gpu

RATES = (1.19, 1.4, 1.64, 1.3, 1.55)  # s_e, s_eps, s_q, s_pi, s_m


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


def run_gpu(lbm, m, tau, steps, dtype, layout="dense_ab", g=(0.0, 0.0, 0.0), fields=None,
            rates=RATES, fullway=False):
    lat = lbm.Lattice3D(m, tau, force=g, dtype=dtype, layout=layout)
    lat.set_mrt(rates)
    if fullway:
        lat.set_bounce_back("fullway")
    if fields is not None:
        lat.init_equilibrium(*fields)
    lat.step(steps)
    f = lat.get_populations()
    lat.close()
    return f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["dense_ab", "dense_aa"])
@pytest.mark.parametrize("force", [True, False])
def test_mrt3_vs_oracle(lbm, oracle_mod, dtype, layout, force):
    """Random solids (12 %), walls in z, random initial fields, 37 steps, ragged nx."""
    announce(f"d3q19 mrt {layout} {dtype} force={force}")
    nx, ny, nz = 70, 16, 12
    m = synthetic.random_mask3(nx, ny, nz, seed=61, solid_fraction=0.12, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=62)
    g = (2e-5, -1e-5, 1e-5) if force else (0.0, 0.0, 0.0)
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.7, 37, g=g, mrt=RATES)
    got = run_gpu(lbm, m, 0.7, 37, dtype, layout, g=g, fields=fields)
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]


def test_mrt3_fullway_vs_oracle(lbm, oracle_mod):
    announce("d3q19 mrt fullway")
    nx, ny, nz = 40, 12, 10
    m = synthetic.random_mask3(nx, ny, nz, seed=63, solid_fraction=0.2, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=64)
    g = (1e-4, 0.0, -5e-5)
    f0 = oracle_mod.fullway_fill3(m, oracle_mod.init3(m, *fields))
    ref = oracle_mod.run3(m, f0, 0.8, 29, g=g, mrt=RATES, fullway=True)
    got = run_gpu(lbm, m, 0.8, 29, "f64", g=g, fields=fields, fullway=True)
    sel = (m[None] == 0) | (ref != 0)
    assert np.abs(got[sel] - ref[sel]).max() <= TOL["f64"]


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s", "bf16s"])
def test_mrt3_ab_aa_bitwise(lbm, dtype):
    announce(f"d3q19 mrt ab/aa bitwise {dtype}")
    nx, ny, nz = 64, 12, 10
    m = synthetic.random_mask3(nx, ny, nz, seed=65, solid_fraction=0.1, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=66)
    for steps in (6, 7):
        a = run_gpu(lbm, m, 0.75, steps, dtype, "dense_ab", g=(1e-5, 0.0, 0.0), fields=fields)
        b = run_gpu(lbm, m, 0.75, steps, dtype, "dense_aa", g=(1e-5, 0.0, 0.0), fields=fields)
        assert np.array_equal(a, b), steps


def test_mrt3_equivalences_and_switches(lbm):
    """All rates omega is BGK and even/odd rates are TRT (FP64, 1e-12); set_mrt(None) is BGK
    bitwise; the last of set_trt / set_mrt wins; invalid rates are refused."""
    announce("d3q19 mrt equivalences")
    nx, ny, nz = 48, 10, 8
    m = synthetic.random_mask3(nx, ny, nz, seed=67, solid_fraction=0.1, walls=True)
    fields = synthetic.random_fields3(nx, ny, nz, seed=68)
    tau, g = 0.8, (1e-4, -3e-5, 2e-5)

    def run(setup):
        lat = lbm.Lattice3D(m, tau, force=g, dtype="f64")
        setup(lat)
        lat.init_equilibrium(*fields)
        lat.step(25)
        f = lat.get_populations()
        lat.close()
        return f

    om = 1.0 / tau
    bgk = run(lambda lat: None)
    assert np.abs(run(lambda lat: lat.set_mrt((om,) * 5)) - bgk).max() <= 1e-12
    magic = 0.2
    sq = 1.0 / (0.5 + magic / (tau - 0.5))
    trt = run(lambda lat: lat.set_trt(magic))
    assert np.abs(run(lambda lat: lat.set_mrt((om, om, sq, om, sq))) - trt).max() <= 1e-12
    assert np.array_equal(run(lambda lat: (lat.set_mrt(RATES), lat.set_mrt(None))), bgk)
    assert np.array_equal(run(lambda lat: (lat.set_mrt(RATES), lat.set_trt(magic))), trt)
    mrt = run(lambda lat: lat.set_mrt(RATES))
    assert np.array_equal(run(lambda lat: (lat.set_trt(magic), lat.set_mrt(RATES))), mrt)
    lat = lbm.Lattice3D(m, tau, dtype="f64")
    for bad in ((0.0, 1, 1, 1, 1), (1, 1, 1, 2.0, 1), (1, 1, 1, 1, float("inf"))):
        with pytest.raises(lbm.LbmError) as e:
            lat.set_mrt(bad)
        assert e.value.status == -1
    lat.close()
