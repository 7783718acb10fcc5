"""D3Q19 parity at the benchmark size (256^3), on sampled outputs the oracle computes one by one,
for the layouts and collision models the benchmark times beyond the dense A-B BGK step: the
sphere packing (fluid fraction 0.4, walls in z, body force) on the fluid-node list and on the AA
layout, and the multiple-relaxation-time collision on the dense A-B layout.

After k steps a node's populations depend only on the initial state within distance k (a node
pulls from its direct neighbours), so the oracle, run on a periodic (2k + 1)^3 window centred on
a sampled node, reproduces that node exactly: the window's wrap-around error moves in from its
edge by one node per step.  Two steps, so that the AA layout runs both its even and its odd
kernel.  Tolerances as everywhere: FP64 max abs 1e-12, FP32 max relative 1e-5.
"""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce

pytestmark = pytest.mark.gpu

N = 256
STEPS = 2
SAMPLES = 200
G = (1e-5, -2e-5, 3e-5)
MRT = (1.19, 1.4, 1.2, 1.3, 1.2)  # s_e, s_eps, s_q, s_pi, s_m


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def spheres(oracle_mod):
    """The benchmark's 256^3 sphere packing at fluid fraction 0.4, random non-equilibrium
    populations on its fluid nodes."""
    m = synthetic.random_spheres3(N, 0.4)
    f0 = synthetic.random_populations(oracle_mod.constants3()[3], (N, N, N), seed=81, amp=0.05)
    f0 *= (m == 0)
    return m, f0


def _sampled_error(oracle_mod, got, m, f0, tau, dtype, seed, mrt=None):
    rng = np.random.default_rng(seed)
    fluid = np.flatnonzero(m == 0)
    worst = 0.0
    for flat in rng.choice(fluid, SAMPLES, replace=False):
        z, y, x = np.unravel_index(flat, m.shape)
        idx = [np.arange(a - STEPS, a + STEPS + 1) % N for a in (z, y, x)]
        wm = np.ascontiguousarray(m[np.ix_(*idx)])
        wf = np.ascontiguousarray(f0[(slice(None),) + np.ix_(*idx)])
        exp = oracle_mod.run3(wm, wf, tau, STEPS, g=G, mrt=mrt)[:, STEPS, STEPS, STEPS]
        val = got[:, z, y, x]
        err = np.abs(val - exp) if dtype == "f64" else np.abs(val - exp) / np.abs(exp)
        worst = max(worst, float(err.max()))
    return worst


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["indirect", "dense_aa"])
def test_spheres_256_sampled(lbm, oracle_mod, spheres, layout, dtype):
    m, f0 = spheres
    announce(f"d3q19 spheres {N}^3 phi=0.4 {layout} {dtype} sampled parity")
    lat = lbm.Lattice3D(m, 0.6, force=G, dtype=dtype, layout=layout)
    assert lat.info()["n_fluid"] == int((m == 0).sum())
    lat.set_populations(f0)
    lat.step(STEPS)
    got = lat.get_populations()
    lat.close()
    assert not np.any(got[:, m == 1])
    assert _sampled_error(oracle_mod, got, m, f0, 0.6, dtype, seed=82) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mrt_256_sampled(lbm, oracle_mod, dtype):
    """256^3 with 5 % random solids, the benchmark's MRT rates, dense A-B."""
    announce(f"d3q19 mrt {N}^3 dense_ab {dtype} sampled parity")
    m = synthetic.random_mask3(N, N, N, seed=83, solid_fraction=0.05)
    f0 = synthetic.random_populations(oracle_mod.constants3()[3], (N, N, N), seed=84, amp=0.05)
    f0 *= (m == 0)
    lat = lbm.Lattice3D(m, 0.8, force=G, dtype=dtype)
    lat.set_mrt(MRT)
    lat.set_populations(f0)
    lat.step(STEPS)
    got = lat.get_populations()
    lat.close()
    assert _sampled_error(oracle_mod, got, m, f0, 0.8, dtype, seed=85, mrt=MRT) <= TOL[dtype]
