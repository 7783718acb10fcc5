"""16-bit shifted storage (FP16 / BF16 deviations, FP32 arithmetic): accuracy against the FP64
path.  Parity unpinned: 16-bit storage is an approximation of the FP64 result, so its error
is measured and reported (printed), with only loose sanity bounds asserted.  The FP64 GPU
path it is compared with is itself pinned to the oracle by the parity tests."""
import numpy as np
import pytest

import synthetic
from gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


def _run(lbm, m, fields, tau, steps, dtype, layout, g=(0.0, 0.0)):
    lat = lbm.Lattice(m, tau, force=g, dtype=dtype, layout=layout)
    if fields is not None:
        lat.init_equilibrium(*fields)
    M0 = lat.mass()
    lat.step(steps)
    rho, ux, uy = lat.macroscopic()
    M1 = lat.mass()
    lat.close()
    return ux, uy, (M1 - M0) / M0


def _l2(a, b, c, d):
    return float(np.sqrt(((a - c) ** 2 + (b - d) ** 2).sum() / (c ** 2 + d ** 2).sum()))


@pytest.mark.parametrize("dtype,bound", [("f16s", 2e-2), ("bf16s", 1e-1), ("f32", 1e-4)])
def test_taylor_green_velocity_error(lbm, dtype, bound):
    """Velocity is a small difference of populations near 0.1, so the FP32 round-off random
    walk of the populations (~1e-7 absolute after 2000 steps) shows up as a few 1e-5 of
    relative velocity error; the populations themselves stay within 1e-6 relative."""
    announce(f"reduced precision taylor-green 512^2 {dtype}")
    n, steps = 512, 2000
    m = synthetic.all_fluid(n, n)
    fields = synthetic.taylor_green(n, 0.01)
    u64, v64, _ = _run(lbm, m, fields, 0.6, steps, "f64", "dense_ab")
    u, v, drift = _run(lbm, m, fields, 0.6, steps, dtype, "dense_ab")
    err = _l2(u, v, u64, v64)
    print(f"\n[reduced] taylor-green {n}^2 {steps} steps {dtype}: velocity L2 rel err {err:.3e}, "
          f"mass drift {drift:.3e}")
    assert np.isfinite(err) and err < bound


@pytest.mark.parametrize("dtype,bound", [("f16s", 1.0), ("bf16s", 1.0), ("f32", 1e-4)])
def test_porous_velocity_error(lbm, dtype, bound):
    """Porous discs, body force 1e-5: the flow's deviations from rest are tiny, so FP16
    deviations are partly subnormal and BF16 keeps only 8 bits: large errors are the finding."""
    announce(f"reduced precision porous 512^2 {dtype}")
    m, _ = synthetic.porous_discs(512, 0.5, rmin=4, rmax=24)
    u64, v64, _ = _run(lbm, m, None, 0.6, 2000, "f64", "indirect", g=(1e-5, 0.0))
    u, v, drift = _run(lbm, m, None, 0.6, 2000, dtype, "indirect", g=(1e-5, 0.0))
    err = _l2(u, v, u64, v64)
    print(f"\n[reduced] porous 512^2 phi=0.5 2000 steps {dtype}: velocity L2 rel err {err:.3e}, "
          f"mass drift {drift:.3e}")
    assert np.isfinite(err) and err < bound
