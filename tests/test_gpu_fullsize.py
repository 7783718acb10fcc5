"""Parity at the full benchmark sizes, on sampled outputs the oracle computes one by one.

After k steps a node's populations depend only on the initial state within distance k (one
node per step), so the oracle, run on a periodic 48 x 48 window centred on a sampled node,
reproduces that node exactly for k <= 11 steps (the window's own wrap-around error travels in
from its edge by one node per step and stays at least 13 nodes away).  Tolerances as
everywhere: FP64 max abs 1e-12, FP32 max relative 1e-5.

Every layout the benchmark times at 4096^2 is sampled in the configuration it is timed in:
the dense A-B and AA steps on the Taylor-Green vortex (AA after an odd step count, whose
canonical view is the gather of reversed slots), and the dense, tiled and indirect steps on
the porous discs at fluid fraction 0.5 with body force (about 51 k kept tiles, the XCD remap
over them and the tile-neighbour table at full size).
"""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce

pytestmark = pytest.mark.gpu

STEPS = 10
HALF = 24


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def porous_mask():
    m, info = synthetic.porous_discs(4096, 0.5)
    return m


def _window(a, y, x):
    n = a.shape[-1]
    ys = np.arange(y - HALF, y + HALF) % a.shape[-2]
    xs = np.arange(x - HALF, x + HALF) % n
    return a[..., ys[:, None], xs[None, :]]


def _check_samples(oracle_mod, f_gpu, mask, fields, tau, g, dtype, seed, n_samples=16,
                   steps=STEPS):
    assert steps <= HALF // 2
    rng = np.random.default_rng(seed)
    fluid = np.argwhere(mask == 0)
    worst = 0.0
    for (y, x) in fluid[rng.choice(len(fluid), n_samples, replace=False)]:
        mw = np.ascontiguousarray(_window(mask, y, x))
        fw = [None if a is None else np.ascontiguousarray(_window(a, y, x)) for a in fields]
        ref = oracle_mod.run(mw, oracle_mod.init(mw, *fw), tau, steps, g=g)[:, HALF, HALF]
        got = f_gpu[:, y, x]
        err = np.abs(got - ref).max() if dtype == "f64" else (np.abs(got - ref) / np.abs(ref)).max()
        worst = max(worst, float(err))
    return worst


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_taylor_green_4096_bench_config(lbm, oracle_mod, dtype):
    """The benchmark's workload and launch configuration: 4096^2 Taylor-Green, dense A-B."""
    announce(f"taylor-green 4096^2 {dtype} dense_ab sampled parity")
    n = 4096
    m = synthetic.all_fluid(n, n)
    fields = synthetic.taylor_green(n, 0.01)
    lat = lbm.Lattice(m, 0.6, dtype=dtype, layout="dense_ab")
    lat.init_equilibrium(*fields)
    M0 = lat.mass()
    lat.step(STEPS)
    f = lat.get_populations()
    M1 = lat.mass()
    lat.close()
    worst = _check_samples(oracle_mod, f, m, fields, 0.6, (0.0, 0.0), dtype, seed=1)
    assert worst <= TOL[dtype]
    assert abs(M1 - M0) / M0 < (1e-13 if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_taylor_green_4096_aa_odd(lbm, oracle_mod, dtype):
    """AA layout at 4096^2 after an odd number of steps (the last step is an odd-step
    kernel writing to the neighbours' slots; the canonical view gathers reversed slots)."""
    announce(f"taylor-green 4096^2 {dtype} dense_aa 11 steps sampled parity")
    n, steps = 4096, 11
    m = synthetic.all_fluid(n, n)
    fields = synthetic.taylor_green(n, 0.01)
    lat = lbm.Lattice(m, 0.6, dtype=dtype, layout="dense_aa")
    lat.init_equilibrium(*fields)
    lat.step(steps)
    f = lat.get_populations()
    lat.close()
    worst = _check_samples(oracle_mod, f, m, fields, 0.6, (0.0, 0.0), dtype, seed=5,
                           steps=steps)
    assert worst <= TOL[dtype]


@pytest.mark.parametrize("layout", ["dense_ab", "tiled16", "indirect"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_porous_4096(lbm, oracle_mod, porous_mask, dtype, layout):
    """4096^2 porous discs at fluid fraction 0.5 with body force, in each sparse-capable
    layout the benchmark times (dense with solid lanes skipped, tiled, indirect)."""
    announce(f"porous 4096^2 phi=0.5 {dtype} {layout} sampled parity")
    m = porous_mask
    g = (1e-6, 0.0)
    lat = lbm.Lattice(m, 0.6, force=g, dtype=dtype, layout=layout)
    lat.step(STEPS)
    f = lat.get_populations()
    lat.close()
    seed = {"dense_ab": 3, "tiled16": 4, "indirect": 2}[layout]
    worst = _check_samples(oracle_mod, f, m, (None, None, None), 0.6, g, dtype, seed=seed,
                           n_samples=24)
    assert worst <= TOL[dtype]


def test_porous_4096_mass_conservation(lbm, porous_mask):
    """Exact mass conservation (to FP64 rounding) over 200 steps of the full porous case,
    tiled layout, FP64."""
    announce("porous 4096^2 phi=0.5 f64 tiled16 mass")
    m = porous_mask
    lat = lbm.Lattice(m, 0.6, force=(1e-6, 0.0), dtype="f64", layout="tiled16")
    M0 = lat.mass()
    lat.step(200)
    M1 = lat.mass()
    lat.close()
    assert M0 == pytest.approx(float((m == 0).sum()), rel=1e-13)
    assert abs(M1 - M0) / M0 < 1e-12
