"""The LDS-staged D3Q19 dense A-B step on lattices large enough to select it, element by element.

The D3Q19 dense A-B launcher picks the LDS-staged segment kernel once a step moves at least
128 MiB (38 population planes of the padded lattice); smaller lattices run the per-node kernel
that the other D3Q19 tests cover.  Inside the segment kernel, whole all-interior 256-node row
segments are staged through LDS (nineteen runs from the nine rows (y +- 1, z +- 1), with the
halo column on either side, which wraps around the periodic x edge), and every other segment
(solids or solid neighbours, or the row's partial last segment) takes the per-node path.

Geometry: nx = 300 (segment 0 whole, segment 1 the ragged tail of 44 nodes); random solids only
inside a box (x in [100, 200), y in [10, 30), z in [10, 25)), so that most rows are
all-interior while rows through the box mix both paths.  Compared with the FP64 D3Q19 oracle
over the whole lattice after 5 steps: BGK with a body force along all three axes, TRT, MRT and
full-way walls (FP64 max abs 1e-12, FP32 max relative 1e-5, as everywhere; wall slots included
for full-way).  16-bit storage: bitwise equal to the node-list layout (one collision function).
The AA layout's odd step runs the same staging (its own kernel): oracle parity after an odd
step count, and 16-bit bitwise equality with the node list.  16-bit MRT stages two y rows per
workgroup (its own kernel); an odd ny case covers the single last row.
"""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce, fp_error

pytestmark = pytest.mark.gpu

STEPS = 5
SHAPES = {"f64": (300, 48, 40), "f32": (300, 64, 48), "f16s": (300, 96, 64),
          "bf16s": (300, 96, 64)}
BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
MRT = (1.19, 1.4, 1.64, 1.3, 1.55)
G = (2e-5, -1e-5, 1e-5)


def _selects_segment_kernel(nx, ny, nz, dtype):
    pitch = (nx + 63) // 64 * 64
    return 38 * pitch * ny * nz * BYTES[dtype] >= 128 * 2**20


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


def _setup(shape):
    nx, ny, nz = shape
    rng = np.random.default_rng(91)
    m = np.zeros((nz, ny, nx), np.uint8)
    m[10:25, 10:30, 100:200] = (rng.random((15, 20, 100)) < 0.2).astype(np.uint8)
    fields = synthetic.random_fields3(nx, ny, nz, seed=92)
    return m, fields


def _model(lat, case):
    if case == "trt":
        lat.set_trt(0.25)
    elif case == "mrt":
        lat.set_mrt(MRT)
    elif case == "fullway":
        lat.set_bounce_back("fullway")


def _run_gpu(lbm, m, fields, dtype, case, layout="dense_ab"):
    lat = lbm.Lattice3D(m, 0.7, force=G, dtype=dtype, layout=layout)
    _model(lat, case)
    lat.init_equilibrium(*fields)
    lat.step(STEPS)
    f = lat.get_populations()
    lat.close()
    return f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["bgk_force", "trt", "mrt", "fullway"])
def test_segment3_vs_oracle(lbm, oracle_mod, dtype, case):
    shape = SHAPES[dtype]
    assert _selects_segment_kernel(*shape, dtype)
    announce(f"d3q19 segment kernel {shape} {dtype} {case}")
    m, fields = _setup(shape)
    got = _run_gpu(lbm, m, fields, dtype, case)
    f0 = oracle_mod.init3(m, *fields)
    kw = {}
    if case == "fullway":
        f0 = oracle_mod.fullway_fill3(m, f0)
        kw["fullway"] = True
    if case == "trt":
        kw["tau_minus"] = oracle_mod.trt_tau_minus(0.7, 0.25)
    if case == "mrt":
        kw["mrt"] = MRT
    ref = oracle_mod.run3(m, f0, 0.7, STEPS, g=G, **kw)
    if case == "fullway":
        sel = (m[None] == 0) | (ref != 0)
        a, b = got[sel], ref[sel]
        err = float(np.abs(a - b).max() if dtype == "f64" else (np.abs(a - b) / np.abs(b)).max())
    else:
        err = fp_error(got, ref, m, dtype)
    print(f"max error {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["bgk_force", "trt"])
def test_segment3_aa_vs_oracle(lbm, oracle_mod, dtype, case):
    """The AA layout's odd step through LDS (reads A_opp(i) from x - c_i, writes A_i(x + c_i)),
    5 steps (ending on an odd step, whose canonical view is the odd read)."""
    shape = SHAPES[dtype]
    assert _selects_segment_kernel(*shape, dtype)
    announce(f"d3q19 segment kernel AA {shape} {dtype} {case}")
    m, fields = _setup(shape)
    got = _run_gpu(lbm, m, fields, dtype, case, layout="dense_aa")
    kw = {"tau_minus": oracle_mod.trt_tau_minus(0.7, 0.25)} if case == "trt" else {}
    ref = oracle_mod.run3(m, oracle_mod.init3(m, *fields), 0.7, STEPS, g=G, **kw)
    err = fp_error(got, ref, m, dtype)
    print(f"max error {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
@pytest.mark.parametrize("case", ["bgk_force", "mrt", "aa"])
def test_segment3_16bit_bitwise(lbm, dtype, case):
    shape = SHAPES[dtype]
    assert _selects_segment_kernel(*shape, dtype)
    announce(f"d3q19 segment kernel {shape} {dtype} {case} bitwise vs node list")
    m, fields = _setup(shape)
    a = _run_gpu(lbm, m, fields, dtype, case, layout="dense_aa" if case == "aa" else "dense_ab")
    b = _run_gpu(lbm, m, fields, dtype, case, layout="indirect")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
def test_segment3_16bit_mrt_two_rows_odd_ny(lbm, dtype):
    """16-bit MRT on a mostly interior lattice runs two y rows per workgroup; with ny odd the
    last row of every z plane is a pair of one (per-node path).  Bitwise equal to the node list."""
    shape = (300, 97, 64)
    assert _selects_segment_kernel(*shape, dtype)
    announce(f"d3q19 two-row segment kernel {shape} {dtype} mrt bitwise vs node list")
    m, fields = _setup(shape)
    a = _run_gpu(lbm, m, fields, dtype, "mrt", layout="dense_ab")
    b = _run_gpu(lbm, m, fields, dtype, "mrt", layout="indirect")
    assert np.array_equal(a, b)

