"""The LDS-staged dense A-B step on lattices large enough to select it, element by element.

The dense A-B launcher picks the LDS-staged segment kernel once a step moves at least
32 MiB (18 population planes of the padded lattice), the AA layout's odd step its LDS kernel
from 128 MiB; smaller lattices run the per-node kernels that the other parity tests cover.  Inside the segment kernel, whole all-interior
256-node row segments are staged through LDS (with the halo column on either side, which
wraps around the periodic x edge), and every other segment (solids or solid neighbours, open
boundary nodes, the row's partial last segment) takes the per-node path.

Geometry: solids only inside a box in the middle of the lattice (x in [260, 500),
y in [100, 700)), so that rows above and below it are all-interior up to the ragged last
segment (nx is no multiple of 256), while rows through it mix both paths; segment 0 of an
interior row reads its left halo from column nx - 1.

Compared with the FP64 oracle over the whole lattice after 12 steps: BGK with body force and
drag field, TRT, MRT, open boundaries between walls, and full-way walls (FP64 max abs 1e-12,
FP32 max relative 1e-5, as everywhere; wall slots included for full-way).  16-bit storage
(two rows per workgroup): bitwise equal to the indirect layout's kernel (one collision
function) at 2000 x 1901, whose last row pair holds a single row.  The AA layout's odd
step runs the same staging (its own kernel) and is compared with the oracle after 13 steps.
"""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce, fp_error, fp_error_w

pytestmark = pytest.mark.gpu

STEPS = 12
SHAPES = {"f64": (1000, 944), "f32": (1500, 1250)}
BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
RATES = (1.19, 1.4, 1.64)


def _step_bytes(nx, ny, dtype):
    pitch = (nx + 63) // 64 * 64
    return 18 * pitch * ny * BYTES[dtype]


def _selects_segment_kernel(nx, ny, dtype):
    """Both LDS kernels (A-B from 32 MiB per step, the odd AA step from 128 MiB)."""
    return _step_bytes(nx, ny, dtype) >= 128 * 2**20


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


def _box_mask(nx, ny, seed):
    rng = np.random.default_rng(seed)
    m = np.zeros((ny, nx), np.uint8)
    box = m[100:700, 260:500]
    box[...] = (rng.random(box.shape) < 0.2).astype(np.uint8)
    return m


def _setup(case, nx, ny):
    """(mask, bc, value, fields, alpha, g) of a case."""
    m = _box_mask(nx, ny, seed=31)
    fields = synthetic.random_fields(nx, ny, seed=17, rho_spread=0.02, u_amp=0.02)
    alpha = synthetic.brinkman_alpha(nx, ny, seed=9, sigma=6.0)
    g = (2e-5, -1e-5)
    bc = val = None
    if case == "open_walls":
        mc, bc, val = synthetic.open_channel(nx, ny, "velocity", u_in=0.05)
        m = np.maximum(m, mc)
        bc[m == 1] = 0
        val[:, m == 1] = 0.0
        alpha = None
    return m, bc, val, fields, alpha, g


def _run_gpu(lbm, case, m, bc, val, fields, alpha, g, dtype, layout="dense_ab", steps=STEPS):
    lat = lbm.Lattice(m, 0.7, force=g, dtype=dtype, layout=layout)
    if case == "trt":
        lat.set_trt(3.0 / 16.0)
    if case == "mrt":
        lat.set_mrt(RATES)
    if case == "fullway":
        lat.set_bounce_back("fullway")
    if bc is not None:
        lat.set_boundaries(bc, val)
    lat.init_equilibrium(*fields)
    if alpha is not None:
        lat.set_porosity(alpha)
    lat.step(steps)
    f = lat.get_populations()
    lat.close()
    return f


def _run_oracle(oracle_mod, case, m, bc, val, fields, alpha, g, steps=STEPS):
    f0 = oracle_mod.init(m, *fields, bc=bc, value=val)
    if case == "fullway":
        f0 = oracle_mod.fullway_fill(m, f0)
    a64 = None if alpha is None else np.asarray(alpha, np.float32).astype(np.float64)
    kw = {}
    if case == "trt":
        kw["tau_minus"] = oracle_mod.trt_tau_minus(0.7, 3.0 / 16.0)
    if case == "mrt":
        kw["mrt"] = RATES
    return oracle_mod.run(m, f0, 0.7, steps, g=g, alpha=a64, bc=bc, value=val,
                          fullway=case == "fullway", **kw)


def _fullway_error(got, ref, m, dtype):
    sel = np.broadcast_to(m[None] == 0, ref.shape) | ((m[None] == 1) & (ref != 0))
    a, b = got[sel], ref[sel]
    if dtype == "f64":
        return float(np.abs(a - b).max())
    return float((np.abs(a - b) / np.abs(b)).max())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["force_drag", "trt", "mrt", "open_walls", "fullway"])
def test_segment_kernel_vs_oracle(lbm, oracle_mod, dtype, case):
    nx, ny = SHAPES[dtype]
    assert _selects_segment_kernel(nx, ny, dtype)
    announce(f"segment kernel {nx}x{ny} {dtype} {case}")
    m, bc, val, fields, alpha, g = _setup(case, nx, ny)
    got = _run_gpu(lbm, case, m, bc, val, fields, alpha, g, dtype)
    ref = _run_oracle(oracle_mod, case, m, bc, val, fields, alpha, g)
    if case == "fullway":
        err = _fullway_error(got, ref, m, dtype)
    elif case == "open_walls":
        err = fp_error_w(got, ref, m, dtype)
    else:
        err = fp_error(got, ref, m, dtype)
    print(f"max error {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype,shape", [("f64", (700, 400)), ("f32", (1000, 600))])
@pytest.mark.parametrize("case", ["force_drag", "open_walls"])
def test_segment_kernel_mid_size(lbm, oracle_mod, dtype, shape, case):
    """Lattices between the two switches (32 to 128 MiB per step): the A-B step through LDS.
    At ny = 400 / 600 the solid box is cut at the lattice's last row."""
    nx, ny = shape
    assert 32 * 2**20 <= _step_bytes(nx, ny, dtype) < 128 * 2**20
    announce(f"segment kernel mid-size {nx}x{ny} {dtype} {case}")
    m, bc, val, fields, alpha, g = _setup(case, nx, ny)
    got = _run_gpu(lbm, case, m, bc, val, fields, alpha, g, dtype)
    ref = _run_oracle(oracle_mod, case, m, bc, val, fields, alpha, g)
    err = (fp_error_w if case == "open_walls" else fp_error)(got, ref, m, dtype)
    print(f"max error {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["force_drag", "mrt", "open_walls"])
def test_segment_kernel_aa_vs_oracle(lbm, oracle_mod, dtype, case):
    """The AA layout's odd step through LDS (the same segment staging, reading A_opp(i) from
    x - c_i, writing A_i(x + c_i)) on the same geometry, 13 steps (ending on an odd step)."""
    nx, ny = SHAPES[dtype]
    assert _selects_segment_kernel(nx, ny, dtype)
    announce(f"segment kernel AA {nx}x{ny} {dtype} {case}")
    m, bc, val, fields, alpha, g = _setup(case, nx, ny)
    got = _run_gpu(lbm, case, m, bc, val, fields, alpha, g, dtype, layout="dense_aa", steps=13)
    ref = _run_oracle(oracle_mod, case, m, bc, val, fields, alpha, g, steps=13)
    err = (fp_error_w if case == "open_walls" else fp_error)(got, ref, m, dtype)
    print(f"max error {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
@pytest.mark.parametrize("case", ["force_drag", "trt", "mrt", "open_walls"])
def test_segment_kernel_16bit_bitwise(lbm, dtype, case):
    nx, ny = 2000, 1901  # odd: the last row pair of the two-row kernel has one row
    assert _selects_segment_kernel(nx, ny, dtype)
    announce(f"segment kernel {nx}x{ny} {dtype} {case} bitwise vs indirect")
    m, bc, val, fields, alpha, g = _setup(case, nx, ny)
    out = [_run_gpu(lbm, case, m, bc, val, fields, alpha, g, dtype, layout)
           for layout in ("dense_ab", "indirect")]
    assert np.array_equal(out[0], out[1])
