"""GPU parity: every layout x storage type of the HIP library against the FP64 oracle.

Tolerances (written here, applied to canonical populations at fluid slots):
  FP64: max |f_gpu - f_oracle| <= 1e-12;   FP32: max |f_gpu - f_oracle| / |f_oracle| <= 1e-5.
Layout variants of the same storage type must agree bitwise (one collision function).
"""
import numpy as np
import pytest

import synthetic
from gpu_util import TOL, announce, fp_error

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


def run_gpu(lbm, mask, tau, steps, dtype, layout, g=(0.0, 0.0), alpha=None, fields=None):
    lat = lbm.Lattice(mask, tau, force=g, dtype=dtype, layout=layout)
    if fields is not None:
        lat.init_equilibrium(*fields)
    if alpha is not None:
        lat.set_porosity(alpha)
    lat.step(steps)
    f = lat.get_populations()
    lat.close()
    return f


def run_oracle(oracle_mod, mask, tau, steps, g=(0.0, 0.0), alpha=None, fields=None):
    f0 = oracle_mod.init(mask, *(fields or (None, None, None)))
    a64 = None if alpha is None else np.asarray(alpha, np.float32).astype(np.float64)
    return oracle_mod.run(mask, f0, tau, steps, g=g, alpha=a64)


# --------------------------------------------------------------- channel --
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_channel_2000_steps_vs_oracle(lbm, oracle_mod, dtype):
    """256 x 64 body-force channel, walls at y = 0 and 63, tau = 0.8, g_x = 1e-6, from
    rest, 2000 steps (the full correctness configuration)."""
    announce(f"channel 256x64 2000 steps {dtype}")
    m = synthetic.channel_mask(256, 64)
    ref = run_oracle(oracle_mod, m, 0.8, 2000, g=(1e-6, 0.0))
    got = run_gpu(lbm, m, 0.8, 2000, dtype, "dense_ab", g=(1e-6, 0.0))
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_porous_all_layouts_vs_oracle(lbm, oracle_mod, dtype, layout):
    """256^2 porous discs (r 4-16, fluid fraction 0.5), walls, body force and a drag field,
    random initial fields, 150 steps (an odd count, so AA ends on an odd step)."""
    announce(f"porous 256 {dtype} {layout}")
    m, _ = synthetic.porous_discs(256, 0.5, rmin=4, rmax=16)
    alpha = synthetic.brinkman_alpha(256, 256, seed=3, sigma=6.0)
    fields = synthetic.random_fields(256, 256, seed=8, rho_spread=0.02, u_amp=0.02)
    g = (2e-5, -1e-5)
    ref = run_oracle(oracle_mod, m, 0.7, 151, g=g, alpha=alpha, fields=fields)
    got = run_gpu(lbm, m, 0.7, 151, dtype, layout, g=g, alpha=alpha, fields=fields)
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["dense_ab", "dense_aa", "indirect"])
@pytest.mark.parametrize("shape", [(300, 37), (1, 5), (65, 1), (257, 70)])
def test_ragged_shapes(lbm, oracle_mod, dtype, layout, shape):
    """Sizes that are not multiples of the 64-element pitch or the 256-lane block, and
    degenerate 1-wide lattices, with random solids (bounce-back everywhere)."""
    nx, ny = shape
    announce(f"ragged {nx}x{ny} {dtype} {layout}")
    m = synthetic.random_mask(nx, ny, seed=nx * 7 + ny, solid_fraction=0.2)
    fields = synthetic.random_fields(nx, ny, seed=5)
    ref = run_oracle(oracle_mod, m, 0.9, 41, g=(1e-4, 2e-5), fields=fields)
    got = run_gpu(lbm, m, 0.9, 41, dtype, layout, g=(1e-4, 2e-5), fields=fields)
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(48, 32), (272, 80)])
def test_tiled_shapes(lbm, oracle_mod, dtype, shape):
    """Tiled layout on multiples of 16 with random solids and empty tiles."""
    nx, ny = shape
    announce(f"tiled {nx}x{ny} {dtype}")
    m = synthetic.random_mask(nx, ny, seed=nx + ny, solid_fraction=0.25)
    m[:, 16:32] = 1  # a column of empty tiles
    fields = synthetic.random_fields(nx, ny, seed=6)
    ref = run_oracle(oracle_mod, m, 0.9, 33, g=(1e-4, 0.0), fields=fields)
    got = run_gpu(lbm, m, 0.9, 33, dtype, "tiled16", g=(1e-4, 0.0), fields=fields)
    assert fp_error(got, ref, m, dtype) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_taylor_green_256(lbm, oracle_mod, dtype):
    announce(f"taylor-green 256 {dtype}")
    m = synthetic.all_fluid(256, 256)
    fields = synthetic.taylor_green(256, 0.01)
    ref = run_oracle(oracle_mod, m, 0.6, 200, fields=fields)
    for layout in ("dense_ab", "dense_aa"):
        got = run_gpu(lbm, m, 0.6, 200, dtype, layout, fields=fields)
        assert fp_error(got, ref, m, dtype) <= TOL[dtype]


# --------------------------------------------------------- exact rationals --
@pytest.mark.parametrize("case", [0, 2])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_exact_rational_4x4(lbm, layout, case):
    """The periodic and the walled-with-force 4x4 exact-rational cases, 3 steps, FP64 GPU
    within 1e-15 of the exact value (tiled needs 16-multiples, so the 4x4 lattice is
    repeated 4 x 4 times, which leaves a periodic solution unchanged).  The drag case
    is below with FP32-exact coefficients (the GPU stores alpha in FP32)."""
    from fractions import Fraction as Fr

    from oracle import exact
    from test_oracle_pins import _exact_case
    announce(f"exact 4x4 case {case} {layout}")
    mask, rho, ux, uy, g, alpha = _exact_case(case)
    ex = exact.run(mask, rho, ux, uy, Fr(4, 5), 3, g=g, alpha=alpha)
    tofl = lambda a: np.array([[float(v) for v in row] for row in a])
    m = np.array(mask, dtype=np.uint8)
    rep = 4 if layout.startswith("tiled16") else 1
    M = np.tile(m, (rep, rep))
    F = [np.tile(tofl(a), (rep, rep)) for a in (rho, ux, uy)]
    got = run_gpu(lbm, M, 0.8, 3, "f64", layout, g=(float(g[0]), float(g[1])), fields=F)
    worst = 0.0
    for (x, y), pops in ex.items():
        for i in range(9):
            worst = max(worst, abs(got[i, y, x] - float(pops[i])))
    assert worst < 1e-15


@pytest.mark.parametrize("layout", ["dense_ab", "dense_aa", "indirect"])
def test_exact_rational_drag_fp32_alpha(lbm, layout):
    """Drag case with alpha values exact in FP32 (multiples of 1/8): FP64 GPU vs the
    exact rational result."""
    from fractions import Fraction as Fr

    from oracle import exact
    announce("exact 4x4 drag with FP32-exact alpha")
    rng = np.random.default_rng(77)
    nx = ny = 4
    mask = [[0] * nx for _ in range(ny)]
    mask[2][1] = 1
    alpha = [[Fr(int(rng.integers(0, 9)), 8) for _ in range(nx)] for _ in range(ny)]
    rho = [[Fr(95 + int(rng.integers(0, 11)), 100) for _ in range(nx)] for _ in range(ny)]
    ux = [[Fr(int(rng.integers(-4, 5)), 100) for _ in range(nx)] for _ in range(ny)]
    uy = [[Fr(int(rng.integers(-4, 5)), 100) for _ in range(nx)] for _ in range(ny)]
    g = (Fr(1, 500), Fr(-1, 1000))
    ex = exact.run(mask, rho, ux, uy, Fr(4, 5), 3, g=g, alpha=alpha)
    tofl = lambda a: np.array([[float(v) for v in row] for row in a])
    got = run_gpu(lbm, np.array(mask, np.uint8), 0.8, 3, "f64", layout,
                  g=(float(g[0]), float(g[1])), alpha=tofl(alpha),
                  fields=[tofl(rho), tofl(ux), tofl(uy)])
    worst = max(abs(got[i, y, x] - float(p[i])) for (x, y), p in ex.items() for i in range(9))
    assert worst < 1e-15


# ------------------------------------------------------- layout agreement --
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s", "bf16s"])
def test_layouts_bitwise_equal(lbm, dtype):
    """A-B, AA (after even and odd step counts), tiled and indirect give bitwise-equal
    canonical populations on the same porous lattice."""
    announce(f"layouts bitwise {dtype}")
    m, _ = synthetic.porous_discs(128, 0.6, rmin=4, rmax=12)
    fields = synthetic.random_fields(128, 128, seed=12, rho_spread=0.02, u_amp=0.02)
    alpha = synthetic.brinkman_alpha(128, 128, seed=5, sigma=4.0)
    for steps in (40, 41):
        ref = run_gpu(lbm, m, 0.75, steps, dtype, "dense_ab", g=(1e-5, 0.0), alpha=alpha,
                      fields=fields)
        for layout in ("dense_aa", "tiled16", "indirect", "tiled16_all"):
            got = run_gpu(lbm, m, 0.75, steps, dtype, layout, g=(1e-5, 0.0), alpha=alpha,
                          fields=fields)
            assert np.array_equal(got, ref), (layout, steps)


# ----------------------------------------------------------- state / views --
@pytest.mark.parametrize("layout", LAYOUTS)
def test_populations_roundtrip(lbm, layout):
    """set_populations then get_populations returns the canonical state exactly (FP64),
    at step 0 and after an odd number of steps (AA odd view)."""
    announce(f"roundtrip {layout}")
    m = synthetic.random_mask(64, 48, seed=1, solid_fraction=0.2)
    rng = np.random.default_rng(0)
    f = np.where(m[None] == 0, 0.05 + 0.1 * rng.random((9, 48, 64)), 0.0)
    lat = lbm.Lattice(m, 0.8, dtype="f64", layout=layout)
    for steps in (0, 3):
        lat.step(steps)
        lat.set_populations(f)
        assert np.array_equal(lat.get_populations(), f)
    lat.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_macroscopic_and_mass(lbm, oracle_mod, layout):
    announce(f"macroscopic {layout}")
    m, _ = synthetic.porous_discs(64, 0.6, rmin=3, rmax=8)
    fields = synthetic.random_fields(64, 64, seed=2)
    alpha = synthetic.brinkman_alpha(64, 64, seed=1, sigma=3.0)
    g = (1e-4, 0.0)
    lat = lbm.Lattice(m, 0.7, force=g, dtype="f64", layout=layout)
    lat.init_equilibrium(*fields)
    lat.set_porosity(alpha)
    M0 = lat.mass()
    lat.step(25)
    rho, ux, uy = lat.macroscopic()
    a64 = alpha.astype(np.float32).astype(np.float64)
    fref = run_oracle(oracle_mod, m, 0.7, 25, g=g, alpha=alpha, fields=fields)
    r2, u2, v2 = oracle_mod.macroscopic(m, fref, g=g, alpha=a64)
    assert np.abs(rho - r2).max() < 1e-12
    assert np.abs(ux - u2).max() < 1e-12
    assert np.abs(uy - v2).max() < 1e-12
    assert np.all(rho[m == 1] == 0)
    assert abs(lat.mass() - M0) / M0 < 1e-13
    assert lat.mass() == pytest.approx(fref.sum(), rel=1e-13)
    lat.close()


def test_state_save_load_bitwise(lbm):
    import torch
    announce("save/load")
    m = synthetic.channel_mask(128, 32)
    lat = lbm.Lattice(m, 0.8, force=(1e-5, 0), dtype="f32", layout="dense_ab")
    lat.step(10)
    buf = torch.empty(lat.state_bytes(), dtype=torch.uint8, device="cuda")
    lat.save_state(buf)
    lat.step(17)
    a = lat.get_populations()
    lat.load_state(buf)
    lat.step(17)
    assert np.array_equal(lat.get_populations(), a)
    lat.close()


def test_objective_matches_oracle(lbm, oracle_mod):
    announce("objective")
    m = synthetic.channel_mask(96, 24)
    alpha = synthetic.brinkman_alpha(96, 24, seed=7, sigma=3.0)
    lat = lbm.Lattice(m, 0.8, force=(1e-5, 0.0), dtype="f64", layout="dense_ab")
    lat.set_porosity(alpha)
    lat.step(300)
    J = lat.objective_outlet_ux(95)
    a64 = alpha.astype(np.float32).astype(np.float64)
    fref = run_oracle(oracle_mod, m, 0.8, 300, g=(1e-5, 0.0), alpha=alpha)
    Jref = oracle_mod.objective_outlet_ux(m, fref, 95, g=(1e-5, 0.0), alpha=a64)
    assert J == pytest.approx(Jref, rel=1e-12)
    lat.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_graph_replay_bitwise(lbm, layout):
    """Steps replayed through captured HIP graphs give bitwise the same populations as steps
    launched one by one, across odd step counts, a force change and a drag change mid-run."""
    announce(f"graph replay {layout}")
    m = synthetic.random_mask(96, 48, seed=21, solid_fraction=0.2)
    alpha = synthetic.brinkman_alpha(96, 48)
    runs = []
    for gsteps in (0, 4, -1):
        lat = lbm.Lattice(m, 0.7, force=(1e-4, 0.0), dtype="f64", layout=layout)
        lat.set_graph_steps(gsteps)
        lat.step(37)
        lat.set_force((2e-4, 1e-5))
        lat.step(41)
        lat.set_porosity(alpha)
        lat.step(9)
        lat.step(64)
        runs.append(lat.get_populations())
        assert lat.info()["time_step"] == 151
        lat.close()
    assert np.array_equal(runs[0], runs[1])
    assert np.array_equal(runs[0], runs[2])


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
@pytest.mark.parametrize("case", ["plain", "force_drag", "trt_open"])
def test_dense_row_pairs_16bit(lbm, dtype, case):
    """The 16-bit dense A-B step runs two rows per workgroup (both rows' loads issued before
    either is computed when both segments are all-interior and the wave is full, else the two
    rows one after the other).  Bitwise equal to the indirect layout's kernel on a 600 x 77
    lattice (odd row count, a ragged last wave) whose solids fill only x < 200, so that
    all-interior segments and segments with solids alternate between row pairs."""
    announce(f"dense row pairs {dtype} {case}")
    nx, ny = 600, 77
    rng = np.random.default_rng(21)
    m = np.zeros((ny, nx), np.uint8)
    m[:, :200] = (rng.random((ny, 200)) < 0.15).astype(np.uint8)
    m[::5, 250] = 1  # a few rows whose second segment is not all-interior
    fields = synthetic.random_fields(nx, ny, seed=4, rho_spread=0.02, u_amp=0.02)
    out = []
    for layout in ("dense_ab", "indirect"):
        g = (1e-5, -2e-6) if case != "plain" else (0.0, 0.0)
        lat = lbm.Lattice(m, 0.7, force=g, dtype=dtype, layout=layout)
        if case == "force_drag":
            lat.set_porosity(synthetic.brinkman_alpha(nx, ny, seed=2, sigma=4.0))
        if case == "trt_open":
            lat.set_trt(3.0 / 16.0)
            bc = np.zeros((ny, nx), np.uint8)
            val = np.zeros((2, ny, nx))
            col = (m[:, nx - 1] == 0)
            bc[col, nx - 1] = synthetic.BC_PRESSURE[(-1, 0)]
            val[0, col, nx - 1] = 1.0
            lat.set_boundaries(bc, val)
        lat.init_equilibrium(*fields)
        lat.step(23)
        out.append(lat.get_populations())
        lat.close()
    assert np.array_equal(out[0], out[1])
