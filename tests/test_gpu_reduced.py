"""Reduced-precision storage (FP32 deviations, FP16 / BF16 shifted deviations, FP32
arithmetic) against the FP64 oracle.

16-bit storage approximates the FP64 result rather than reaching it, so its accuracy is a
measured figure: each bound below sits about 3x above the error measured on MI355X (printed
by the test), so that a change in the storage rounding, the shift or the collision arithmetic
shows up.  Cases: the 256^2 Taylor-Green vortex (tau = 0.6, u0 = 0.01) and 256^2 porous discs
(fluid fraction 0.5, radii 4-16, tau = 0.6, body force g_x = 1e-6, where the FP16 deviations
of the moving populations are mostly subnormal), 5000 steps each, the step count of the
reduced-precision benchmark; dense A-B for the vortex, the tiled layout for the discs.
Reported: relative L2 error of the velocity field over the fluid nodes, and the relative mass
drift (exact in FP64 up to rounding; the 16-bit roundings break it).
"""
import numpy as np
import pytest

import synthetic
from gpu_util import announce

pytestmark = pytest.mark.gpu

STEPS = 5000
N = 256

# (case, dtype) -> (velocity L2 bound, |mass drift| bound), about 3x the values measured on
# MI355X: Taylor-Green f32 6.2e-5 / 3.4e-9, f16s 1.74e-2 / 1.1e-5, bf16s 1.80e-2 / 1.2e-4;
# porous f32 2.8e-6 / 1.2e-10, f16s 5.4e-3 / 7.5e-7, bf16s 4.9e-3 / 4.3e-8
BOUNDS = {
    ("tgv", "f32"): (2e-4, 1e-8),
    ("tgv", "f16s"): (5e-2, 3e-5),
    ("tgv", "bf16s"): (5e-2, 4e-4),
    ("porous", "f32"): (1e-5, 4e-10),
    ("porous", "f16s"): (1.6e-2, 2.5e-6),
    ("porous", "bf16s"): (1.5e-2, 1.5e-7),
}


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


def case_setup(case):
    """(mask, initial fields or None, tau, g, layout) of a case."""
    if case == "tgv":
        return synthetic.all_fluid(N, N), synthetic.taylor_green(N, 0.01), 0.6, (0.0, 0.0), \
            "dense_ab"
    m, _ = synthetic.porous_discs(N, 0.5, rmin=4, rmax=16)
    return m, None, 0.6, (1e-6, 0.0), "tiled16"


_ORACLE = {}


def oracle_velocity(oracle_mod, case):
    """The oracle's (u_x, u_y) after STEPS steps (computed once per case)."""
    if case not in _ORACLE:
        m, fields, tau, g, _ = case_setup(case)
        f0 = oracle_mod.init(m, *fields) if fields is not None else oracle_mod.init(m)
        f = oracle_mod.run(m, f0, tau, STEPS, g=g)
        _, ux, uy = oracle_mod.macroscopic(m, f, g=g)
        _ORACLE[case] = (ux, uy)
    return _ORACLE[case]


def l2_rel(ux, uy, rx, ry, fluid):
    num = ((ux - rx) ** 2 + (uy - ry) ** 2)[fluid].sum()
    den = (rx ** 2 + ry ** 2)[fluid].sum()
    return float(np.sqrt(num / den))


def reduced_error(lbm, oracle_mod, case, dtype):
    """(velocity L2 error against the oracle, relative mass drift) of `dtype` storage."""
    m, fields, tau, g, layout = case_setup(case)
    lat = lbm.Lattice(m, tau, force=g, dtype=dtype, layout=layout)
    if fields is not None:
        lat.init_equilibrium(*fields)
    M0 = lat.mass()
    lat.step(STEPS)
    _, ux, uy = lat.macroscopic()
    M1 = lat.mass()
    lat.close()
    rx, ry = oracle_velocity(oracle_mod, case)
    return l2_rel(ux, uy, rx, ry, m == 0), (M1 - M0) / M0


@pytest.mark.parametrize("dtype", ["f32", "f16s", "bf16s"])
@pytest.mark.parametrize("case", ["tgv", "porous"])
def test_reduced_storage_against_oracle(lbm, oracle_mod, case, dtype):
    announce(f"reduced precision {case} {N}^2 {STEPS} steps {dtype} vs oracle")
    err, drift = reduced_error(lbm, oracle_mod, case, dtype)
    print(f"\n[reduced] {case} {N}^2 {STEPS} steps {dtype}: velocity L2 rel err vs oracle "
          f"{err:.3e}, mass drift {drift:.3e}")
    eb, mb = BOUNDS[(case, dtype)]
    assert np.isfinite(err) and err <= eb
    assert abs(drift) <= mb


def test_fp64_reaches_oracle(lbm, oracle_mod):
    """The FP64 path on the same cases agrees with the oracle to rounding (the reference the
    reduced-precision errors are read against)."""
    for case in ("tgv", "porous"):
        announce(f"reduced precision reference {case} f64")
        err, drift = reduced_error(lbm, oracle_mod, case, "f64")
        assert err <= 1e-10
        assert abs(drift) <= 1e-12
