"""The sparse-study geometries of Sec. 4.3 (regular 8 x 8 circle arrays and random circles with
r in [8, 256] on n x n, walls at the top and bottom, constant-pressure inlet and outlet) and
the porosity / sparse-efficiency arithmetic of Eqs. 8 and 9."""
import numpy as np
import pytest

import synthetic
from paper_2108_13241_amd import metrics


def _check_open_ends(m, bc, value):
    n = m.shape[0]
    assert m[0].all() and m[n - 1].all()
    inl = (bc[:, 0] == synthetic.BC_PRESSURE[(1, 0)])
    out = (bc[:, n - 1] == synthetic.BC_PRESSURE[(-1, 0)])
    rows = np.arange(n)
    assert np.array_equal(inl, (m[:, 0] == 0) & (rows > 0) & (rows < n - 1))
    assert np.array_equal(out, (m[:, n - 1] == 0) & (rows > 0) & (rows < n - 1))
    assert np.all(value[0, inl, 0] == 1.016) and np.all(value[0, out, n - 1] == 1.0)
    bc_inner = bc.copy()
    bc_inner[:, 0] = 0
    bc_inner[:, n - 1] = 0
    assert not bc_inner.any()


@pytest.mark.parametrize("phi", [0.9, 0.6, 0.3])
def test_circle_array(phi):
    n = 512
    m, bc, value, info = synthetic.circle_array(n, phi)
    got = metrics.porosity(int((m == 0).sum()), n * n)
    assert got == info["phi_achieved"]
    # the largest radius with porosity >= phi: one node more of radius drops below
    assert phi <= got < phi + 4 * 8 * 8 * 2 * np.pi * info["radius"] / (n * n)
    # 64 equal circles: every cell of the 8 x 8 array holds the same number of solid nodes
    inner = m.copy()
    inner[0] = inner[n - 1] = 0
    cells = inner.reshape(8, n // 8, 8, n // 8).sum(axis=(1, 3))
    assert np.all(cells == cells[3, 3])
    _check_open_ends(m, bc, value)
    with pytest.raises(ValueError):
        synthetic.circle_array(n, 0.25)


@pytest.mark.parametrize("phi", [0.8, 0.4, 0.1])
def test_random_circles(phi):
    n = 1024
    m, bc, value, info = synthetic.random_circles(n, phi)
    m2, _, _, _ = synthetic.random_circles(n, phi)
    assert np.array_equal(m, m2)  # seeded
    assert info["phi_achieved"] <= phi
    # the last circle added has r <= 256: it removes at most pi 256^2 fluid nodes
    assert info["phi_achieved"] > phi - np.pi * 257 ** 2 / (n * n)
    _check_open_ends(m, bc, value)


def test_open_box_and_efficiency():
    m, bc, value, info = synthetic.open_box(64)
    assert info["phi_achieved"] == metrics.porosity(64 * 62, 64 * 64)
    _check_open_ends(m, bc, value)
    assert metrics.sparse_efficiency(30.0, 40.0) == 0.75
