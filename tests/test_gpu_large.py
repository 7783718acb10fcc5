"""Dense lattices beyond 2^32 population elements (64-bit row offsets), D2Q9 and D3Q19.

Geometry: a periodic lattice driven by a uniform body force from rest, with one small solid
obstacle copied into several windows: one at low offsets, one that wraps around the last
row / column (and plane) to the first, one astride the row (plane) where the element
offset of population 0 passes 2^32, and one wholly above it.  After T steps an obstacle's
influence has spread T nodes (one node per step), so:

* inside each window the fields equal the oracle's fields on a small periodic box holding
  the same obstacle at the same place relative to the window (FP64: 1e-12 absolute; FP32:
  rho 1e-5 relative, u 2e-6 absolute), and every window equals the first one bitwise
  (translation invariance);
* every node outside the windows holds the same far-field values as the box's far field;
* the total mass is conserved (FP64, FP32; 16-bit storage rounds it).

The GPU needs about 125 GB for the largest case (the MI355X holds 288 GB); the test skips on
smaller devices.
"""
import numpy as np
import pytest

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


def _need_device_bytes(nbytes):
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes:
        pytest.skip(f"needs {nbytes / 2**30:.0f} GiB of free device memory")


def _release():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------- D2Q9 --
NX, NY = 24576, 20480  # pitch 24576: 9 * NY * pitch = 4.53e9 elements
L2, T2 = 80, 20        # oracle box and steps: obstacle 10 x 10 at the box centre
ROW_2_32 = (1 << 32) // (9 * NX)  # first row whose population-0 offset exceeds 2^32


def _obstacle2():
    rng = np.random.default_rng(404)
    blob = (rng.random((10, 10)) < 0.55).astype(np.uint8)
    blob[4:6, 4:6] = 1
    return blob


def _windows2():
    # centres (x, y): low offsets; wrapping the last row and column; astride the 2^32 row;
    # above it
    return [(200, 300), (NX - 1, NY - 1), (NX // 2, ROW_2_32), (5000, NY - 400)]


def _axes(c, n, L):
    return (c - L // 2 + np.arange(L)) % n


def _box2(blob):
    m = np.zeros((L2, L2), np.uint8)
    o = L2 // 2 - blob.shape[0] // 2
    m[o:o + blob.shape[0], o:o + blob.shape[1]] = blob
    return m


def _big_mask2(blob):
    m = np.zeros((NY, NX), np.uint8)
    box = _box2(blob)
    for cx, cy in _windows2():
        rows, cols = _axes(cy, NY, L2), _axes(cx, NX, L2)
        m[np.ix_(rows, cols)] |= box
    return m


@pytest.mark.parametrize("dtype,layout", [("f64", "dense_ab"), ("f32", "dense_aa"),
                                          ("f16s", "dense_ab")])
def test_d2q9_beyond_2_32_elements(lbm, oracle_mod, dtype, layout):
    import torch
    announce(f"large d2q9 {NX}x{NY} {dtype} {layout}")
    assert 9 * NY * NX > 1 << 32 and NY - 1 > ROW_2_32
    s_d = {"f64": 8, "f32": 4, "f16s": 2}[dtype]
    lattices = 9 * NX * NY * s_d * (1 if layout == "dense_aa" else 2)
    _need_device_bytes(lattices + 9 * NX * NY * 8 + 3 * NX * NY * 8 + (4 << 30))
    tau, g = 0.7, (2e-5, -7e-6)
    blob = _obstacle2()
    m = _big_mask2(blob)
    lat = lbm.Lattice(m, tau, force=g, dtype=dtype, layout=layout)
    M0 = lat.mass()
    lat.step(T2)
    M1 = lat.mass()
    fields = [torch.empty((NY, NX), dtype=torch.float64, device="cuda") for _ in range(3)]
    lat.macroscopic_device(*fields)
    torch.cuda.synchronize()
    lat.close()
    del m

    wins = []
    for cx, cy in _windows2():
        rows = torch.as_tensor(_axes(cy, NY, L2), device="cuda")
        cols = torch.as_tensor(_axes(cx, NX, L2), device="cuda")
        wins.append((rows, cols, [f[rows[:, None], cols[None, :]].cpu().numpy() for f in fields]))
    # translation invariance: every window equals the first one bitwise
    for _, _, w in wins[1:]:
        for a, b in zip(w, wins[0][2]):
            assert np.array_equal(a, b)
    # far field: every node outside the windows equals one value per field
    far = [float(f[NY // 2 + 7, NX // 3].item()) for f in fields]
    diff = torch.zeros((NY, NX), dtype=torch.bool, device="cuda")
    for f, v in zip(fields, far):
        diff |= f != v
    for rows, cols, _ in wins:
        diff[rows[:, None], cols[None, :]] = False
    assert int(diff.sum().item()) == 0
    del diff, fields
    _release()

    if dtype == "f16s":
        return  # 16-bit storage is an approximation: translation and far field only
    assert abs(M1 - M0) <= (1e-12 if dtype == "f64" else 1e-5) * M0
    box = _box2(blob)
    ref = oracle_mod.run(box, oracle_mod.init(box), tau, T2, g=g)
    exp = oracle_mod.macroscopic(box, ref, g=g)
    got = wins[0][2]
    for v, e in zip(far, exp):
        if dtype == "f64":
            assert abs(v - e[1, 1]) <= 1e-12
    if dtype == "f64":
        for a, b in zip(got, exp):
            assert np.abs(a - b).max() <= 1e-12
    else:
        fl = box == 0
        assert (np.abs(got[0] - exp[0])[fl] / exp[0][fl]).max() <= 1e-5
        assert np.abs(got[1] - exp[1]).max() <= 2e-6
        assert np.abs(got[2] - exp[2]).max() <= 2e-6


# ---------------------------------------------------------------------- D3Q19 --
NX3, NY3, NZ3 = 256, 256, 3500  # 19 * nodes = 4.36e9 elements
L3, T3 = 40, 12                 # oracle box and steps: obstacle 6^3 at the box centre
PLANE_2_32 = (1 << 32) // (19 * NX3 * NY3)


def _obstacle3():
    rng = np.random.default_rng(405)
    blob = (rng.random((6, 6, 6)) < 0.5).astype(np.uint8)
    blob[2:4, 2:4, 2:4] = 1
    return blob


def _windows3():
    # centres (x, y, z)
    return [(60, 60, 60), (NX3 - 1, NY3 - 1, NZ3 - 1), (128, 128, PLANE_2_32),
            (200, 50, NZ3 - 20)]


def _box3(blob):
    m = np.zeros((L3, L3, L3), np.uint8)
    o = L3 // 2 - blob.shape[0] // 2
    m[o:o + 6, o:o + 6, o:o + 6] = blob
    return m


def test_d3q19_beyond_2_32_elements(lbm, oracle_mod):
    announce(f"large d3q19 {NX3}x{NY3}x{NZ3} f64")
    n = NX3 * NY3 * NZ3
    assert 19 * n > 1 << 32 and NZ3 - 1 > PLANE_2_32
    _need_device_bytes(2 * 19 * n * 8 + 19 * n * 8 + 4 * n * 8 + (4 << 30))
    tau, g = 0.75, (1e-5, -4e-6, 3e-6)
    blob = _obstacle3()
    box = _box3(blob)
    m = np.zeros((NZ3, NY3, NX3), np.uint8)
    axes = []
    for cx, cy, cz in _windows3():
        ax = (_axes(cz, NZ3, L3), _axes(cy, NY3, L3), _axes(cx, NX3, L3))
        m[np.ix_(*ax)] |= box
        axes.append(ax)
    lat = lbm.Lattice3D(m, tau, force=g, dtype="f64")
    M0 = lat.mass()
    lat.step(T3)
    M1 = lat.mass()
    out = lat.macroscopic()
    lat.close()
    del m
    _release()
    assert abs(M1 - M0) <= 1e-12 * M0

    wins = [[f[np.ix_(*ax)] for f in out] for ax in axes]
    for w in wins[1:]:
        for a, b in zip(w, wins[0]):
            assert np.array_equal(a, b)
    far = [float(f[NZ3 // 2, 100, 30]) for f in out]
    for f, v in zip(out, far):
        d = f != v
        for ax in axes:
            d[np.ix_(*ax)] = False
        assert not d.any()
    del out

    ref = oracle_mod.run3(box, oracle_mod.init3(box), tau, T3, g=g)
    exp = oracle_mod.macroscopic3(box, ref, g=g)
    for v, e in zip(far, exp):
        assert abs(v - e[1, 1, 1]) <= 1e-12
    for a, b in zip(wins[0], exp):
        assert np.abs(a - b).max() <= 1e-12
