"""Host-side checks of the C ABI (no GPU needed): the library loads and exports every
function include/*.h declares, argument validation fails with the documented status
before touching the device, and the geometry planners agree with brute force."""
import glob
import os
import re

import numpy as np
import pytest

import synthetic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for path in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        hdr = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names |= set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(lbm\w*_\w+)\s*\(",
                                hdr, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    import paper_2108_13241_amd as m
    return m.load()


def test_all_declared_symbols_exported(lib):
    names = declared_functions()
    assert len(names) >= 40
    assert "lbm3d_step" in names and "lbm_step" in names
    from paper_2108_13241_amd._lib import SIGNATURES
    for n in names:
        assert hasattr(lib, n), n
        assert n in SIGNATURES, n


def test_error_strings(lib):
    for st in (0, -1, -2, -3, -4, -5):
        assert lib.lbm_error_string(st)
    assert lib.lbm_error_string(42) == b"unknown status"


def _create(lib, nx, ny, mask, tau=0.8, force=(0.0, 0.0), dtype=0, layout=0):
    import ctypes
    ctx = ctypes.c_void_p()
    g = (ctypes.c_double * 2)(*force)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    st = lib.lbm_create(ctypes.byref(ctx), nx, ny,
                        m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), tau, g, dtype, layout)
    return st, ctx


@pytest.mark.parametrize("kw,status", [
    ({"tau": 0.5}, -1), ({"tau": float("nan")}, -1), ({"force": (float("inf"), 0.0)}, -1),
    ({"dtype": 7}, -1), ({"layout": 9}, -1), ({"layout": 5}, -1), ({"layout": 2}, -4),
    ({"layout": 4}, -4)])
def test_create_validation(lib, kw, status):
    m = np.zeros((10, 20), np.uint8)
    st, ctx = _create(lib, 20, 10, m, **kw)
    assert st == status
    assert not ctx.value
    assert lib.lbm_last_error(None)


@pytest.mark.parametrize("nx,ny,layout", [
    (65536, 32768, 0),        # dense: ny * pitch = 2^31 nodes
    (65536, 32768, 1),
    (29826162, 1, 0),         # dense: 9 * pitch >= 2^28 (lane column offsets)
    (32768, 16384, 3),        # indirect: 9 * ny * pitch >= 2^32
    (32768, 16384, 2),        # tiled
])
def test_create_size_limits(lib, nx, ny, layout):
    """Meshes beyond a layout's offset range are refused before the mask is read (the
    one-byte mask passed here would otherwise be overrun)."""
    st, ctx = _create(lib, nx, ny, np.zeros(1, np.uint8), layout=layout)
    assert st == -4
    assert not ctx.value
    assert b"too large" in lib.lbm_last_error(None)


def test_create_rejects_bad_mask(lib):
    m = np.zeros((8, 8), np.uint8)
    m[3, 3] = 2
    st, _ = _create(lib, 8, 8, m)
    assert st == -1
    assert b"node_type" in lib.lbm_last_error(None)


def test_null_context(lib):
    import ctypes
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_mass(None, ctypes.byref(ctypes.c_double())) == -1
    assert lib.lbm_set_mrt(None, None) == -1
    lib.lbm_destroy(None)


def _create3(lib, nx, ny, nz, m, tau=0.8, force=None, dtype=0, layout=0):
    import ctypes
    ctx = ctypes.c_void_p(1)
    g = (ctypes.c_double * 3)(*force) if force is not None else None
    st = lib.lbm3d_create(ctypes.byref(ctx), nx, ny, nz,
                          m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), tau, g, dtype,
                          layout)
    return st, ctx


@pytest.mark.parametrize("args,status", [
    (dict(nx=0), -1), (dict(nz=0), -1), (dict(tau=0.5), -1), (dict(tau=float("nan")), -1),
    (dict(force=(0.0, float("inf"), 0.0)), -1), (dict(dtype=4), -1), (dict(dtype=-1), -1),
    (dict(layout=7), -1),
    # the tiled layout (4 x 4 x 4 blocks) on a mesh whose ny = 10 is no multiple of 4
    (dict(layout=2), -4), (dict(layout=4), -4),
    # nz * ny * pitch >= 2^31 nodes, or 19 * pitch >= 2^28, is refused before the
    # mask is read or anything is allocated
    (dict(nx=1024, ny=2048, nz=1024), -4), (dict(nx=14128700, ny=1, nz=1), -4),
])
def test_create3d_validation(lib, args, status):
    kw = dict(nx=12, ny=10, nz=6)
    kw.update(args)
    nx, ny, nz = kw.pop("nx"), kw.pop("ny"), kw.pop("nz")
    m = np.zeros(max(nx * ny * nz, 1) if status != -4 else 1, np.uint8)
    st, ctx = _create3(lib, nx, ny, nz, m, **kw)
    assert st == status
    assert not ctx.value
    assert lib.lbm3d_last_error(None)


def test_create3d_rejects_bad_mask(lib):
    m = np.zeros((4, 5, 6), np.uint8)
    m[1, 2, 3] = 7
    st, _ = _create3(lib, 6, 5, 4, m)
    assert st == -1
    assert b"node_type" in lib.lbm3d_last_error(None)


def test_null_context3d(lib):
    import ctypes
    assert lib.lbm3d_step(None, 1) == -1
    assert lib.lbm3d_mass(None, ctypes.byref(ctypes.c_double())) == -1
    assert lib.lbm3d_get_info(None, None) == -1
    assert lib.lbm3d_set_trt(None, 0.25) == -1
    assert lib.lbm3d_set_bounce_back(None, 1) == -1
    lib.lbm3d_destroy(None)


def test_allocator_pairing(lib):
    import ctypes
    from paper_2108_13241_amd._lib import ALLOC_FN
    cb = ALLOC_FN(lambda n, u: None)
    assert lib.lbm_set_allocator(ctypes.cast(cb, ctypes.c_void_p), None, None) == -1
    assert lib.lbm_set_allocator(None, None, None) == 0


def _brute_tiles(m):
    ny, nx = m.shape
    tyn, txn = ny // 16, nx // 16
    keep = {}
    for ty in range(tyn):
        for tx in range(txn):
            if (m[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] == 0).any():
                keep[(tx, ty)] = len(keep)
    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    xy = np.array(list(keep.keys()), dtype=np.int32).reshape(-1, 2)
    nb = np.full((len(keep), 9), -1, np.int32)
    for (tx, ty), k in keep.items():
        for d in range(9):
            nb[k, d] = keep.get(((tx + cx[d]) % txn, (ty + cy[d]) % tyn), -1)
    return xy, nb


@pytest.mark.parametrize("seed", [0, 1])
def test_plan_tiles_vs_brute_force(seed):
    import paper_2108_13241_amd as lbm
    m, _ = synthetic.porous_discs(128, 0.4, seed=seed, rmin=6, rmax=20)
    m[:, 32:64] = 1
    xy, nb = lbm.plan_tiles(m)
    bxy, bnb = _brute_tiles(m)
    assert np.array_equal(xy, bxy)
    assert np.array_equal(nb, bnb)
    assert np.all(nb[:, 0] == np.arange(len(nb)))


def test_plan_tiles_rejects_ragged():
    import paper_2108_13241_amd as lbm
    with pytest.raises(lbm.LbmError):
        lbm.plan_tiles(np.zeros((20, 32), np.uint8))


@pytest.mark.parametrize("shape", [(37, 23), (64, 64), (1, 9)])
def test_plan_indirect_vs_brute_force(shape):
    import paper_2108_13241_amd as lbm
    nx, ny = shape
    m = synthetic.random_mask(nx, ny, seed=nx + ny, solid_fraction=0.3)
    xy, nb = lbm.plan_indirect(m)
    fl = [(x, y) for y in range(ny) for x in range(nx) if m[y, x] == 0]
    assert [tuple(p) for p in xy] == fl
    index = {p: k for k, p in enumerate(fl)}
    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    for k, (x, y) in enumerate(fl):
        for i in range(1, 9):
            src = ((x - cx[i]) % nx, (y - cy[i]) % ny)
            assert nb[i - 1, k] == index.get(src, -1)


def test_porous_generator_deterministic():
    a, ia = synthetic.porous_discs(256, 0.5, rmin=4, rmax=16)
    b, ib = synthetic.porous_discs(256, 0.5, rmin=4, rmax=16)
    assert np.array_equal(a, b)
    assert abs(ia["phi_achieved"] - 0.5) < 0.01
    assert (a[0] == 1).all() and (a[-1] == 1).all()


def test_allocator_hooks_outlive_switch(lib):
    """The torch allocator callbacks are made once and stay referenced after the hook is
    switched off (contexts created with them call them at destroy time)."""
    import paper_2108_13241_amd as pkg
    pkg._install_torch_allocator()
    hooks = pkg._hooks
    assert hooks is not None and pkg._hook_active
    pkg._uninstall_torch_allocator()
    assert pkg._hooks is hooks and not pkg._hook_active
    pkg._install_torch_allocator()
    assert pkg._hooks is hooks and pkg._hook_active


def test_device_buffer_checks():
    """Caller buffers handed to the library are checked in the binding: CPU tensors, too
    small, wrong dtype or non-contiguous tensors raise before any call; raw addresses pass."""
    import torch

    from paper_2108_13241_amd import _dev
    assert _dev(None, 8, "x", optional=True) is None
    assert _dev(12345, 8, "x") == 12345
    with pytest.raises(ValueError, match="required"):
        _dev(None, 8, "x")
    with pytest.raises(ValueError, match="CUDA"):
        _dev(torch.zeros(4), 8, "x")
    with pytest.raises(ValueError, match="CUDA"):
        _dev(np.zeros(4), 8, "x")
