"""Failure handling through the C ABI on a GPU: every rejected call returns its documented
status, leaves the context usable, and no kernel is launched with bad arguments."""
import ctypes

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


def _status(exc):
    return exc.value.status


def test_invalid_calls_leave_context_usable(lbm):
    import torch
    announce("error paths")
    m = synthetic.channel_mask(64, 16)
    m[:, 10] = 1  # a fully solid column
    lat = lbm.Lattice(m, 0.8, force=(1e-5, 0.0), dtype="f64", layout="dense_ab")
    M0 = lat.mass()
    with pytest.raises(lbm.LbmError) as e:
        lat.set_porosity(np.full((16, 64), 1.5, np.float32))
    assert _status(e) == -1
    bad = lat.get_populations()
    bad[3, 5, 7] = np.nan
    with pytest.raises(lbm.LbmError) as e:
        lat.set_populations(bad)
    assert _status(e) == -1
    with pytest.raises(lbm.LbmError) as e:
        lat.init_equilibrium(np.zeros((16, 64)))
    assert _status(e) == -1
    with pytest.raises(lbm.LbmError) as e:
        lat.objective_outlet_ux(10)
    assert _status(e) == -1
    with pytest.raises(lbm.LbmError) as e:
        lat.objective_outlet_ux(64)
    assert _status(e) == -1
    with pytest.raises(lbm.LbmError) as e:
        lat.step(-1)
    assert _status(e) == -1
    ab, _ = lat.adjoint_bytes()
    mu = torch.zeros(ab, dtype=torch.uint8, device="cuda")
    st = torch.zeros(lat.state_bytes(), dtype=torch.uint8, device="cuda")
    gg = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(lbm.LbmError) as e:
        lat.adjoint_step(st, mu, mu, None, gg)
    assert _status(e) == -1
    # still usable
    lat.step(20)
    assert lat.mass() == pytest.approx(M0, rel=1e-13)
    assert lat.info()["time_step"] == 20
    lat.close()


@pytest.mark.parametrize("layout,dtype", [("tiled16", "f64"), ("indirect", "f32"),
                                          ("dense_ab", "f16s")])
def test_adjoint_unsupported(lbm, layout, dtype):
    m = synthetic.channel_mask(64, 32)
    lat = lbm.Lattice(m, 0.8, dtype=dtype, layout=layout)
    with pytest.raises(lbm.LbmError) as e:
        lat.adjoint_bytes()
    assert _status(e) == -4
    lat.close()


def test_allocator_failure_reports_nomem(lbm):
    """An allocator hook that returns NULL makes lbm_create fail with LBM_ERR_NOMEM and leak
    nothing; restoring the hooks makes creation work again."""
    announce("allocator failure")
    from paper_2108_13241_amd import _install_torch_allocator, _uninstall_torch_allocator
    from paper_2108_13241_amd._lib import ALLOC_FN, FREE_FN
    L = lbm.load()
    calls = {"alloc": 0, "free": 0}

    def alloc(n, u):
        calls["alloc"] += 1
        return None

    def free(p, u):
        calls["free"] += 1

    a, f = ALLOC_FN(alloc), FREE_FN(free)
    assert L.lbm_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p),
                               None) == 0
    try:
        ctx = ctypes.c_void_p()
        m = np.zeros((16, 16), np.uint8)
        g = (ctypes.c_double * 2)(0.0, 0.0)
        st = L.lbm_create(ctypes.byref(ctx), 16, 16,
                          m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 0.8, g, 0, 0)
        assert st == -2
        assert not ctx.value
        assert calls["alloc"] >= 1
        # D3Q19 contexts take their memory from the same hook
        n0 = calls["alloc"]
        m3 = np.zeros((4, 8, 8), np.uint8)
        g3 = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
        st = L.lbm3d_create(ctypes.byref(ctx), 8, 8, 4,
                            m3.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 0.8, g3, 0, 0)
        assert st == -2
        assert not ctx.value
        assert calls["alloc"] > n0
        assert L.lbm3d_last_error(None)
    finally:
        import paper_2108_13241_amd as pkg
        pkg._hook_active = False  # the hook was replaced by hand above
        _install_torch_allocator()
    lat = lbm.Lattice(np.zeros((16, 16), np.uint8), 0.8)
    lat.step(3)
    lat.close()


def test_hipmalloc_path(lbm):
    """Contexts created without the torch allocator (plain hipMalloc) work the same."""
    m = synthetic.random_mask(48, 40, seed=9, solid_fraction=0.2)
    a = lbm.Lattice(m, 0.7, force=(1e-4, 0.0), dtype="f64", layout="indirect", torch_memory=False)
    a.step(30)
    fa = a.get_populations()
    a.close()
    b = lbm.Lattice(m, 0.7, force=(1e-4, 0.0), dtype="f64", layout="indirect", torch_memory=True)
    b.step(30)
    assert np.array_equal(b.get_populations(), fa)
    b.close()


def test_device_buffer_validation(lbm):
    """Wrong caller buffers raise ValueError in the binding (nothing is overrun); the context
    stays usable; a refused adjoint query names its reason."""
    import torch
    announce("device buffer validation")
    m = synthetic.channel_mask(64, 16)
    lat = lbm.Lattice(m, 0.8, force=(1e-5, 0.0), dtype="f32")
    sb = lat.state_bytes()
    with pytest.raises(ValueError, match="bytes"):
        lat.save_state(torch.empty(sb - 1, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError, match="contiguous"):
        lat.load_state(torch.empty((2, sb), dtype=torch.uint8, device="cuda")[:, 0])
    with pytest.raises(ValueError, match="float64"):
        lat.macroscopic_device(torch.empty((16, 64), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="bytes"):
        lat.macroscopic_device(None, torch.empty((16, 63), dtype=torch.float64, device="cuda"))
    ab, _ = lat.adjoint_bytes()
    mu = torch.zeros(ab, dtype=torch.uint8, device="cuda")
    gg = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="mu"):
        lat.adjoint_seed_outlet_ux(63, 1.0, mu[:-8], None, gg)
    with pytest.raises(ValueError, match="grad_g"):
        lat.adjoint_seed_outlet_ux(63, 1.0, mu, None, gg[:1])
    with pytest.raises(ValueError, match="ckpt"):
        lat.run_checkpointed(10, 4, torch.empty(2 * sb, dtype=torch.uint8, device="cuda"))
    out = torch.zeros((16, 64), dtype=torch.float64, device="cuda")
    lat.step(5)
    lat.macroscopic_device(None, out, None)
    torch.cuda.synchronize()
    assert float(out[8, 10].item()) > 0.0
    lat.set_trt(0.25)
    with pytest.raises(lbm.LbmError) as e:
        lat.adjoint_bytes()
    assert e.value.status == -4 and "BGK" in str(e.value)
    lat.close()


def test_allocator_switch_keeps_older_contexts(lbm):
    """A context created with torch's allocator keeps it after the hook is switched off for
    newer contexts: it still steps, and closing it returns its blocks to torch (the callbacks
    outlive the switch and a garbage collection)."""
    import gc

    import torch
    announce("allocator switch")
    m = synthetic.random_mask(64, 32, seed=12, solid_fraction=0.2)
    a = lbm.Lattice(m, 0.7, force=(1e-4, 0.0), dtype="f32", torch_memory=True)
    b = lbm.Lattice(m, 0.7, force=(1e-4, 0.0), dtype="f32", torch_memory=False)
    gc.collect()
    a.step(9)
    b.step(9)
    assert np.array_equal(a.get_populations(), b.get_populations())
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    a.close()
    assert torch.cuda.memory_allocated() <= before - 2 * 9 * 32 * 64 * 4
    b.close()
    from paper_2108_13241_amd import _install_torch_allocator
    _install_torch_allocator()
    c = lbm.Lattice(m, 0.7, dtype="f32")
    c.step(2)
    c.close()


def test_d3q19_memory_paths(lbm):
    """A D3Q19 context created while torch's allocator is registered takes its lattices from
    torch (torch.cuda.memory_allocated grows by at least the two lattices); one created with
    plain hipMalloc gives bitwise the same populations."""
    import torch
    announce("d3q19 memory paths")
    m = synthetic.random_mask3(40, 12, 10, seed=3, solid_fraction=0.1)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    a = lbm.Lattice3D(m, 0.7, force=(1e-4, 0.0, 0.0), dtype="f64", torch_memory=True)
    grown = torch.cuda.memory_allocated() - before
    assert grown >= 2 * 19 * 10 * 12 * 64 * 8
    assert a.info()["device_bytes"] <= grown + (1 << 20)
    a.step(12)
    fa = a.get_populations()
    a.close()
    b = lbm.Lattice3D(m, 0.7, force=(1e-4, 0.0, 0.0), dtype="f64", torch_memory=False)
    b.step(12)
    assert np.array_equal(b.get_populations(), fa)
    b.close()
    from paper_2108_13241_amd import _install_torch_allocator
    _install_torch_allocator()
