"""MI355X-native D2Q9 / D3Q19 lattice-Boltzmann library: Python binding of include/lbm.h and
include/lbm3d.h.

Every step of the method runs in the HIP kernels of ``liblbm_hip.so``; this module only
marshals arguments.  PyTorch supplies device memory (its caching allocator is
registered with ``lbm_set_allocator``) and streams (``torch.cuda.current_stream``).

    import paper_2108_13241_amd as lbm
    lat = lbm.Lattice(mask, tau=0.8, force=(1e-6, 0.0), dtype="f64", layout="dense_ab")
    lat.step(2000)
    rho, ux, uy = lat.macroscopic()
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import DTYPES, LAYOUTS, POP_BYTES, Lbm3dInfo, LbmError, LbmInfo, check, check3, load

__all__ = ["Lattice", "Lattice3D", "LbmError", "DTYPES", "LAYOUTS", "plan_tiles", "plan_indirect",
           "copy_kernel", "ChannelObjective", "load"]

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)

# ------------------------------------------------------------ torch memory --
_torch_blocks = {}
# The ctypes callbacks are made once and kept for the life of the process: a
# context keeps the allocator it was created with, so its free callback must
# stay callable after the hook is switched off for newer contexts.
_hooks = None
_hook_active = False


def _install_torch_allocator():
    """Route the library's device allocations through torch's caching allocator."""
    global _hooks, _hook_active
    if _hook_active:
        return
    if _hooks is None:
        import torch

        from ._lib import ALLOC_FN, FREE_FN

        def _alloc(nbytes, _user):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            except Exception:  # noqa: BLE001 - report NULL to the library (LBM_ERR_NOMEM)
                return None
            p = t.data_ptr()
            _torch_blocks[p] = t
            return p

        def _free(ptr, _user):
            _torch_blocks.pop(ptr, None)

        _hooks = (ALLOC_FN(_alloc), FREE_FN(_free))
    check(load().lbm_set_allocator(ctypes.cast(_hooks[0], ctypes.c_void_p),
                                   ctypes.cast(_hooks[1], ctypes.c_void_p), None))
    _hook_active = True


def _uninstall_torch_allocator():
    """Back to hipMalloc / hipFree for contexts created from now on (contexts created with
    torch memory keep it)."""
    global _hook_active
    check(load().lbm_set_allocator(None, None, None))
    _hook_active = False


def _ptr(t):
    """Device pointer of a torch tensor (or an int address / None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _dev(t, nbytes, what, dtype=None, optional=False):
    """Address of a caller-owned device buffer for the library to read or write: a CUDA torch
    tensor, checked here (on a GPU, contiguous, at least `nbytes` long, of `dtype` if given),
    so that a wrong buffer raises instead of being overrun; or a raw int address, taken as
    is (the caller vouches for its size)."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{what}: a device buffer is required")
    if isinstance(t, int):
        return t
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what}: expected a CUDA tensor or a device address")
    if not t.is_contiguous():
        raise ValueError(f"{what}: the tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what}: expected {dtype}, got {t.dtype}")
    if t.nbytes < nbytes:
        raise ValueError(f"{what}: needs {nbytes} bytes, the tensor has {t.nbytes}")
    return t.data_ptr()


def _f64t():
    import torch
    return torch.float64


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


class Lattice:
    """One D2Q9 lattice on the current GPU (a thin wrapper of lbm_ctx)."""

    def __init__(self, mask, tau, force=(0.0, 0.0), dtype="f64", layout="dense_ab",
                 stream=None, torch_memory=True):
        import torch

        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.ndim != 2:
            raise ValueError("mask must be [ny, nx]")
        self.ny, self.nx = mask.shape
        self.mask = mask
        self.dtype = dtype
        self.layout = layout
        self._lib = load()
        if torch_memory:
            _install_torch_allocator()
        else:
            _uninstall_torch_allocator()
        self._ctx = ctypes.c_void_p()
        g = (ctypes.c_double * 2)(float(force[0]), float(force[1]))
        st = self._lib.lbm_create(ctypes.byref(self._ctx), self.nx, self.ny,
                                  mask.ctypes.data_as(_u8p), float(tau), g, DTYPES[dtype],
                                  LAYOUTS[layout])
        check(st, None)
        self.set_stream(stream if stream is not None else torch.cuda.current_stream())

    # -- plumbing ----------------------------------------------------------
    def _check(self, status):
        check(status, self._ctx)

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def set_stream(self, stream):
        """stream: torch.cuda.Stream, a raw hipStream_t address, or 0 (default stream)."""
        raw = getattr(stream, "cuda_stream", stream)
        self.stream = stream
        self._check(self._lib.lbm_set_stream(self._ctx, ctypes.c_void_p(int(raw or 0))))

    # -- state -----------------------------------------------------------------
    def init_equilibrium(self, rho=None, ux=None, uy=None):
        s = (self.ny, self.nx)
        rho, ux, uy = _f64(rho, s), _f64(ux, s), _f64(uy, s)
        self._check(self._lib.lbm_init_equilibrium(self._ctx, _dptr(rho), _dptr(ux), _dptr(uy)))

    def set_porosity(self, alpha):
        if alpha is None:
            self._check(self._lib.lbm_set_porosity(self._ctx, None))
            return
        a = np.ascontiguousarray(alpha, dtype=np.float32)
        if a.shape != (self.ny, self.nx):
            raise ValueError("alpha must be [ny, nx]")
        self._check(self._lib.lbm_set_porosity(self._ctx,
                                               a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def set_boundaries(self, bc, value=None):
        """Open boundaries (constant velocity / pressure, Zou-He): bc uint8 [ny, nx] with codes
        0 none, 1..4 velocity with inward normal +x, -x, +y, -y, 5..8 pressure with the same
        normals; value float64 [2, ny, nx] = (u_x, u_y) or (rho, -).  bc None removes them."""
        if bc is None:
            self._check(self._lib.lbm_set_boundaries(self._ctx, None, None))
            return
        b = np.ascontiguousarray(bc, dtype=np.uint8)
        v = np.ascontiguousarray(value, dtype=np.float64)
        if b.shape != (self.ny, self.nx) or v.shape != (2, self.ny, self.nx):
            raise ValueError("bc must be [ny, nx] and value [2, ny, nx]")
        self._check(self._lib.lbm_set_boundaries(self._ctx, b.ctypes.data, v.ctypes.data))

    def set_trt(self, magic):
        """Two-relaxation-time collision with parameter Lambda = magic (0 = BGK)."""
        self._check(self._lib.lbm_set_trt(self._ctx, float(magic)))

    def set_mrt(self, rates):
        """Multiple-relaxation-time collision with rates (s_e, s_eps, s_q) for the energy,
        energy-square and energy-flux moments (the shear moments relax with 1 / tau); None
        switches it off (BGK)."""
        if rates is None:
            self._check(self._lib.lbm_set_mrt(self._ctx, None))
            return
        r = np.ascontiguousarray(rates, dtype=np.float64)
        if r.shape != (3,):
            raise ValueError("MRT takes three rates (s_e, s_eps, s_q)")
        self._check(self._lib.lbm_set_mrt(self._ctx, r.ctypes.data))

    def set_bounce_back(self, mode):
        """"halfway" (default) or "fullway" wall rule (0 / 1); under full-way the canonical
        populations include the wall slots of solid nodes next to fluid."""
        m = {"halfway": 0, "fullway": 1}.get(mode, mode)
        self._check(self._lib.lbm_set_bounce_back(self._ctx, int(m)))

    def set_force(self, g):
        arr = (ctypes.c_double * 2)(float(g[0]), float(g[1]))
        self._check(self._lib.lbm_set_force(self._ctx, arr))

    def set_graph_steps(self, steps):
        """-1 auto, 0 off, or an even number of steps per replayed HIP graph."""
        self._check(self._lib.lbm_set_graph_steps(self._ctx, int(steps)))

    def step(self, n=1):
        self._check(self._lib.lbm_step(self._ctx, int(n)))

    def macroscopic(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(3)]
        self._check(self._lib.lbm_macroscopic(self._ctx, *[_dptr(o) for o in out]))
        return tuple(out)

    def macroscopic_device(self, rho=None, ux=None, uy=None):
        """Fields into device FP64 [ny, nx] tensors (None: skipped); asynchronous."""
        n, d = 8 * self.ny * self.nx, _f64t()
        self._check(self._lib.lbm_macroscopic_device(
            self._ctx, _dev(rho, n, "rho", d, True), _dev(ux, n, "ux", d, True),
            _dev(uy, n, "uy", d, True)))

    def get_populations(self):
        f = np.zeros((9, self.ny, self.nx))
        self._check(self._lib.lbm_get_populations(self._ctx, _dptr(f)))
        return f

    def set_populations(self, f):
        f = _f64(f, (9, self.ny, self.nx))
        self._check(self._lib.lbm_set_populations(self._ctx, _dptr(f)))

    def mass(self):
        m = ctypes.c_double()
        self._check(self._lib.lbm_mass(self._ctx, ctypes.byref(m)))
        return m.value

    def state_bytes(self):
        b = ctypes.c_size_t()
        self._check(self._lib.lbm_state_bytes(self._ctx, ctypes.byref(b)))
        return b.value

    def save_state(self, dst):
        self._check(self._lib.lbm_save_state(self._ctx, _dev(dst, self.state_bytes(), "dst")))

    def load_state(self, src):
        self._check(self._lib.lbm_load_state(self._ctx, _dev(src, self.state_bytes(), "src")))

    def objective_outlet_ux(self, x_col):
        J = ctypes.c_double()
        self._check(self._lib.lbm_objective_outlet_ux(self._ctx, int(x_col), ctypes.byref(J)))
        return J.value

    def info(self):
        i = LbmInfo()
        self._check(self._lib.lbm_get_info(self._ctx, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in LbmInfo._fields_}

    # -- adjoint -----------------------------------------------------------------
    def adjoint_bytes(self):
        b = ctypes.c_size_t()
        p = ctypes.c_int32()
        self._check(self._lib.lbm_adjoint_bytes(self._ctx, ctypes.byref(b), ctypes.byref(p)))
        return b.value, p.value

    def _mu(self, mu, what):
        return _dev(mu, self._adjoint_nbytes(), what)

    def _adjoint_nbytes(self):
        if getattr(self, "_adj_nbytes", None) is None:
            self._adj_nbytes = self.adjoint_bytes()[0]
        return self._adj_nbytes

    def _grads(self, grad_alpha, grad_g):
        d = _f64t()
        return (_dev(grad_alpha, 8 * self.ny * self.nx, "grad_alpha", d, True),
                _dev(grad_g, 16, "grad_g", d))

    def _slots(self, T, K):
        """Checkpoint slots of a T-step run with interval K (0 for arguments the library
        refuses anyway)."""
        return (int(T) + int(K) - 1) // int(K) if int(K) > 0 and int(T) > 0 else 0

    def adjoint_get(self, mu):
        """Adjoint field -> host FP64 [9, ny, nx]."""
        out = np.zeros((9, self.ny, self.nx))
        self._check(self._lib.lbm_adjoint_get(self._ctx, self._mu(mu, "mu"), _dptr(out)))
        return out

    def adjoint_set(self, mu, values):
        v = _f64(values, (9, self.ny, self.nx))
        self._check(self._lib.lbm_adjoint_set(self._ctx, self._mu(mu, "mu"), _dptr(v)))

    def adjoint_seed_outlet_ux(self, x_col, dJ, mu, grad_alpha, grad_g):
        self._check(self._lib.lbm_adjoint_seed_outlet_ux(self._ctx, int(x_col), float(dJ),
                                                         self._mu(mu, "mu"),
                                                         *self._grads(grad_alpha, grad_g)))

    def adjoint_step(self, state, mu_in, mu_out, grad_alpha, grad_g):
        self._check(self._lib.lbm_adjoint_step(
            self._ctx, _dev(state, self.state_bytes(), "state"), self._mu(mu_in, "mu_in"),
            self._mu(mu_out, "mu_out"), *self._grads(grad_alpha, grad_g)))

    def adjoint_step_noalloc(self, state, mu_in, mu_out, grad_alpha, grad_g):
        """adjoint_step without any device allocation (partials in the library's fixed
        per-device scratch array; lattices up to 16376 row segments of 256 nodes)."""
        self._check(self._lib.lbm_adjoint_step_noalloc(
            self._ctx, _dev(state, self.state_bytes(), "state"), self._mu(mu_in, "mu_in"),
            self._mu(mu_out, "mu_out"), *self._grads(grad_alpha, grad_g)))

    def run_checkpointed(self, T, K, ckpt):
        n = self._slots(T, K) * self.state_bytes()
        self._check(self._lib.lbm_run_checkpointed(self._ctx, int(T), int(K),
                                                   _dev(ckpt, n, "ckpt")))

    def adjoint_checkpointed(self, T, K, ckpt, seg, x_col, dJ, grad_alpha, grad_g):
        sb = self.state_bytes()
        self._check(self._lib.lbm_adjoint_checkpointed(
            self._ctx, int(T), int(K), _dev(ckpt, self._slots(T, K) * sb, "ckpt"),
            _dev(seg, max(int(K), 0) * sb, "seg"), int(x_col), float(dJ),
            *self._grads(grad_alpha, grad_g)))


# ------------------------------------------------------------ host planning --
def _force3(g):
    g = [float(v) for v in g]
    if len(g) != 3:
        raise ValueError("a D3Q19 force has three components (g_x, g_y, g_z)")
    return (ctypes.c_double * 3)(*g)


class Lattice3D:
    """One D3Q19 lattice on the current GPU (a thin wrapper of lbm3d_ctx): dense A-B, AA,
    fluid-node-list ("indirect") or 4 x 4 x 4-block tiled ("tiled16", "tiled16_all") layout; BGK, TRT or MRT collision with Guo forcing; halfway
    (or, except on AA, full-way) bounce-back.  Arrays are [nz, ny, nx]; canonical populations
    [19, nz, ny, nx] in the velocity order of include/lbm3d.h."""

    def __init__(self, mask, tau, force=(0.0, 0.0, 0.0), dtype="f64", stream=None,
                 torch_memory=True, layout="dense_ab"):
        import torch

        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.ndim != 3:
            raise ValueError("mask must be [nz, ny, nx]")
        self.nz, self.ny, self.nx = mask.shape
        self.shape = mask.shape
        self.mask = mask
        self.dtype = dtype
        self._lib = load()
        if torch_memory:
            _install_torch_allocator()
        else:
            _uninstall_torch_allocator()
        self._ctx = ctypes.c_void_p()
        g = _force3(force)
        check3(self._lib.lbm3d_create(ctypes.byref(self._ctx), self.nx, self.ny, self.nz,
                                      mask.ctypes.data_as(_u8p), float(tau), g, DTYPES[dtype],
                                      LAYOUTS[layout]),
               None)
        self.layout = layout
        self.set_stream(stream if stream is not None else torch.cuda.current_stream())

    def _check(self, status):
        check3(status, self._ctx)

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm3d_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def set_stream(self, stream):
        raw = getattr(stream, "cuda_stream", stream)
        self.stream = stream
        self._check(self._lib.lbm3d_set_stream(self._ctx, ctypes.c_void_p(int(raw or 0))))

    def init_equilibrium(self, rho=None, ux=None, uy=None, uz=None):
        f = [_f64(a, self.shape) for a in (rho, ux, uy, uz)]
        self._check(self._lib.lbm3d_init_equilibrium(self._ctx, *[_dptr(a) for a in f]))

    def set_force(self, g):
        self._check(self._lib.lbm3d_set_force(self._ctx, _force3(g)))

    def set_trt(self, magic):
        """Two-relaxation-time collision with parameter Lambda = magic (0 = BGK)."""
        self._check(self._lib.lbm3d_set_trt(self._ctx, float(magic)))

    def set_mrt(self, rates):
        """Multiple-relaxation-time collision with rates (s_e, s_eps, s_q, s_pi, s_m) (the
        shear moments relax with 1 / tau); None switches it off (BGK)."""
        if rates is None:
            self._check(self._lib.lbm3d_set_mrt(self._ctx, None))
            return
        r = np.ascontiguousarray(rates, dtype=np.float64)
        if r.shape != (5,):
            raise ValueError("D3Q19 MRT takes five rates (s_e, s_eps, s_q, s_pi, s_m)")
        self._check(self._lib.lbm3d_set_mrt(self._ctx, r.ctypes.data))

    def set_bounce_back(self, mode):
        """"halfway" (default) or "fullway" wall rule (0 / 1); under full-way the canonical
        populations include the wall slots of solid nodes next to fluid."""
        m = {"halfway": 0, "fullway": 1}.get(mode, mode)
        self._check(self._lib.lbm3d_set_bounce_back(self._ctx, int(m)))

    def step(self, n=1):
        self._check(self._lib.lbm3d_step(self._ctx, int(n)))

    def macroscopic(self):
        out = [np.zeros(self.shape) for _ in range(4)]
        self._check(self._lib.lbm3d_macroscopic(self._ctx, *[_dptr(o) for o in out]))
        return tuple(out)

    def macroscopic_device(self, rho, ux, uy, uz):
        """Fields into device FP64 [nz, ny, nx] tensors (all four); asynchronous."""
        n, d = 8 * self.nx * self.ny * self.nz, _f64t()
        self._check(self._lib.lbm3d_macroscopic_device(
            self._ctx, _dev(rho, n, "rho", d), _dev(ux, n, "ux", d), _dev(uy, n, "uy", d),
            _dev(uz, n, "uz", d)))

    def state_bytes(self):
        b = ctypes.c_size_t()
        self._check(self._lib.lbm3d_state_bytes(self._ctx, ctypes.byref(b)))
        return b.value

    def save_state(self, dst):
        self._check(self._lib.lbm3d_save_state(self._ctx, _dev(dst, self.state_bytes(), "dst")))

    def load_state(self, src):
        self._check(self._lib.lbm3d_load_state(self._ctx, _dev(src, self.state_bytes(), "src")))

    def get_populations(self):
        f = np.zeros((19,) + self.shape)
        self._check(self._lib.lbm3d_get_populations(self._ctx, _dptr(f)))
        return f

    def set_populations(self, f):
        f = _f64(f, (19,) + self.shape)
        self._check(self._lib.lbm3d_set_populations(self._ctx, _dptr(f)))

    def mass(self):
        m = ctypes.c_double()
        self._check(self._lib.lbm3d_mass(self._ctx, ctypes.byref(m)))
        return m.value

    def info(self):
        i = Lbm3dInfo()
        self._check(self._lib.lbm3d_get_info(self._ctx, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in Lbm3dInfo._fields_}


def plan_tiles(mask):
    """(tile_xy [n, 2], tile_nbr [n, 9]) of the compacted 16x16 tile list."""
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    ny, nx = m.shape
    L = load()
    n = ctypes.c_int64()
    check(L.lbm_plan_tiles(nx, ny, m.ctypes.data_as(_u8p), ctypes.byref(n), None, None))
    xy = np.zeros((n.value, 2), dtype=np.int32)
    nb = np.zeros((n.value, 9), dtype=np.int32)
    check(L.lbm_plan_tiles(nx, ny, m.ctypes.data_as(_u8p), ctypes.byref(n),
                           xy.ctypes.data_as(_i32p), nb.ctypes.data_as(_i32p)))
    return xy, nb


def plan_indirect(mask):
    """(fluid_xy [n, 2], nbr [8, n]) of the compacted fluid-node list."""
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    ny, nx = m.shape
    L = load()
    n = ctypes.c_int64()
    check(L.lbm_plan_indirect(nx, ny, m.ctypes.data_as(_u8p), ctypes.byref(n), None, None))
    xy = np.zeros((n.value, 2), dtype=np.int32)
    nb = np.zeros((8, n.value), dtype=np.int32)
    check(L.lbm_plan_indirect(nx, ny, m.ctypes.data_as(_u8p), ctypes.byref(n),
                              xy.ctypes.data_as(_i32p), nb.ctypes.data_as(_i32p)))
    return xy, nb


def copy_kernel(src, dst, nbytes, stream=None):
    raw = getattr(stream, "cuda_stream", stream) or 0
    n = int(nbytes)
    check(load().lbm_copy_kernel(_dev(src, n, "src"), _dev(dst, n, "dst"), n,
                                 ctypes.c_void_p(int(raw))))


from .adjoint import ChannelObjective  # noqa: E402
