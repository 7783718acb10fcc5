"""Plain FP64 CPU oracle for the D2Q9 BGK lattice-Boltzmann step (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The GPU library shares no code with it:
the oracle is plain C (``lbm_oracle.c``, compiled with gcc) plus an exact-rational
brute force in pure Python (``exact.py``).

Array conventions (numpy, C order):
  mask   uint8  [ny, nx]      0 fluid, 1 solid
  f      float64 [9, ny, nx]  canonical pre-collision populations f_i(x, t), the
                              left-hand side of the LB update (Sec. 2.2, Eq. 3);
                              solid slots are 0
  alpha  float64 [ny, nx]     Brinkman drag coefficient (None = 0)
  bc     uint8  [ny, nx]      open-boundary code (Sec. 3, Zou-He): 0 none, 1..4 constant
                              velocity with inward normal +x, -x, +y, -y, 5..8 constant
                              pressure with the same normals (None = no open boundaries)
  value  float64 [2, ny, nx]  boundary values: (u_x, u_y) at velocity nodes, (rho, -) at
                              pressure nodes

Pins (tests/test_oracle_*.py) check it against what the paper and the mathematics
fix: closed-form moments of the equilibrium (Eq. 6) and of the forcing term,
conservation of mass and momentum, the equilibrium fixed point, lattice symmetry,
the exact steady and start-up Poiseuille profiles, the Taylor-Green decay rate
(viscosity from Eq. 5), the Brinkman momentum recurrence, exact-rational brute force
on 4x4 lattices, and finite differences of the forward map for the gradient.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SRC3 = os.path.join(_HERE, "lbm_oracle_d3q19.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, _SRC3, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.oracle_constants.argtypes = [_ip, _ip, _dp, _ip]
        L.oracle_equilibrium.argtypes = [ctypes.c_double] * 3 + [_dp]
        L.oracle_guo_source.argtypes = [ctypes.c_double] * 4 + [_dp]
        L.oracle_node_velocity.argtypes = [_dp] + [ctypes.c_double] * 3 + [_dp]
        L.oracle_collide.argtypes = [_dp] + [ctypes.c_double] * 4 + [_dp]
        L.oracle_collide_jacobian.argtypes = [_dp] + [ctypes.c_double] * 4 + [_dp, _dp, _dp]
        L.oracle_init.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, _dp, _dp, _dp]
        L.oracle_init.restype = ctypes.c_int
        L.oracle_run.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, _dp, ctypes.c_long, ctypes.c_int]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_macroscopic.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_double,
                                         ctypes.c_double, _dp, _dp, _dp, _dp]
        L.oracle_macroscopic.restype = ctypes.c_int
        L.oracle_objective_outlet_ux.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp,
                                                 ctypes.c_double, ctypes.c_double, _dp,
                                                 ctypes.c_int, _dp]
        L.oracle_objective_outlet_ux.restype = ctypes.c_int
        L.oracle_outlet_ux_gradient.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                _dp, ctypes.c_long, ctypes.c_int, _dp, _dp, _dp]
        L.oracle_outlet_ux_gradient.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_zou_he.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_zou_he.restype = ctypes.c_int
        L.oracle_apply_boundaries.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _u8p, _dp, _dp]
        L.oracle_apply_boundaries.restype = ctypes.c_int
        L.oracle_run_bc.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, _dp, _u8p, _dp,
                                    ctypes.c_long, ctypes.c_int]
        L.oracle_run_bc.restype = ctypes.c_int
        L.oracle_collide_trt.argtypes = [_dp] + [ctypes.c_double] * 5 + [_dp]
        L.oracle3_constants.argtypes = [_ip, _ip, _ip, _dp, _ip]
        L.oracle3_equilibrium.argtypes = [ctypes.c_double] * 4 + [_dp]
        L.oracle3_guo_source.argtypes = [ctypes.c_double] * 6 + [_dp]
        L.oracle3_node_velocity.argtypes = [_dp] + [ctypes.c_double] * 3 + [_dp]
        L.oracle3_collide.argtypes = [_dp] + [ctypes.c_double] * 4 + [_dp]
        L.oracle3_init.argtypes = [ctypes.c_int] * 3 + [_u8p, _dp, _dp, _dp, _dp, _dp]
        L.oracle3_init.restype = ctypes.c_int
        L.oracle3_run.argtypes = [ctypes.c_int] * 3 + [_u8p, _dp] + [ctypes.c_double] * 4 + \
            [ctypes.c_long, ctypes.c_int]
        L.oracle3_run.restype = ctypes.c_int
        L.oracle3_run_trt.argtypes = [ctypes.c_int] * 3 + [_u8p, _dp] + [ctypes.c_double] * 5 + \
            [ctypes.c_long, ctypes.c_int]
        L.oracle3_run_trt.restype = ctypes.c_int
        L.oracle3_collide_trt.argtypes = [_dp] + [ctypes.c_double] * 5 + [_dp]
        L.oracle3_run_walls.argtypes = L.oracle3_run_trt.argtypes + [ctypes.c_int]
        L.oracle3_mrt_matrix.argtypes = [_dp]
        L.oracle3_collide_mrt.argtypes = [_dp] + [ctypes.c_double] * 3 + [_dp, _dp]
        L.oracle3_run_mrt.argtypes = [ctypes.c_int] * 3 + [_u8p, _dp, ctypes.c_double, _dp] + \
            [ctypes.c_double] * 3 + [ctypes.c_long, ctypes.c_int, ctypes.c_int]
        L.oracle3_run_mrt.restype = ctypes.c_int
        L.oracle3_run_walls.restype = ctypes.c_int
        L.oracle3_fullway_fill.argtypes = [ctypes.c_int] * 3 + [_u8p, _dp]
        L.oracle3_fullway_fill.restype = ctypes.c_int
        L.oracle3_macroscopic.argtypes = [ctypes.c_int] * 3 + [_u8p, _dp] + \
            [ctypes.c_double] * 3 + [_dp] * 4
        L.oracle3_macroscopic.restype = ctypes.c_int
        L.oracle_run_trt.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _u8p,
                                     _dp, ctypes.c_long, ctypes.c_int]
        L.oracle_run_trt.restype = ctypes.c_int
        L.oracle_run_walls.argtypes = L.oracle_run_trt.argtypes + [ctypes.c_int]
        L.oracle_run_walls.restype = ctypes.c_int
        L.oracle_mrt_matrix.argtypes = [_dp]
        L.oracle_collide_mrt.argtypes = [_dp] + [ctypes.c_double] * 3 + [_dp, _dp]
        L.oracle_run_mrt.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp] + \
            [ctypes.c_double] * 6 + [_dp, _u8p, _dp, ctypes.c_long, ctypes.c_int, ctypes.c_int]
        L.oracle_run_mrt.restype = ctypes.c_int
        L.oracle_fullway_fill.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp]
        L.oracle_fullway_fill.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _mask(m):
    m = np.ascontiguousarray(m, dtype=np.uint8)
    if m.ndim != 2:
        raise ValueError("mask must be [ny, nx]")
    return m


def constants():
    """(cx, cy, w, opp) as the oracle uses them."""
    cx = (ctypes.c_int * 9)()
    cy = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    opp = (ctypes.c_int * 9)()
    lib().oracle_constants(cx, cy, w, opp)
    return (np.array(cx[:]), np.array(cy[:]), np.array(w[:]), np.array(opp[:]))


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    lib().oracle_equilibrium(rho, ux, uy, _d(out))
    return out


def guo_source(ux, uy, Fx, Fy):
    out = np.zeros(9)
    lib().oracle_guo_source(ux, uy, Fx, Fy, _d(out))
    return out


def node_velocity(f, alpha=0.0, g=(0.0, 0.0)):
    f = _f64(f)
    out = np.zeros(3)
    lib().oracle_node_velocity(_d(f), alpha, g[0], g[1], _d(out))
    return out


def collide(f, omega, alpha=0.0, g=(0.0, 0.0)):
    f = _f64(f)
    out = np.zeros(9)
    lib().oracle_collide(_d(f), alpha, g[0], g[1], omega, _d(out))
    return out


def collide_trt(f, omega_p, omega_m, alpha=0.0, g=(0.0, 0.0)):
    """Two-relaxation-time collision (omega_m = omega_p is BGK)."""
    f = _f64(f)
    out = np.zeros(9)
    lib().oracle_collide_trt(_d(f), alpha, g[0], g[1], omega_p, omega_m, _d(out))
    return out


def mrt_matrix():
    """The MRT moment matrix M [9, 9] (rows: rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy)."""
    M = np.zeros((9, 9))
    lib().oracle_mrt_matrix(_d(M))
    return M


def collide_mrt(f, rates, alpha=0.0, g=(0.0, 0.0)):
    """Multiple-relaxation-time collision with the nine moment rates `rates` (row order of
    mrt_matrix)."""
    f = _f64(f)
    r = np.ascontiguousarray(rates, dtype=np.float64)
    if r.shape != (9,):
        raise ValueError("rates must hold 9 values")
    out = np.zeros(9)
    lib().oracle_collide_mrt(_d(f), alpha, g[0], g[1], _d(r), _d(out))
    return out


def trt_tau_minus(tau, magic):
    """Antisymmetric relaxation time for the parameter Lambda = (tau - 1/2)(tau_m - 1/2)."""
    return 0.5 + magic / (tau - 0.5)


def collide_jacobian(f, omega, alpha=0.0, g=(0.0, 0.0)):
    """(d fstar/d f [9,9], d fstar/d alpha [9], d fstar/d g [9,2])."""
    f = _f64(f)
    dfdf = np.zeros((9, 9))
    dfda = np.zeros(9)
    dfdg = np.zeros((9, 2))
    lib().oracle_collide_jacobian(_d(f), alpha, g[0], g[1], omega, _d(dfdf), _d(dfda), _d(dfdg))
    return dfdf, dfda, dfdg


def zou_he(f, kind, normal, value):
    """One Zou-He boundary node: kind "velocity" (value = (u_x, u_y)) or "pressure"
    (value = (rho, -)), inward unit normal (n_x, n_y) along an axis."""
    f = _f64(f)
    out = np.zeros(9)
    k = {"velocity": 1, "pressure": 2}[kind]
    rc = lib().oracle_zou_he(_d(f), k, int(normal[0]), int(normal[1]), float(value[0]),
                             float(value[1]), _d(out))
    if rc:
        raise ValueError("bad normal")
    return out


def _bc_args(m, bc, value):
    if bc is None:
        return None, None
    ny, nx = m.shape
    bc = np.ascontiguousarray(bc, dtype=np.uint8)
    value = np.ascontiguousarray(value, dtype=np.float64)
    if bc.shape != (ny, nx) or value.shape != (2, ny, nx):
        raise ValueError("bc must be [ny, nx] and value [2, ny, nx]")
    return bc, value


def apply_boundaries(mask, f, bc, value):
    """Return a copy of f with the open-boundary conditions applied."""
    m = _mask(mask)
    ny, nx = m.shape
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    bc, value = _bc_args(m, bc, value)
    rc = lib().oracle_apply_boundaries(nx, ny, m.ctypes.data_as(_u8p), bc.ctypes.data_as(_u8p),
                                       _d(value), _d(f))
    if rc:
        raise ValueError("bad boundary code (or a code at a solid node)")
    return f


def init(mask, rho0=None, ux0=None, uy0=None, bc=None, value=None):
    """Equilibrium initial state (Algorithm 1, first loop); with open boundaries the
    boundary conditions are then applied, so that every state satisfies them."""
    m = _mask(mask)
    ny, nx = m.shape
    f = np.zeros((9, ny, nx))
    rho0, ux0, uy0 = _f64(rho0), _f64(ux0), _f64(uy0)
    rc = lib().oracle_init(nx, ny, m.ctypes.data_as(_u8p), _d(rho0), _d(ux0), _d(uy0), _d(f))
    if rc:
        raise ValueError("oracle_init failed")
    if bc is not None:
        f = apply_boundaries(m, f, bc, value)
    return f


def run(mask, f, tau, steps, g=(0.0, 0.0), alpha=None, threads=0, bc=None, value=None,
        tau_minus=None, fullway=False, mrt=None):
    """Advance a copy of f by `steps` time steps; returns the new array.  tau_minus: the
    antisymmetric relaxation time of the two-relaxation-time collision (None: BGK).
    mrt: (s_e, s_eps, s_q) selects the multiple-relaxation-time collision (shear rate
    1 / tau).  fullway: full-way bounce-back (f then includes the wall slots of solid nodes
    next to fluid)."""
    m = _mask(mask)
    ny, nx = m.shape
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    if f.shape != (9, ny, nx):
        raise ValueError("f must be [9, ny, nx]")
    alpha = _f64(alpha)
    bc, value = _bc_args(m, bc, value)
    if mrt is not None:
        if tau_minus is not None:
            raise ValueError("tau_minus and mrt are exclusive")
        se, sp, sq = (float(v) for v in mrt)
        rc = lib().oracle_run_mrt(nx, ny, m.ctypes.data_as(_u8p), _d(f), tau, se, sp, sq, g[0],
                                  g[1], _d(alpha), None if bc is None else bc.ctypes.data_as(_u8p),
                                  _d(value), int(steps), int(threads), int(bool(fullway)))
        if rc:
            raise ValueError(f"oracle_run failed ({rc})")
        return f
    tm = float(tau) if tau_minus is None else float(tau_minus)
    rc = lib().oracle_run_walls(nx, ny, m.ctypes.data_as(_u8p), _d(f), tau, tm, g[0], g[1],
                                _d(alpha), None if bc is None else bc.ctypes.data_as(_u8p),
                                _d(value), int(steps), int(threads), int(bool(fullway)))
    if rc:
        raise ValueError(f"oracle_run failed ({rc})")
    return f


def fullway_fill(mask, f):
    """Copy of f whose wall slots (solid nodes next to fluid) hold the full-way initial
    values: slot i of wall node w = f_i of the fluid node w - c_i, else 0."""
    m = _mask(mask)
    ny, nx = m.shape
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    if f.shape != (9, ny, nx):
        raise ValueError("f must be [9, ny, nx]")
    if lib().oracle_fullway_fill(nx, ny, m.ctypes.data_as(_u8p), _d(f)):
        raise ValueError("oracle_fullway_fill failed")
    return f


def macroscopic(mask, f, g=(0.0, 0.0), alpha=None):
    m = _mask(mask)
    ny, nx = m.shape
    f = _f64(f)
    rho, ux, uy = (np.zeros((ny, nx)) for _ in range(3))
    alpha = _f64(alpha)
    lib().oracle_macroscopic(nx, ny, m.ctypes.data_as(_u8p), _d(f), g[0], g[1], _d(alpha),
                             _d(rho), _d(ux), _d(uy))
    return rho, ux, uy


def objective_outlet_ux(mask, f, x_out, g=(0.0, 0.0), alpha=None):
    m = _mask(mask)
    ny, nx = m.shape
    f = _f64(f)
    J = ctypes.c_double()
    rc = lib().oracle_objective_outlet_ux(nx, ny, m.ctypes.data_as(_u8p), _d(f), g[0], g[1],
                                          _d(_f64(alpha)), x_out, ctypes.byref(J))
    if rc:
        raise ValueError("no fluid node in the outlet column")
    return J.value


def outlet_ux_gradient(mask, f0, tau, steps, x_out, g=(0.0, 0.0), alpha=None):
    """(J, dJ/dalpha [ny, nx], dJ/dg [2]) by reverse mode over `steps` steps from f0."""
    m = _mask(mask)
    ny, nx = m.shape
    f0 = _f64(f0)
    ga = np.zeros((ny, nx))
    gg = np.zeros(2)
    J = ctypes.c_double()
    rc = lib().oracle_outlet_ux_gradient(nx, ny, m.ctypes.data_as(_u8p), _d(f0), tau, g[0], g[1],
                                         _d(_f64(alpha)), int(steps), int(x_out), ctypes.byref(J),
                                         _d(ga), _d(gg))
    if rc:
        raise ValueError(f"oracle_outlet_ux_gradient failed ({rc})")
    return J.value, ga, gg


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# ------------------------------------------------------------------- D3Q19 --
# Arrays: mask uint8 [nz, ny, nx]; f float64 [19, nz, ny, nx]; g = (g_x, g_y, g_z).

def constants3():
    """(cx, cy, cz, w, opp) of the D3Q19 oracle."""
    c = [(ctypes.c_int * 19)() for _ in range(3)]
    w = (ctypes.c_double * 19)()
    opp = (ctypes.c_int * 19)()
    lib().oracle3_constants(c[0], c[1], c[2], w, opp)
    return tuple(np.array(a[:]) for a in c) + (np.array(w[:]), np.array(opp[:]))


def equilibrium3(rho, ux, uy, uz):
    out = np.zeros(19)
    lib().oracle3_equilibrium(rho, ux, uy, uz, _d(out))
    return out


def guo_source3(u, F):
    out = np.zeros(19)
    lib().oracle3_guo_source(u[0], u[1], u[2], F[0], F[1], F[2], _d(out))
    return out


def node_velocity3(f, g=(0.0, 0.0, 0.0)):
    f = _f64(f)
    out = np.zeros(4)
    lib().oracle3_node_velocity(_d(f), g[0], g[1], g[2], _d(out))
    return out


def collide3(f, omega, g=(0.0, 0.0, 0.0)):
    f = _f64(f)
    out = np.zeros(19)
    lib().oracle3_collide(_d(f), g[0], g[1], g[2], omega, _d(out))
    return out


def collide3_trt(f, omega_p, omega_m, g=(0.0, 0.0, 0.0)):
    """D3Q19 two-relaxation-time collision (omega_m = omega_p is BGK)."""
    f = _f64(f)
    out = np.zeros(19)
    lib().oracle3_collide_trt(_d(f), g[0], g[1], g[2], omega_p, omega_m, _d(out))
    return out


def _mask3(m):
    m = np.ascontiguousarray(m, dtype=np.uint8)
    if m.ndim != 3:
        raise ValueError("mask must be [nz, ny, nx]")
    return m


def init3(mask, rho0=None, ux0=None, uy0=None, uz0=None):
    m = _mask3(mask)
    nz, ny, nx = m.shape
    f = np.zeros((19, nz, ny, nx))
    fl = [_f64(a) for a in (rho0, ux0, uy0, uz0)]
    if lib().oracle3_init(nx, ny, nz, m.ctypes.data_as(_u8p), *[_d(a) for a in fl], _d(f)):
        raise ValueError("oracle3_init failed")
    return f


def mrt_matrix3():
    """The D3Q19 MRT moment matrix M [19, 19] (row order of oracle3_collide_mrt)."""
    M = np.zeros((19, 19))
    lib().oracle3_mrt_matrix(_d(M))
    return M


def collide3_mrt(f, rates, g=(0.0, 0.0, 0.0)):
    """D3Q19 multiple-relaxation-time collision with the 19 moment rates `rates`."""
    f = _f64(f)
    r = np.ascontiguousarray(rates, dtype=np.float64)
    if r.shape != (19,):
        raise ValueError("rates must hold 19 values")
    out = np.zeros(19)
    lib().oracle3_collide_mrt(_d(f), g[0], g[1], g[2], _d(r), _d(out))
    return out


def run3(mask, f, tau, steps, g=(0.0, 0.0, 0.0), threads=0, tau_minus=None, fullway=False,
         mrt=None):
    """Advance a copy of the D3Q19 state f by `steps` steps.  tau_minus: antisymmetric
    relaxation time of the two-relaxation-time collision (None: BGK).  mrt: (s_e, s_eps, s_q,
    s_pi, s_m) selects the multiple-relaxation-time collision (shear rate 1 / tau).  fullway:
    full-way bounce-back (f includes the wall slots)."""
    m = _mask3(mask)
    nz, ny, nx = m.shape
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    if f.shape != (19, nz, ny, nx):
        raise ValueError("f must be [19, nz, ny, nx]")
    if mrt is not None:
        if tau_minus is not None:
            raise ValueError("tau_minus and mrt are exclusive")
        r5 = np.ascontiguousarray(mrt, dtype=np.float64)
        if r5.shape != (5,):
            raise ValueError("mrt takes five rates (s_e, s_eps, s_q, s_pi, s_m)")
        rc = lib().oracle3_run_mrt(nx, ny, nz, m.ctypes.data_as(_u8p), _d(f), tau, _d(r5), g[0],
                                   g[1], g[2], int(steps), int(threads), int(bool(fullway)))
        if rc:
            raise ValueError(f"oracle3_run failed ({rc})")
        return f
    tm = float(tau) if tau_minus is None else float(tau_minus)
    rc = lib().oracle3_run_walls(nx, ny, nz, m.ctypes.data_as(_u8p), _d(f), tau, tm, g[0], g[1],
                                 g[2], int(steps), int(threads), int(bool(fullway)))
    if rc:
        raise ValueError(f"oracle3_run failed ({rc})")
    return f


def fullway_fill3(mask, f):
    """Copy of the D3Q19 state f with the full-way initial wall slots (slot i of wall node w =
    f_i of the fluid node w - c_i, else 0)."""
    m = _mask3(mask)
    nz, ny, nx = m.shape
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    if f.shape != (19, nz, ny, nx):
        raise ValueError("f must be [19, nz, ny, nx]")
    if lib().oracle3_fullway_fill(nx, ny, nz, m.ctypes.data_as(_u8p), _d(f)):
        raise ValueError("oracle3_fullway_fill failed")
    return f


def macroscopic3(mask, f, g=(0.0, 0.0, 0.0)):
    m = _mask3(mask)
    nz, ny, nx = m.shape
    f = _f64(f)
    out = [np.zeros((nz, ny, nx)) for _ in range(4)]
    lib().oracle3_macroscopic(nx, ny, nz, m.ctypes.data_as(_u8p), _d(f), g[0], g[1], g[2],
                              *[_d(a) for a in out])
    return tuple(out)
