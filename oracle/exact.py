"""Exact-rational brute force of the D2Q9 update on tiny lattices (test infrastructure).

TEST INFRASTRUCTURE ONLY.  A second, independent statement of the same update in
pure Python with ``fractions.Fraction``: no rounding at all, so on a 4x4 lattice it
gives the exact value the FP64 oracle approximates.  It is written node by node from
the definitions, without arrays or loops shared with the C oracle:

  * moments (Sec. 2.2, Eq. 2) with the half-force velocity and implicit drag,
  * equilibrium (Eq. 6) and the BGK relaxation (Eqs. 3-5) plus Guo's forcing term,
  * streaming by pushing each post-collision population to x + v_i, bouncing back
    to the origin node with the reversed direction when x + v_i is solid.

With tau a rational number (omega = 1/tau rational) and rational initial fields and
forces, every intermediate value stays rational.
"""
from __future__ import annotations

from fractions import Fraction as Fr

# Lattice velocities in the paper's Fig. 1 numbering, written as (direction, vector).
VELOCITIES = {
    0: (0, 0),
    1: (1, 0),
    2: (0, 1),
    3: (-1, 0),
    4: (0, -1),
    5: (1, 1),
    6: (-1, 1),
    7: (-1, -1),
    8: (1, -1),
}
WEIGHTS = {0: Fr(4, 9), 1: Fr(1, 9), 2: Fr(1, 9), 3: Fr(1, 9), 4: Fr(1, 9),
           5: Fr(1, 36), 6: Fr(1, 36), 7: Fr(1, 36), 8: Fr(1, 36)}


def reverse(i):
    cx, cy = VELOCITIES[i]
    for j, (dx, dy) in VELOCITIES.items():
        if (dx, dy) == (-cx, -cy):
            return j
    raise AssertionError


def feq(rho, u):
    out = {}
    uu = u[0] * u[0] + u[1] * u[1]
    for i, (cx, cy) in VELOCITIES.items():
        cu = cx * u[0] + cy * u[1]
        out[i] = WEIGHTS[i] * rho * (1 + 3 * cu + Fr(9, 2) * cu * cu - Fr(3, 2) * uu)
    return out


def velocity(pops, alpha, g):
    rho = sum(pops[i] for i in range(9))
    mx = sum(VELOCITIES[i][0] * pops[i] for i in range(9))
    my = sum(VELOCITIES[i][1] * pops[i] for i in range(9))
    D = 1 + alpha / 2
    return rho, ((mx / rho + g[0] / 2) / D, (my / rho + g[1] / 2) / D)


def collide(pops, omega, alpha, g):
    rho, u = velocity(pops, alpha, g)
    F = (rho * (g[0] - alpha * u[0]), rho * (g[1] - alpha * u[1]))
    eq = feq(rho, u)
    out = {}
    for i, (cx, cy) in VELOCITIES.items():
        cu = cx * u[0] + cy * u[1]
        cF = cx * F[0] + cy * F[1]
        S = WEIGHTS[i] * (3 * ((cx - u[0]) * F[0] + (cy - u[1]) * F[1]) + 9 * cu * cF)
        out[i] = pops[i] - omega * (pops[i] - eq[i]) + (1 - omega / 2) * S
    return out


def step(state, solid, nx, ny, omega, alpha, g):
    """state: {(x, y): {i: Fraction}} for fluid nodes. Returns the next state."""
    post = {node: collide(p, omega, alpha.get(node, Fr(0)), g) for node, p in state.items()}
    nxt = {node: {} for node in state}
    for (x, y), p in post.items():
        for i, (cx, cy) in VELOCITIES.items():
            dest = ((x + cx) % nx, (y + cy) % ny)
            if dest in solid:
                nxt[(x, y)][reverse(i)] = p[i]
            else:
                nxt[dest][i] = p[i]
    return nxt


def run(mask, rho0, ux0, uy0, tau, steps, g=(Fr(0), Fr(0)), alpha=None):
    """Exact run.  mask: nested lists [ny][nx] of 0/1; fields: nested lists of Fractions.
    Returns {(x, y): {i: Fraction}} for fluid nodes after `steps` steps."""
    ny, nx = len(mask), len(mask[0])
    solid = {(x, y) for y in range(ny) for x in range(nx) if mask[y][x]}
    alpha_map = {}
    if alpha is not None:
        alpha_map = {(x, y): alpha[y][x] for y in range(ny) for x in range(nx)}
    state = {}
    for y in range(ny):
        for x in range(nx):
            if (x, y) not in solid:
                state[(x, y)] = feq(rho0[y][x], (ux0[y][x], uy0[y][x]))
    omega = 1 / Fr(tau)
    for _ in range(steps):
        state = step(state, solid, nx, ny, omega, alpha_map, g)
    return state
