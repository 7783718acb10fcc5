"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds geometry masks and initial / parameter fields only; it contains none
of the lattice-Boltzmann arithmetic, and neither the GPU library nor the oracle imports
the other through it.  Every generator is deterministic for a given seed.

Workloads (the paper measures on synthetic geometries of its own; these stand in):
  * channel: solid rows y = 0 and y = ny - 1, periodic in x (channel flow, Sec. 4.1);
  * Taylor-Green vortex: fully periodic, all fluid (stands in for the dense-geometry
    timing of Sec. 4.3, which used an all-fluid cavity: same traffic per node);
  * porous medium: random solid discs on a square domain with walls at y = 0 and
    y = ny - 1 (the sparse geometries of Sec. 4.3, built from circles of random radius);
  * Brinkman field: a smooth random drag-coefficient field in [0, 1];
  * open channels (Sec. 4.1, chan_v / chan_p): walls at y = 0 and y = ny - 1, a constant
    velocity or constant pressure inlet column at x = 0 and a constant pressure outlet
    column at x = nx - 1;
  * lid-driven cavity (Sec. 4.1): solid side and bottom walls, a constant-velocity lid;
  * 3-D (D3Q19) inputs, arrays [nz, ny, nx]: the three-dimensional Taylor-Green vortex
    (all fluid, periodic), random solids with optional walls at z = 0 and z = nz - 1,
    random fields, and random populations scaled per direction.

Open-boundary codes (one byte per node): 0 none, 1..4 constant velocity with inward
normal +x, -x, +y, -y, 5..8 constant pressure with the same normals; values [2, ny, nx]
hold (u_x, u_y) at velocity nodes and (rho, 0) at pressure nodes.
"""
from __future__ import annotations

import math

import numpy as np


def channel_mask(nx: int, ny: int) -> np.ndarray:
    """uint8 [ny, nx]: 1 on rows 0 and ny-1, 0 elsewhere."""
    m = np.zeros((ny, nx), dtype=np.uint8)
    m[0, :] = 1
    m[ny - 1, :] = 1
    return m


def all_fluid(nx: int, ny: int) -> np.ndarray:
    return np.zeros((ny, nx), dtype=np.uint8)


def taylor_green(n: int, u0: float = 0.01, ny: int | None = None):
    """Decaying Taylor-Green vortex on a periodic n x n lattice (node indices x, y),
    k = 2 pi / n:  u_x = -u0 cos(k x) sin(k y),  u_y = u0 sin(k x) cos(k y),
    rho = 1 - (3 u0^2 / 4) (cos 2kx + cos 2ky)  (pressure p = rho / 3).
    Returns (rho, ux, uy) as float64 [n, n]."""
    ny = n if ny is None else ny
    if ny != n:
        raise ValueError("the Taylor-Green initial field is defined on square lattices here")
    k = 2.0 * math.pi / n
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    rho = 1.0 - 0.75 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return (np.ascontiguousarray(rho), np.ascontiguousarray(ux), np.ascontiguousarray(uy))


def random_fields(nx: int, ny: int, seed: int, rho_spread: float = 0.05, u_amp: float = 0.05):
    """Random smooth-free fields: rho in [1-spread, 1+spread], |u_a| <= u_amp."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rho_spread * (2.0 * rng.random((ny, nx)) - 1.0)
    ux = u_amp * (2.0 * rng.random((ny, nx)) - 1.0)
    uy = u_amp * (2.0 * rng.random((ny, nx)) - 1.0)
    return rho, ux, uy


def random_mask(nx: int, ny: int, seed: int, solid_fraction: float = 0.2,
                walls: bool = False) -> np.ndarray:
    """Independent random solid nodes (a harsh bounce-back test geometry)."""
    rng = np.random.default_rng(seed)
    m = (rng.random((ny, nx)) < solid_fraction).astype(np.uint8)
    if walls:
        m[0, :] = 1
        m[ny - 1, :] = 1
    if not (m == 0).any():
        m[ny // 2, nx // 2] = 0
    return m


def porous_discs(n: int, phi: float, seed: int | None = None, rmin: int = 8, rmax: int = 64,
                 jam_limit: int = 5000, ny: int | None = None):
    """Porous medium of random solid discs with fluid fraction close to `phi`.

    Square n x ny domain (ny defaults to n); solid rows y = 0 and y = ny - 1; periodic in x.
    Radii are uniform integers in [rmin, rmax]; centres uniform in [0, n) x [1, ny - 1).
    Node (x, y) is solid if dx^2 + dy^2 <= r^2 (dx periodic in x, dy not wrapped).
    Discs are placed without overlap (centre distance >= r1 + r2 + 1) until the solid
    fraction reaches 1 - phi; after `jam_limit` consecutive rejected candidates, overlap
    is allowed (random non-overlapping placement jams well below 80 % coverage).

    Returns (mask uint8 [ny, n], info dict with the achieved fluid fraction, the number of
    discs and whether overlap had to be allowed)."""
    ny = n if ny is None else ny
    if seed is None:
        seed = 1000 + int(round(100 * phi))
    rng = np.random.default_rng(seed)
    m = np.zeros((ny, n), dtype=np.uint8)
    m[0, :] = 1
    m[ny - 1, :] = 1
    target_solid = int(math.ceil((1.0 - phi) * n * ny))
    solid = int(m.sum())
    # clear[y, x] = min over placed discs j of (|(x, y) - c_j| - r_j), kept exactly where it
    # can still reject a candidate (below rmax + 1); a candidate (c, r) is free of overlap
    # iff clear[c] >= r + 1, which is the pairwise rule |c - c_j| >= r + r_j + 1.
    clear = np.full((ny, n), np.inf)
    k = 0
    rejects = 0
    overlap = False
    batch = 4096
    while solid < target_solid:
        rs = rng.integers(rmin, rmax + 1, size=batch)
        cxs = rng.integers(0, n, size=batch)
        cys = rng.integers(1, ny - 1, size=batch)
        j = 0
        while j < batch and solid < target_solid:
            if not overlap:
                ok = clear[cys[j:], cxs[j:]] >= rs[j:] + 1
                idx = np.flatnonzero(ok)
                first = j + int(idx[0]) if idx.size else batch
                gap = first - j
                if rejects + gap >= jam_limit:
                    # jammed: the candidate after the jam_limit-th consecutive rejection on
                    # is accepted with overlap allowed
                    j = j + (jam_limit - rejects)
                    rejects = 0
                    overlap = True
                    continue
                rejects += gap
                if first >= batch:
                    break
                j = first
            r, cx, cy = int(rs[j]), int(cxs[j]), int(cys[j])
            j += 1
            rejects = 0
            k += 1
            y0, y1 = max(cy - r, 0), min(cy + r, ny - 1)
            ys = np.arange(y0, y1 + 1)[:, None]
            xs = np.arange(cx - r, cx + r + 1)[None, :]
            inside = (xs - cx) ** 2 + (ys - cy) ** 2 <= r * r
            cols = np.mod(xs[0], n)
            block = m[y0:y1 + 1][:, cols]
            solid += int((inside & (block == 0)).sum())
            block[inside] = 1
            m[y0:y1 + 1, cols] = block
            if not overlap:
                reach = r + rmax + 1
                wy0, wy1 = max(cy - reach, 0), min(cy + reach, ny - 1)
                wys = np.arange(wy0, wy1 + 1)[:, None]
                wxs = np.arange(cx - reach, cx + reach + 1)[None, :]
                dist = np.sqrt(((wxs - cx) ** 2 + (wys - cy) ** 2).astype(np.float64)) - r
                wcols = np.mod(wxs[0], n)
                win = clear[wy0:wy1 + 1][:, wcols]
                clear[wy0:wy1 + 1, wcols] = np.minimum(win, dist)
    info = {
        "phi_target": phi,
        "phi_achieved": float((m == 0).sum()) / (n * ny),
        "discs": k,
        "overlap_allowed": overlap,
        "seed": seed,
    }
    return m, info


def brinkman_alpha(nx: int, ny: int, seed: int = 7, sigma: float = 8.0) -> np.ndarray:
    """Smooth random drag-coefficient field in [0, 1]: white noise (seeded) filtered by a
    Gaussian of width `sigma` nodes (periodic, by FFT), standardised to s, then
    alpha = (1 + tanh(2 (s - 1))) / 2.  Mostly close to 0 with blobs close to 1."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (math.pi ** 2) * (sigma ** 2) * (kx ** 2 + ky ** 2))
    s = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))
    s = (s - s.mean()) / (s.std() + 1e-300)
    return np.ascontiguousarray(0.5 * (1.0 + np.tanh(2.0 * (s - 1.0))))


BC_VELOCITY = {(1, 0): 1, (-1, 0): 2, (0, 1): 3, (0, -1): 4}
BC_PRESSURE = {(1, 0): 5, (-1, 0): 6, (0, 1): 7, (0, -1): 8}


def open_channel(nx: int, ny: int, inlet: str = "velocity", u_in: float = 0.1,
                 rho_in: float = 1.016, rho_out: float = 1.0):
    """Channel with walls at y = 0 and ny - 1, inlet column x = 0 (constant velocity
    (u_in, 0) or constant density rho_in) and outlet column x = nx - 1 (constant density
    rho_out).  Returns (mask, bc, value)."""
    if nx < 3 or ny < 3:
        raise ValueError("open channel needs nx, ny >= 3")
    mask = channel_mask(nx, ny)
    bc = np.zeros((ny, nx), dtype=np.uint8)
    value = np.zeros((2, ny, nx), dtype=np.float64)
    if inlet == "velocity":
        bc[1:ny - 1, 0] = BC_VELOCITY[(1, 0)]
        value[0, 1:ny - 1, 0] = u_in
    elif inlet == "pressure":
        bc[1:ny - 1, 0] = BC_PRESSURE[(1, 0)]
        value[0, 1:ny - 1, 0] = rho_in
    else:
        raise ValueError("inlet is 'velocity' or 'pressure'")
    bc[1:ny - 1, nx - 1] = BC_PRESSURE[(-1, 0)]
    value[0, 1:ny - 1, nx - 1] = rho_out
    return mask, bc, value


def lid_cavity(n: int, u_lid: float = 0.1, ny: int | None = None):
    """Square cavity: solid columns x = 0 and x = n - 1 and solid row y = 0; the top row
    y = ny - 1 (x = 1 .. n - 2) is a constant-velocity lid moving with (u_lid, 0).
    Returns (mask, bc, value)."""
    ny = n if ny is None else ny
    if n < 3 or ny < 3:
        raise ValueError("cavity needs n, ny >= 3")
    mask = np.zeros((ny, n), dtype=np.uint8)
    mask[:, 0] = 1
    mask[:, n - 1] = 1
    mask[0, :] = 1
    bc = np.zeros((ny, n), dtype=np.uint8)
    value = np.zeros((2, ny, n), dtype=np.float64)
    bc[ny - 1, 1:n - 1] = BC_VELOCITY[(0, -1)]
    value[0, ny - 1, 1:n - 1] = u_lid
    return mask, bc, value


# ---------------------------------------------------------------- sparse study --
# The paper's sparse geometries (Sec. 4.3, Fig. 7 and 8): square n x n domains filled with
# solid circles, bounce-back walls at y = 0 and y = n - 1, constant-pressure inlet (left,
# rho = 1.016) and outlet (right, rho = 1.0).  Porosity phi (Eq. 8) counts every non-solid
# node over all nodes.

def _paint_circle(m, cx, cy, r):
    """Mark the nodes with (x - cx)^2 + (y - cy)^2 <= r^2 solid (clipped to the domain, no
    wrap); returns the number of nodes that became solid."""
    ny, nx = m.shape
    y0, y1 = max(int(math.floor(cy - r)), 0), min(int(math.ceil(cy + r)), ny - 1)
    x0, x1 = max(int(math.floor(cx - r)), 0), min(int(math.ceil(cx + r)), nx - 1)
    if y0 > y1 or x0 > x1:
        return 0
    ys = np.arange(y0, y1 + 1, dtype=np.float64)[:, None]
    xs = np.arange(x0, x1 + 1, dtype=np.float64)[None, :]
    inside = (xs - cx) ** 2 + (ys - cy) ** 2 <= r * r
    block = m[y0:y1 + 1, x0:x1 + 1]
    new = int((inside & (block == 0)).sum())
    block[inside] = 1
    return new


def _open_ends(m, rho_in=1.016, rho_out=1.0):
    """Pressure inlet on the fluid nodes of column 0, outlet on those of column n - 1."""
    ny, nx = m.shape
    bc = np.zeros((ny, nx), dtype=np.uint8)
    value = np.zeros((2, ny, nx), dtype=np.float64)
    rows = np.arange(1, ny - 1)
    inl = rows[m[rows, 0] == 0]
    out = rows[m[rows, nx - 1] == 0]
    bc[inl, 0] = BC_PRESSURE[(1, 0)]
    value[0, inl, 0] = rho_in
    bc[out, nx - 1] = BC_PRESSURE[(-1, 0)]
    value[0, out, nx - 1] = rho_out
    return bc, value


def _walls(n):
    m = np.zeros((n, n), dtype=np.uint8)
    m[0, :] = 1
    m[n - 1, :] = 1
    return m


def circle_array(n: int, phi: float, k: int = 8):
    """Regular arrangement (Sec. 4.3): a k x k array of equal solid circles centred at
    ((i + 1/2) n / k, (j + 1/2) n / k); the radius is the largest (to 1e-6 node) whose
    porosity is still >= phi.  phi < 0.3 is refused: the circles then overlap and close
    the domain walls (why the paper stops there).  Returns (mask, bc, value, info)."""
    if phi < 0.3 or phi > 1.0:
        raise ValueError("the regular circle array is defined for 0.3 <= phi <= 1")
    centres = [((i + 0.5) * n / k, (j + 0.5) * n / k) for j in range(k) for i in range(k)]

    def build(r):
        m = _walls(n)
        for cx, cy in centres:
            _paint_circle(m, cx, cy, r)
        return m

    def porosity(m):
        return float((m == 0).sum()) / (n * n)

    lo, hi = 0.0, n / (2.0 * k) * math.sqrt(2.0) + 1.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if porosity(build(mid)) >= phi:
            lo = mid
        else:
            hi = mid
    m = build(lo)
    bc, value = _open_ends(m)
    return m, bc, value, {"kind": "regular", "phi_target": phi, "phi_achieved": porosity(m),
                          "radius": lo, "circles": k * k}


def random_circles(n: int, phi: float, seed: int | None = None, rmin: int = 8, rmax: int = 256):
    """Random arrangement (Sec. 4.3): circles with integer radii uniform in [rmin, rmax] and
    centres uniform over the domain (overlap allowed, clipped at the domain edges) are added
    until the porosity falls to phi or below.  Seeded by 2000 + round(100 phi) by default.
    Returns (mask, bc, value, info)."""
    if seed is None:
        seed = 2000 + int(round(100 * phi))
    rng = np.random.default_rng(seed)
    m = _walls(n)
    solid = int(m.sum())
    target = int(math.ceil((1.0 - phi) * n * n))
    count = 0
    while solid < target:
        r = int(rng.integers(rmin, rmax + 1))
        cx, cy = int(rng.integers(0, n)), int(rng.integers(0, n))
        solid += _paint_circle(m, cx, cy, r)
        count += 1
    bc, value = _open_ends(m)
    return m, bc, value, {"kind": "random", "phi_target": phi,
                          "phi_achieved": float((m == 0).sum()) / (n * n), "circles": count,
                          "seed": seed}


def open_box(n: int):
    """The dense counterpart of the sparse geometries: walls, pressure inlet and outlet, no
    obstacles (the reference geometry of the sparse efficiency, Eq. 9)."""
    m = _walls(n)
    bc, value = _open_ends(m)
    return m, bc, value, {"kind": "dense", "phi_achieved": float((m == 0).sum()) / (n * n)}


# ------------------------------------------------------------------ 3-D inputs --
def taylor_green3(n: int, u0: float = 0.01):
    """Three-dimensional Taylor-Green vortex on a periodic n^3 lattice, k = 2 pi / n:
    u_x = u0 sin(kx) cos(ky) cos(kz), u_y = -u0 cos(kx) sin(ky) cos(kz), u_z = 0,
    p - p0 = (u0^2 / 16) (cos 2kx + cos 2ky)(cos 2kz + 2) with rho = 1 + 3 (p - p0).
    Returns (rho, ux, uy, uz) as float64 [n, n, n] (index [z, y, x])."""
    k = 2.0 * math.pi / n
    c = np.arange(n, dtype=np.float64) * k
    x, y, z = c[None, None, :], c[None, :, None], c[:, None, None]
    ux = u0 * np.sin(x) * np.cos(y) * np.cos(z)
    uy = -u0 * np.cos(x) * np.sin(y) * np.cos(z)
    uz = np.zeros((n, n, n))
    rho = 1.0 + 3.0 * (u0 * u0 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    return tuple(np.ascontiguousarray(np.broadcast_to(a, (n, n, n))) for a in (rho, ux, uy, uz))


def random_mask3(nx: int, ny: int, nz: int, seed: int, solid_fraction: float = 0.15,
                 walls: bool = False) -> np.ndarray:
    """Independent random solid nodes [nz, ny, nx]; walls: solid planes z = 0 and nz - 1."""
    rng = np.random.default_rng(seed)
    m = (rng.random((nz, ny, nx)) < solid_fraction).astype(np.uint8)
    if walls:
        m[0] = 1
        m[nz - 1] = 1
    if not (m == 0).any():
        m[nz // 2, ny // 2, nx // 2] = 0
    return m


def random_spheres3(n: int, phi: float, seed: int | None = None, rmin: int = 4,
                    rmax: int = 16) -> np.ndarray:
    """n^3 mask (uint8 [nz, ny, nx]) of a 3-D porous medium: solid spheres with integer radii
    uniform in [rmin, rmax] and centres uniform over the periodic box (overlap allowed), added
    until the fluid fraction is <= phi; walls at z = 0 and n - 1.  Seeded by
    default_rng(3000 + round(100 phi)) unless `seed` is given."""
    rng = np.random.default_rng(3000 + int(round(100 * phi)) if seed is None else seed)
    m = np.zeros((n, n, n), np.uint8)
    m[0] = 1
    m[n - 1] = 1
    target = (1.0 - phi) * m.size
    solid = int(m.sum())
    while solid < target:
        r = int(rng.integers(rmin, rmax + 1))
        c = rng.integers(0, n, size=3)
        d = np.arange(-r, r + 1)
        dz, dy, dx = np.meshgrid(d, d, d, indexing="ij")
        inside = dx * dx + dy * dy + dz * dz <= r * r
        zz, yy, xx = ((c[0] + dz) % n)[inside], ((c[1] + dy) % n)[inside], ((c[2] + dx) % n)[inside]
        solid += int((m[zz, yy, xx] == 0).sum())  # distinct cells: 2 r + 1 <= n
        m[zz, yy, xx] = 1
    return m


def random_fields3(nx: int, ny: int, nz: int, seed: int, rho_spread: float = 0.03,
                   u_amp: float = 0.03):
    """rho in [1 - spread, 1 + spread], each velocity component in [-u_amp, u_amp]."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rho_spread * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    u = [u_amp * (2.0 * rng.random((nz, ny, nx)) - 1.0) for _ in range(3)]
    return (rho, *u)


def random_populations(scale, shape, seed: int, amp: float = 0.05) -> np.ndarray:
    """Populations scale[i] * (1 + amp * U(-1, 1)) of shape [len(scale), *shape] (float64):
    a state away from equilibrium, so that the collision's relaxation is exercised."""
    rng = np.random.default_rng(seed)
    scale = np.asarray(scale, np.float64).reshape((-1,) + (1,) * len(shape))
    f = rng.random((scale.shape[0],) + tuple(shape))
    f *= 2.0 * amp
    f += 1.0 - amp
    f *= scale
    return f
