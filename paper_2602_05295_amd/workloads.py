"""Seeded synthetic inputs for the HOME-LBM step.

Shared by the tests, the benchmark and the oracle checks.  It holds none of
the method's arithmetic: it only produces densities, velocities, random
moment fields, solid masks and domain tables, all from
``numpy.random.default_rng(seed)``.  Arrays are x-fastest: scalar fields have
shape (nz, ny, nx), vector fields (3, nz, ny, nx), moment fields
(10, nz, ny, nx).

The shapes and distributions stand in for the paper's scenes (Sec. 6): a
Taylor-Green vortex, decaying turbulence in a periodic box, a double shear
layer (the bit-allocation study), a channel with many obstacles, many small
domains, and a box with spheres.
"""
from __future__ import annotations

import numpy as np

CS = 1.0 / np.sqrt(3.0)  # lattice sound speed (cs^2 = 1/3, Sec. 3.2)


# ------------------------------------------------------------------ flows ---

def taylor_green_2d(nx: int, ny: int, nz: int, U0: float = 0.05):
    """2D Taylor-Green vortex, uniform in z, wavenumber k = 2 pi / nx (nx == ny).

    u_x = -U0 cos(kx) sin(ky), u_y = U0 sin(kx) cos(ky), u_z = 0 and the
    matching pressure, rho = 1 - (3 U0^2 / 4)(cos 2kx + cos 2ky).
    Returns (rho (nz, ny, nx), u (3, nz, ny, nx)).
    """
    if nx != ny:
        raise ValueError("taylor_green_2d needs nx == ny")
    k = 2.0 * np.pi / nx
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.zeros((nz, 1, 1))
    ux = -U0 * np.cos(k * x) * np.sin(k * y) + z
    uy = U0 * np.sin(k * x) * np.cos(k * y) + z
    uz = np.zeros_like(ux)
    rho = 1.0 - 0.75 * U0 * U0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) + z
    return rho, np.stack([ux, uy, uz])


def double_shear_layer(nx: int, ny: int, nz: int, U0: float = 0.04, width: float = 1.0 / 80.0,
                       amp: float = 0.05, zamp: float = 0.02, seed: int = 0):
    """A 3D analogue of the double-layer vortex: two periodic shear layers,
    u_x = U0 tanh((y/ny - 1/4)/width) below y = ny/2 and
    U0 tanh((3/4 - y/ny)/width) above, perturbed by
    u_y = amp U0 sin(2 pi (x/nx + 1/4)) and a small seeded random z
    modulation of that perturbation (so the roll-up is three-dimensional);
    rho = 1.  Returns (rho, u)."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    yy = (y + 0.5) / ny
    ux = np.where(yy <= 0.5, np.tanh((yy - 0.25) / width), np.tanh((0.75 - yy) / width))
    phase = rng.uniform(0, 2 * np.pi, 2)
    mod = 1.0 + zamp / amp * 0.5 * (np.sin(2 * np.pi * z / nz + phase[0]) + np.sin(4 * np.pi * z / nz + phase[1]))
    uy = amp * np.sin(2 * np.pi * (x / nx + 0.25)) * mod
    u = np.stack([U0 * ux, U0 * uy, np.zeros_like(ux)])
    return np.ones((nz, ny, nx)), u


def random_solenoidal(nx: int, ny: int, nz: int, kmax: float, umax: float, seed: int = 0):
    """Divergence-free random velocity field.

    iid complex-Gaussian vector amplitudes on the integer wavevectors
    0 < |n| <= kmax, each projected perpendicular to n; the real part of the
    inverse transform, scaled so that max |u| = umax.  Returns (3, nz, ny, nx).
    """
    rng = np.random.default_rng(seed)
    kk = int(np.floor(kmax))
    rngs = np.arange(-kk, kk + 1)
    n = np.stack(np.meshgrid(rngs, rngs, rngs, indexing="ij"), axis=-1).reshape(-1, 3)
    n2 = (n * n).sum(1)
    n = n[(n2 > 0) & (n2 <= kmax * kmax)]
    amp = rng.standard_normal((n.shape[0], 3)) + 1j * rng.standard_normal((n.shape[0], 3))
    amp -= n * ((amp * n).sum(1) / (n * n).sum(1))[:, None]
    spec = np.zeros((3, nz, ny, nx), dtype=np.complex128)
    # n = (nx-index, ny-index, nz-index); array axes are (z, y, x)
    spec[:, n[:, 2] % nz, n[:, 1] % ny, n[:, 0] % nx] = amp.T
    u = np.fft.ifftn(spec, axes=(1, 2, 3)).real
    speed = np.sqrt((u * u).sum(0)).max()
    return u * (umax / speed)


def random_moments(nx: int, ny: int, nz: int, seed: int = 0, drho: float = 0.01, dj: float = 0.03,
                   dp: float = 0.005):
    """An arbitrary smooth-free moment field near rest: rho = 1 + drho N(0,1),
    j = dj N(0,1), P = dp N(0,1) (symmetric entries drawn independently).
    Shape (10, nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    m = np.empty((10, nz, ny, nx))
    m[0] = 1.0 + drho * rng.standard_normal((nz, ny, nx))
    m[1:4] = dj * rng.standard_normal((3, nz, ny, nx))
    m[4:10] = dp * rng.standard_normal((6, nz, ny, nx))
    return m


# ------------------------------------------------------------------ masks ---

def _rasterize(mask, kind, center, half, periodic):
    """Set the cells of one axis-aligned ellipsoid (kind 0) or box (kind 1)."""
    nz, ny, nx = mask.shape
    lo = np.floor(center - half).astype(int)
    hi = np.ceil(center + half).astype(int) + 1
    idx = []
    for a, n in enumerate((nx, ny, nz)):
        r = np.arange(lo[a], hi[a])
        if not periodic:
            r = r[(r >= 0) & (r < n)]
        idx.append(r)
    if any(r.size == 0 for r in idx):
        return
    X = idx[0][None, None, :] + 0.0
    Y = idx[1][None, :, None] + 0.0
    Z = idx[2][:, None, None] + 0.0
    dx, dy, dz = (X - center[0]) / half[0], (Y - center[1]) / half[1], (Z - center[2]) / half[2]
    if kind == 0:
        inside = dx * dx + dy * dy + dz * dz <= 1.0
    else:
        inside = (np.abs(dx) <= 1.0) & (np.abs(dy) <= 1.0) & (np.abs(dz) <= 1.0)
    zi, yi, xi = (np.mod(idx[2], nz), np.mod(idx[1], ny), np.mod(idx[0], nx))
    sub = mask[np.ix_(zi, yi, xi)]
    mask[np.ix_(zi, yi, xi)] = sub | inside.astype(np.uint8)


def channel_obstacles(nx=1000, ny=400, nz=400, count=300, target=0.06, seed=0):
    """Obstacle table for the channel: half ellipsoids (semi-axes U[8,32] s),
    half boxes (half-extents U[6,26] s), axis-aligned, centres
    x in [0.15, 0.85] nx, y, z in [0.1, 0.9] ny/nz.  Returns (kinds, centres,
    unit sizes); the scale s is fixed by channel_mask."""
    rng = np.random.default_rng(seed)
    kinds = (np.arange(count) % 2).astype(int)
    rng.shuffle(kinds)
    cx = rng.uniform(0.15 * nx, 0.85 * nx, count)
    cy = rng.uniform(0.1 * ny, 0.9 * ny, count)
    cz = rng.uniform(0.1 * nz, 0.9 * nz, count)
    size = np.where(kinds[:, None] == 0, rng.uniform(8, 32, (count, 3)), rng.uniform(6, 26, (count, 3)))
    return kinds, np.stack([cx, cy, cz], 1), size


def _objects_mask(shape, kinds, centres, sizes, scale, periodic):
    mask = np.zeros(shape, dtype=np.uint8)
    for k, c, h in zip(kinds, centres, sizes):
        _rasterize(mask, k, c, np.maximum(h * scale, 0.5), periodic)
    return mask


def channel_mask(nx=1000, ny=400, nz=400, count=300, target=0.06, seed=0, tol=0.003):
    """Solid mask (nz, ny, nx) uint8 of the obstacle channel.  The scale s is
    bisected on a 4x coarser grid so that the union's solid fraction is
    target +- tol, then the mask is drawn at full resolution.  Cells within 2
    of the x faces stay fluid."""
    kinds, centres, sizes = channel_obstacles(nx, ny, nz, count, target, seed)
    c = 4
    shape_c = (max(1, nz // c), max(1, ny // c), max(1, nx // c))
    lo, hi = 0.05, 4.0
    s = 1.0
    for _ in range(30):
        s = 0.5 * (lo + hi)
        frac = _objects_mask(shape_c, kinds, centres / c, sizes / c, s, False).mean()
        if abs(frac - target) < 0.25 * tol:
            break
        if frac < target:
            lo = s
        else:
            hi = s
    mask = _objects_mask((nz, ny, nx), kinds, centres, sizes, s, False)
    mask[:, :, :3] = 0
    mask[:, :, nx - 3:] = 0
    return mask


def sphere_mask(nx, ny, nz, phi, rmin, rmax, seed=0, periodic=True, max_spheres=100000):
    """Random spheres (radius U[rmin, rmax], periodic wrap) added until the
    solid fraction is >= phi.  Shape (nz, ny, nx) uint8."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    if phi <= 0:
        return mask
    for _ in range(max_spheres):
        if mask.mean() >= phi:
            break
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0, 1, 3) * np.array([nx, ny, nz])
        _rasterize(mask, 0, c, np.array([r, r, r]), periodic)
    return mask


# ------------------------------------------------------------ workloads -----

def batched_domains(count=128, seed=0, nmin=24, nmax=96):
    """Table of small periodic domains: dims ~ U{nmin..nmax} per axis,
    tau ~ U[0.52, 0.8], solid fraction phi ~ U[0, 0.10] from spheres of radius
    U[3, 0.25 min(dims)], random solenoidal field (|n| <= 4, max|u| = 0.05)."""
    rng = np.random.default_rng(seed)
    doms = []
    for d in range(count):
        nx, ny, nz = (int(v) for v in rng.integers(nmin, nmax + 1, 3))
        tau = float(rng.uniform(0.52, 0.8))
        phi = float(rng.uniform(0.0, 0.10))
        sub = int(rng.integers(0, 2**31 - 1))
        doms.append(dict(dims=(nx, ny, nz), tau=tau, phi=phi, seed=sub))
    return doms


def batched_domain_fields(dom):
    """(mask, u) for one entry of batched_domains."""
    nx, ny, nz = dom["dims"]
    rmax = max(3.0, 0.25 * min(nx, ny, nz))
    mask = sphere_mask(nx, ny, nz, dom["phi"], 3.0, rmax, seed=dom["seed"])
    u = random_solenoidal(nx, ny, nz, 4.0, 0.05, seed=dom["seed"] + 1)
    return mask, u
