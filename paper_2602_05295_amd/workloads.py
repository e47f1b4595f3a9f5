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


def _channel_scale(nx, ny, nz, kinds, centres, sizes, target, tol=0.003):
    """The obstacle scale s: bisected on a 4x coarser grid until the union's
    solid fraction is target +- tol/4."""
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
    return s


def channel_mask(nx=1000, ny=400, nz=400, count=300, target=0.06, seed=0, tol=0.003):
    """Solid mask (nz, ny, nx) uint8 of the obstacle channel.  The scale s is
    bisected on a 4x coarser grid so that the union's solid fraction is
    target +- tol, then the mask is drawn at full resolution.  Cells within 2
    of the x faces stay fluid."""
    kinds, centres, sizes = channel_obstacles(nx, ny, nz, count, target, seed)
    s = _channel_scale(nx, ny, nz, kinds, centres, sizes, target, tol)
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


# ------------------------------------------------------------------ meshes ---
# Triangle meshes of the channel's obstacles, for the per-triangle solid
# correction.  Every obstacle is a closed convex polyhedron: an axis-aligned
# box whose faces are cut into small triangles, or a latitude-longitude
# polyhedron inscribed in an axis-aligned ellipsoid.  The solid mask of a mesh
# scene marks the lattice points inside a polyhedron (on its surface counts as
# inside), so every link from a fluid cell to a solid one crosses a mesh.

def _sphere_grid(nt: int, nph: int):
    """Unit-sphere vertices V[k, l] (k = 0..nt polar, l = 0..nph azimuthal,
    column nph repeating column 0)."""
    th = np.pi * np.arange(nt + 1) / nt
    ph = 2.0 * np.pi * (np.arange(nph + 1) % nph) / nph
    st, ct = np.sin(th)[:, None], np.cos(th)[:, None]
    return np.stack([st * np.cos(ph)[None, :], st * np.sin(ph)[None, :], np.broadcast_to(ct, (nt + 1, nph + 1))], -1)


def _sphere_facets(nt: int, nph: int):
    """Triangles (T, 3, 3) of the unit polyhedron with nt bands and nph
    sectors, and its facet planes n.x <= d per (band, sector): n (nt, nph, 3),
    d (nt, nph).  Band quads are planar (two triangles, one plane); the polar
    bands are fans of single triangles."""
    V = _sphere_grid(nt, nph)
    k = np.arange(nt)[:, None]
    l = np.arange(nph)[None, :]
    v00, v01, v10, v11 = V[k, l], V[k, l + 1], V[k + 1, l], V[k + 1, l + 1]
    # plane of each facet from three of its distinct corners
    a = np.where((k == 0)[..., None], v00, v00)
    b = np.where((k == nt - 1)[..., None], v10, v10)
    c = np.where((k == nt - 1)[..., None], v01, v11)
    n = np.cross(b - a, c - a)
    n = n / np.linalg.norm(n, axis=-1, keepdims=True)
    d = (n * a).sum(-1)
    flip = d < 0
    n[flip] *= -1.0
    d[flip] *= -1.0
    tris = []
    tris.append(np.stack([v00[0], v10[0], v11[0]], 1))                 # north fan
    if nt > 2:
        mid = slice(1, nt - 1)
        tris.append(np.stack([v00[mid], v10[mid], v11[mid]], 2).reshape(-1, 3, 3))
        tris.append(np.stack([v00[mid], v11[mid], v01[mid]], 2).reshape(-1, 3, 3))
    tris.append(np.stack([v00[nt - 1], v10[nt - 1], v01[nt - 1]], 1))  # south fan
    return np.concatenate(tris, 0), n, d


def ellipsoid_mesh(center, semi, edge: float = 1.5):
    """Mesh of the polyhedron inscribed in an axis-aligned ellipsoid, with
    edges of about `edge` cells: (triangles (T, 3, 3), (nt, nph))."""
    a = np.asarray(semi, float)
    nt = max(4, int(np.ceil(np.pi * a.max() / edge)))
    nph = max(8, int(np.ceil(2.0 * np.pi * a.max() / edge)))
    unit, _, _ = _sphere_facets(nt, nph)
    return np.asarray(center, float) + unit * a, (nt, nph)


def inside_ellipsoid_mesh(points, center, semi, grid):
    """Whether points (..., 3) lie inside (or on) the inscribed polyhedron of
    ellipsoid_mesh: in the frame where the ellipsoid is the unit sphere, the
    facets near the point's direction (one band and sector either side of
    the one it points into) must all hold it."""
    nt, nph = grid
    _, n, d = _sphere_facets(nt, nph)
    q = (np.asarray(points, float) - np.asarray(center, float)) / np.asarray(semi, float)
    r = np.linalg.norm(q, axis=-1)
    th = np.arccos(np.clip(q[..., 2] / np.maximum(r, 1e-300), -1.0, 1.0))
    ph = np.mod(np.arctan2(q[..., 1], q[..., 0]), 2.0 * np.pi)
    k0 = np.clip((th / (np.pi / nt)).astype(int), 0, nt - 1)
    l0 = np.clip((ph / (2.0 * np.pi / nph)).astype(int), 0, nph - 1)
    inside = r <= 1.0
    for dk in (-1, 0, 1):
        kk = np.clip(k0 + dk, 0, nt - 1)
        for dl in (-1, 0, 1):
            ll = np.mod(l0 + dl, nph)
            inside &= (n[kk, ll] * q).sum(-1) <= d[kk, ll]
    return inside


def box_mesh(center, half, edge: float = 1.5):
    """Mesh of an axis-aligned box (center, half-extents): every face cut
    into a grid of quads of about `edge` cells, two triangles each."""
    c = np.asarray(center, float)
    h = np.asarray(half, float)
    tris = []
    for ax in range(3):
        u, v = [a for a in range(3) if a != ax]
        nu = max(1, int(np.ceil(2.0 * h[u] / edge)))
        nv = max(1, int(np.ceil(2.0 * h[v] / edge)))
        su = -h[u] + 2.0 * h[u] * np.arange(nu + 1) / nu
        sv = -h[v] + 2.0 * h[v] * np.arange(nv + 1) / nv
        for sgn in (-1.0, 1.0):
            P = np.zeros((nu + 1, nv + 1, 3))
            P[..., ax] = sgn * h[ax]
            P[..., u] = su[:, None]
            P[..., v] = sv[None, :]
            p00, p10, p01, p11 = P[:-1, :-1], P[1:, :-1], P[:-1, 1:], P[1:, 1:]
            tris.append(np.stack([p00, p10, p11], 2).reshape(-1, 3, 3))
            tris.append(np.stack([p00, p11, p01], 2).reshape(-1, 3, 3))
    return c + np.concatenate(tris, 0)


def mesh_scene(shape, objects, edge: float = 1.5):
    """Solid mask and triangle list of closed convex obstacles.  objects:
    (kind, center (x, y, z), size (3), id) with kind 0 an ellipsoid
    (semi-axes) and kind 1 a box (half-extents), id in 1..255 (the mask value
    of its cells and the object of its triangles).  Returns (mask (nz, ny, nx)
    uint8, triangles (T, 9) float32 as x0 y0 z0 x1 ... z2, object id per
    triangle (T,) uint8).  The mask marks the lattice points inside a
    polyhedron of the exact geometry; the triangles are its vertices rounded
    to float32, so a lattice point within rounding distance (about 1e-7 of
    its coordinates) of a facet may lie on the other side of the rounded
    mesh."""
    nz, ny, nx = shape
    mask = np.zeros(shape, dtype=np.uint8)
    tris, ids = [], []
    for kind, c, size, oid in objects:
        c = np.asarray(c, float)
        size = np.asarray(size, float)
        if kind == 0:
            t, grid = ellipsoid_mesh(c, size, edge)
        else:
            t = box_mesh(c, size, edge)
        lo = np.maximum(np.floor(c - size).astype(int) - 1, 0)
        hi = np.minimum(np.ceil(c + size).astype(int) + 2, [nx, ny, nz])
        if np.any(hi <= lo):
            continue
        Z, Y, X = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]), np.arange(lo[0], hi[0]),
                              indexing="ij")
        pts = np.stack([X, Y, Z], -1).astype(float)
        if kind == 0:
            ins = inside_ellipsoid_mesh(pts, c, size, grid)
        else:
            ins = np.all(np.abs(pts - c) <= size, axis=-1)
        sub = mask[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub[ins] = np.uint8(oid)
        tris.append(t.reshape(-1, 9))
        ids.append(np.full(t.shape[0], oid, np.uint8))
    if not tris:
        return mask, np.zeros((0, 9), np.float32), np.zeros(0, np.uint8)
    return mask, np.concatenate(tris).astype(np.float32), np.concatenate(ids)


def channel_mesh(nx=1000, ny=400, nz=400, count=300, target=0.06, seed=0, edge=1.5):
    """The obstacle channel of channel_mask with its ellipsoids and boxes as
    triangle meshes (object id 1 for all): (mask, triangles, ids).  The
    ellipsoids' polyhedra are inscribed, so the solid fraction is a little
    below channel_mask's."""
    kinds, centres, sizes = channel_obstacles(nx, ny, nz, count, target, seed)
    s = _channel_scale(nx, ny, nz, kinds, centres, sizes, target)
    objs = [(int(k), c, np.maximum(h * s, 0.5), 1) for k, c, h in zip(kinds, centres, sizes)]
    mask, tris, ids = mesh_scene((nz, ny, nx), objs, edge)
    mask[:, :, :3] = 0
    mask[:, :, nx - 3:] = 0
    return mask, tris, ids
