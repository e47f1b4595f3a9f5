"""Linear stability of the D3Q27 HOME-LBM step -- TEST INFRASTRUCTURE.

Not part of the product.  The 3D counterpart of the D2Q9 analysis in
``d2q9.py``: the moment-space amplification matrix of the oracle's own step
and the largest drift speed at which it stays von Neumann stable, for the 3D
models and for the 2D ones.  Run as a script it prints the table of those
speed limits.

Source: "High-Performance Moment-Encoded Lattice Boltzmann Method with
Stability-Guided Quantization" (arXiv 2602.05295), Sec. 5.1-5.2 (plane-wave
analysis of the collide-and-stream map, G(k) = D(k) times the Jacobian of the
post-collision map, stable when max |lambda| <= 1) and Sec. 5.3 (the velocity
range is to lie inside the stable region).

In moment space the step maps the ten stored moments m(x) to
m'(x) = sum_i phi(c_i) f+_i(x - c_i), with f+ = h(collide(m)) and phi the
moment weights (1, c, c c - cs^2 delta).  A plane wave m = m^ exp(i k.x)
therefore has G(k) = sum_i exp(-i k.c_i) phi(c_i) d f+_i / d m, the moment
form of Eq. Mo-NOCM for this step; the cell Jacobian d f+ / d m comes from
complex steps through the C oracle.
"""
from __future__ import annotations

import itertools

import numpy as np

import oracle as orc
from oracle import d2q9

CS2 = 1.0 / 3.0
_H = 1e-30


def moment_weights(c):
    """phi(c_i): rows 1, c_x, c_y, c_z, then c_a c_b - cs^2 delta_ab in the
    stored order xx, yy, zz, xy, xz, yz (Eq. rho_u_stress)."""
    cx, cy, cz = np.asarray(c, float).T
    return np.stack([np.ones_like(cx), cx, cy, cz, cx * cx - CS2, cy * cy - CS2, cz * cz - CS2,
                     cx * cy, cx * cz, cy * cz], 1)


def cell_jacobian(tau, rho, u):
    """d f+ / d m (27 x 10) of the oracle's collide-and-reconstruct at the
    uniform equilibrium (rho, u)."""
    P = orc.make_params((4, 4, 4), tau)
    m0 = orc.equilibrium_moments(np.array(float(rho)), np.asarray(u, float))
    J = np.zeros((27, 10))
    for q in range(10):
        im = np.zeros(10)
        im[q] = _H
        J[:, q] = orc.post_collision_f(P, m0, im).imag / _H
    return J


def amplification_grid_3d(ks, tau, rho, u):
    """G(k) (10 x 10) for each wave vector of ks[..., 3]."""
    c = orc.lattice()[0]
    phi = moment_weights(c)
    J = cell_jacobian(tau, rho, u)
    ph = np.exp(-1j * (np.asarray(ks, float) @ c.T))
    return np.einsum("...i,ia,ib->...ab", ph, phi, J)


def wave_grid(dim, n):
    """n^dim wave vectors 2 pi j / n, j = 0 .. n-1 per axis (the full
    Brillouin zone of a periodic n^dim grid)."""
    axis = 2 * np.pi * np.arange(n) / n
    return np.array(list(itertools.product(axis, repeat=dim)))


def max_growth(dim, model, tau, u, n):
    """max |lambda| over the wave grid at drift u (3D: the oracle's step;
    2D: one of d2q9.MODELS)."""
    ks = wave_grid(dim, n)
    if dim == 3:
        G = amplification_grid_3d(ks, tau, 1.0, u)
    else:
        G = d2q9.amplification_grid(model, ks, 1.0, u[0], u[1], tau)
    return np.abs(np.linalg.eigvals(G)).max()


def speed_limit(dim, model, tau, direction, n, hi=0.6, iters=12):
    """The largest |u| along `direction` with max |lambda| <= 1 on the wave
    grid, by bisection on [0, hi] (assumes one crossing; hi if none)."""
    dvec = np.asarray(direction, float)
    dvec = dvec / np.linalg.norm(dvec)
    unstable = lambda s: max_growth(dim, model, tau, s * dvec, n) > 1 + 1e-10
    if not unstable(hi):
        return hi
    lo = 0.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if unstable(mid):
            hi = mid
        else:
            lo = mid
    return lo


def _print_limits():
    print("largest drift speed with max|lambda| <= 1 (bisection to 1.5e-4)")
    print("3D HOME-LBM step (App. A collision), 16^3 wave grid")
    for nu in (1e-2, 1e-3, 1e-4, 1e-5):
        tau = 0.5 + nu / CS2
        lims = [speed_limit(3, None, tau, dvec, 16) for dvec in ((1, 0, 0), (1, 1, 0), (1, 1, 1))]
        print(f"  nu {nu:<7g} x {lims[0]:.3f}  xy {lims[1]:.3f}  xyz {lims[2]:.3f}", flush=True)
    print("2D models, 64^2 wave grid: x / diagonal")
    for nu in (1e-3, 1e-4, 1e-5):
        tau = d2q9.tau_of_nu(nu)
        row = []
        for m in d2q9.MODELS:
            a = speed_limit(2, m, tau, (1, 0), 64)
            b = speed_limit(2, m, tau, (1, 1), 64)
            row.append(f"{m} {a:.3f}/{b:.3f}")
        print(f"  nu {nu:<7g} " + "  ".join(row), flush=True)


if __name__ == "__main__":
    _print_limits()
