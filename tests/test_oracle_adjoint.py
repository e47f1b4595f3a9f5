"""Pins of the oracle's FP64 adjoint step: the dot-product identity
<J v, w> = <v, J^T w> (J v by complex step of the forward step) and central
finite differences of a multi-step loss, with walls and with open faces."""
import numpy as np
import pytest

from paper_2602_05295_amd import workloads as W


def _setup(orc, inflow):
    n = (7, 6, 5)
    mask = W.sphere_mask(*n, phi=0.12, rmin=1.0, rmax=1.8, seed=3)
    if inflow:
        mask[:, :, :3] = 0
        mask[:, :, -3:] = 0
    m = W.random_moments(*n, seed=6)
    m[0][mask == 1] = 1.0
    P = orc.make_params(n, 0.62, inflow=inflow, u_in=(0.06, 0.01, -0.02))
    return n, mask, m, P


@pytest.mark.parametrize("inflow", [False, True])
def test_adjoint_dot_product(orc, inflow):
    n, mask, m, P = _setup(orc, inflow)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(m.shape)
    w = rng.standard_normal(m.shape)
    Jv = orc.step_complex(P, m + 1j * 1e-30 * v, mask).imag / 1e-30
    JTw = orc.adjoint_step(P, m, w, mask)
    lhs, rhs = (Jv * w).sum(), (v * JTw).sum()
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.abs(Jv).sum())


@pytest.mark.parametrize("inflow", [False, True])
def test_adjoint_finite_differences(orc, inflow):
    n, mask, m0, P = _setup(orc, inflow)
    T = 4
    rng = np.random.default_rng(2)
    target = rng.standard_normal(m0.shape) * 0.01

    def loss(m):
        for _ in range(T):
            m = orc.step(P, m, mask)
        return 0.5 * ((m - target) ** 2).sum()

    traj = [m0]
    for _ in range(T):
        traj.append(orc.step(P, traj[-1], mask))
    lam = traj[-1] - target
    for t in range(T - 1, -1, -1):
        lam = orc.adjoint_step(P, traj[t], lam, mask)
    h = 1e-6
    for d in range(5):
        v = rng.standard_normal(m0.shape)
        v[:, mask == 1] = 0
        fd = (loss(m0 + h * v) - loss(m0 - h * v)) / (2 * h)
        ad = (lam * v).sum()
        assert abs(fd - ad) <= 1e-7 * abs(ad), (d, fd, ad)


@pytest.mark.parametrize("case", ["periodic", "walls", "faces"])
def test_gathered_adjoint_equals_scattered(orc, case):
    """adjoint_step_cells (gathered per source cell, used at sampled cells of
    large grids) equals adjoint_step (scattered per output cell) at every
    cell: periodic, with walls, and with open faces and walls."""
    dims = (9, 7, 6)
    mask = None
    inflow = case == "faces"
    if case != "periodic":
        mask = W.sphere_mask(*dims, phi=0.12, rmin=1.0, rmax=1.8, seed=2)
        if inflow:
            mask[:, :, :3] = 0
            mask[:, :, -3:] = 0
            mask[:, 2:5, 3:6] = 1
        assert mask.any()
    m = W.random_moments(*dims, seed=11, dj=0.02, dp=0.003)
    lam = np.random.default_rng(12).standard_normal(m.shape)
    P = orc.make_params(dims, 0.6, inflow=inflow, u_in=(0.05, 0.01, -0.02))
    ref = orc.adjoint_step(P, m, lam, mask)
    cells = np.arange(np.prod(dims))
    got = orc.adjoint_step_cells(P, m, lam, cells, mask)
    assert np.abs(got.T - ref.reshape(10, -1)).max() < 1e-13 * np.abs(ref).max()
