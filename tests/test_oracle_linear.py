"""Pins of the oracle's linearised step (Sec. 5.1-5.2).

The complex-step Jacobian of the whole periodic step at a uniform state is
block circulant; its block Fourier transform must equal the 10x10 moment-space
amplification matrix G(k) = sum_i exp(-i k.c_i) phi(c_i) d f+_i / d m, the
moment form of Eq. (Mo-NOCM) for pull streaming.  G(0) has the closed-form
spectrum {1 (x4), 0, 1 - 1/tau (x5)}; small-k modes follow Eqs. (shear_mode,
acoustic_modes), the sound modes decaying with the bulk viscosity of App. A's
trace reset; and the von Neumann criterion max|lambda| <= 1 holds at u = 0
and at the drift speeds of the benchmark workloads."""
import itertools

import numpy as np
import pytest

import oracle as orc_mod
from oracle import stability

CS2 = 1.0 / 3.0
H = 1e-30


def _phi(c):
    cx, cy, cz = c.T
    return np.stack([np.ones(27), cx, cy, cz, cx * cx - CS2, cy * cy - CS2, cz * cz - CS2, cx * cy, cx * cz, cy * cz],
                    1).astype(float)


def _cell_jac(orc, P, m0):
    J = np.zeros((27, 10))
    for k in range(10):
        im = np.zeros(10)
        im[k] = H
        J[:, k] = orc.post_collision_f(P, m0, im).imag / H
    return J


def _G(c, PHI, J, k):
    ph = np.exp(-1j * (c @ k))
    return (PHI.T * ph) @ J


def _uniform(orc, rho, u, neq=None):
    m = orc.equilibrium_moments(np.array(rho), np.asarray(u, float))
    if neq is not None:
        m[4:] += neq
    return m


def test_full_jacobian_equals_fourier_symbol(orc):
    c, w, _ = orc.lattice()
    PHI = _phi(c)
    N = 4
    P = orc.make_params((N, N, N), 0.6)
    m0 = _uniform(orc, 1.02, [0.05, -0.03, 0.02], np.array([1e-3, -2e-3, 5e-4, 3e-4, -1e-4, 2e-4]))
    J = _cell_jac(orc, P, m0)
    Nc = N ** 3
    M = np.repeat(m0[:, None], Nc, axis=1).reshape(10, N, N, N)
    # columns of the full Jacobian restricted to output cell 0
    rows = np.arange(10) * Nc
    Jcol = np.zeros((10, 10 * Nc))
    for q in range(10 * Nc):
        im = np.zeros(10 * Nc)
        im[q] = H
        Jcol[:, q] = orc.step_complex(P, M + 1j * im.reshape(M.shape)).imag.ravel()[rows] / H
    worst = 0.0
    for kk in itertools.product(range(N), repeat=3):
        k = 2 * np.pi * np.array(kk) / N
        Jh = np.zeros((10, 10), complex)
        for z, y, x in itertools.product(range(N), repeat=3):
            cell = x + N * (y + N * z)
            d = np.array([-x % N, -y % N, -z % N])
            Jh += Jcol[:, np.arange(10) * Nc + cell] * np.exp(-1j * (k @ d))
        worst = max(worst, np.abs(Jh - _G(c, PHI, J, k)).max())
    assert worst < 1e-12


@pytest.mark.parametrize("tau", [0.51, 0.6, 1.0, 1.5])
def test_zero_wavenumber_spectrum(orc, tau):
    c, w, _ = orc.lattice()
    PHI = _phi(c)
    P = orc.make_params((4, 4, 4), tau)
    m0 = _uniform(orc, 0.97, [0.1, 0.05, -0.08], np.array([2e-3, 0, -1e-3, 4e-4, 1e-4, -3e-4]))
    ev = np.linalg.eigvals(_G(c, PHI, _cell_jac(orc, P, m0), np.zeros(3)))
    ref = np.array([1.0] * 4 + [0.0] + [1 - 1 / tau] * 5)
    assert np.abs(np.sort(ev.real) - np.sort(ref)).max() < 1e-12
    assert np.abs(ev.imag).max() < 1e-12


def test_small_k_hydrodynamic_modes(orc):
    """|k| = 2 pi / 64 along x: shear modes omega = k u - i nu k^2 (nu within
    1%), acoustic phases k u +- cs |k| within 1%."""
    c, w, _ = orc.lattice()
    PHI = _phi(c)
    tau = 0.6
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / 64
    for ux in (0.0, 0.05):
        P = orc.make_params((4, 4, 4), tau)
        J = _cell_jac(orc, P, _uniform(orc, 1.0, [ux, 0, 0]))
        lam = np.linalg.eigvals(_G(c, PHI, J, np.array([k, 0, 0])))
        om = 1j * np.log(lam)
        hydro = om[np.abs(om.real) < 0.2]
        hydro = hydro[np.argsort(hydro.real)]
        assert hydro.size == 4
        ac_lo, sh1, sh2, ac_hi = hydro
        for s in (sh1, sh2):
            assert abs(s.real - k * ux) < 1e-3 * k * ux + 1e-12
            assert abs(-s.imag / (nu * k * k) - 1) < 0.01
        cs = np.sqrt(CS2)
        assert abs(ac_hi.real - (k * ux + cs * k)) < 0.01 * cs * k
        assert abs(ac_lo.real - (k * ux - cs * k)) < 0.01 * cs * k
        assert ac_hi.imag < 0 and ac_lo.imag < 0


@pytest.mark.parametrize("tau", [0.505, 0.51, 0.6, 0.8, 1.0])
def test_von_neumann_bound_at_rest(orc, tau):
    """max |lambda(k)| <= 1 over a 16^3 wavenumber grid at u = 0 (Sec. 5.2)."""
    c, w, _ = orc.lattice()
    PHI = _phi(c)
    P = orc.make_params((4, 4, 4), tau)
    J = _cell_jac(orc, P, _uniform(orc, 1.0, [0, 0, 0]))
    K = 16
    ks = 2 * np.pi * np.array(list(itertools.product(range(K), repeat=3))) / K
    ph = np.exp(-1j * (ks @ c.T))                      # (nk, 27)
    G = np.einsum("ki,ia,ib->kab", ph, PHI, J)        # (nk, 10, 10)
    lam = np.abs(np.linalg.eigvals(G)).max()
    assert lam <= 1 + 1e-12


def test_sound_attenuation_follows_the_bulk_rate():
    """App. A sets the trace of S to |u|^2 (bulk relaxation rate 1), so by
    Eq. acoustic_modes with D = 3 the sound modes decay at
    k^2 (2 nu / 3 + mu_v / 2), mu_v = (2/3) cs^2 (1 - 1/2) = 1/9."""
    from oracle import d2q9
    c, w, _ = orc_mod.lattice()
    for tau in (0.53, 0.6):
        nu = (tau - 0.5) / 3
        k = 2 * np.pi / 64
        lam = np.linalg.eigvals(stability.amplification_grid_3d(np.array([k, 0, 0]), tau, 1.0, [0, 0, 0]))
        om = 1j * np.log(lam)
        hydro = om[np.abs(om.real) < 0.2]
        hydro = hydro[np.argsort(hydro.real)]
        damp = k * k * (2 * nu / 3 + 0.5 * d2q9.bulk_viscosity(1.0, D=3))
        for ac in (hydro[0], hydro[-1]):
            assert abs(-ac.imag / damp - 1) < 0.01


@pytest.mark.parametrize("tau", [0.51, 0.52, 0.6])
def test_stable_at_the_workload_speeds(tau):
    """The step is von Neumann stable (max |lambda| <= 1 on a 12^3 wave grid)
    at drift speeds up to 0.12 along x, xy and xyz for the relaxation times
    the benchmarks use (their largest speed is the channel's inflow, 0.08)."""
    for dvec in ((1, 0, 0), (1, 1, 0), (1, 1, 1)):
        u = 0.12 * np.array(dvec, float) / np.linalg.norm(dvec)
        assert stability.max_growth(3, None, tau, u, 12) <= 1 + 1e-10


def test_amplification_matches_the_cell_symbol():
    """stability.amplification_grid_3d is the symbol checked against the full
    Jacobian above."""
    c, w, _ = orc_mod.lattice()
    PHI = _phi(c)
    tau = 0.57
    u = [0.04, -0.02, 0.03]
    k = np.array([0.4, -1.3, 2.2])
    m0 = _uniform(orc_mod, 1.0, u)
    J = _cell_jac(orc_mod, orc_mod.make_params((4, 4, 4), tau), m0)
    assert np.abs(stability.amplification_grid_3d(k, tau, 1.0, u) - _G(c, PHI, J, k)).max() < 1e-14
