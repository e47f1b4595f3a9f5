"""Pins of the oracle's per-cell pieces against what the paper and the
mathematics fix: D3Q27 quadrature moments, Hermite moment recovery
(Eq. three_order_f against Eq. rho_u_stress), and the App. A collision's
invariants written in an independent (deviatoric) closed form."""
import itertools

import numpy as np
import pytest

CS2 = 1.0 / 3.0


def test_lattice_weights_and_isotropy(orc):
    c, w, opp = orc.lattice()
    # textbook D3Q27 weights: 8/27 rest, 2/27 faces, 1/54 edges, 1/216 corners
    nz = np.abs(c).sum(1)
    for n, val in [(0, 8 / 27), (1, 2 / 27), (2, 1 / 54), (3, 1 / 216)]:
        assert np.allclose(w[nz == n], val, atol=1e-16)
    assert abs(w.sum() - 1) < 1e-15
    assert np.all(c[opp] == -c)
    assert np.all(c[13] == 0)
    # quadrature moments up to 4th order (and 6th along axes) of the Maxwellian
    d = np.eye(3)
    for a, b in itertools.product(range(3), repeat=2):
        assert abs((w * c[:, a] * c[:, b]).sum() - CS2 * d[a, b]) < 1e-15
    for a, b, g in itertools.product(range(3), repeat=3):
        assert abs((w * c[:, a] * c[:, b] * c[:, g]).sum()) < 1e-15
    for a, b, g, e in itertools.product(range(3), repeat=4):
        ref = CS2 * CS2 * (d[a, b] * d[g, e] + d[a, g] * d[b, e] + d[a, e] * d[b, g])
        assert abs((w * c[:, a] * c[:, b] * c[:, g] * c[:, e]).sum() - ref) < 1e-15


def _H3(c, a, b, g):
    d = np.eye(3)
    return (c[:, a] * c[:, b] * c[:, g]
            - CS2 * (c[:, a] * d[b, g] + c[:, b] * d[a, g] + c[:, g] * d[a, b]))


def _sym(S6):
    S = np.zeros((3, 3))
    for p, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        S[a, b] = S[b, a] = S6[p]
    return S


@pytest.mark.parametrize("seed", range(5))
def test_hermite_moment_recovery(orc, seed):
    """m(h(rho, u, S)) = (rho, rho u, rho S) (Hermite orthogonality), and the
    reconstruction carries the third moments rho T of Sec. 3.2 (reading R1)."""
    rng = np.random.default_rng(seed)
    rho = 1 + 0.2 * rng.standard_normal()
    u = 0.1 * rng.standard_normal(3)
    S6 = 0.05 * rng.standard_normal(6)
    f = orc.reconstruct(rho, u, S6)
    m = orc.project(f)
    assert np.abs(m - np.r_[rho, rho * u, rho * S6]).max() < 1e-14
    c, w, _ = orc.lattice()
    S = _sym(S6)
    for a, b, g in [(0, 0, 1), (0, 1, 1), (0, 0, 2), (0, 2, 2), (1, 2, 2), (1, 1, 2), (0, 1, 2)]:
        T = S[a, b] * u[g] + S[a, g] * u[b] + S[b, g] * u[a] - 2 * u[a] * u[b] * u[g]
        assert abs((f * _H3(c, a, b, g)).sum() - rho * T) < 1e-14
    # the printed coefficient on the xyz term (literal reading) halves that moment
    fl = orc.reconstruct(rho, u, S6, literal_xyz=True)
    Txyz = S[0, 1] * u[2] + S[0, 2] * u[1] + S[1, 2] * u[0] - 2 * u[0] * u[1] * u[2]
    assert abs((fl * _H3(c, 0, 1, 2)).sum() - 0.5 * rho * Txyz) < 1e-14


def test_equilibrium_reconstruction_is_maxwellian_expansion(orc):
    """At S = u u the reconstruction equals the textbook third-order Hermite
    equilibrium, including the rest weights at u = 0."""
    c, w, _ = orc.lattice()
    rho, u = 1.03, np.array([0.04, -0.02, 0.07])
    S6 = np.array([u[0] ** 2, u[1] ** 2, u[2] ** 2, u[0] * u[1], u[0] * u[2], u[1] * u[2]])
    f = orc.reconstruct(rho, u, S6)
    cu = c @ u
    uu = u @ u
    # third-order truncation of the D3Q27 Maxwellian (terms with H3_aaa vanish on the lattice)
    h3 = 0.0
    for a, b, g in itertools.product(range(3), repeat=3):
        h3 = h3 + _H3(c, a, b, g) * u[a] * u[b] * u[g]
    feq = rho * w * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu + 4.5 * h3)
    assert np.abs(f - feq).max() < 1e-15
    assert np.abs(orc.reconstruct(1.0, np.zeros(3), np.zeros(6)) - w).max() < 1e-16


@pytest.mark.parametrize("tau", [0.51, 0.6, 0.8, 1.0, 1.7])
def test_collision_deviatoric_form(orc, tau):
    """App. A with F = 0 equals S+ = u u + (1 - 1/tau) dev(S - u u): rho and u
    kept, trace of S+ reset to |u|^2, deviator of S - u u scaled by 1 - 1/tau."""
    rng = np.random.default_rng(int(tau * 100))
    for _ in range(5):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.1 * rng.standard_normal(3)
        S6 = 0.05 * rng.standard_normal(6)
        out = orc.collide(rho, u, S6, tau)
        assert out[0] == rho
        assert np.abs(out[1:4] - u).max() == 0
        S = _sym(S6)
        UU = np.outer(u, u)
        D = S - UU
        ref = UU + (1 - 1 / tau) * (D - np.trace(D) / 3 * np.eye(3))
        assert np.abs(_sym(out[4:]) - ref).max() < 1e-15
        assert abs(np.trace(_sym(out[4:])) - u @ u) < 1e-15


def test_collision_equilibrium_fixed_point_and_force(orc):
    rng = np.random.default_rng(7)
    u = 0.1 * rng.standard_normal(3)
    S6 = np.array([u[0] ** 2, u[1] ** 2, u[2] ** 2, u[0] * u[1], u[0] * u[2], u[1] * u[2]])
    out = orc.collide(1.1, u, S6, 0.7)
    assert np.abs(out[4:] - S6).max() < 1e-16
    # the force shifts u by F/(2 rho) (so rho u+ = rho u + F/2) ...
    F = np.array([1e-3, -2e-3, 5e-4])
    out = orc.collide(1.1, u, S6, 0.7, F)
    assert np.abs(1.1 * out[1:4] - (1.1 * u + F / 2)).max() < 1e-16
    # ... and at tau = 1 App. A's stress is the equilibrium of the mean of
    # pre- and post-force velocities to first order in F: S+ = u u + (F u + u F)/(2 rho)
    out1 = orc.collide(1.1, u, S6, 1.0, F)
    ref = np.outer(u, u) + (np.outer(F, u) + np.outer(u, F)) / (2 * 1.1)
    assert np.abs(_sym(out1[4:]) - ref).max() < 1e-15


def test_post_collision_f_conserves_mass_and_momentum(orc):
    """f+ = h(collide(m)) carries the same rho and rho u as the stored moments."""
    rng = np.random.default_rng(3)
    P = orc.make_params((4, 4, 4), 0.6)
    for _ in range(5):
        m = np.r_[1 + 0.05 * rng.standard_normal(), 0.05 * rng.standard_normal(3), 0.01 * rng.standard_normal(6)]
        f = orc.post_collision_f(P, m)
        mm = orc.project(f)
        assert abs(mm[0] - m[0]) < 1e-15 and np.abs(mm[1:4] - m[1:4]).max() < 1e-16
