"""Pins of the D2Q9 oracle and its linear stability analysis (Sec. 5.1-5.2,
App. B-E).

Each pin comes from outside the code it checks: the Maxwellian's moments,
Hermite orthogonality, the complex-step Jacobian of the nonlinear step on a
periodic grid (against the closed-form amplification matrices), the textbook
reduction of MRT with equal rates to BGK, the k = 0 spectra, and the
Navier-Stokes modes of Eqs. shear_mode and acoustic_modes at small k."""
import itertools

import numpy as np
import pytest

from oracle import d2q9 as d

CS2 = 1.0 / 3.0
H = 1e-30
STATE = (1.02, 0.05, -0.03)           # rho, ux, uy of a drifting uniform state


def test_lattice_isotropy():
    c, w = d.C, d.W
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - CS2 * np.eye(2)).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ig->abg", w, c, c, c)).max() < 1e-15
    m4 = np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c)
    I = np.eye(2)
    ref = CS2 ** 2 * (np.einsum("ab,gd->abgd", I, I) + np.einsum("ag,bd->abgd", I, I)
                      + np.einsum("ad,bg->abgd", I, I))
    assert np.abs(m4 - ref).max() < 1e-15


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (0.9, 0.2, -0.1), (1.3, -0.35, 0.4)])
def test_equilibrium_has_maxwellian_moments(rho, ux, uy):
    """R19: every raw moment sum c_x^a c_y^b f_eq (a, b <= 2) is the
    Maxwellian's, rho E[X^a] E[Y^b] with X ~ N(u_x, cs^2), Y ~ N(u_y, cs^2);
    the central moments of M^NOCM(u) are (rho, 0, 0, 2 rho cs^2, 0, 0, 0, 0,
    rho cs^4)."""
    f = d.feq(rho, ux, uy)
    gauss = lambda a, u: (1.0, u, u * u + CS2)[a]
    for a, b in itertools.product(range(3), repeat=2):
        assert abs((f * d.CX ** a * d.CY ** b).sum() - rho * gauss(a, ux) * gauss(b, uy)) < 1e-14
    k = d.m_nocm(ux, uy) @ f
    ref = np.array([rho, 0, 0, 2 * rho * CS2, 0, 0, 0, 0, rho * CS2 ** 2])
    assert np.abs(k - ref).max() < 1e-14


def test_printed_quartic_equilibrium_loses_mass():
    """The reason for R19: the fourth-order equilibrium as printed in App. E
    sums to rho (1 - 9/4 |u|^4) over the lattice."""
    rho, ux, uy = 1.0, 0.1, 0.1
    cu = d.CX * ux + d.CY * uy
    usq = ux * ux + uy * uy
    printed = d.W * rho * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - usq / (2 * CS2)
                           - (d.CX * ux ** 3 + d.CY * uy ** 3) / (2 * CS2 ** 2) + cu ** 3 / (6 * CS2 ** 3)
                           + usq ** 2 / (8 * CS2 ** 2) - (d.CX ** 2 + d.CY ** 2) * usq ** 2 / (4 * CS2 ** 3)
                           + cu ** 4 / (24 * CS2 ** 4))
    assert abs(printed.sum() - rho * (1 - 2.25 * usq ** 2)) < 1e-15
    assert abs(d.feq(rho, ux, uy).sum() - rho) < 1e-15


@pytest.mark.parametrize("of", ["feq", "heq"])
def test_equilibrium_derivatives(of):
    """The closed-form derivatives behind Lambda against complex steps."""
    fn = d.feq if of == "feq" else d.heq
    der = d.feq_derivatives if of == "feq" else d.heq_derivatives
    rho, ux, uy = STATE
    num = (fn(rho + 1j * H, ux, uy).imag / H, fn(rho, ux + 1j * H, uy).imag / H,
           fn(rho, ux, uy + 1j * H).imag / H)
    for a, b in zip(der(rho, ux, uy), num):
        assert np.abs(a - b).max() < 1e-15


def test_reconstruction_moments():
    """h(rho, u, S) carries rho, rho u and rho S exactly (Hermite projection)
    and its third-order Hermite coefficients are rho T_xxy and rho T_xyy with
    T_abg = S_ab u_g + S_ag u_b + S_bg u_a - 2 u_a u_b u_g (App. D recursion
    for the non-equilibrium part)."""
    rho, ux, uy = STATE
    sxx, sxy, syy = ux * ux + 0.01, ux * uy - 0.004, uy * uy + 0.006
    h = d.reconstruct(rho, ux, uy, sxx, sxy, syy)
    assert np.allclose(d.moments(h), (rho, ux, uy, sxx, sxy, syy), rtol=0, atol=1e-15)
    txxy = sxx * uy + 2 * sxy * ux - 2 * ux * ux * uy
    txyy = syy * ux + 2 * sxy * uy - 2 * ux * uy * uy
    assert abs((h * d.CY * (d.CX ** 2 - CS2)).sum() - rho * txxy) < 1e-15
    assert abs((h * d.CX * (d.CY ** 2 - CS2)).sum() - rho * txyy) < 1e-15


def test_qb_is_the_linearised_reconstruction():
    """R20: (A2 + A3 R_u) B applied to a perturbation whose second moments are
    delta(rho S) gives exactly the change of h at fixed rho and u."""
    rho, ux, uy = STATE
    rng = np.random.default_rng(3)
    df = rng.standard_normal(9) * 1e-3
    dP = np.array([((d.CX ** 2 - CS2) * df).sum(), (d.CX * d.CY * df).sum(), ((d.CY ** 2 - CS2) * df).sum()])
    base = (ux * ux, ux * uy, uy * uy)
    dh = d.reconstruct(rho, ux, uy, *(b + p / rho for b, p in zip(base, dP))) - d.heq(rho, ux, uy)
    assert np.abs(d.hermite_qb(ux, uy) @ df - dh).max() < 1e-16


def _grid_symbol(model, tau, nx=4, ny=3):
    """Fourier symbols of the complex-step Jacobian of the periodic nx x ny
    step at the model's uniform fixed point, for every grid wave vector."""
    rho, ux, uy = STATE
    f0 = d.rest_state(model, rho, ux, uy)
    F = np.broadcast_to(f0[:, None, None], (9, ny, nx)).astype(complex)
    assert np.abs(d.step(model, F.real, tau) - F.real).max() < 1e-15
    n = 9 * nx * ny
    Jcol = np.zeros((9, n))
    for q in range(n):
        P = np.zeros(n, complex)
        P[q] = 1j * H
        Jcol[:, q] = d.step(model, F + P.reshape(F.shape), tau).imag[:, 0, 0] / H
    out = []
    for kx, ky in itertools.product(range(nx), range(ny)):
        k = 2 * np.pi * np.array([kx / nx, ky / ny])
        Jh = np.zeros((9, 9), complex)
        for y, x in itertools.product(range(ny), range(nx)):
            cell = x + nx * y
            Jh += Jcol[:, np.arange(9) * nx * ny + cell] * np.exp(1j * (k @ np.array([x, y])))
        out.append((k, Jh))
    return out


@pytest.mark.parametrize("model", d.MODELS)
def test_grid_jacobian_equals_amplification_matrix(model):
    """G(k) of App. B / Eq. Mo-NOCM (with R19-R21, R24) is the exact
    linearisation of the nonlinear collide-and-pull-stream step."""
    tau = 0.6
    for k, Jh in _grid_symbol(model, tau):
        assert np.abs(Jh - d.amplification(model, k, *STATE, tau)).max() < 1e-13


@pytest.mark.parametrize("tau", [0.5003, 0.6, 1.0, 1.7])
def test_zero_wavenumber_spectra(tau):
    """At k = 0 the conserved rho, j give eigenvalue 1 and each relaxed moment
    1 - r_i; the HOME composites keep rho, j, S only (three zeros)."""
    def ev(m, r=None):
        return np.sort(np.linalg.eigvals(d.amplification(m, [0, 0], *STATE, tau, r)).real)
    s = 1 / tau
    assert np.abs(ev("bgk") - np.sort([1, 1, 1] + [1 - s] * 6)).max() < 1e-12
    for m in ("rm", "nocm"):
        assert np.abs(ev(m) - np.sort(1 - d.rates(m, tau))).max() < 1e-12
    assert np.abs(ev("home") - np.sort([1, 1, 1] + [1 - s] * 3 + [0] * 3)).max() < 1e-12
    assert np.abs(ev("home_appa") - np.sort([1, 1, 1, 0] + [1 - s] * 2 + [0] * 3)).max() < 1e-12


@pytest.mark.parametrize("model", ["rm", "nocm"])
def test_equal_rates_reduce_to_bgk(model):
    """MRT with every non-conserved rate equal to 1/tau is BGK."""
    tau = 0.57
    r = np.array([0, 0, 0] + [1 / tau] * 6)
    for k in ([0.3, -1.1], [2.0, 0.7]):
        G = d.amplification(model, k, *STATE, tau, r)
        assert np.abs(G - d.amplification("bgk", k, *STATE, tau)).max() < 1e-13


BULK_RATE = {"bgk": None, "rm": 1.64, "nocm": None, "home": None, "home_appa": 1.0}


@pytest.mark.parametrize("model", d.MODELS)
@pytest.mark.parametrize("phi", [0.0, np.pi / 4])
def test_small_k_hydrodynamic_modes(model, phi):
    """|k| = 2 pi / 64 at rest: the three least damped modes follow
    Eqs. shear_mode and acoustic_modes with D = 2: shear decay nu k^2 within
    1%, sound speed cs within 0.1%, sound decay k^2 (nu/2 + mu_v/2) within 1%,
    mu_v the bulk viscosity of the model's trace relaxation rate (BGK, NOCM,
    HOME: 1/tau, so mu_v = nu; RM-MRT: 1.64; App. A in 2D: 1)."""
    tau = 0.53
    nu = d.nu_of_tau(tau)
    k = 2 * np.pi / 64
    lam = np.linalg.eigvals(d.amplification(model, k * np.array([np.cos(phi), np.sin(phi)]), 1.0, 0.0, 0.0, tau))
    om = d.omega(lam[np.abs(lam) > 0.9])
    om = om[np.argsort(om.real)]
    assert om.size == 3
    ac_m, shear, ac_p = om
    rate = BULK_RATE[model] or 1 / tau
    sh_ref = d.shear_mode(k, 0.0, phi, nu)
    ap_ref, am_ref = d.acoustic_modes(k, 0.0, phi, nu, d.bulk_viscosity(rate))
    assert abs(shear.imag / sh_ref.imag - 1) < 0.01 and abs(shear.real) < 1e-12
    for got, ref in ((ac_p, ap_ref), (ac_m, am_ref)):
        assert abs(got.real / ref.real - 1) < 1e-3
        assert abs(got.imag / ref.imag - 1) < 0.01


def test_shear_mode_advects_with_the_flow():
    """Galilean-invariant models carry the shear mode at k u cos(phi) with its
    decay nu k^2 unchanged (u = 0.05 along x, k along x and at 45 degrees)."""
    tau = 0.53
    nu = d.nu_of_tau(tau)
    k, u = 2 * np.pi / 64, 0.05
    for model in ("nocm", "home", "home_appa"):
        for phi in (0.0, np.pi / 4):
            lam = np.linalg.eigvals(d.amplification(model, k * np.array([np.cos(phi), np.sin(phi)]), 1.0, u, 0.0, tau))
            om = d.omega(lam[np.abs(lam) > 0.9])
            om = om[np.argsort(om.real)]
            ref = d.shear_mode(k, u, phi, nu)
            assert abs(om[1].real - ref.real) < 2e-3 * abs(ref.real)
            assert abs(om[1].imag / ref.imag - 1) < 0.02


@pytest.mark.parametrize("nu", [1e-3, 1e-4, 1e-5])
def test_von_neumann_bound_at_rest(nu):
    """max |lambda(k)| <= 1 over k in [-pi, pi]^2 at u = 0 for every model
    (Sec. 5.1's criterion)."""
    g = np.linspace(-np.pi, np.pi, 41)
    K2 = np.stack(np.meshgrid(g, g, indexing="ij"), -1)
    for model in d.MODELS:
        lam = np.abs(np.linalg.eigvals(d.amplification_grid(model, K2, 1.0, 0.0, 0.0, d.tau_of_nu(nu)))).max()
        assert lam <= 1 + 1e-12, model


@pytest.mark.parametrize("nu", [1e-3, 1e-4, 1e-5])
def test_home_margin_overlaps_nocm_at_rest(nu):
    """Sec. 5.2's stability-margin comparison: along k_x at u = 0 the HOME
    composite's max |lambda| equals NOCM-MRT's."""
    kx = np.linspace(0.0, np.pi, 129)
    ks = np.stack([kx, 0 * kx], 1)
    tau = d.tau_of_nu(nu)
    a = np.abs(np.linalg.eigvals(d.amplification_grid("home", ks, 1.0, 0.0, 0.0, tau))).max(-1)
    b = np.abs(np.linalg.eigvals(d.amplification_grid("nocm", ks, 1.0, 0.0, 0.0, tau))).max(-1)
    assert np.abs(a - b).max() < 1e-10


def test_nonlinear_growth_follows_the_linear_rate():
    """An eigenmode of G(k) seeded into the nonlinear NOCM-MRT step grows as
    |lambda|^t: the instability that the analysis finds at u = (0.1, 0.1),
    nu = 1e-4 is the model's, not the analysis's."""
    n = 16
    tau = d.tau_of_nu(1e-4)
    k = 2 * np.pi * np.array([2, 2]) / n
    lam, vec = np.linalg.eig(d.amplification("nocm", k, 1.0, 0.1, 0.1, tau))
    j = np.argmax(np.abs(lam))
    assert np.abs(lam[j]) > 1.01
    y, x = np.mgrid[0:n, 0:n]
    mode = (vec[:, j][:, None, None] * np.exp(1j * (k[0] * x + k[1] * y))).real
    f0 = d.feq(np.ones((n, n)), np.full((n, n), 0.1), np.full((n, n), 0.1))
    phase = np.exp(-1j * (k[0] * x + k[1] * y))
    coeff = lambda g: np.abs(((g - f0) * phase).sum((1, 2))).max()
    f = f0 + 1e-10 * mode
    start = coeff(f)
    steps = 60
    for _ in range(steps):
        f = d.step("nocm", f, tau)
    assert abs(coeff(f) / start / np.abs(lam[j]) ** steps - 1) < 1e-3


def test_study_tables_have_their_shapes():
    """The study behind the reported tables runs and fills every entry
    (coarse grids here)."""
    s = d.study(nk=9, nk2=5)
    assert len(s["margin"]) == 3 * len(d.MODELS) and all(v.shape == (9,) for v in s["margin"].values())
    assert len(s["dissipation"]) == 4 * len(d.MODELS) and all(v.shape == (5, 5) for v in s["dissipation"].values())
    for om in s["dispersion"].values():
        assert om.shape == (8, 3) and np.all(np.abs(om[:, 1].real) < 1e-9)    # shear branch at rest
        assert np.all(om[:, 2].real > 0) and np.all(om[:, 0].real < 0)


def test_speed_limit_brackets_the_crossing():
    """stability.speed_limit returns a speed that is stable while a slightly
    larger one is not (2D HOME composite, nu = 1e-3, coarse wave grid)."""
    from oracle import stability
    tau = d.tau_of_nu(1e-3)
    s = stability.speed_limit(2, "home", tau, (1, 0), 16, iters=8)
    assert 0.0 < s < 0.6
    assert stability.max_growth(2, "home", tau, (s, 0.0), 16) <= 1 + 1e-10
    assert stability.max_growth(2, "home", tau, (s + 0.6 / 2 ** 8 * 1.01, 0.0), 16) > 1 + 1e-10
