"""D2Q9 lattice Boltzmann models and their linear stability -- TEST INFRASTRUCTURE.

Not part of the product: only the tests (and a reader running this module as a
script to print the study tables) use it.  Plain FP64 numpy, written to be
checked against the paper by eye; every array routine also runs on complex
input, so complex-step derivatives of the nonlinear maps are exact.

Source: "High-Performance Moment-Encoded Lattice Boltzmann Method with
Stability-Guided Quantization" (arXiv 2602.05295).
  lattice, weights, c_s              App. C.4 (D2Q9 lattice definitions)
  BGK collision                      App. C.1 (Eq. bgk_collision)
  RM-MRT collision and M^RM          App. C.2 (Eq. mrt_rm_collision), App. C.4
  NOCM-MRT collision and M^NOCM(u)   App. C.3 (Eq. cm_collision), App. C.4
  relaxation rates                   App. C.4 (relaxation rates)
  moments m(f) = (rho, u, S)         Sec. 3.1 (Eq. rho_u_stress)
  third-order reconstruction h       Sec. 3.2 (Eq. three_order_f), restricted
                                     to two dimensions
  HOME composite g = h(m(f+))        Sec. 5.2 (Eq. home_mapping,
                                     Eq. home_postcollision)
  A2, A3, R_u, B                     App. D (Eq. a3_neq, Eq. fneq_base)
  equilibrium Jacobian Lambda        Sec. 5.1 (Eq. Lambda_chainrule), App. E
  amplification matrices G(k)        Sec. 5.1 (G = D(k)[I + K(Lambda - I)]),
                                     App. B (Eq. G_differentcollision),
                                     Sec. 5.2 (Eq. Mo-NOCM)
  hydrodynamic modes                 Sec. 5.2 (Eqs. shear_mode, acoustic_modes)

Readings taken where the paper is ambiguous, garbled or at odds with itself:
  R19 The equilibrium of BGK, RM-MRT and NOCM-MRT is the D2Q9 product form
      f_eq_i = rho psi(c_ix, u_x) psi(c_iy, u_y), psi(0, u) = 1 - cs^2 - u^2,
      psi(+-1, u) = (cs^2 + u^2 +- u)/2: every raw moment sum c_x^a c_y^b f
      with a, b <= 2 equals the Maxwellian's, and its central moments are
      (rho, 0, 0, 2 rho cs^2, 0, 0, 0, 0, rho cs^4).  The fourth-order form
      printed in App. E does not conserve mass (its quartic terms sum to
      -9/4 rho |u|^4 over the lattice).
  R20 The linear map a2_neq -> f_neq is the one the f_neq formula of App. D
      defines: f_neq_i = w_i [H2_i : a2 / (2 cs^4)
      + (H_i,xxy a3_xxy + H_i,xyy a3_xyy) / (2 cs^6)], with a3 from the
      recursion.  Written as (A2 + A3 R_u) B, each symmetric-tensor component
      carries its multiplicity once (2 for xy in A2, 3 for xxy and xyy in A3)
      and B returns plain components (a_xx, a_xy, a_yy).  The printed A2, A3
      and Voigt B disagree with that formula by these factors.
  R21 In Eq. Mo-NOCM the leading Lambda is the Jacobian of the
      reconstruction's own equilibrium h(rho, u, u u); the Lambda inside the
      NOCM-MRT collision is that of the R19 equilibrium.  (B Lambda is the same
      for both, since both carry exact second moments.)  With this reading the
      closed form is the exact linearisation of g = h(m(f+)).
  R22 s_nu = r_nu = 1 / (1/2 + nu / cs^2) = 1 / tau.
  R23 The direction order of App. C.4 is used everywhere; B (whose table lists
      another order) is built from its defining formula.
  R24 HOME-LBM in two dimensions ("home_appa") is App. A's moment collision
      written for D = 2: off-diagonal S relaxed with 1/tau toward u u, the
      deviatoric part of the diagonal likewise, the trace set to |u|^2.  In
      the language of Eq. Mo-NOCM that is the NOCM-MRT projection with the
      bulk row (X^2 + Y^2) at rate 1.  The paper's HOME curves ("home")
      use the NOCM-MRT rates as printed, bulk at s_nu.
  R25 Plane waves are exp(i(k.x - omega t)), so an eigenvalue lambda of G(k)
      gives omega = i log(lambda): Im omega = log|lambda| (> 0 grows) and
      Re omega = -arg(lambda).
  R9  (as in the D3Q27 oracle) nu = cs^2 (tau - 1/2): App. C.1 prints
      1/(3 nu + 1/2) as tau, which is the rate 1/tau = r_nu of App. C.4.

Distributions are arrays f[9, ny, nx] (x fastest); a uniform state is f[9].
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0

# App. C.4: directions i = 0..8 and their weights.
C = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=float)
CX, CY = C[:, 0], C[:, 1]
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)

MODELS = ("bgk", "rm", "nocm", "home", "home_appa")


def nu_of_tau(tau):
    """R9: nu = cs^2 (tau - 1/2); the relaxation rate 1/tau is r_nu of App. C.4."""
    return CS2 * (tau - 0.5)


def tau_of_nu(nu):
    return 0.5 + nu / CS2


# ------------------------------------------------------------ moments --------

def _cell(a, f):
    """Broadcast a per-direction vector a[9] against f[9, ...]."""
    return a.reshape((9,) + (1,) * (np.ndim(f) - 1))


def moments(f):
    """Eq. rho_u_stress without force: rho = sum f, u = sum c f / rho,
    S = sum (c c - cs^2 delta) f / rho, returned as (rho, ux, uy, Sxx, Sxy, Syy)."""
    rho = f.sum(0)
    ux = (_cell(CX, f) * f).sum(0) / rho
    uy = (_cell(CY, f) * f).sum(0) / rho
    sxx = (_cell(CX * CX - CS2, f) * f).sum(0) / rho
    sxy = (_cell(CX * CY, f) * f).sum(0) / rho
    syy = (_cell(CY * CY - CS2, f) * f).sum(0) / rho
    return rho, ux, uy, sxx, sxy, syy


# --------------------------------------------------------- equilibria --------

def _psi(c, u):
    """One-dimensional three-velocity factor of the R19 equilibrium."""
    return np.where(c == 0, 1.0 - CS2 - u * u, 0.5 * (CS2 + u * u + c * u))


def _dpsi(c, u):
    return np.where(c == 0, -2.0 * u, u + 0.5 * c)


def feq(rho, ux, uy):
    """R19 equilibrium, shape (9,) + shape of rho."""
    rho, ux, uy = np.broadcast_arrays(*(np.asarray(v) for v in (rho, ux, uy)))
    shp = (9,) + (1,) * rho.ndim
    cx, cy = CX.reshape(shp), CY.reshape(shp)
    return rho * _psi(cx, ux) * _psi(cy, uy)


def feq_derivatives(rho, ux, uy):
    """d f_eq / d(rho, ux, uy) at a uniform state, each of shape (9,)."""
    d_rho = _psi(CX, ux) * _psi(CY, uy)
    d_ux = rho * _dpsi(CX, ux) * _psi(CY, uy)
    d_uy = rho * _psi(CX, ux) * _dpsi(CY, uy)
    return d_rho, d_ux, d_uy


def reconstruct(rho, ux, uy, sxx, sxy, syy):
    """Eq. three_order_f on D2Q9: the second-order Hermite term with S and the
    third-order terms xxy and xyy with T_abg = S_ab u_g + S_ag u_b + S_bg u_a
    - 2 u_a u_b u_g (H_xxx and H_yyy vanish on this lattice)."""
    shp = (9,) + (1,) * np.ndim(rho)
    cx, cy, w = CX.reshape(shp), CY.reshape(shp), W.reshape(shp)
    hxx, hxy, hyy = cx * cx - CS2, cx * cy, cy * cy - CS2
    hxxy, hxyy = cy * (cx * cx - CS2), cx * (cy * cy - CS2)
    txxy = sxx * uy + 2.0 * sxy * ux - 2.0 * ux * ux * uy
    txyy = syy * ux + 2.0 * sxy * uy - 2.0 * ux * uy * uy
    return w * rho * (1.0 + (cx * ux + cy * uy) / CS2
                      + (hxx * sxx + 2.0 * hxy * sxy + hyy * syy) / (2.0 * CS2 ** 2)
                      + (hxxy * txxy + hxyy * txyy) / (2.0 * CS2 ** 3))


def heq(rho, ux, uy):
    """The reconstruction's equilibrium h(rho, u, u u)."""
    return reconstruct(rho, ux, uy, ux * ux, ux * uy, uy * uy)


def heq_derivatives(rho, ux, uy):
    """d h(rho, u, u u) / d(rho, ux, uy) at a uniform state, each (9,)."""
    hxx, hxy, hyy = CX * CX - CS2, CX * CY, CY * CY - CS2
    hxxy, hxyy = CY * (CX * CX - CS2), CX * (CY * CY - CS2)
    d_rho = heq(1.0, ux, uy)
    d_ux = rho * W * (CX / CS2 + (2.0 * hxx * ux + 2.0 * hxy * uy) / (2.0 * CS2 ** 2)
                      + (2.0 * hxxy * ux * uy + hxyy * uy * uy) / (2.0 * CS2 ** 3))
    d_uy = rho * W * (CY / CS2 + (2.0 * hxy * ux + 2.0 * hyy * uy) / (2.0 * CS2 ** 2)
                      + (hxxy * ux * ux + 2.0 * hxyy * ux * uy) / (2.0 * CS2 ** 3))
    return d_rho, d_ux, d_uy


# ------------------------------------------------- transformation matrices ---

# App. C.4, printed as is.
M_RM = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 1, 1, 1, 1, 2, 2, 2, 2],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
    [0, 1, 0, -1, 0, 2, -2, -2, 2],
    [0, 0, 1, 0, -1, 2, 2, -2, -2],
    [0, 0, 0, 0, 0, 1, 1, 1, 1],
], dtype=float)


def m_nocm(ux, uy):
    """App. C.4: rows 1, X, Y, X^2 + Y^2, X^2 - Y^2, X Y, X^2 Y, X Y^2, X^2 Y^2
    of the shifted velocities X = c_x - u_x, Y = c_y - u_y.  For arrays of
    velocities the result has shape ux.shape + (9, 9)."""
    ux, uy = np.asarray(ux), np.asarray(uy)
    X = CX - ux[..., None]
    Y = CY - uy[..., None]
    rows = [np.ones_like(X), X, Y, X * X + Y * Y, X * X - Y * Y, X * Y, X * X * Y, X * Y * Y, X * X * Y * Y]
    return np.stack(rows, axis=-2)


def rates(model, tau):
    """App. C.4 relaxation rates (R22: s_nu = r_nu = 1/tau); R24 for home_appa."""
    r = 1.0 / tau
    if model == "rm":
        return np.array([0, 0, 0, 1.64, r, r, 1.9, 1.9, 1.54])
    if model in ("nocm", "home"):
        return np.array([0, 0, 0, r, r, r, 1.0, 1.0, 1.0])
    if model == "home_appa":
        return np.array([0, 0, 0, 1.0, r, r, 1.0, 1.0, 1.0])
    raise ValueError(model)


# --------------------------------------------------------- collisions --------

def _mrt(f, M, r):
    """f - M^-1 R M (f - f_eq) per cell (Eqs. mrt_rm_collision, cm_collision).
    M has shape (9, 9) or cells + (9, 9)."""
    rho, ux, uy = moments(f)[:3]
    d = np.moveaxis(f - feq(rho, ux, uy), 0, -1)[..., None]        # cells + (9, 1)
    Md = (M @ d)[..., 0] * r
    corr = np.linalg.solve(np.broadcast_to(M, Md.shape + (9,)), Md[..., None])[..., 0]
    return f - np.moveaxis(corr, -1, 0)


def collide(model, f, tau, r=None):
    """Post-collision distributions g(f) of Eq. g_mapping for one model.

    bgk        Eq. bgk_collision
    rm         Eq. mrt_rm_collision with M^RM
    nocm       Eq. cm_collision with M^NOCM(u) of each cell
    home       Eq. home_mapping: h(m(f+)), f+ the NOCM-MRT post-collision state
    home_appa  h applied to App. A's collision (D = 2) of m(f) (R24)
    r overrides the rate vector of the MRT models."""
    if model == "bgk":
        rho, ux, uy = moments(f)[:3]
        return f - (f - feq(rho, ux, uy)) / tau
    if r is None and model != "home_appa":
        r = rates(model, tau)
    if model == "rm":
        return _mrt(f, M_RM, r)
    if model in ("nocm", "home"):
        rho, ux, uy = moments(f)[:3]
        fp = _mrt(f, m_nocm(ux, uy), r)
        if model == "nocm":
            return fp
        return reconstruct(*moments(fp))
    if model == "home_appa":
        rho, ux, uy, sxx, sxy, syy = moments(f)
        om = 1.0 / tau
        usq = ux * ux + uy * uy
        pxy = (1 - om) * sxy + om * ux * uy
        pxx = (tau - 1) / (2 * tau) * (sxx - syy) + 0.5 * usq + om * 0.5 * (ux * ux - uy * uy)
        pyy = (tau - 1) / (2 * tau) * (syy - sxx) + 0.5 * usq + om * 0.5 * (uy * uy - ux * ux)
        return reconstruct(rho, ux, uy, pxx, pxy, pyy)
    raise ValueError(model)


def stream(g):
    """Pull streaming on a periodic grid: f_i(x, t + 1) = g_i(x - c_i)."""
    out = np.empty_like(g)
    for i in range(9):
        out[i] = np.roll(g[i], shift=(int(CY[i]), int(CX[i])), axis=(0, 1))
    return out


def step(model, f, tau, r=None):
    """One collide-and-stream step, Eq. lbe_without_force_update."""
    return stream(collide(model, f, tau, r))


def rest_state(model, rho, ux, uy):
    """The uniform fixed point of the model's step: f_eq, or h(rho, u, u u)
    for the HOME composites."""
    if model in ("home", "home_appa"):
        return heq(rho, ux, uy)
    return feq(rho, ux, uy)


# ---------------------------------------------- linearised operators ---------

def equilibrium_jacobian(rho, ux, uy, of="feq"):
    """Eq. Lambda_chainrule: Lambda_ij = d f_eq_i/d rho * 1
    + sum_a d f_eq_i / d u_a * (c_ja - u_a) / rho, at a uniform state."""
    d_rho, d_ux, d_uy = (feq_derivatives if of == "feq" else heq_derivatives)(rho, ux, uy)
    return (np.outer(d_rho, np.ones(9)) + np.outer(d_ux, (CX - ux) / rho)
            + np.outer(d_uy, (CY - uy) / rho))


def hermite_qb(ux, uy):
    """(A2 + A3 R_u) B of App. D under reading R20: a 9x9 matrix taking a
    perturbation of f to the f_neq that h reconstructs from its a2."""
    hxx, hxy, hyy = CX * CX - CS2, CX * CY, CY * CY - CS2
    hxxx, hyyy = CX ** 3 - 3 * CS2 * CX, CY ** 3 - 3 * CS2 * CY
    hxxy, hxyy = CY * (CX * CX - CS2), CX * (CY * CY - CS2)
    A2 = (W / (2 * CS2 ** 2))[:, None] * np.stack([hxx, 2 * hxy, hyy], 1)
    A3 = (W / (6 * CS2 ** 3))[:, None] * np.stack([hxxx, 3 * hxxy, 3 * hxyy, hyyy], 1)
    Ru = np.array([[3 * ux, 0, 0], [uy, 2 * ux, 0], [0, 2 * uy, ux], [0, 0, 3 * uy]])
    B = np.stack([CX * CX - CS2, CX * CY, CY * CY - CS2], 0)
    return (A2 + A3 @ Ru) @ B


def advection(k):
    """D(k) = diag(exp(-i k . c_i))."""
    return np.diag(np.exp(-1j * (C @ np.asarray(k, float))))


def collision_operator(model, rho, ux, uy, tau, r=None):
    """The bracket of G(k) = D(k)[...]: the Jacobian of g at the uniform state.

    bgk            I - (I - Lambda)/tau                       (App. B)
    rm, nocm       I - M^-1 R M (I - Lambda)                  (App. B)
    home, appa     Lambda_h + QB (I - M^-1 R M (I - Lambda) - Lambda)
                                                    (Eq. Mo-NOCM, R20, R21)"""
    I = np.eye(9)
    lam = equilibrium_jacobian(rho, ux, uy)
    if model == "bgk":
        return I - (I - lam) / tau
    if r is None:
        r = rates(model, tau)
    M = M_RM if model == "rm" else m_nocm(ux, uy)
    relax = np.linalg.solve(M, np.diag(r) @ M) @ (I - lam)
    if model in ("rm", "nocm"):
        return I - relax
    lam_h = equilibrium_jacobian(rho, ux, uy, of="heq")
    return lam_h + hermite_qb(ux, uy) @ (I - relax - lam)


def amplification(model, k, rho, ux, uy, tau, r=None):
    """G(k) of Sec. 5.1 / App. B / Eq. Mo-NOCM."""
    return advection(k) @ collision_operator(model, rho, ux, uy, tau, r)


def amplification_grid(model, ks, rho, ux, uy, tau, r=None):
    """G(k) for an array of wave vectors ks[..., 2]: shape ks.shape[:-1] + (9, 9)."""
    K = collision_operator(model, rho, ux, uy, tau, r)
    ph = np.exp(-1j * (np.asarray(ks, float) @ C.T))
    return ph[..., :, None] * K


def omega(lam):
    """R25: omega = i log(lambda)."""
    return 1j * np.log(lam)


# ------------------------------------------------------------- theory --------

def shear_mode(k, u, phi, nu):
    """Eq. shear_mode."""
    return k * u * np.cos(phi) - 1j * k * k * nu


def acoustic_modes(k, u, phi, nu, mu_v, D=2):
    """Eq. acoustic_modes: the (+, -) pair."""
    damp = k * k * ((D - 1) / D * nu + 0.5 * mu_v)
    base = k * u * np.cos(phi)
    cs = np.sqrt(CS2)
    return base + k * cs - 1j * damp, base - k * cs - 1j * damp


def bulk_viscosity(rate_bulk, D=2):
    """Bulk viscosity of a scheme whose trace of the non-equilibrium second
    moment relaxes at rate_bulk: (2/D) cs^2 (1/rate_bulk - 1/2) (Chapman-Enskog
    at first order; equal to (2/D) nu when the trace relaxes with the shear)."""
    return 2.0 / D * CS2 * (1.0 / rate_bulk - 0.5)


# -------------------------------------------------------------- study --------

def hydrodynamic_branches(model, kx, rho, ux, uy, tau):
    """omega of the three hydrodynamic modes (acoustic -, shear, acoustic +)
    along k = (kx, 0), kx ascending from a small nonzero value (where the three
    are distinct), sorted by Re omega there: at the first wave number the
    three eigenvalues nearest 1, then at each next one the eigenvalues nearest
    the branch's previous value."""
    lam = np.linalg.eigvals(amplification_grid(model, np.stack([kx, 0 * kx], 1), rho, ux, uy, tau))
    cur = lam[0][np.argsort(np.abs(lam[0] - 1))[:3]]
    out = np.empty((len(kx), 3), complex)
    for n in range(len(kx)):
        pick = []
        for v in cur:
            cand = [i for i in np.argsort(np.abs(lam[n] - v)) if i not in pick]
            pick.append(cand[0])
        cur = lam[n][pick]
        out[n] = cur
    om = omega(out)
    return np.take_along_axis(om, np.argsort(om.real[:1], axis=1).repeat(len(kx), 0), 1)


def study(nk=129, nk2=65):
    """The three experiments of Sec. 5.2 (Numerical Spectral Analysis), as
    numbers: the stability margin max|lambda(k_x)| at u = 0 for
    nu in {1e-3, 1e-4, 1e-5}; max Im omega over k in [0, pi]^2 for
    u = (0,0) ... (0.3,0.3) at nu = 1e-4; the dispersion omega(k_x) of the
    three hydrodynamic branches at nu = 1e-4, u = 0."""
    out = {"margin": {}, "dissipation": {}, "dispersion": {}}
    kx = np.linspace(0.0, np.pi, nk)
    ks = np.stack([kx, np.zeros_like(kx)], 1)
    for nu in (1e-3, 1e-4, 1e-5):
        tau = tau_of_nu(nu)
        for m in MODELS:
            lam = np.abs(np.linalg.eigvals(amplification_grid(m, ks, 1.0, 0.0, 0.0, tau))).max(-1)
            out["margin"][(m, nu)] = lam
    g = np.linspace(0.0, np.pi, nk2)
    K2 = np.stack(np.meshgrid(g, g, indexing="ij"), -1)
    tau = tau_of_nu(1e-4)
    for uu in (0.0, 0.1, 0.2, 0.3):
        for m in MODELS:
            lam = np.linalg.eigvals(amplification_grid(m, K2, 1.0, uu, uu, tau))
            out["dissipation"][(m, uu)] = np.log(np.abs(lam)).max(-1)
    kd = np.linspace(np.pi / (nk - 1), np.pi, nk - 1)
    for m in MODELS:
        out["dispersion"][m] = hydrodynamic_branches(m, kd, 1.0, 0.0, 0.0, tau)
    out["kd"] = kd
    out["kx"], out["k2"] = kx, g
    return out


def _print_study():
    s = study()
    kx = s["kx"]
    idx = [0, 16, 32, 48, 64, 80, 96, 112, 128]
    print("stability margin max|lambda| at u = 0 (k_y = 0)")
    print("nu      model      " + " ".join(f"{kx[i]:7.3f}" for i in idx) + "   min")
    for (m, nu), lam in s["margin"].items():
        print(f"{nu:<7g} {m:<10} " + " ".join(f"{lam[i]:7.5f}" for i in idx) + f"  {lam.min():7.5f}")
    print("\nmax Im omega over k in [0, pi]^2, nu = 1e-4: max, unstable fraction")
    for (m, uu), im in s["dissipation"].items():
        print(f"u=({uu},{uu}) {m:<10} {im.max():+.3e}  {np.mean(im > 1e-12):.4f}")
    print("\ndispersion: Re omega of the acoustic + branch / (cs k) and of the shear branch, nu = 1e-4, u = 0")
    kd = s["kd"]
    jdx = [i - 1 for i in idx[1:]]
    print("model      " + " ".join(f"{kd[i]:13.3f}" for i in jdx))
    for m, om in s["dispersion"].items():
        print(f"{m:<10} " + " ".join(f"{om[i, 2].real / (np.sqrt(CS2) * kd[i]):6.3f}/{om[i, 1].real:+.3f}"
                                     for i in jdx))


if __name__ == "__main__":
    _print_study()
