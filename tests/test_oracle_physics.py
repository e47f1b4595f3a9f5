"""Pins of the oracle's whole step against conservation laws, fixed points and
closed-form flows: mass and momentum conservation on periodic grids, the
rest and uniform-flow fixed points, Taylor-Green decay exp(-2 nu k^2 t),
shear-wave advection (the dispersion relation of Sec. 5.2 Eq. shear_mode:
omega = k.u - i nu k^2), the Poiseuille profile with bounce-back walls, and
uniform flow through the inflow/outflow faces."""
import numpy as np
import pytest

from paper_2602_05295_amd import workloads as W


def test_conservation_periodic(orc):
    """Collision keeps rho and rho u and streaming permutes: totals are invariant."""
    n = (9, 7, 5)
    m = W.random_moments(*n, seed=1)
    P = orc.make_params(n, 0.56)
    tot0 = m[:4].reshape(4, -1).sum(1)
    for t in range(20):
        m = orc.step(P, m)
    tot = m[:4].reshape(4, -1).sum(1)
    assert abs(tot[0] - tot0[0]) / tot0[0] < 1e-13 * 20
    assert np.abs(tot[1:] - tot0[1:]).max() < 1e-13 * 20 * np.prod(n) * 0.03


def test_mass_conservation_with_walls(orc):
    n = (8, 9, 7)
    mask = W.sphere_mask(*n, phi=0.15, rmin=1.5, rmax=2.5, seed=4)
    m = W.random_moments(*n, seed=2)
    P = orc.make_params(n, 0.6)
    m = orc.step(P, m, mask)  # solid cells -> rest
    fl = mask == 0
    mass0 = m[0][fl].sum()
    for t in range(20):
        m = orc.step(P, m, mask)
        assert np.all(m[0][~fl] == 1.0) and np.all(m[1:][:, ~fl] == 0.0)
    assert abs(m[0][fl].sum() - mass0) / mass0 < 1e-13 * 20


def test_rest_and_uniform_flow_fixed_points(orc):
    n = (5, 4, 3)
    P = orc.make_params(n, 0.7)
    rest = orc.equilibrium_moments(np.ones(n[::-1]), np.zeros((3,) + n[::-1]))
    assert np.abs(orc.step(P, rest) - rest).max() < 1e-15
    u0 = np.array([0.05, -0.02, 0.03])
    uni = orc.equilibrium_moments(np.full(n[::-1], 1.02), np.broadcast_to(u0[:, None, None, None], (3,) + n[::-1]))
    assert np.abs(orc.step(P, uni) - uni).max() < 1e-15


def test_uniform_state_maps_to_its_collision(orc):
    """For a uniform field, streaming is the identity and m(h(.)) = id, so one
    step is the collision alone (computed by App. A's deviatoric form)."""
    n = (4, 3, 5)
    tau = 0.65
    rho, u = 1.04, np.array([0.03, 0.01, -0.05])
    S = np.outer(u, u) + np.array([[2e-3, 1e-3, -5e-4], [1e-3, -1e-3, 3e-4], [-5e-4, 3e-4, 4e-4]])
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    m = np.zeros((10,) + n[::-1])
    m[0] = rho
    m[1:4] = (rho * u)[:, None, None, None]
    for p, (a, b) in enumerate(pairs):
        m[4 + p] = rho * S[a, b]
    D = S - np.outer(u, u)
    Sp = np.outer(u, u) + (1 - 1 / tau) * (D - np.trace(D) / 3 * np.eye(3))
    out = orc.step(orc.make_params(n, tau), m)
    assert np.abs(out[0] - rho).max() < 1e-15
    assert np.abs(out[1:4] - (rho * u)[:, None, None, None]).max() < 1e-16
    for p, (a, b) in enumerate(pairs):
        assert np.abs(out[4 + p] - rho * Sp[a, b]).max() < 1e-16


def _tgv_rate_error(orc, n, steps, U0, tau=0.6):
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / n
    rho, u = W.taylor_green_2d(n, n, 1, U0)
    m = orc.equilibrium_moments(rho, u)
    P = orc.make_params((n, n, 1), tau)
    x = np.arange(n)[None, None, :]
    y = np.arange(n)[None, :, None]
    basis = -np.cos(k * x) * np.sin(k * y)
    amps = []
    for t in range(steps + 1):
        amps.append(((m[1] / m[0]) * basis).sum() / (basis * basis).sum())
        if t < steps:
            m = orc.step(P, m)
    amps = np.array(amps)
    ts = np.arange(steps + 1)
    sel = ts >= steps // 5
    rate = -np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]
    return rate / (2 * nu * k * k) - 1, amps[-1] / amps[0]


def test_taylor_green_decay(orc):
    """Velocity amplitude decays as exp(-2 nu k^2 t), nu = (tau - 1/2)/3
    (reading R9); at 32^2, tau = 0.6, U0 = 0.05 that is 0.7734 after 100 steps.
    Under diffusive scaling (n doubled, U0 halved, 4x steps) the error shrinks."""
    e32, ratio = _tgv_rate_error(orc, 32, 100, 0.05)
    assert abs(e32) < 0.02
    k = 2 * np.pi / 32
    assert abs(ratio - np.exp(-2 * (0.1 / 3) * k * k * 100)) < 0.01
    e64, _ = _tgv_rate_error(orc, 64, 400, 0.025)
    assert abs(e64) * 2.5 <= abs(e32)


def test_shear_wave_advection_and_decay(orc):
    """A transverse wave u_y = A sin(kx) on a uniform flow U e_x moves with the
    flow and decays at nu k^2: omega = k U - i nu k^2 (Eq. shear_mode).  The
    phase pins the streaming direction (f_i(x) = f+_i(x - c_i))."""
    n, tau, U, A = 64, 0.8, 0.05, 1e-3
    nu, k = (tau - 0.5) / 3, 2 * np.pi / n
    x = np.arange(n)
    rho = np.ones((1, 1, n))
    u = np.zeros((3, 1, 1, n))
    u[0] = U
    u[1, 0, 0] = A * np.sin(k * x)
    m = orc.equilibrium_moments(rho, u)
    P = orc.make_params((n, 1, 1), tau)
    amp = []
    T = 200
    for t in range(T + 1):
        amp.append(((m[2] / m[0])[0, 0] * np.exp(-1j * k * x)).sum())
        if t < T:
            m = orc.step(P, m)
    amp = np.array(amp)
    ts = np.arange(T + 1)
    sel = ts >= 20
    phase = np.unwrap(np.angle(amp / amp[0]))
    slope = np.polyfit(ts[sel], phase[sel], 1)[0]
    decay = -np.polyfit(ts[sel], np.log(np.abs(amp / amp[0]))[sel], 1)[0]
    assert abs(slope / (-k * U) - 1) < 1e-3
    assert abs(decay / (nu * k * k) - 1) < 0.01


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0])
def test_poiseuille_profile(orc, tau):
    """Force-driven channel between halfway bounce-back walls at y = 0.5 and
    y = H + 0.5: u(y) = F/(2 rho nu) (y - 1/2)(H + 1/2 - y)."""
    H, F = 16, 1e-6
    nx = nz = 4
    ny = H + 2
    nu = (tau - 0.5) / 3
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, H + 1, :] = 1
    y = np.arange(ny)
    prof = F / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
    prof[0] = prof[-1] = 0
    u = np.zeros((3, nz, ny, nx))
    u[0] = prof[None, :, None]
    m = orc.equilibrium_moments(np.ones((nz, ny, nx)), u)
    P = orc.make_params((nx, ny, nz), tau, F=(F, 0, 0))
    for it in range(6000):
        m2 = orc.step(P, m, mask)
        done = np.abs(m2 - m).max() < 1e-14
        m = m2
        if done:
            break
    ux = (m[1] / m[0])[0, 1:H + 1, 0]
    ref = prof[1:H + 1]
    assert np.linalg.norm(ux - ref) / np.linalg.norm(ref) < 0.02


def test_uniform_inflow_outflow_is_steady(orc):
    """With the inflow velocity everywhere, the face rules (R11) leave the flow
    unchanged: the inflow face's moment boundary reproduces the interior state
    and the zero-gradient outflow copies it."""
    n = (6, 4, 3)
    u_in = np.array([0.08, 0.0, 0.0])
    m = orc.equilibrium_moments(np.ones(n[::-1]), np.broadcast_to(u_in[:, None, None, None], (3,) + n[::-1]))
    P = orc.make_params(n, 0.52, inflow=True, u_in=u_in)
    out = m
    for _ in range(5):
        out = orc.step(P, out)
    assert np.abs(out - m).max() < 1e-15


def test_inflow_drives_flow_from_rest(orc):
    """Starting at rest, the inflow face injects momentum along +x."""
    n = (12, 3, 3)
    m = orc.equilibrium_moments(np.ones(n[::-1]), np.zeros((3,) + n[::-1]))
    P = orc.make_params(n, 0.8, inflow=True, u_in=(0.05, 0, 0))
    for _ in range(30):
        m = orc.step(P, m)
    jx = m[1].mean(axis=(0, 1))
    assert jx[0] > 0.02 and np.all(jx > 0)
    assert np.abs(m[2:4]).max() < 1e-15


def test_step_cells_matches_full_step(orc):
    n = (7, 6, 5)
    mask = W.sphere_mask(*n, phi=0.1, rmin=1.0, rmax=2.0, seed=9)
    mask[:, :, :3] = 0
    mask[:, :, -3:] = 0
    m = W.random_moments(*n, seed=5)
    P = orc.make_params(n, 0.6, inflow=True, u_in=(0.05, 0.01, 0))
    full = orc.step(P, m, mask)
    cells = np.arange(np.prod(n))[::3]
    part = orc.step_cells(P, m, cells, mask)
    assert np.abs(part - full.reshape(10, -1)[:, cells].T).max() == 0


def test_float_instantiation_floor(orc):
    """The float-instantiated oracle on the 32^2 Taylor-Green case stays within
    1e-4 (relative, per moment group) of FP64 after 100 steps; the value is the
    intrinsic single-precision floor of the plain formulation."""
    rho, u = W.taylor_green_2d(32, 32, 1, 0.05)
    m = orc.equilibrium_moments(rho, u)
    P = orc.make_params((32, 32, 1), 0.6)
    m32 = m.astype(np.float32)
    for _ in range(100):
        m = orc.step(P, m)
        m32 = orc.step_f32(P, m32)
    for g in (slice(0, 1), slice(1, 4), slice(4, 10)):
        err = np.abs(m32[g] - m[g]).max() / np.abs(m[g]).max()
        assert err < 1e-4, (g, err)


# ------------------------------------------- moment wall and wall forces ---
# R16: the solid coupling of Sec. 3.2 (f_i(x) = h_i(rho^x, u^p, S^p)); its
# distribution does not depend on where along the link p lies, so on a voxel
# mask the no-slip point sits at the solid node: plane Couette flow between
# walls at y = 0 and y = W + 1 is exactly linear.  R17: momentum exchange.

def _channel(orc, rule, F=0.0, U=0.0, tau=0.8, Wd=16, steps=4000):
    nx = nz = 4
    ny = Wd + 2
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, Wd + 1, :] = 2
    obj = np.zeros((256, 9))
    obj[2, 3] = U
    obj[1, :3] = obj[2, :3] = ((nx - 1) / 2, (Wd + 1) / 2, (nz - 1) / 2)
    P = orc.make_params((nx, ny, nz), tau, F=(F, 0, 0), wall_rule=rule, objects=obj)
    m = orc.equilibrium_moments(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    m = orc.run(P, m, steps, mask, nthreads=1)
    return m, orc.object_forces(P, m, mask), (nx, ny, nz, Wd, (tau - 0.5) / 3)


def test_moment_wall_couette_is_exactly_linear(orc):
    U = 0.01
    m, fo, (nx, ny, nz, Wd, nu) = _channel(orc, 1, U=U)
    y = np.arange(1, Wd + 1)
    ux = (m[1] / m[0])[:, 1:Wd + 1, :]
    ref = (U * y / (Wd + 1))[None, :, None]
    assert np.abs(ux - ref).max() < 1e-5 * U
    # wall shear: the fluid pushes the still wall along +x and holds the moving one back
    sig = nu * U / (Wd + 1) * nx * nz
    assert abs(fo[1, 0] / sig - 1) < 1e-4 and abs(fo[2, 0] / sig + 1) < 1e-4
    # torque about the channel's center: the shear couple, counter-clockwise about z
    tz = fo[1, 5] + fo[2, 5]
    assert 0.85 * Wd * sig < tz < 1.05 * Wd * sig


@pytest.mark.parametrize("rule", [0, 1])
def test_wall_forces_balance_the_body_force(orc, rule):
    """At steady state every unit of momentum the body force puts into the
    fluid goes into the walls: sum of F_x over objects = F x (fluid cells)."""
    F = 1e-5
    m, fo, (nx, ny, nz, Wd, nu) = _channel(orc, rule, F=F, steps=6000)
    assert abs((fo[1, 0] + fo[2, 0]) / (F * nx * nz * Wd) - 1) < 1e-6
    assert abs(fo[1, 1] + fo[2, 1]) < 1e-9 * abs(fo[1, 1])  # wall pressures cancel


def test_moment_wall_keeps_rest(orc):
    dims = (12, 10, 9)
    mask = W.sphere_mask(*dims, phi=0.1, rmin=1.5, rmax=3.0, seed=2)
    m = orc.equilibrium_moments(np.ones(dims[::-1]), np.zeros((3,) + dims[::-1]))
    P = orc.make_params(dims, 0.7, wall_rule=1)
    out = orc.run(P, m, 3, mask)
    fl = mask == 0
    assert np.abs(out[:, fl] - m[:, fl]).max() < 1e-15


def test_torque_moves_with_the_center(orc):
    """tau about C2 = tau about C1 + (C1 - C2) x F, for moving objects in a
    random state: the torque is taken about the object's center."""
    dims = (14, 12, 10)
    mask = W.sphere_mask(*dims, phi=0.12, rmin=1.5, rmax=3.0, seed=4).astype(np.uint8)
    rng = np.random.default_rng(0)
    mask[mask > 0] = 1
    mask[:, :, :6][mask[:, :, :6] > 0] = 7  # a second object
    m = W.random_moments(*dims, seed=9, dj=0.02, dp=0.003).astype(np.float64)
    obj1 = np.zeros((256, 9))
    obj1[:, :3] = rng.uniform(0, 10, (256, 3))
    obj1[:, 3:] = rng.uniform(-0.02, 0.02, (256, 6))
    obj2 = obj1.copy()
    obj2[:, :3] = rng.uniform(0, 10, (256, 3))
    P1 = orc.make_params(dims, 0.7, wall_rule=1, objects=obj1)
    f1 = orc.object_forces(P1, m, mask)
    # the wall velocity changes with the center: keep u^p by moving V with it
    obj2[:, 3:6] = obj1[:, 3:6] + np.cross(obj1[:, 6:], obj2[:, :3] - obj1[:, :3])
    P2 = orc.make_params(dims, 0.7, wall_rule=1, objects=obj2)
    f2 = orc.object_forces(P2, m, mask)
    for k in (1, 7):
        assert np.abs(f1[k, :3]).max() > 0
        np.testing.assert_allclose(f2[k, :3], f1[k, :3], rtol=1e-12, atol=1e-15)
        want = f1[k, 3:] + np.cross(obj1[k, :3] - obj2[k, :3], f1[k, :3])
        np.testing.assert_allclose(f2[k, 3:], want, rtol=1e-10, atol=1e-13)


# --------------------------------------- the paper's mixed-precision pipeline ---
# Storing post-collision instead of post-stream moments moves the storage
# point by half a step: without quantization, stream(collide(m)) is the step.

@pytest.mark.parametrize("case", ["periodic", "walls", "faces"])
def test_mixed_pipeline_is_the_step_shifted(orc, case):
    dims = (14, 11, 9)
    mask, inflow, rule = None, False, 0
    if case != "periodic":
        mask = W.sphere_mask(*dims, phi=0.1, rmin=1.5, rmax=2.5, seed=3)
    if case == "walls":
        rule = 1
    if case == "faces":
        mask[:, :, :3] = 0
        mask[:, :, -3:] = 0
        inflow = True
    P = orc.make_params(dims, 0.62, inflow=inflow, u_in=(0.05, 0.01, 0.0), wall_rule=rule)
    m = W.random_moments(*dims, seed=7, dj=0.02, dp=0.003).astype(np.float64)
    if mask is not None:
        m[:, mask > 0] = np.array([1, 0, 0, 0, 0, 0, 0, 0, 0, 0])[:, None]
    want = orc.step(P, m, mask)
    got = orc.stream_post(P, orc.collide_field(P, m, mask), mask)
    assert np.abs(got - want).max() < 1e-14


def test_mixed_q16_step_keeps_rest_and_mass(orc):
    dims = (10, 9, 8)
    rest = orc.q16_encode(orc.equilibrium_moments(np.ones(dims[::-1]), np.zeros((3,) + dims[::-1])))
    # the rest codes decode to N = +Delta/2 (reading R14); at tau = 1 the
    # collision sets N to 0, whose code is the rest code again
    out, m_ps = orc.mixed_q16_step(orc.make_params(dims, 1.0), rest, mode=0)
    assert np.array_equal(out, rest)
    P = orc.make_params(dims, 0.6)
    # streaming moves mass and momentum without loss: the post-stream sums equal
    # the decoded post-collision sums
    w = orc.q16_encode(W.random_moments(*dims, seed=2, dj=0.02, dp=0.003))
    post = orc.q16_decode(w)
    out, m_ps = orc.mixed_q16_step(P, w, t=1, seed=3, mode=1)
    for k in range(4):
        assert abs(m_ps[k].sum() - post[k].sum()) < 1e-10 * max(1.0, abs(post[k].sum()))


# ---------------------------------------------------------- open faces (R11) --

def test_outflow_of_an_x_invariant_field_is_the_periodic_step(orc):
    """A field that does not depend on x has a zero x-gradient everywhere, so
    the zero-gradient outflow face must pull exactly what the periodic step
    pulls: f_i(nx-1, y, z) = f+_i(nx-1, y - c_y, z - c_z) for c_x = -1.  Cells
    x >= 1 pull nothing from the inflow rule either, so every cell but the
    inflow plane matches the periodic step.  The field has (y, z) structure in
    every moment, so a source without the transverse shift fails."""
    nx, ny, nz = 6, 7, 5
    g = W.random_moments(1, ny, nz, seed=21, dj=0.04, dp=0.004)       # (10, nz, ny, 1)
    m = np.ascontiguousarray(np.broadcast_to(g, (10, nz, ny, nx)))
    for inflow_u in ((0.06, 0.0, 0.0), (0.03, 0.01, -0.02)):
        Po = orc.make_params((nx, ny, nz), 0.57, inflow=True, u_in=inflow_u)
        Pp = orc.make_params((nx, ny, nz), 0.57)
        open_ = orc.step(Po, m)
        per = orc.step(Pp, m)
        assert np.abs(open_[..., 1:] - per[..., 1:]).max() < 1e-14
        # and the inflow plane does differ: the inflow rule is in force
        assert np.abs(open_[..., 0] - per[..., 0]).max() > 1e-4


@pytest.mark.parametrize("tau", [0.53, 0.8])
def test_inflow_keeps_a_uniform_state_with_stress(orc, tau):
    """A uniform state whose velocity equals u_in, with a non-equilibrium
    stress, must map to its own collision at every cell, face cells included:
    the inflow's moment boundary S^p = u_in u_in + (S^x - u^x u^x) then
    rebuilds exactly the cell's post-collision distribution (Sec. 3.2), and
    the outflow's zero gradient copies it.  Dropping the non-equilibrium
    carry-over changes the inflow cells."""
    n = (5, 4, 3)
    u = np.array([0.07, -0.01, 0.02])
    rho = 1.03
    Sneq = np.array([[2e-3, 1e-3, -5e-4], [1e-3, -1e-3, 3e-4], [-5e-4, 3e-4, 4e-4]])
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    S = np.outer(u, u) + Sneq
    m = np.zeros((10,) + n[::-1])
    m[0] = rho
    m[1:4] = (rho * u)[:, None, None, None]
    for p, (a, b) in enumerate(pairs):
        m[4 + p] = rho * S[a, b]
    post = orc.collide(rho, u, [S[a, b] for a, b in pairs], tau)
    want = np.r_[post[0], post[0] * post[1:4], post[0] * post[4:]]
    Po = orc.make_params(n, tau, inflow=True, u_in=u)
    out = orc.step(Po, m)
    assert np.abs(out - want[:, None, None, None]).max() < 1e-15
    # the same field with the wrong inflow velocity is not kept
    Pw = orc.make_params(n, tau, inflow=True, u_in=u + np.array([0.01, 0, 0]))
    assert np.abs(orc.step(Pw, m)[..., 0] - want[:, None, None]).max() > 1e-4


def test_open_channel_settles_to_the_inflow(orc):
    """An obstacle-free channel with periodic y, z started at rest: once the
    start-up transient has left, the mass flux through the inflow plane equals
    the flux through the outflow plane and the inflow plane moves at u_in."""
    n = (32, 4, 4)
    u_in = 0.05
    m = orc.equilibrium_moments(np.ones(n[::-1]), np.zeros((3,) + n[::-1]))
    P = orc.make_params(n, 0.8, inflow=True, u_in=(u_in, 0, 0))
    for _ in range(3000):
        m = orc.step(P, m)
    jx = m[1].mean(axis=(0, 1))
    ux = (m[1] / m[0]).mean(axis=(0, 1))
    assert abs(jx[0] - jx[-1]) / jx[0] < 1e-3, (jx[0], jx[-1])
    assert abs(ux[0] - u_in) / u_in < 1e-3, ux[0]
    assert np.abs(m[2:4]).max() < 1e-15


# ----------------------------------------------------- body force (App. A) --

def _d3q27():
    c = np.array([(x, y, z) for z in (-1, 0, 1) for y in (-1, 0, 1) for x in (-1, 0, 1)], float)
    w1 = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
    w = np.array([w1[int(a)] * w1[int(b)] * w1[int(g)] for a, b, g in c])
    return c, w


def _guo_bgk(f, F, tau):
    """One BGK collision with Guo's forcing term, written on the 27
    distributions (Guo, Zheng & Shi, Phys. Rev. E 65, 046308 (2002)):
    f+ = f - (f - f_eq)/tau + (1 - 1/(2 tau)) w [(c - u)/cs^2 + (c.u) c/cs^4].F,
    u = (sum c f + F/2)/rho, f_eq the second-order Hermite equilibrium."""
    c, w = _d3q27()
    rho = f.sum()
    u = (c.T @ f + F / 2) / rho
    cu = c @ u
    feq = rho * w * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
    src = w * (3 * ((c - u) @ F) + 9 * cu * (c @ F))
    return f - (f - feq) / tau + (1 - 1 / (2 * tau)) * src


@pytest.mark.parametrize("tau", [0.55, 0.7, 1.6])
def test_forced_collision_is_guo_forcing_in_moments(orc, tau):
    """App. A's forced collision equals the moments of a distribution-level
    collision with Guo's forcing: the shear part (off-diagonal entries and
    the deviator of the diagonal) at rate 1/tau, the trace at rate 1 (R8),
    and the momentum rho u + F/2 after the collision.  Each force term of
    App. A is pinned away from tau = 1."""
    c, w = _d3q27()
    rng = np.random.default_rng(int(100 * tau))
    H2 = np.einsum("ia,ib->iab", c, c) - np.eye(3) / 3
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for _ in range(6):
        f = w * (1 + 0.3 * rng.standard_normal(27))               # arbitrary positive set
        F = 1e-2 * rng.standard_normal(3)
        rho = f.sum()
        u = (c.T @ f + F / 2) / rho                             # stored j includes F/2
        Pi = np.einsum("i,iab->ab", f, H2)
        out = orc.collide(rho, u, [Pi[a, b] / rho for a, b in pairs], tau, F)
        Splus = np.zeros((3, 3))
        for p, (a, b) in enumerate(pairs):
            Splus[a, b] = Splus[b, a] = out[4 + p]
        g_shear = _guo_bgk(f, F, tau)
        g_bulk = _guo_bgk(f, F, 1.0)
        Pi_s = np.einsum("i,iab->ab", g_shear, H2)
        Pi_b = np.einsum("i,iab->ab", g_bulk, H2)
        dev = lambda A: A - np.trace(A) / 3 * np.eye(3)
        assert np.abs(dev(rho * Splus) - dev(Pi_s)).max() < 1e-15
        assert abs(np.trace(rho * Splus) - np.trace(Pi_b)) < 1e-15
        assert np.abs(rho * out[1:4] - c.T @ g_shear).max() < 1e-15
