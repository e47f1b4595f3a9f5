"""Long-horizon GPU checks against the FP64 oracle.

* Statistics of a chaotic flow: a 64^3 analogue of the decaying-turbulence
  configuration (tau = 0.51, seeded solenoidal field on |k| <= 4, max |u| =
  0.1 cs), 1000 steps in FP32 and in 16-bit moments.  Pointwise values part
  ways (the flow is chaotic); kinetic energy and enstrophy must stay within
  0.5% of the oracle's unquantized FP64 run at t = 100, 500 and 1000.  The
  16-bit run's RMS velocity error and energy-decay deviation from FP64 are
  printed (physics fidelity, not parity).
* 16-bit against unquantized FP64 on the 32^3 Taylor-Green vortex over 100
  steps: decoded velocity within 2 Delta_u sqrt(t) of the exact FP64 step at
  every cell, and a decay rate within 2% of the closed form exp(-2 nu k^2 t).
* 16-bit codes over 20 steps of a 200 x 100 x 100 crop of the obstacle
  channel against the oracle's 16-bit run with the same dither: decoded
  codec variables within 2 Delta sqrt(t).
* The adjoint at the benchmark horizon: 400 steps with a checkpoint every 20,
  spheres at ~5%, tau = 0.6, on a 32^3 box (the size the oracle affords):
  GPU d loss / d u0 within 1e-3 relative L2 of the oracle's gradient.
"""
import numpy as np
import pytest

from helpers import DELTA, codec_vars
from paper_2602_05295_amd import workloads as W

pytestmark = pytest.mark.gpu


def _note(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def H():
    from paper_2602_05295_amd import homelbm
    homelbm.lib()
    return homelbm


def _stats(m):
    """Kinetic energy sum(rho |u|^2)/2 and enstrophy sum |curl u|^2 / 2
    (central differences, periodic) of a moment field (10, nz, ny, nx)."""
    m = np.asarray(m, dtype=np.float64)
    rho = m[0]
    u = m[1:4] / rho
    ke = 0.5 * (rho * (u * u).sum(0)).sum()

    def d(f, axis):  # derivative along array axis (0 = z, 1 = y, 2 = x)
        return 0.5 * (np.roll(f, -1, axis) - np.roll(f, 1, axis))

    wx = d(u[2], 1) - d(u[1], 0)
    wy = d(u[0], 0) - d(u[2], 2)
    wz = d(u[1], 2) - d(u[0], 1)
    ens = 0.5 * (wx * wx + wy * wy + wz * wz).sum()
    return ke, ens


def test_turbulence_64_statistics_1000_steps(H, orc):
    n, tau = 64, 0.51
    _note("turbulence 64^3 statistics 1000 steps")
    u = W.random_solenoidal(n, n, n, 4.0, 0.1 * W.CS, seed=3).astype(np.float32)
    rho = np.ones((n, n, n), np.float32)
    marks = [100, 500, 1000]
    got = {}
    for fmt in ("fp32", "q16"):
        with H.HomeLBM((n, n, n), tau, fmt=fmt) as s:
            s.set_options(dither_mode=1, seed=0)
            s.set_equilibrium(rho, u)
            if fmt == "fp32":
                m0 = s.get_moments().astype(np.float64)
            t = 0
            for T in marks:
                s.step(T - t)
                t = T
                got[(fmt, T)] = s.get_moments().astype(np.float64)
    P = orc.make_params((n, n, n), tau)
    ref = {}
    m = m0
    t = 0
    for T in marks:
        m = orc.run(P, m, T - t)
        t = T
        ref[T] = m
    ke0 = _stats(m0)[0]
    for T in marks:
        ke_r, ens_r = _stats(ref[T])
        for fmt in ("fp32", "q16"):
            ke, ens = _stats(got[(fmt, T)])
            assert abs(ke - ke_r) / ke_r < 5e-3, (fmt, T, ke, ke_r)
            assert abs(ens - ens_r) / ens_r < 5e-3, (fmt, T, ens, ens_r)
        uq = got[("q16", T)][1:4] / got[("q16", T)][0]
        ur = ref[T][1:4] / ref[T][0]
        rms = np.sqrt(((uq - ur) ** 2).sum(0).mean()) / np.sqrt((ur * ur).sum(0).mean())
        keq = _stats(got[("q16", T)])[0]
        print(f"q16 vs fp64 at t={T}: rms velocity error {rms:.3e} (relative), "
              f"energy decay KE/KE0 {keq / ke0:.6f} vs {ke_r / ke0:.6f} "
              f"(deviation {(keq - ke_r) / ke_r:+.2e})", flush=True)


def test_q16_taylor_green_against_unquantized(H, orc):
    n, tau, U0, T = 32, 0.6, 0.05, 100
    _note("q16 taylor-green vs fp64", n, T)
    rho, u = W.taylor_green_2d(n, n, n, U0)
    with H.HomeLBM((n, n, n), tau, fmt="q16") as s:
        s.set_options(dither_mode=1, seed=7)
        s.set_equilibrium(rho.astype(np.float32), u.astype(np.float32))
        m0 = s.get_moments().astype(np.float64)  # the decoded initial state
        traj = [m0]
        for _ in range(T):
            s.step(1)
            traj.append(s.get_moments().astype(np.float64))
    P = orc.make_params((n, n, n), tau)
    m = m0
    k = 2 * np.pi / n
    nu = (tau - 0.5) / 3
    x = np.arange(n)[None, None, :]
    y = np.arange(n)[None, :, None]
    basis = -np.cos(k * x) * np.sin(k * y)
    amps = []
    worst = 0.0
    for t in range(1, T + 1):
        m = orc.step(P, m)
        vq = codec_vars(traj[t])
        vr = codec_vars(m)
        err = np.abs(vq[1:4] - vr[1:4]).max()
        worst = max(worst, err / (DELTA[1] * np.sqrt(t)))
        assert err <= 2 * DELTA[1] * np.sqrt(t), (t, err)
        amps.append(((traj[t][1] / traj[t][0]) * basis).sum() / (basis * basis).sum())
    ts = np.arange(1, T + 1)
    sel = ts >= T // 5
    rate = -np.polyfit(ts[sel], np.log(np.array(amps)[sel]), 1)[0]
    assert abs(rate / (2 * nu * k * k) - 1) < 0.02, rate / (2 * nu * k * k)
    print(f"q16 taylor-green: max |u_q16 - u_fp64| / (Delta_u sqrt(t)) = {worst:.3f}; "
          f"decay rate / closed form = {rate / (2 * nu * k * k):.5f}", flush=True)


def test_q16_channel_crop_20_steps(H, orc):
    _note("q16 channel crop 20 steps")
    full = W.channel_mask(1000, 400, 400, seed=0)
    mask = np.ascontiguousarray(full[150:250, 150:250, 400:600])
    del full
    mask[:, :, :3] = 0
    mask[:, :, -3:] = 0
    nz, ny, nx = mask.shape
    T, seed = 20, 11
    u = np.zeros((3, nz, ny, nx), np.float32)
    rho = np.ones((nz, ny, nx), np.float32)
    with H.HomeLBM((nx, ny, nz), 0.52, mask=mask, fmt="q16") as s:
        # the impulsive start drives a few stress codes of the crop to the end
        # of their range (saturation, reading R5, which the oracle applies too)
        s.set_options(inflow=True, u_in=(0.08, 0, 0), dither_mode=1, seed=seed, check_health=False)
        s.set_equilibrium(rho, u)
        s.step(5)  # the inflow has started to drive the flow
        t0 = s.step_count
        w = s.get_raw().copy()
        s.step(T)
        got = s.get_moments().astype(np.float64)
    P = orc.make_params((nx, ny, nz), 0.52, inflow=True, u_in=(0.08, 0.0, 0.0))
    for t in range(T):
        w = orc.q16_step(P, w, mask, t=t0 + t, seed=seed, mode=1)
    ref = orc.q16_decode(w)
    fl = mask == 0
    vg = codec_vars(got)[:, fl]
    vr = codec_vars(ref)[:, fl]
    d = np.abs(vg - vr).max(axis=1)
    bound = 2 * DELTA * np.sqrt(T)
    assert np.all(d <= bound), (d / DELTA, bound / DELTA)
    print("q16 channel crop: max |difference| / Delta per variable after 20 steps:",
          np.round(d / DELTA, 2).tolist(), flush=True)


def _oracle_gradient(orc, P, mask, u0, target, T):
    """d loss / d u0 with the oracle: forward (all states kept), the adjoint
    steps (the transpose gathered per cell, the same map as the scattered
    adjoint), then the equilibrium map and the loss by complex step."""
    rho0 = np.ones(u0.shape[1:])
    m = orc.equilibrium_moments(rho0, u0)
    m[:, mask == 1] = 0.0
    m[0][mask == 1] = 1.0
    traj = [m]
    for _ in range(T):
        traj.append(orc.step(P, traj[-1], mask))
    fl = mask == 0

    def loss_cells(mm):
        uu = mm[1:4] / mm[0]
        return 0.5 * (((uu - target) ** 2).sum(0) * fl)

    h = 1e-30
    lam = np.zeros_like(m)
    for k in range(10):
        mc = traj[-1].astype(complex)
        mc[k] += 1j * h
        lam[k] = loss_cells(mc).imag / h
    cells = np.arange(m[0].size)
    for t in range(T - 1, -1, -1):
        lam = orc.adjoint_step_cells(P, traj[t], lam, cells, mask).T.reshape(m.shape)
    g = np.zeros_like(u0)
    for a in range(3):
        uc = u0.astype(complex)
        uc[a] += 1j * h
        dm = orc.equilibrium_moments(rho0.astype(complex), uc).imag / h
        g[a] = (lam * dm).sum(0)
    g[:, mask == 1] = 0.0
    return g, loss_cells(traj[-1]).sum()


def test_adjoint_gradient_at_the_benchmark_horizon(H, orc):
    import torch
    from paper_2602_05295_amd.adjoint import rollout
    n, T, every = 32, 400, 20
    _note("adjoint gradient horizon", n, T, every)
    mask = W.sphere_mask(n, n, n, phi=0.05, rmin=2.0, rmax=4.0, seed=5)
    u0 = W.random_solenoidal(n, n, n, 4.0, 0.05, seed=11)
    tgt = W.random_solenoidal(n, n, n, 4.0, 0.05, seed=12)
    with H.HomeLBM((n, n, n), 0.6, mask=mask) as s:
        s.set_options(check_health=False)
        u = torch.tensor(u0, dtype=torch.float32, device="cuda", requires_grad=True)
        out = rollout(s, u, T, every)
        vel = out[1:4] / out[0]
        t = torch.tensor(tgt, dtype=torch.float32, device="cuda")
        w = torch.tensor(mask == 0, dtype=torch.float32, device="cuda")
        loss = 0.5 * (((vel - t) ** 2).sum(0) * w).sum()
        loss.backward()
        g_gpu = u.grad.detach().cpu().numpy().astype(np.float64)
        loss_gpu = float(loss.detach())
    P = orc.make_params((n, n, n), 0.6)
    g_orc, loss_orc = _oracle_gradient(orc, P, mask, u0.astype(np.float32).astype(np.float64), tgt, T)
    assert abs(loss_gpu - loss_orc) / loss_orc < 1e-4
    rel = np.linalg.norm(g_gpu - g_orc) / np.linalg.norm(g_orc)
    print(f"adjoint at {T} steps: relative L2 gradient difference {rel:.3e}", flush=True)
    assert rel < 1e-3, rel
