"""GPU adjoint against the FP64 oracle's adjoint (itself checked against
central differences and the dot-product identity on the CPU).

One step: lam_prev = J(m)^T lam_next per moment group within 2e-5 (relative
to the group's largest value).  A checkpointed 40-step rollout on a 24^3 box
with spheres: d loss / d u0 within 1e-4 relative L2 of the oracle's gradient.
"""
import numpy as np
import pytest

from paper_2602_05295_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _note(*a):
    print("CASE", *a, flush=True)


def _raw_from_moments(m):
    r = m.astype(np.float32).copy()
    r[0] = r[0] - np.float32(1.0)
    return r


@pytest.mark.parametrize("case", ["periodic", "walls", "faces"])
def test_adjoint_step_matches_oracle(orc, torch_mod, case):
    torch = torch_mod
    from paper_2602_05295_amd.homelbm import HomeLBM
    dims = (29, 22, 17)
    _note("adjoint step", case, dims)
    mask = None
    inflow = case == "faces"
    if case != "periodic":
        mask = W.sphere_mask(*dims, phi=0.08, rmin=1.5, rmax=3.0, seed=4)
        if inflow:
            mask[:, :, :3] = 0
            mask[:, :, -3:] = 0
    m = W.random_moments(*dims, seed=3, dj=0.02, dp=0.003)
    if mask is not None:
        m[:, mask == 1] = 0.0
        m[0][mask == 1] = 1.0
    raw = _raw_from_moments(m)
    lam = np.random.default_rng(5).standard_normal(m.shape).astype(np.float32)
    u_in = (0.05, 0.01, -0.02)
    with HomeLBM(dims, 0.6, mask=mask) as s:
        if inflow:
            s.set_options(inflow=True, u_in=u_in)
        mt = torch.from_numpy(raw).cuda()
        ln = torch.from_numpy(lam).cuda()
        lp = torch.empty_like(ln)
        s.adjoint_step(mt, ln, lp)
        s.synchronize()
        got = lp.cpu().numpy()
    m64 = raw.astype(np.float64)
    m64[0] += 1.0
    P = orc.make_params(dims, 0.6, inflow=inflow, u_in=u_in)
    ref = orc.adjoint_step(P, m64, lam.astype(np.float64), mask)
    for g in (slice(0, 1), slice(1, 4), slice(4, 10)):
        err = np.abs(got[g] - ref[g]).max() / np.abs(ref[g]).max()
        assert err < 2e-5, (case, g, err)


def _oracle_gradient(orc, P, mask, u0, target, T):
    """d loss / d u0 with the oracle: forward, adjoint, then the equilibrium
    map and the loss taken by complex step (cellwise maps)."""
    rho0 = np.ones(u0.shape[1:])
    m = orc.equilibrium_moments(rho0, u0)
    if mask is not None:
        m[:, mask == 1] = 0.0
        m[0][mask == 1] = 1.0
    traj = [m]
    for _ in range(T):
        traj.append(orc.step(P, traj[-1], mask))
    fl = np.ones(u0.shape[1:], bool) if mask is None else (mask == 0)

    def loss_cells(mm):
        u = mm[1:4] / mm[0]
        return 0.5 * (((u - target) ** 2).sum(0) * fl)

    h = 1e-30
    lam = np.zeros_like(m)
    for k in range(10):
        mc = traj[-1].astype(complex)
        mc[k] += 1j * h
        lam[k] = loss_cells(mc).imag / h
    for t in range(T - 1, -1, -1):
        lam = orc.adjoint_step(P, traj[t], lam, mask)
    g = np.zeros_like(u0)
    for a in range(3):
        uc = u0.astype(complex)
        uc[a] += 1j * h
        dm = orc.equilibrium_moments(rho0.astype(complex), uc).imag / h
        g[a] = (lam * dm).sum(0)
    if mask is not None:
        g[:, mask == 1] = 0.0
    loss = loss_cells(traj[-1]).sum()
    return g, loss


def test_rollout_gradient_matches_oracle(orc, torch_mod):
    torch = torch_mod
    from paper_2602_05295_amd.adjoint import rollout
    from paper_2602_05295_amd.homelbm import HomeLBM
    n, T, every = 24, 40, 10
    _note("rollout gradient", n, T)
    mask = W.sphere_mask(n, n, n, phi=0.05, rmin=2.0, rmax=4.0, seed=7)
    u0 = W.random_solenoidal(n, n, n, 4.0, 0.05, seed=1)
    tgt = W.random_solenoidal(n, n, n, 4.0, 0.05, seed=2)
    fl = (mask == 0)
    with HomeLBM((n, n, n), 0.6, mask=mask) as s:
        u = torch.tensor(u0, dtype=torch.float32, device="cuda", requires_grad=True)
        out = rollout(s, u, T, every)
        vel = out[1:4] / out[0]
        t = torch.tensor(tgt, dtype=torch.float32, device="cuda")
        w = torch.tensor(fl, dtype=torch.float32, device="cuda")
        loss = 0.5 * (((vel - t) ** 2).sum(0) * w).sum()
        loss.backward()
        g_gpu = u.grad.detach().cpu().numpy().astype(np.float64)
        loss_gpu = float(loss.detach())
    P = orc.make_params((n, n, n), 0.6)
    g_orc, loss_orc = _oracle_gradient(orc, P, mask, u0.astype(np.float32).astype(np.float64), tgt, T)
    assert abs(loss_gpu - loss_orc) / loss_orc < 1e-4
    rel = np.linalg.norm(g_gpu - g_orc) / np.linalg.norm(g_orc)
    assert rel < 1e-4, rel


def test_adjoint_step_full_size_sampled(orc, torch_mod):
    """The adjoint benchmark's configuration: 128^3 with ~5% sphere obstacles,
    FP32, tau = 0.6, at the state reached after 10 steps from its initial
    field.  One adjoint step, lam_prev at 3000+ sampled cells (among them
    fluid cells next to a wall) against the oracle's transpose gathered at
    those cells, within 2e-5 per moment group."""
    torch = torch_mod
    from paper_2602_05295_amd.homelbm import HomeLBM
    n = 128
    dims = (n, n, n)
    _note("adjoint step full size sampled", dims)
    mask = W.sphere_mask(n, n, n, phi=0.05, rmin=4.0, rmax=12.0, seed=0)
    u0 = W.random_solenoidal(n, n, n, 4.0, 0.05, seed=0).astype(np.float32)
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((10, n, n, n)).astype(np.float32)
    with HomeLBM(dims, 0.6, mask=mask) as s:
        s.set_equilibrium(np.ones((n, n, n), np.float32), u0)
        s.step(10)
        m = s.get_moments()
        raw = _raw_from_moments(m)
        mt = torch.from_numpy(raw).cuda()
        ln = torch.from_numpy(lam).cuda()
        lp = torch.empty_like(ln)
        s.adjoint_step(mt, ln, lp)
        s.synchronize()
        got = lp.cpu().numpy().reshape(10, -1)
    fluid = np.flatnonzero(mask.ravel() == 0)
    solid = np.flatnonzero(mask.ravel() != 0)
    near = (rng.choice(solid, 1500) + rng.choice([-1, 1, -n, n, -n * n, n * n], 1500)) % (n ** 3)
    near = near[mask.ravel()[near] == 0]
    cells = np.unique(np.concatenate([rng.choice(fluid, 2000, replace=False), near]))
    m64 = raw.astype(np.float64)
    m64[0] += 1.0
    P = orc.make_params(dims, 0.6)
    ref = orc.adjoint_step_cells(P, m64, lam.astype(np.float64), cells, mask).T
    g = got[:, cells]
    for grp in (slice(0, 1), slice(1, 4), slice(4, 10)):
        err = np.abs(g[grp] - ref[grp]).max() / np.abs(ref[grp]).max()
        assert err < 2e-5, (grp, err)
