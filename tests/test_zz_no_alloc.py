"""The allocation-free adjoint entry point (lbm_adjoint_step_noalloc) against
lbm_adjoint_step, called through the C ABI on two contexts in a row, the
second smaller than the first, so the second call runs over flags the first
one left in the shared device array.  Both run the same kernels on the same
inputs, so the outputs must be identical."""
import numpy as np
import pytest

from paper_2602_05295_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(torch, H, dims, seed, inflow):
    mask = W.sphere_mask(*dims, phi=0.08, rmin=1.5, rmax=3.0, seed=seed)
    if inflow:
        mask[:, :, :3] = 0
        mask[:, :, -3:] = 0
    m = W.random_moments(*dims, seed=seed + 1, dj=0.02, dp=0.003)
    m[:, mask == 1] = 0.0
    m[0][mask == 1] = 1.0
    raw = m.astype(np.float32)
    raw[0] -= np.float32(1.0)
    lam = np.random.default_rng(seed + 2).standard_normal(m.shape).astype(np.float32)
    L = H.lib()
    with H.HomeLBM(dims, 0.6, mask=mask) as s:
        if inflow:
            s.set_options(inflow=True, u_in=(0.05, 0.01, -0.02))
        s.step(1)  # builds the boundary list for the face setting
        mt = torch.from_numpy(raw).cuda()
        ln = torch.from_numpy(lam).cuda()
        ref = torch.full_like(ln, float("nan"))
        got = torch.full_like(ln, float("nan"))
        assert L.lbm_adjoint_step(s._h, mt.data_ptr(), ln.data_ptr(), ref.data_ptr()) == H.OK
        st = L.lbm_adjoint_step_noalloc(s._h, mt.data_ptr(), ln.data_ptr(), got.data_ptr())
        assert st == H.OK, L.lbm_last_error(s._h)
        s.synchronize()
        return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_adjoint_equals_adjoint_step():
    import torch
    from paper_2602_05295_amd import homelbm as H
    for dims, seed, inflow in [((48, 40, 36), 3, True), ((30, 21, 17), 9, False)]:
        print("CASE noalloc adjoint", dims, seed, inflow, flush=True)
        ref, got = _case(torch, H, dims, seed, inflow)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(got, ref), np.abs(got - ref).max()


def test_noalloc_adjoint_seeded_sequence():
    """Eight contexts in a row with seeded shapes, growing and shrinking,
    spheres always and open faces or not: every call equals lbm_adjoint_step."""
    import torch
    from paper_2602_05295_amd import homelbm as H
    rng = np.random.default_rng(17)
    for k in range(8):
        dims = (int(rng.integers(8, 80)), int(rng.integers(6, 40)), int(rng.integers(6, 30)))
        inflow = bool(rng.integers(0, 2))
        print("CASE noalloc adjoint sequence", k, dims, inflow, flush=True)
        ref, got = _case(torch, H, dims, 100 + k, inflow)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(got, ref), (k, np.abs(got - ref).max())


def test_noalloc_adjoint_rejects_what_it_cannot_do():
    import torch
    from paper_2602_05295_amd import homelbm as H
    L = H.lib()
    print("CASE noalloc adjoint errors", flush=True)
    dims = (12, 10, 8)
    with H.HomeLBM(dims, 0.6, fmt="q16") as s:
        buf = torch.zeros(10 * s.N, device="cuda")
        out = torch.zeros_like(buf)
        assert L.lbm_adjoint_step_noalloc(s._h, buf.data_ptr(), buf.data_ptr(), out.data_ptr()) == H.ERR_UNSUPPORTED
    with H.HomeLBM(dims, 0.6) as s:
        buf = torch.zeros(10 * s.N, device="cuda")
        assert L.lbm_adjoint_step_noalloc(s._h, buf.data_ptr(), buf.data_ptr(), buf.data_ptr()) == H.ERR_INVALID_ARG
    # one cell more than the scratch array holds: refused before any launch
    with H.HomeLBM((512, 256, 257), 0.6) as s:
        a, b, c = (torch.zeros(16, device="cuda") for _ in range(3))
        assert L.lbm_adjoint_step_noalloc(s._h, a.data_ptr(), b.data_ptr(), c.data_ptr()) == H.ERR_INVALID_ARG
        assert b"33554432" in L.lbm_last_error(s._h)
