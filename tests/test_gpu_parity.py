"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

FP32 storage: per moment group, max |gpu - oracle| / max |oracle| <= 1e-5.
Q16 storage: from identical codes, one step gives codes within 1 LSB of the
oracle's with fewer than 1% differing; over t steps the decoded codec
variables stay within 2 Delta sqrt(t) of the oracle's (Delta = one
quantization step of that variable).
"""
import numpy as np
import pytest

from helpers import DELTA, codec_vars, group_rel_err, unpack
from paper_2602_05295_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def H():
    from paper_2602_05295_amd import homelbm
    homelbm.lib()
    return homelbm


def _note(*a):
    print("CASE", *a, flush=True)


def _orc_params(orc, dims, tau, inflow=False, u_in=(0, 0, 0), F=(0, 0, 0)):
    return orc.make_params(dims, tau, F=F, inflow=inflow, u_in=u_in)


def _faces_clear(mask):
    mask[:, :, :3] = 0
    mask[:, :, -3:] = 0
    return mask


# ------------------------------------------------------------------ FP32 ---

@pytest.mark.parametrize("dims", [(37, 29, 23), (64, 17, 9), (5, 3, 2), (1, 1, 1), (31, 45, 3), (2, 33, 4)])
def test_fp32_one_step_random(H, orc, dims):
    _note("fp32 one step", dims)
    m = W.random_moments(*dims, seed=sum(dims)).astype(np.float32)
    with H.HomeLBM(dims, 0.57) as s:
        s.set_moments(m)
        s.step(1)
        got = s.get_moments()
    ref = orc.step(_orc_params(orc, dims, 0.57), m.astype(np.float64))
    err = group_rel_err(got, ref)
    assert max(err.values()) <= TOL32, err


@pytest.mark.parametrize("rows", [8, 10, 12, 13])
def test_fp32_tile_heights_agree_with_oracle_and_each_other(H, orc, rows):
    """Every tile height, with ragged tiles in x and y and several z segments,
    gives the oracle's step and the same bits as the automatic choice (the
    height the context times as fastest, which leaves the state alone)."""
    dims = (130, 53, 40)
    _note("fp32 tile rows", rows, dims)
    m = W.random_moments(*dims, seed=21).astype(np.float32)
    outs = {}
    for tr in (0, rows):
        with H.HomeLBM(dims, 0.57) as s:
            s.set_options(tile_rows=tr)
            s.set_moments(m)
            before = s.get_raw().copy()
            assert s.tile_rows == tr  # 0: not timed yet
            s.prepare(2)  # times the heights when tr is 0; takes no step
            assert s.step_count == 0 and np.array_equal(s.get_raw(), before)
            assert s.tile_rows == (tr if tr else s.tile_rows) and s.tile_rows in (8, 10, 12, 13)
            s.step(2)
            outs[tr] = s.get_raw()
    assert np.array_equal(outs[0], outs[rows])
    P = _orc_params(orc, dims, 0.57)
    ref = orc.step(P, orc.step(P, m.astype(np.float64)))
    got = outs[rows].astype(np.float64)
    got[0] += 1.0
    err = group_rel_err(got, ref)
    assert max(err.values()) <= TOL32, err


@pytest.mark.parametrize("rows", [8, 13])
def test_q16_tile_heights_same_codes(H, rows):
    dims = (97, 40, 33)
    _note("q16 tile rows", rows, dims)
    m = W.random_moments(*dims, seed=22, dj=0.02, dp=0.003).astype(np.float32)
    outs = {}
    for tr in (0, rows):
        with H.HomeLBM(dims, 0.58, fmt="q16") as s:
            s.set_options(tile_rows=tr, dither_mode=1, seed=3)
            s.set_moments(m)
            s.step(3)
            outs[tr] = s.get_raw()
    assert np.array_equal(outs[0], outs[rows])


def test_fp32_taylor_green_100_steps(H, orc):
    _note("fp32 TGV 32^3 100 steps")
    rho, u = W.taylor_green_2d(32, 32, 32, 0.05)
    with H.HomeLBM((32, 32, 32), 0.6) as s:
        s.set_equilibrium(rho.astype(np.float32), u.astype(np.float32))
        m0 = s.get_moments()
        s.step(100)
        got = s.get_moments()
    ref = orc.run(_orc_params(orc, (32, 32, 32), 0.6), m0.astype(np.float64), 100)
    err = group_rel_err(got, ref)
    assert max(err.values()) <= TOL32, err


@pytest.mark.parametrize("inflow", [False, True])
def test_fp32_solids_and_faces(H, orc, inflow):
    dims = (26, 19, 13)
    _note("fp32 solids", dims, "inflow", inflow)
    mask = W.sphere_mask(*dims, phi=0.08, rmin=1.5, rmax=3.0, seed=5)
    if inflow:
        mask = _faces_clear(mask)
    m = W.random_moments(*dims, seed=3).astype(np.float32)
    u_in = (0.06, 0.01, -0.02)
    with H.HomeLBM(dims, 0.62, mask=mask) as s:
        if inflow:
            s.set_options(inflow=True, u_in=u_in)
        s.set_moments(m)
        m0 = s.get_moments()
        s.step(5)
        got = s.get_moments()
        nfl, nso = s.boundary_counts()
        assert nfl > 0 and nso > 0
    P = _orc_params(orc, dims, 0.62, inflow, u_in)
    ref = orc.run(P, m0.astype(np.float64), 5, mask)
    err = group_rel_err(got, ref)
    assert max(err.values()) <= TOL32, err


def test_fp32_rest_is_exact_fixed_point(H):
    _note("fp32 rest")
    dims = (20, 12, 7)
    mask = W.sphere_mask(*dims, phi=0.1, rmin=1.5, rmax=2.5, seed=1)
    with H.HomeLBM(dims, 0.6, mask=mask) as s:
        r0 = s.get_raw().copy()
        s.step(7)
        assert np.array_equal(s.get_raw(), r0)


def test_fp32_bitwise_reproducible(H):
    _note("fp32 reproducible")
    dims = (40, 30, 20)
    mask = W.sphere_mask(*dims, phi=0.05, rmin=2, rmax=4, seed=2)
    m = W.random_moments(*dims, seed=4).astype(np.float32)
    outs = []
    for _ in range(2):
        with H.HomeLBM(dims, 0.55, mask=mask) as s:
            s.set_moments(m)
            s.step(10)
            outs.append(s.get_raw())
    assert np.array_equal(outs[0], outs[1])


# ------------------------------------------------------------------- Q16 ---

def _q16_step_compare(H, orc, dims, tau, mask=None, inflow=False, mode=1, seed=7, t0=3, steps=1, F=(0, 0, 0)):
    m = W.random_moments(*dims, seed=11, dj=0.02, dp=0.003)
    u_in = (0.05, 0.0, 0.01)
    with H.HomeLBM(dims, tau, mask=mask, fmt="q16") as s:
        s.set_options(dither_mode=mode, seed=seed, inflow=inflow, u_in=u_in, force=F)
        s.set_moments(m.astype(np.float32))
        s.step_count = t0
        w0 = s.get_raw().copy()
        s.step(steps)
        got = s.get_raw()
    P = _orc_params(orc, dims, tau, inflow, u_in, F)
    w = w0
    for k in range(steps):
        w = orc.q16_step(P, w, mask, t=t0 + k, seed=seed, mode=mode)
    return got, w


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("dims", [(37, 29, 23), (8, 5, 3), (1, 1, 1)])
def test_q16_one_step_codes(H, orc, dims, mode):
    _note("q16 one step", dims, "dither", mode)
    got, ref = _q16_step_compare(H, orc, dims, 0.58, mode=mode)
    d = np.abs(unpack(got) - unpack(ref))
    assert d.max() <= 1, d.max()
    assert (d > 0).mean() < 0.01, (d > 0).mean()


@pytest.mark.parametrize("inflow", [False, True])
def test_q16_one_step_solids_faces(H, orc, inflow):
    dims = (30, 21, 11)
    _note("q16 solids", dims, "inflow", inflow)
    mask = W.sphere_mask(*dims, phi=0.08, rmin=1.5, rmax=3.0, seed=6)
    if inflow:
        mask = _faces_clear(mask)
    got, ref = _q16_step_compare(H, orc, dims, 0.6, mask=mask, inflow=inflow)
    fl = (mask == 0)
    d = np.abs(unpack(got) - unpack(ref))[:, fl]
    assert d.max() <= 1, d.max()
    assert (d > 0).mean() < 0.01, (d > 0).mean()


def test_q16_taylor_green_100_steps(H, orc):
    _note("q16 TGV 32^3 100 steps")
    n, T = 32, 100
    rho, u = W.taylor_green_2d(n, n, n, 0.05)
    P = _orc_params(orc, (n, n, n), 0.6)
    with H.HomeLBM((n, n, n), 0.6, fmt="q16") as s:
        s.set_options(dither_mode=1, seed=1)
        s.set_equilibrium(rho.astype(np.float32), u.astype(np.float32))
        w = s.get_raw().copy()
        s.step(T)
        got = s.get_raw()
    for k in range(T):
        w = orc.q16_step(P, w, t=k, seed=1, mode=1)
    vg = codec_vars(orc.q16_decode(got))
    vo = codec_vars(orc.q16_decode(w))
    err = np.abs(vg - vo).reshape(10, -1).max(1)
    assert np.all(err <= 2 * DELTA * np.sqrt(T)), err / DELTA


def test_q16_memory_is_half(H):
    _note("memory")
    dims = (30, 20, 10)
    with H.HomeLBM(dims, 0.6) as a, H.HomeLBM(dims, 0.6, fmt="q16") as b:
        sa, _ = a.memory_bytes()
        sb, _ = b.memory_bytes()
    assert sa == 2 * 40 * 6000 and sb == 2 * 20 * 6000 and sb * 2 == sa


# ------------------------------------------------------- full-size samples ---

def _sample_cells(rng, N, mask=None, k=3000, extra=None):
    cells = rng.choice(N, size=k, replace=False)
    if extra is not None:
        cells = np.concatenate([cells, extra])
    cells = np.unique(cells)
    if mask is not None:
        cells = cells[mask.ravel()[cells] == 0]
    return cells


def _plan_edge_cells(n, rows):
    """Cells of an n^3 grid on the fluid pass's work boundaries: the first and
    last x and y of tiles, the first and last plane of every z segment and of
    the z tail, as the plan for n^3 with `rows`-row tiles (the height the
    context ran) lays them out."""
    import torch
    from paper_2602_05295_amd import homelbm
    plan = homelbm.fluid_plan((n, n, n), tile_rows=rows, cus=torch.cuda.get_device_properties(0).multi_processor_count)
    zt = n - plan["tail"]
    zs = set()
    for sg in range(plan["nseg"]):
        za, zb = zt * sg // plan["nseg"], zt * (sg + 1) // plan["nseg"]
        zs.update({za, zb - 1})
    if plan["tail"]:
        zs.update({zt, n - 1})
    xs = sorted({v for t in range(plan["ntx"]) for v in (64 * t, min(64 * t + 63, n - 1))})
    ys = sorted({v for t in range(plan["nty"]) for v in (plan["rows"] * t, min(plan["rows"] * (t + 1) - 1, n - 1))})
    rng = np.random.default_rng(7)
    z = np.array(sorted(zs))
    pts = [(x, y, zz) for zz in z for x, y in zip(rng.choice(xs, 24), rng.choice(ys, 24))]
    return np.array([x + n * (y + n * zz) for x, y, zz in pts])


def test_fp32_256cubed_sampled(H, orc):
    """The 256^3 decaying-turbulence configuration, one step, sampled cells
    (random ones and cells on the work split's tile, segment and tail
    boundaries)."""
    n = 256
    _note("fp32 256^3 sampled")
    u = W.random_solenoidal(n, n, n, 8.0, 0.1 / np.sqrt(3), seed=0).astype(np.float32)
    rho = np.ones((n, n, n), np.float32)
    with H.HomeLBM((n, n, n), 0.51) as s:
        s.set_equilibrium(rho, u)
        s.step(3)
        m0 = s.get_moments()
        s.step(1)
        got = s.get_moments()
        rows = s.tile_rows
    rng = np.random.default_rng(0)
    cells = _sample_cells(rng, n ** 3, extra=np.concatenate([np.array([0, n - 1, n * n - 1, n ** 3 - 1]),
                                                             _plan_edge_cells(n, rows)]))
    ref = orc.step_cells(_orc_params(orc, (n, n, n), 0.51), m0.astype(np.float64), cells)
    g = got.reshape(10, -1)[:, cells]
    err = group_rel_err(g, ref.T)
    assert max(err.values()) <= TOL32, err


def test_q16_256cubed_sampled(H, orc):
    """The headline configuration: 256^3 decaying turbulence in 16-bit
    moments with dither per step, as the benchmark runs it (same launch
    plan), one step; sampled codes within one code of the oracle's and at
    most 1% off by one."""
    n = 256
    _note("q16 256^3 sampled")
    u = W.random_solenoidal(n, n, n, 8.0, 0.1 / np.sqrt(3), seed=0).astype(np.float32)
    rho = np.ones((n, n, n), np.float32)
    with H.HomeLBM((n, n, n), 0.51, fmt="q16") as s:
        s.set_options(dither_mode=1, seed=0)
        s.set_equilibrium(rho, u)
        s.step(3)
        w0 = s.get_raw()
        t0 = s.step_count
        s.step(1)
        got = s.get_raw()
        rows = s.tile_rows
    rng = np.random.default_rng(2)
    cells = _sample_cells(rng, n ** 3, extra=np.concatenate([np.array([0, n - 1, n * n - 1, n ** 3 - 1]),
                                                             _plan_edge_cells(n, rows)]))
    ref = orc.q16_step_cells(_orc_params(orc, (n, n, n), 0.51), w0, cells, None, t=t0, seed=0, mode=1)
    g = got.reshape(5, -1)[:, cells]
    d = np.abs(unpack(g) - unpack(ref.T))
    assert d.max() <= 1, d.max()
    assert (d > 0).mean() < 0.01, (d > 0).mean()


def test_q16_channel_sampled(H, orc):
    """The 1000x400x400 obstacle channel in Q16, one step, sampled cells
    including boundary cells, and sampled solid cells."""
    nx, ny, nz = 1000, 400, 400
    _note("q16 channel 1000x400x400 sampled")
    mask = W.channel_mask(nx, ny, nz, seed=0)
    u = np.zeros((3, nz, ny, nx), np.float32)
    u[0] = 0.08
    u[:, mask == 1] = 0
    rho = np.ones((nz, ny, nx), np.float32)
    with H.HomeLBM((nx, ny, nz), 0.52, mask=mask, fmt="q16") as s:
        s.set_options(dither_mode=1, seed=3, inflow=True, u_in=(0.08, 0, 0))
        s.set_equilibrium(rho, u)
        s.step(2)
        w0 = s.get_raw()
        t0 = s.step_count
        s.step(1)
        got = s.get_raw()
    rng = np.random.default_rng(1)
    # boundary cells: fluid neighbours of solids, and the two open faces
    solid_idx = np.flatnonzero(mask.ravel())
    near = rng.choice(solid_idx, 2000) + rng.choice([-1, 1, -nx, nx], 2000)
    faces = np.concatenate([rng.integers(0, ny * nz, 300) * nx, rng.integers(0, ny * nz, 300) * nx + nx - 1])
    cells = _sample_cells(rng, nx * ny * nz, mask, k=3000, extra=np.concatenate([near % (nx * ny * nz), faces]))
    P = _orc_params(orc, (nx, ny, nz), 0.52, True, (0.08, 0, 0))
    ref = orc.q16_step_cells(P, w0, cells, mask, t=t0, seed=3, mode=1)
    g = got.reshape(5, -1)[:, cells].T
    d = np.abs(unpack(g.T) - unpack(ref.T))
    assert d.max() <= 1, d.max()
    assert (d > 0).mean() < 0.01, (d > 0).mean()
    # solid cells, interior ones included, hold the oracle's rest codes
    sol = np.unique(rng.choice(solid_idx, 2000))
    ref_s = orc.q16_step_cells(P, w0, sol, mask, t=t0, seed=3, mode=1)
    assert np.array_equal(got.reshape(5, -1)[:, sol].T, ref_s)


# ------------------------------------------------------------- interfaces ---

def test_dither_known_answers(H, orc):
    _note("dither KAT")
    rng = np.random.default_rng(5)
    idx = rng.integers(0, 2**32, 500, dtype=np.uint64).astype(np.uint32)
    for t, seed, mode in [(0, 0, 1), (17, 99, 1), (5, 7, 2), (6, 7, 2)]:
        dev = H.debug_dither(idx, t, seed, mode)
        for k in range(0, 500, 25):
            _, h = orc.dither(int(idx[k]), t, seed, mode)
            assert (int(dev[k, 0]), int(dev[k, 1])) == h


def test_set_get_roundtrip(H, orc):
    _note("set/get")
    dims = (13, 7, 5)
    m = W.random_moments(*dims, seed=2).astype(np.float32)
    with H.HomeLBM(dims, 0.6) as s:
        s.set_moments(m)
        assert np.array_equal(s.get_moments(), m)
    with H.HomeLBM(dims, 0.6, fmt="q16") as s:
        s.set_moments(m)
        codes = unpack(s.get_raw())
    ref = unpack(orc.q16_encode(m.astype(np.float64)))
    assert np.abs(codes - ref).max() <= 1 and (codes != ref).mean() < 0.01


def test_invalid_arguments(H):
    _note("invalid args")
    with pytest.raises(H.LBMError) as e:
        H.HomeLBM((0, 4, 4), 0.6)
    assert e.value.status == H.ERR_INVALID_ARG
    with pytest.raises(H.LBMError):
        H.HomeLBM((4, 4, 4), 0.5)
    ids = np.zeros(64, np.uint8)
    ids[21] = 2  # mask values 1..255 name solid objects
    with H.HomeLBM((4, 4, 4), 0.6, mask=ids) as s:
        assert s.boundary_counts()[1] == 1
    with pytest.raises(H.LBMError):
        H.HomeLBM((1 << 11, 1 << 10, 1 << 10), 0.6)
    mask = np.zeros((4, 4, 10), np.uint8)
    mask[:, :, 1] = 1
    with H.HomeLBM((10, 4, 4), 0.6, mask=mask) as s:
        with pytest.raises(H.LBMError):
            s.set_options(inflow=True, u_in=(0.05, 0, 0))
        with pytest.raises(H.LBMError):
            s.step(-1)


def test_health_check_flags_nan_and_saturation(H):
    _note("health")
    dims = (8, 8, 8)
    m = W.random_moments(*dims, seed=1).astype(np.float32)
    m[1, 3, 3, 3] = np.nan
    with H.HomeLBM(dims, 0.6) as s:
        s.set_moments(m)
        with pytest.raises(H.LBMError) as e:
            s.step(1)
        assert e.value.status == H.ERR_UNSTABLE
    m = W.random_moments(*dims, seed=1).astype(np.float32)
    m[1] = 0.6 * m[0]  # u = 0.6 is outside the [-0.4, 0.4] code range
    with H.HomeLBM(dims, 0.6, fmt="q16") as s:
        s.set_moments(m)
        assert s.check() > 0


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_set_raw_puts_listed_solid_cells_back_at_rest(H, fmt):
    """The boundary pass relies on solid cells next to fluid holding the rest
    state; a raw state with anything else there must give the same step."""
    dims = (26, 19, 14)
    _note("set_raw solid rest", fmt)
    mask = W.sphere_mask(*dims, phi=0.1, rmin=1.5, rmax=3.5, seed=9)
    m = W.random_moments(*dims, seed=12, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, 0.6, mask=mask, fmt=fmt) as s:
        s.set_options(dither_mode=1, seed=5)
        s.set_moments(m)
        raw = s.get_raw().copy()
        s.step(2)
        ref = s.get_raw().copy()
    bad = raw.copy()
    rng = np.random.default_rng(1)
    noise = rng.integers(0, 2**32, size=bad.shape, dtype=np.uint64).astype(np.uint32)
    if fmt == "fp32":
        bad[:, mask == 1] = rng.standard_normal((10, int(mask.sum()))).astype(np.float32)
    else:
        bad[:, mask == 1] = noise[:, mask == 1]
    with H.HomeLBM(dims, 0.6, mask=mask, fmt=fmt) as s:
        s.set_options(dither_mode=1, seed=5)
        s.set_raw(bad)
        s.step(2)
        got = s.get_raw()
    fl = mask == 0
    assert np.array_equal(got[:, fl], ref[:, fl])



@pytest.mark.parametrize("fmt", ["fp32", "q16"])
@pytest.mark.parametrize("inflow", [False, True])
def test_step_into_matches_step(H, fmt, inflow):
    """lbm_step_into from a raw state gives the same state as lbm_step from
    it (same dither, same boundary handling), and leaves the context's own
    state and the input buffer alone."""
    import torch
    dims = (70, 23, 11)
    _note("step_into", fmt, "inflow", inflow)
    mask = W.sphere_mask(*dims, phi=0.08, rmin=1.5, rmax=3.0, seed=21)
    if inflow:
        mask = _faces_clear(mask)
    m = W.random_moments(*dims, seed=4, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, 0.58, mask=mask, fmt=fmt) as s:
        s.set_options(dither_mode=1, seed=3, inflow=inflow, u_in=(0.05, 0.0, 0.01))
        s.set_moments(m)
        s.step(2)
        t = s.step_count
        raw0 = s.get_raw().copy()
        s.step(3)
        want = s.get_raw().copy()
        tt = torch.float32 if fmt == "fp32" else torch.int32
        a = torch.from_numpy(raw0.view(np.float32 if fmt == "fp32" else np.int32)).cuda()
        b, c = torch.empty_like(a), torch.empty_like(a)
        assert a.dtype == tt
        s.step_count = t
        s.step_into(a, b)
        s.step_into(b, c)
        s.step_into(c, b)
        assert s.step_count == t + 3
        own = s.get_raw()
        torch.cuda.synchronize()
        got = b.cpu().numpy().view(want.dtype)
        assert np.array_equal(got, want)
        assert np.array_equal(a.cpu().numpy().view(raw0.dtype), raw0)
        assert np.array_equal(own, want)  # the context's own state: still the state after its 5 steps
        with pytest.raises(H.LBMError):
            s.step_into(a, a)



# ------------------------------------------------------------ body force ---
# App. A with a uniform force F (the stored momentum holds F/2, Eq.
# rho_u_stress).  The oracle applies App. A's printed formulas literally; the
# kernels use their non-equilibrium form.

FORCE = (2e-3, -1e-3, 5e-4)


def _force_mask(dims, case, seed):
    if case == "periodic":
        return None, False
    mask = W.sphere_mask(*dims, phi=0.08, rmin=1.5, rmax=3.0, seed=seed)
    if case == "faces":
        return _faces_clear(mask), True
    return mask, False


@pytest.mark.parametrize("case", ["periodic", "solids", "faces"])
def test_fp32_body_force_steps(H, orc, case):
    dims = (26, 19, 13)
    _note("fp32 body force", case)
    mask, inflow = _force_mask(dims, case, 5)
    m = W.random_moments(*dims, seed=3).astype(np.float32)
    u_in = (0.06, 0.01, -0.02)
    with H.HomeLBM(dims, 0.62, mask=mask) as s:
        s.set_options(inflow=inflow, u_in=u_in, force=FORCE)
        s.set_moments(m)
        m0 = s.get_moments()
        s.step(5)
        got = s.get_moments()
    P = _orc_params(orc, dims, 0.62, inflow, u_in, FORCE)
    ref = orc.run(P, m0.astype(np.float64), 5, mask)
    err = group_rel_err(got, ref)
    assert max(err.values()) <= TOL32, err
    # the force is not a no-op at this tolerance
    ref0 = orc.run(_orc_params(orc, dims, 0.62, inflow, u_in), m0.astype(np.float64), 5, mask)
    assert max(group_rel_err(ref0, ref).values()) > 100 * TOL32


@pytest.mark.parametrize("case", ["periodic", "solids", "faces"])
def test_q16_body_force_one_step_codes(H, orc, case):
    dims = (30, 21, 11)
    _note("q16 body force", case)
    mask, inflow = _force_mask(dims, case, 6)
    got, ref = _q16_step_compare(H, orc, dims, 0.6, mask=mask, inflow=inflow, F=FORCE)
    fl = np.ones(dims[::-1], bool) if mask is None else (mask == 0)
    d = np.abs(unpack(got) - unpack(ref))[:, fl]
    assert d.max() <= 1, d.max()
    assert (d > 0).mean() < 0.01, (d > 0).mean()


def test_body_force_rejected_where_unsupported(H):
    with H.HomeLBM((8, 8, 8), 0.6) as s:
        with pytest.raises(H.LBMError):
            s.set_options(force=(0.02, 0.0, 0.0))  # |F_a| > 0.01
        with pytest.raises(H.LBMError):
            s.set_options(force=(float("nan"), 0.0, 0.0))
        import torch
        s.set_options(force=(1e-3, 0.0, 0.0))
        m = torch.zeros((10, 8, 8, 8), device="cuda")
        with pytest.raises(H.LBMError):
            s.adjoint_step(m, m.clone(), m.clone())


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_poiseuille_with_body_force(H, orc, fmt):
    """Force-driven channel between halfway bounce-back walls at y = 1/2 and
    y = W + 1/2: the steady profile is u(y) = F/(2 rho nu) (y - 1/2)(W + 1/2 - y)
    to within 2% (relative L2), and the FP32 run lands on the oracle's
    steady state."""
    Wd, F, tau = 16, 1e-5, 0.8
    nx = nz = 4
    ny = Wd + 2
    dims = (nx, ny, nz)
    _note("poiseuille", fmt)
    nu = (tau - 0.5) / 3
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, Wd + 1, :] = 1
    y = np.arange(ny)
    prof = F / (2 * nu) * (y - 0.5) * (Wd + 0.5 - y)
    prof[0] = prof[-1] = 0
    u = np.zeros((3, nz, ny, nx), np.float32)
    u[0] = prof[None, :, None]
    rho = np.ones((nz, ny, nx), np.float32)
    steps = 3000
    with H.HomeLBM(dims, tau, mask=mask, fmt=fmt) as s:
        s.set_options(force=(F, 0.0, 0.0))
        s.set_equilibrium(rho, u)
        m0 = s.get_moments()
        s.step(steps)
        m = s.get_moments()
    ux = (m[1] / m[0])[:, 1:Wd + 1, :]
    ref = prof[1:Wd + 1][None, :, None]
    rel = np.linalg.norm((ux - ref).ravel()) / (np.linalg.norm(ref) * np.sqrt(nx * nz))
    assert rel < 0.02, rel
    if fmt == "fp32":
        mo = orc.run(orc.make_params(dims, tau, F=(F, 0, 0)), m0.astype(np.float64), steps, mask)
        uo = (mo[1] / mo[0])[:, 1:Wd + 1, :]
        assert np.abs(ux - uo).max() <= 1e-4 * np.abs(uo).max()
