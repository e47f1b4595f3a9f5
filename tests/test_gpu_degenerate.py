"""The method's degenerate cases against the FP64 oracle: a domain with no
fluid at all, a single fluid cell walled in on all 26 sides, relaxation
times near 1/2 and large, and 16-bit states at the edges of the codec's
ranges (some codes saturated).  Bars as in the fixed parity tests:
FP32 within 1e-5 per moment group, 16-bit codes within one code of the
oracle's with almost all equal."""
import numpy as np
import pytest

from helpers import group_rel_err, unpack
from paper_2602_05295_amd import workloads as W

pytestmark = pytest.mark.gpu


def _note(*a):
    print("CASE", *a, flush=True)


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_all_solid_domain_stays_at_rest(orc, fmt):
    from paper_2602_05295_amd import homelbm as H
    dims = (20, 9, 7)
    _note("all solid", fmt)
    mask = np.ones(dims[::-1], np.uint8)
    m = W.random_moments(*dims, seed=1, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, 0.6, mask=mask, fmt=fmt) as s:
        s.set_moments(m)
        s.step(3)
        got = s.get_moments()
        assert s.boundary_counts()[0] == 0
        with pytest.raises(H.LBMError):  # open faces need fluid next to both faces
            s.set_options(inflow=True, u_in=(0.05, 0.0, 0.0))
    ref = orc.run(orc.make_params(dims, 0.6), m.astype(np.float64), 3, mask)
    np.testing.assert_array_equal(ref[0], 1.0)
    np.testing.assert_array_equal(ref[1:], 0.0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=0)


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_single_fluid_cell_walled_in(orc, fmt):
    """Every one of the cell's 26 links meets a wall: its new state is its own
    post-collision populations sent back."""
    from paper_2602_05295_amd import homelbm as H
    dims = (7, 6, 5)
    _note("single fluid cell", fmt)
    mask = np.ones(dims[::-1], np.uint8)
    mask[2, 3, 3] = 0
    m = W.random_moments(*dims, seed=2, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, 0.7, mask=mask, fmt=fmt) as s:
        s.set_options(dither_mode=1, seed=3)
        s.set_moments(m)
        assert s.boundary_counts()[0] == 1
        if fmt == "fp32":
            m0 = s.get_moments().astype(np.float64)
            s.step(4)
            err = group_rel_err(s.get_moments(), orc.run(orc.make_params(dims, 0.7), m0, 4, mask))
            assert max(err.values()) <= 1e-5, err
        else:
            for t in range(4):
                s.step_count = t
                w0 = s.get_raw().copy()
                s.step(1)
                ref = orc.q16_step(orc.make_params(dims, 0.7), w0, mask, t=t, seed=3, mode=1)
                d = np.abs(unpack(s.get_raw()) - unpack(ref))[:, 2, 3, 3]
                assert d.max() <= 1, (t, d)


@pytest.mark.parametrize("tau", [0.5001, 0.505, 2.0, 20.0])
def test_fp32_relaxation_time_extremes(orc, tau):
    from paper_2602_05295_amd import homelbm as H
    dims = (41, 13, 9)
    _note("fp32 tau", tau)
    mask = W.sphere_mask(*dims, phi=0.06, rmin=1.5, rmax=2.5, seed=4)
    m = W.random_moments(*dims, seed=5, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, tau, mask=mask) as s:
        s.set_moments(m)
        m0 = s.get_moments().astype(np.float64)
        s.step(2)
        got = s.get_moments()
    err = group_rel_err(got, orc.run(orc.make_params(dims, tau), m0, 2, mask))
    assert max(err.values()) <= 1e-5, err


@pytest.mark.parametrize("edge", ["fast", "dense", "rare"])
def test_q16_at_the_codec_range_edges(orc, edge):
    """States at and past the ends of the codec's ranges (speed near 0.4,
    density near either end), so that some codes sit saturated at 0 or
    65535: one step from them, as on the oracle."""
    from paper_2602_05295_amd import homelbm as H
    dims = (33, 11, 7)
    _note("q16 range edge", edge)
    rng = np.random.default_rng(6)
    shape = dims[::-1]
    rho = np.ones(shape) + rng.uniform(-0.01, 0.01, shape)
    u = rng.uniform(-0.02, 0.02, (3,) + shape)
    if edge == "fast":
        u[0] += 0.385
        u[1] -= 0.385
    elif edge == "dense":
        rho += 0.495  # the codec's density range is [0.8, 1.5] (Sec. 5.3)
    else:
        rho -= 0.195
    with H.HomeLBM(dims, 0.6, fmt="q16") as s:
        s.set_options(dither_mode=1, seed=8, check_health=False)
        s.set_equilibrium(rho.astype(np.float32), u.astype(np.float32))
        s.step_count = 2
        w0 = s.get_raw().copy()
        s.step(1)
        got = s.get_raw()
    ref = orc.q16_step(orc.make_params(dims, 0.6), w0, None, t=2, seed=8, mode=1)
    k = {"fast": 1, "dense": 0, "rare": 0}[edge]  # the saturated code: u_x, or rho
    assert np.any(unpack(w0)[k] == (0 if edge == "rare" else 65535))
    d = np.abs(unpack(got) - unpack(ref))
    assert d.max() <= 1, d.max()
    assert (d > 0).mean() < 0.01, (d > 0).mean()
