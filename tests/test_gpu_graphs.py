"""Captured step sequences (lbm_options.graph_steps) against kernel-by-kernel
launches: the same raw state, bit for bit, after several lbm_step calls that
replay cached graphs (chunks of graph_steps steps, a remainder, single steps
launched eagerly), with the context's own eager work between the replays;
16-bit with per-step dither (each step's key from the device-side counter),
FP32, walls and open faces.  lbm_prepare captures ahead what a later
lbm_step replays and leaves the state and the step count alone."""
import numpy as np
import pytest

from paper_2602_05295_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(H, fmt, graph_steps, calls, prepare=()):
    dims = (40, 30, 24)
    mask = W.sphere_mask(*dims, phi=0.06, rmin=1.5, rmax=3.0, seed=3)
    mask[:, :, :3] = 0
    mask[:, :, -3:] = 0
    m = W.random_moments(*dims, seed=4, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, 0.56, mask=mask, fmt=fmt) as s:
        s.set_options(dither_mode=1, seed=9, inflow=True, u_in=(0.05, 0.0, 0.01), graph_steps=graph_steps)
        s.set_moments(m)
        before = s.get_raw().copy()
        for n in prepare:
            s.prepare(n)
        assert s.step_count == 0 and np.array_equal(s.get_raw(), before)
        states = []
        for n in calls:
            s.step(n)
            states.append(s.get_raw().copy())  # eager work between replays
        return states, s.step_count


@pytest.mark.parametrize("fmt", ["q16", "fp32"])
def test_graph_replay_equals_eager(fmt):
    from paper_2602_05295_amd import homelbm as H
    calls = [1, 300, 7, 7, 2, 1]
    print("CASE graph replay", fmt, calls, flush=True)
    ref, t_ref = _run(H, fmt, 0, calls)
    for g in (256, 5):
        got, t_got = _run(H, fmt, g, calls)
        assert t_got == t_ref
        for k, (a, b) in enumerate(zip(got, ref)):
            assert np.array_equal(a, b), (fmt, g, k)


@pytest.mark.parametrize("fmt", ["q16", "fp32"])
def test_prepared_sequences_equal_eager(fmt):
    from paper_2602_05295_amd import homelbm as H
    calls = [5, 20, 20, 300, 1]
    print("CASE prepared graphs", fmt, calls, flush=True)
    ref, t_ref = _run(H, fmt, 0, calls)
    got, t_got = _run(H, fmt, 256, calls, prepare=(5, 20, 300))
    assert t_got == t_ref
    for k, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(a, b), (fmt, k)
