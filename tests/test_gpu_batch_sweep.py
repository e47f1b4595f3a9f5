"""Seeded sweep of batches against the FP64 oracle.

Each case draws a batch of 1-12 domains from a generator seeded by the case
number: ragged shapes from single cells to strips wider than a wavefront,
spheres or none per domain, a relaxation time per domain, the storage format,
the strip kernel's block size (among those wide enough), the dither mode and
the step count.  Every domain must match the oracle to the bars of the fixed batch tests: FP32
within 1e-5 per moment group of the oracle's run; 16-bit codes, stepped one
step at a time from the device's own codes, within one code of the oracle's
step on every fluid cell with almost all codes equal.
"""
import numpy as np
import pytest

from helpers import group_rel_err, unpack
from paper_2602_05295_amd import workloads as W

CASES = 24


@pytest.fixture(scope="module")
def H():
    from paper_2602_05295_amd import homelbm
    homelbm.lib()
    return homelbm


def draw(case):
    """The configuration of one batch (host-side choices only)."""
    rng = np.random.default_rng(5000 + case)
    dims, masks, taus = [], [], []
    total = 0
    for k in range(int(rng.integers(1, 13))):
        nx, ny, nz = int(rng.integers(1, 101)), int(rng.integers(1, 41)), int(rng.integers(1, 17))
        if total + nx * ny * nz > 80000:
            break
        total += nx * ny * nz
        d = (nx, ny, nz)
        dims.append(d)
        taus.append(float(rng.uniform(0.52, 0.9)))
        mask = None
        if min(d) >= 6 and rng.integers(0, 2):
            mask = W.sphere_mask(*d, phi=0.06, rmin=1.5, rmax=2.5, seed=100 * case + k)
            if not mask.any():
                mask = None
        masks.append(mask)
    # a workgroup of B threads takes domains at most B / 3 cells wide
    blocks = [b for b in (256, 512, 1024) if max(d[0] for d in dims) <= b // 3]
    return dict(dims=dims, masks=masks, taus=taus, fmt="fp32" if case % 2 == 0 else "q16",
                block=int(rng.choice(blocks)), mode=int(rng.integers(0, 3)),
                seed=int(rng.integers(0, 2 ** 31)), t0=int(rng.integers(0, 1000)), steps=int(rng.integers(1, 3)))


def test_the_batch_sweep_spans_the_configurations():
    cs = [draw(k) for k in range(CASES)]
    assert all(len(c["dims"]) >= 1 for c in cs) and max(len(c["dims"]) for c in cs) >= 8
    assert any(len(c["dims"]) == 1 for c in cs) or min(len(c["dims"]) for c in cs) <= 3
    assert {c["block"] for c in cs} == {256, 512, 1024}
    doms = [(d, m) for c in cs for d, m in zip(c["dims"], c["masks"])]
    assert any(m is not None for _, m in doms) and any(m is None for _, m in doms)
    assert any(d[0] > 64 for d, _ in doms) and any(d[0] < 8 for d, _ in doms)
    assert any(d[1] < 4 for d, _ in doms) and any(d[2] < 3 for d, _ in doms)


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(CASES))
def test_batch_sweep_case(H, orc, case):
    c = draw(case)
    dims, masks, taus, fmt = c["dims"], c["masks"], c["taus"], c["fmt"]
    print("CASE batch sweep", case, fmt, "block", c["block"], "mode", c["mode"], "steps", c["steps"],
          [(d, m is not None) for d, m in zip(dims, masks)], flush=True)
    with H.HomeLBMBatch(dims, taus, masks, fmt=fmt) as b:
        b.set_options(dither_mode=c["mode"], seed=c["seed"])
        b.set_tuning(c["block"], 1)
        for k, d in enumerate(dims):
            b.set_moments(k, W.random_moments(*d, seed=7 * case + k, dj=0.02, dp=0.003).astype(np.float32))
        if fmt == "fp32":
            m0 = [b.get_moments(k).astype(np.float64) for k in range(len(dims))]
            b.step(c["steps"])
            for k, d in enumerate(dims):
                ref = orc.run(orc.make_params(d, taus[k]), m0[k], c["steps"], masks[k])
                err = group_rel_err(b.get_moments(k), ref)
                assert max(err.values()) <= 1e-5, (k, d, err)
            return
        b.step_count = c["t0"]
        for s in range(c["steps"]):
            w0 = [b.get_raw(k).copy() for k in range(len(dims))]
            b.step(1)
            for k, d in enumerate(dims):
                ref = orc.q16_step(orc.make_params(d, taus[k]), w0[k], masks[k], t=c["t0"] + s, seed=c["seed"],
                                   mode=c["mode"])
                diff = np.abs(unpack(b.get_raw(k)) - unpack(ref))
                if masks[k] is not None:
                    diff = diff[:, masks[k] == 0]
                assert diff.max() <= 1, (s, k, d, diff.max())
                assert (diff > 0).sum() <= max(3, 0.01 * diff.size), (s, k, d, (diff > 0).sum(), diff.size)


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(0, CASES, 3))
def test_batch_sweep_graphs_equal_eager(H, case):
    """The same batch stepped through its captured graphs and kernel by
    kernel: the same bits in every domain after each of three step calls."""
    c = draw(case)
    print("CASE batch sweep graphs", case, c["fmt"], "block", c["block"], len(c["dims"]), flush=True)
    out = {}
    for eager in (False, True):
        with H.HomeLBMBatch(c["dims"], c["taus"], c["masks"], fmt=c["fmt"]) as b:
            b.set_options(dither_mode=c["mode"], seed=c["seed"])
            b.set_tuning(c["block"], 1)
            for k, d in enumerate(c["dims"]):
                b.set_moments(k, W.random_moments(*d, seed=7 * case + k, dj=0.02, dp=0.003).astype(np.float32))
            states = []
            for n in (1, 9, 4):
                (b.step_eager if eager else b.step)(n)
                states.append([b.get_raw(k).copy() for k in range(len(c["dims"]))])
            out[eager] = states
    for s, (g, e) in enumerate(zip(out[False], out[True])):
        for k in range(len(c["dims"])):
            assert np.array_equal(g[k], e[k]), (case, s, k)


@pytest.mark.gpu
@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_batch_of_many_tiny_domains(H, orc, fmt):
    """3000 domains of 1..6 cells a side, many to a workgroup and packed
    across wavefront boundaries, spheres in some: every domain against the
    oracle after one step (16-bit from identical codes)."""
    rng = np.random.default_rng(21)
    dims = [tuple(int(v) for v in rng.integers(1, 7, 3)) for _ in range(3000)]
    taus = [float(v) for v in rng.uniform(0.52, 0.9, len(dims))]
    masks = []
    for k, d in enumerate(dims):
        mk = None
        if min(d) >= 4 and k % 3 == 0:
            mk = W.sphere_mask(*d, phi=0.1, rmin=0.8, rmax=1.5, seed=k)
            if not mk.any() or mk.all():
                mk = None
        masks.append(mk)
    print("CASE batch many tiny domains", fmt, len(dims), sum(m is not None for m in masks), flush=True)
    with H.HomeLBMBatch(dims, taus, masks, fmt=fmt) as b:
        b.set_options(dither_mode=1, seed=5)
        for k, d in enumerate(dims):
            b.set_moments(k, W.random_moments(*d, seed=k, dj=0.02, dp=0.003).astype(np.float32))
        b.step_count = 3
        before = [(b.get_moments(k) if fmt == "fp32" else b.get_raw(k)).copy() for k in range(len(dims))]
        b.step(1)
        for k, d in enumerate(dims):
            P = orc.make_params(d, taus[k])
            if fmt == "fp32":
                err = group_rel_err(b.get_moments(k), orc.step(P, before[k].astype(np.float64), masks[k]))
                assert max(err.values()) <= 1e-5, (k, d, err)
            else:
                ref = orc.q16_step(P, before[k], masks[k], t=3, seed=5, mode=1)
                diff = np.abs(unpack(b.get_raw(k)) - unpack(ref))
                if masks[k] is not None:
                    diff = diff[:, masks[k] == 0]
                assert diff.max() <= 1, (k, d, diff.max())
