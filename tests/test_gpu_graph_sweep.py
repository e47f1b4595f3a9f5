"""Seeded sweep of captured step sequences (lbm_options.graph_steps) against
kernel-by-kernel launches: the same raw state, bit for bit, after every one
of several lbm_step calls, with the context's own eager work (a state read)
between the replays.

Each case draws its domain shape, storage format, solids, open x faces,
body force, wall rule, dither mode, tile height, the chunk length of the
captured sequences and the lengths of the step calls from a generator
seeded by the case number.
"""
import numpy as np
import pytest

from paper_2602_05295_amd import workloads as W

CASES = 12
FMTS = ["fp32", "q16", "p16_15", "p13_12"]


def draw(case):
    """The configuration of one case (host-side choices only)."""
    rng = np.random.default_rng(13000 + case)
    while True:
        d = (int(rng.integers(6, 100)), int(rng.integers(1, 30)), int(rng.integers(1, 20)))
        if d[0] * d[1] * d[2] <= 40000:
            break
    inflow = d[0] >= 8 and bool(rng.integers(0, 2))
    mask = None
    if min(d) >= 6 and rng.integers(0, 2):
        mask = W.sphere_mask(*d, phi=0.06, rmin=1.5, rmax=2.5, seed=case)
        if inflow:
            mask[:, :, :3] = 0  # solids stay clear of the open faces
            mask[:, :, -3:] = 0
        if not mask.any():
            mask = None
    F = tuple(float(v) for v in rng.uniform(-2e-5, 2e-5, 3)) if rng.integers(0, 2) else (0.0, 0.0, 0.0)
    calls = [int(v) for v in rng.integers(1, 60, int(rng.integers(3, 7)))]
    return dict(dims=d, fmt=FMTS[case % len(FMTS)], inflow=inflow, mask=mask, F=F,
                rule=int(rng.integers(0, 2)) if mask is not None else 0, mode=int(rng.integers(0, 3)),
                rows=int(rng.choice([0, 8, 10, 12, 13])), chunk=int(rng.integers(2, 65)), calls=calls,
                tau=float(rng.uniform(0.52, 0.9)), seed=int(rng.integers(0, 2 ** 31)),
                u_in=tuple(float(v) for v in rng.uniform(-0.05, 0.05, 3)))


def test_the_graph_sweep_spans_the_configurations():
    cs = [draw(k) for k in range(CASES)]
    assert {c["fmt"] for c in cs} == set(FMTS)
    assert any(c["inflow"] for c in cs) and any(c["mask"] is not None for c in cs)
    assert any(c["rule"] == 1 for c in cs) and any(c["F"] != (0.0, 0.0, 0.0) for c in cs)
    # some calls are longer than a chunk, so a call replays whole chunks and a remainder
    assert any(max(c["calls"]) > c["chunk"] for c in cs)


def _run(H, c, chunk):
    with H.HomeLBM(c["dims"], c["tau"], mask=c["mask"], fmt=c["fmt"]) as s:
        s.set_options(dither_mode=c["mode"], seed=c["seed"], inflow=c["inflow"], u_in=c["u_in"], force=c["F"],
                      wall_rule=c["rule"], tile_rows=c["rows"], graph_steps=chunk)
        s.set_moments(W.random_moments(*c["dims"], seed=7, dj=0.02, dp=0.003).astype(np.float32))
        states = []
        for n in c["calls"]:
            s.step(n)
            states.append(s.get_raw().copy())
        return states, s.step_count


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(CASES))
def test_graph_sweep_case(case):
    from paper_2602_05295_amd import homelbm as H
    c = draw(case)
    print("CASE graph sweep", case, c["dims"], c["fmt"], "mask", c["mask"] is not None, "inflow", c["inflow"],
          "rule", c["rule"], "rows", c["rows"], "chunk", c["chunk"], "calls", c["calls"], flush=True)
    ref, t_ref = _run(H, c, 0)
    got, t_got = _run(H, c, c["chunk"])
    assert t_got == t_ref == sum(c["calls"])
    for k, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(a, b), (case, k)
