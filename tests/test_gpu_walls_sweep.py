"""Seeded sweep of the solid coupling with moving objects against the FP64
oracle (readings R16, R17).

Each case draws its domain shape, storage format, wall rule (bounce-back or
the moment wall at the link midpoint), open x faces or periodic x, body
force, the objects (ids, centers, velocities, angular velocities) and the
step count from a generator seeded by the case number.  Bars as in the fixed
wall tests: FP32 within 1e-5 per moment group of the oracle's run, and the
first step's force and torque on every object within 1e-4 of the oracle's
momentum exchange where forces are tracked; 16-bit codes, one step at a time
from the device's codes, within one code of the oracle's step on every fluid
cell with almost all codes equal.
"""
import numpy as np
import pytest

from helpers import group_rel_err, unpack
from paper_2602_05295_amd import workloads as W

CASES = 24


def draw(case):
    """The configuration of one case (host-side choices only)."""
    rng = np.random.default_rng(7000 + case)
    while True:
        d = (int(rng.integers(6, 91)), int(rng.integers(6, 29)), int(rng.integers(6, 19)))
        if d[0] * d[1] * d[2] <= 30000:
            break
    inflow = d[0] >= 8 and bool(rng.integers(0, 2))
    mask = W.sphere_mask(*d, phi=0.08, rmin=1.5, rmax=3.0, seed=case)
    if inflow:
        mask[:, :, :3] = 0  # solids stay clear of the open faces
        mask[:, :, -3:] = 0
    # the solid cells split into three objects by x position
    idv = [int(v) for v in rng.choice(np.arange(1, 256), 3, replace=False)]
    xs = np.broadcast_to(np.arange(d[0])[None, None, :], mask.shape)
    ids = np.zeros_like(mask)
    for k, (lo, hi) in enumerate(((0, d[0] // 3), (d[0] // 3, 2 * d[0] // 3), (2 * d[0] // 3, d[0]))):
        ids[(mask > 0) & (xs >= lo) & (xs < hi)] = idv[k]
    obj = np.zeros((256, 9))
    for k in idv:
        obj[k, :3] = rng.uniform(0, min(d), 3)
        obj[k, 3:6] = rng.uniform(-0.03, 0.03, 3)
        obj[k, 6:9] = rng.uniform(-0.003, 0.003, 3)
    fmt = "fp32" if case % 2 == 0 else "q16"
    F = tuple(float(v) for v in rng.uniform(-5e-4, 5e-4, 3)) if rng.integers(0, 2) else (0.0, 0.0, 0.0)
    rule = int(rng.integers(0, 2))
    track = fmt == "fp32" and not inflow  # forces are tracked without a body force
    if track:
        F = (0.0, 0.0, 0.0)
    return dict(dims=d, ids=ids, idv=idv, obj=obj, fmt=fmt, inflow=inflow, F=F, rule=rule, track=track,
                tau=float(rng.uniform(0.55, 0.9)), steps=int(rng.integers(1, 4)),
                u_in=tuple(float(v) for v in rng.uniform(-0.05, 0.05, 3)), seed=int(rng.integers(0, 2 ** 31)),
                t0=int(rng.integers(0, 1000)))


def test_the_walls_sweep_spans_the_configurations():
    cs = [draw(k) for k in range(CASES)]
    assert {c["rule"] for c in cs} == {0, 1} and {c["fmt"] for c in cs} == {"fp32", "q16"}
    assert any(c["inflow"] for c in cs) and any(not c["inflow"] for c in cs)
    assert any(c["F"] != (0.0, 0.0, 0.0) for c in cs) and any(c["track"] for c in cs)
    assert any(c["rule"] == 1 and c["inflow"] for c in cs)
    assert all(len(set(c["idv"])) == 3 for c in cs)


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(CASES))
def test_walls_sweep_case(orc, case):
    from paper_2602_05295_amd import homelbm as H
    c = draw(case)
    dims, ids, obj, fmt = c["dims"], c["ids"], c["obj"], c["fmt"]
    print("CASE walls sweep", case, dims, fmt, "rule", c["rule"], "inflow", c["inflow"], "F", c["F"],
          "track", c["track"], "steps", c["steps"], flush=True)
    P = orc.make_params(dims, c["tau"], F=c["F"], inflow=c["inflow"], u_in=c["u_in"], wall_rule=c["rule"],
                        objects=obj)
    m = W.random_moments(*dims, seed=case, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, c["tau"], mask=ids, fmt=fmt) as s:
        s.set_options(inflow=c["inflow"], u_in=c["u_in"], force=c["F"], wall_rule=c["rule"],
                      track_forces=c["track"], dither_mode=1, seed=c["seed"])
        for k in c["idv"]:
            s.set_object(k, obj[k, :3], obj[k, 3:6], obj[k, 6:9])
        s.set_moments(m)
        if fmt == "fp32":
            m0 = s.get_moments().astype(np.float64)
            s.step(1)
            if c["track"]:
                got = s.object_forces()
                ref = orc.object_forces(P, m0, ids)
                for k in c["idv"]:
                    for part in (slice(0, 3), slice(3, 6)):
                        den = np.abs(ref[k, part]).max()
                        assert np.abs(got[k, part] - ref[k, part]).max() <= 1e-4 * max(den, 1e-12), (k, part)
            s.step(c["steps"] - 1)
            err = group_rel_err(s.get_moments(), orc.run(P, m0, c["steps"], ids))
            assert max(err.values()) <= 1e-5, err
            return
        s.step_count = c["t0"]
        fl = ids == 0
        for k in range(c["steps"]):
            w0 = s.get_raw().copy()
            s.step(1)
            ref = orc.q16_step(P, w0, ids, t=c["t0"] + k, seed=c["seed"], mode=1)
            d = np.abs(unpack(s.get_raw()) - unpack(ref))[:, fl]
            assert d.max() <= 1, (k, d.max())
            assert (d > 0).sum() <= max(3, 0.01 * d.size), (k, (d > 0).sum(), d.size)
