"""Seeded sweep of step configurations against the FP64 oracle.

Each case draws its own domain shape (ragged in every direction, down to one
cell), storage format, solid mask, open x faces, body force, tile height,
dither mode and step count from a generator seeded by the case number, so the
sweep reaches combinations no hand-written case names.  The bars are those of
the fixed parity tests: FP32 storage within 1e-5 per moment group of the
oracle's run; integer storage, stepped one step at a time from the device's
own codes, within one code of the oracle's step on every fluid cell with
almost all codes equal.
"""
import numpy as np
import pytest

from helpers import group_rel_err, unpack, unpack_packed
from paper_2602_05295_amd import workloads as W

TOL32 = 1e-5
CASES = 96
FMTS = ["fp32", "q16", "p16_15", "p15_14", "p14_13", "p13_12", "p12_11"]


@pytest.fixture(scope="module")
def H():
    from paper_2602_05295_amd import homelbm
    homelbm.lib()
    return homelbm


def draw(case):
    """The configuration of one case (host-side choices only)."""
    rng = np.random.default_rng(1000 + case)
    while True:
        nx = int(rng.integers(1, 141))
        ny = int(rng.integers(1, 41))
        nz = int(rng.integers(1, 25))
        if nx * ny * nz <= 60000:
            break
    dims = (nx, ny, nz)
    fmt = FMTS[0] if case % 3 == 0 else ("q16" if case % 3 == 1 else FMTS[2 + int(rng.integers(0, 5))])
    inflow = nx >= 8 and bool(rng.integers(0, 2))
    masked = min(dims) >= 6 and bool(rng.integers(0, 2))
    mask = None
    if masked:
        mask = W.sphere_mask(*dims, phi=0.06, rmin=1.5, rmax=2.5, seed=case)
        if inflow:
            mask[:, :, :3] = 0  # solids stay clear of the open faces
            mask[:, :, -3:] = 0
        if not mask.any():
            mask = None
    F = tuple(float(v) for v in rng.uniform(-2e-5, 2e-5, 3)) if rng.integers(0, 2) else (0.0, 0.0, 0.0)
    return dict(dims=dims, fmt=fmt, inflow=inflow, mask=mask, F=F,
                tau=float(rng.uniform(0.52, 0.9)), rows=int(rng.choice([8, 10, 12, 13])),
                mode=int(rng.integers(0, 3)), seed=int(rng.integers(0, 2 ** 31)), t0=int(rng.integers(0, 1000)),
                steps=int(rng.integers(1, 4)), u_in=tuple(float(v) for v in rng.uniform(-0.05, 0.05, 3)))


def test_the_sweep_spans_the_configurations():
    """The drawn cases cover every format family, both face kinds, masks,
    body forces, every tile height and shapes below one tile in each direction."""
    cs = [draw(k) for k in range(CASES)]
    assert {c["fmt"] for c in cs} >= {"fp32", "q16"} and any(c["fmt"].startswith("p") for c in cs)
    assert any(c["inflow"] for c in cs) and any(not c["inflow"] for c in cs)
    assert any(c["mask"] is not None and c["inflow"] for c in cs)
    assert any(c["mask"] is not None and not c["inflow"] for c in cs)
    assert any(c["F"] != (0.0, 0.0, 0.0) for c in cs)
    assert {c["rows"] for c in cs} == {8, 10, 12, 13}
    assert any(c["dims"][0] < 64 for c in cs) and any(c["dims"][0] > 64 and c["dims"][0] % 64 for c in cs)
    assert any(c["dims"][1] < 8 for c in cs) and any(c["dims"][2] < 3 for c in cs)


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(CASES))
def test_sweep_case(H, orc, case):
    c = draw(case)
    dims, fmt, mask = c["dims"], c["fmt"], c["mask"]
    print("CASE sweep", case, dims, fmt, "mask", mask is not None, "inflow", c["inflow"], "F", c["F"],
          "rows", c["rows"], "mode", c["mode"], "steps", c["steps"], flush=True)
    P = orc.make_params(dims, c["tau"], F=c["F"], inflow=c["inflow"], u_in=c["u_in"])
    m = W.random_moments(*dims, seed=case, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, c["tau"], mask=mask, fmt=fmt) as s:
        s.set_options(tile_rows=c["rows"], dither_mode=c["mode"], seed=c["seed"], inflow=c["inflow"],
                      u_in=c["u_in"], force=c["F"])
        s.set_moments(m)
        if fmt == "fp32":
            m0 = s.get_moments().astype(np.float64)
            s.step(c["steps"])
            err = group_rel_err(s.get_moments(), orc.run(P, m0, c["steps"], mask))
            assert max(err.values()) <= TOL32, err
            return
        s.step_count = c["t0"]
        fl = np.ones(dims[::-1], bool) if mask is None else (mask == 0)
        for k in range(c["steps"]):
            w0 = s.get_raw().copy()
            s.step(1)
            got = s.get_raw()
            t = c["t0"] + k
            if fmt == "q16":
                ref = orc.q16_step(P, w0, mask, t=t, seed=c["seed"], mode=c["mode"])
                d = np.abs(unpack(got) - unpack(ref))[:, fl]
            else:
                b1, b2 = H.BITS[H.FORMATS[fmt]]
                ref = orc.qb_step(P, w0, b1, b2, mask, t=t, seed=c["seed"], mode=c["mode"])
                d = np.abs(unpack_packed(got, b1, b2) - unpack_packed(ref, b1, b2))[:, fl]
            assert d.max() <= 1, (k, d.max())
            assert (d > 0).sum() <= max(3, 0.01 * d.size), (k, (d > 0).sum(), d.size)
