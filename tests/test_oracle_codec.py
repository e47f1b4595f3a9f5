"""Pins of the oracle's 16-bit codec (Sec. 5.3) and its dither generator.

Known answers follow from the printed formulas: q = floor(m' (2^b-1) + 1/2)
with m' = (m - min)/(max - min), so min -> 0, max -> 2^16 - 1, the midpoint
rounds half up, and decode(q) = min + q (max - min)/(2^b - 1).  The ranges
and bit width are the paper's printed constants (tests/golden/paper_codec.json).
The dither must be zero-mean and uniform on (-1/2, 1/2) LSB."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2602_05295_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper():
    with open(os.path.join(GOLD, "paper_codec.json")) as fh:
        return json.load(fh)


def test_ranges_match_paper(orc):
    p = _paper()
    assert list(orc.Q_LO[:1]) + list(orc.Q_HI[:1]) == p["rho_range"]["value"]
    assert np.all(orc.Q_LO[1:4] == p["u_range"]["value"][0]) and np.all(orc.Q_HI[1:4] == p["u_range"]["value"][1])
    assert np.all(orc.Q_LO[4:] == p["stress_neq_range"]["value"][0])
    assert np.all(orc.Q_HI[4:] == p["stress_neq_range"]["value"][1])
    full = p["stress_full_range"]["value"]
    red = p["stress_neq_range"]["value"]
    assert (full[1] - full[0]) / (red[1] - red[0]) > 3  # the reduction buys over 3x resolution
    assert p["bits"]["value"] == 16 and p["words_per_node"]["value"] == 5


@pytest.mark.parametrize("k", range(10))
def test_codec_known_answers(orc, k):
    lo, hi = orc.Q_LO[k], orc.Q_HI[k]
    assert orc.encode_one(lo, k) == 0
    assert orc.encode_one(hi, k) == 65535
    d = (hi - lo) / 65535
    # the range midpoint is the half-way value 32767.5 (+1/2): just above it
    # rounds up to 32768, just below it to 32767.
    mid = 0.5 * (lo + hi)
    assert orc.encode_one(mid + 0.05 * d, k) == 32768 and orc.encode_one(mid - 0.05 * d, k) == 32767
    assert orc.encode_one(hi + 1.0, k) == 65535 and orc.encode_one(lo - 1.0, k) == 0   # saturation
    assert orc.decode_one(0, k) == lo and abs(orc.decode_one(65535, k) - hi) < 1e-15
    for q in (1, 17, 4096, 32767, 65534):
        assert abs(orc.decode_one(q, k) - (lo + q * d)) < 1e-15
        # values a little above / below the half-way point between q and q+1
        assert orc.encode_one(lo + (q + 0.5 + 0.05) * d, k) == q + 1
        assert orc.encode_one(lo + (q + 0.5 - 0.05) * d, k) == q
        assert orc.encode_one(lo + (q + 0.05) * d, k) == q


def test_codec_round_trip_error_bounds(orc):
    rng = np.random.default_rng(0)
    for k in range(10):
        lo, hi = orc.Q_LO[k], orc.Q_HI[k]
        d = (hi - lo) / 65535
        for m in rng.uniform(lo, hi, 300):
            e = abs(orc.decode_one(orc.encode_one(m, k), k) - m)
            assert e <= 0.5 * d * (1 + 1e-9)
            xi = rng.uniform(-0.5, 0.5)
            e = abs(orc.decode_one(orc.encode_one(m, k, xi), k) - m)
            assert e < d * (1 + 1e-9)


def test_dither_values_are_zero_mean_uniform(orc):
    # every xi is (v + 1/2)/64 - 1/2 for a 6-bit v: the 64 levels average to 0 exactly
    levels = (np.arange(64) + 0.5) / 64 - 0.5
    assert levels.sum() == 0.0 and levels.min() > -0.5 and levels.max() < 0.5
    n = 20000
    xs = np.array([orc.dither(i, 3, 11, 1)[0] for i in range(n)])
    v = np.rint((xs + 0.5) * 64 - 0.5).astype(int)
    assert np.all(np.abs(((v + 0.5) / 64 - 0.5) - xs) < 1e-15)
    for k in range(10):
        counts = np.bincount(v[:, k], minlength=64)
        chi2 = ((counts - n / 64) ** 2 / (n / 64)).sum()
        assert chi2 < 140, (k, chi2)                           # 63 dof, p ~ 1e-7 bound
        assert abs(xs[:, k].mean()) < 4 * np.sqrt(1 / 12 / n)
    cc = np.corrcoef(xs.T)
    assert np.abs(cc - np.eye(10)).max() < 0.05


def test_dither_modes(orc):
    a, _ = orc.dither(100, 1, 5, 1)
    b, _ = orc.dither(100, 2, 5, 1)
    assert np.any(a != b)                                  # per-step dither changes with t
    a, _ = orc.dither(100, 1, 5, 2)
    b, _ = orc.dither(100, 2, 5, 2)
    assert np.all(a == b)                                  # static pattern does not
    z, _ = orc.dither(100, 1, 5, 0)
    assert np.all(z == 0)


def test_pcg_hash_is_a_permutation_with_avalanche(orc):
    xs = np.arange(1 << 16, dtype=np.uint64) * 65537 + 12345
    hs = {orc.pcg_hash(int(x) & 0xFFFFFFFF) for x in xs}
    assert len(hs) == xs.size
    rng = np.random.default_rng(1)
    flips = []
    for x in rng.integers(0, 2**32, 300):
        h0 = orc.pcg_hash(int(x))
        bit = int(rng.integers(0, 32))
        flips.append(bin(h0 ^ orc.pcg_hash(int(x) ^ (1 << bit))).count("1"))
    assert 14 < np.mean(flips) < 18


def test_oracle_known_answers_unchanged(orc):
    with open(os.path.join(GOLD, "oracle_kat.json")) as fh:
        kat = json.load(fh)
    for c in kat["dither"]:
        xi, h = orc.dither(c["idx"], c["t"], c["seed"], c["mode"])
        assert (h[0], h[1]) == (c["h1"], c["h2"])
        assert np.all(xi == np.array(c["xi"]))
    for v, h in kat["pcg_hash"].items():
        assert orc.pcg_hash(int(v)) == h
    for c in kat["encode"]:
        assert orc.encode_one(c["m"], c["k"], c["xi"]) == c["q"]


def test_field_codec_and_rest_fixed_point(orc):
    n = (6, 5, 4)
    P = orc.make_params(n, 0.6)
    rest = orc.equilibrium_moments(np.ones(n[::-1]), np.zeros((3,) + n[::-1]))
    w = orc.q16_encode(rest)
    # With symmetric ranges and 2^16 - 1 steps, zero sits at code 32767.5, so u
    # and N of the rest state decode to +Delta/2.  The decoded state is uniform,
    # so without dither every cell keeps the same codes, and rho and u (which
    # the collision conserves) keep their codes exactly.
    q0 = orc.unpack_codes(w)
    assert np.all(q0[1:4] == 32768) and np.all(q0[4:] == 32768)
    w1 = w
    for _ in range(3):
        w1 = orc.q16_step(P, w1, mode=0)
        q1 = orc.unpack_codes(w1)
        assert np.all(q1[:4] == q0[:4])
        assert np.all(q1 == q1[:, :1, :1, :1])
    m = orc.equilibrium_moments(*W.taylor_green_2d(6, 6, 4, 0.05)[:1], W.taylor_green_2d(6, 6, 4, 0.05)[1])
    P = orc.make_params((6, 6, 4), 0.6)
    w = orc.q16_encode(m)
    mhat = orc.q16_decode(w)
    ref = orc.step(P, mhat)                         # exact step of the decoded state
    for mode in (0, 1):
        got = orc.q16_decode(orc.q16_step(P, w, t=3, seed=1, mode=mode))
        # compare in codec variables: each within one quantization step
        for k, (a, b) in enumerate(zip(_codec_vars(got), _codec_vars(ref))):
            d = (orc.Q_HI[k] - orc.Q_LO[k]) / 65535
            lim = (0.5 if mode == 0 else 1.0) * d * (1 + 1e-3) + 4e-7 * np.abs(b).max()
            assert np.abs(a - b).max() <= lim, (mode, k)


def _codec_vars(m):
    rho = m[0]
    u = m[1:4] / rho
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    N = [m[4 + p] - rho * u[a] * u[b] for p, (a, b) in enumerate(pairs)]
    return [rho, *u, *N]


def test_q16_step_cells_matches_full(orc):
    n = (7, 5, 6)
    mask = W.sphere_mask(*n, phi=0.1, rmin=1.0, rmax=2.0, seed=2)
    m = W.random_moments(*n, seed=8)
    w = orc.q16_encode(m, mask)
    P = orc.make_params(n, 0.57)
    full = orc.q16_step(P, w, mask, t=11, seed=4, mode=1)
    cells = np.arange(np.prod(n))[1::4]
    part = orc.q16_step_cells(P, w, cells, mask, t=11, seed=4, mode=1)
    assert np.all(part == full.reshape(5, -1)[:, cells].T)


# ------------------------------------------- b_rho_u / b_S allocation (R18) ---
CONFIGS = [(16, 16), (16, 15), (15, 14), (14, 13), (13, 12), (12, 11)]


def _unpack_stream(w, b1, b2):
    """The ten codes of each cell, read back by treating its words as one
    little-endian integer (word i = bits 32 i .. 32 i + 31)."""
    W = w.shape[0]
    flat = w.reshape(W, -1)
    out = np.zeros((10, flat.shape[1]), np.int64)
    for c in range(flat.shape[1]):
        s = 0
        for i in range(W):
            s |= int(flat[i, c]) << (32 * i)
        o = 0
        for k in range(10):
            b = b1 if k < 4 else b2
            out[k, c] = (s >> o) & ((1 << b) - 1)
            o += b
    return out.reshape((10,) + w.shape[1:])


def test_packed_16_16_is_the_paired_layout(orc):
    m = W.random_moments(7, 5, 3, seed=1, dj=0.02, dp=0.003)
    for mode in (0, 1):
        assert np.array_equal(orc.qb_encode(m, 16, 16, t=4, seed=2, mode=mode), orc.q16_encode(m, t=4, seed=2, mode=mode))


@pytest.mark.parametrize("b1,b2", CONFIGS)
def test_packed_layout(orc, b1, b2):
    rng = np.random.default_rng(b1 * 100 + b2)
    q = np.stack([rng.integers(0, 1 << (b1 if k < 4 else b2), size=(3, 4, 5)) for k in range(10)]).astype(np.uint32)
    w = orc.qb_pack(q, b1, b2)
    assert w.shape[0] == -(-(4 * b1 + 6 * b2) // 32)
    assert np.array_equal(_unpack_stream(w, b1, b2), q)


@pytest.mark.parametrize("b1,b2", CONFIGS)
def test_packed_known_answers(orc, b1, b2):
    """min -> 0, max -> 2^b - 1, the range midpoint rounds half up (Sec. 5.3
    with b bits), for every code of a cell."""
    lo, hi = np.array(orc.Q_LO), np.array(orc.Q_HI)
    b = np.array([b1] * 4 + [b2] * 6)
    qmax = (1 << b) - 1
    d = (hi - lo) / qmax
    mid = 0.5 * (lo + hi)
    vs = [lo, hi, mid + 0.05 * d, mid - 0.05 * d]
    want = [np.zeros(10, int), qmax, (qmax + 1) // 2, (qmax - 1) // 2]
    v = np.stack(vs, axis=1)  # codec variables (rho, u, N) of 4 cells
    m = np.empty_like(v)
    m[0] = v[0]
    m[1:4] = v[0] * v[1:4]
    pa, pb = [0, 1, 2, 0, 0, 1], [0, 1, 2, 1, 2, 2]
    for p in range(6):
        m[4 + p] = v[4 + p] + v[0] * v[1 + pa[p]] * v[1 + pb[p]]
    w = orc.qb_encode(m.reshape(10, 1, 1, 4), b1, b2)
    got = _unpack_stream(w, b1, b2).reshape(10, 4)
    for c in range(4):
        assert np.array_equal(got[:, c], want[c]), (c, got[:, c], want[c])


@pytest.mark.parametrize("b1,b2", CONFIGS)
def test_packed_round_trip_error(orc, b1, b2):
    m = W.random_moments(9, 7, 5, seed=3, dj=0.02, dp=0.003)
    lo, hi = np.array(orc.Q_LO), np.array(orc.Q_HI)
    d = (hi - lo) / ((1 << np.array([b1] * 4 + [b2] * 6)) - 1)

    def cvars(x):
        rho = x[0]
        u = x[1:4] / rho
        pa, pb = [0, 1, 2, 0, 0, 1], [0, 1, 2, 1, 2, 2]
        return np.stack([rho, *u, *[x[4 + p] - rho * u[pa[p]] * u[pb[p]] for p in range(6)]])

    v = cvars(m)
    for mode, bound in ((0, 0.5), (1, 1.0)):
        r = cvars(orc.qb_decode(orc.qb_encode(m, b1, b2, t=1, seed=5, mode=mode), b1, b2))
        err = np.abs(r - v).reshape(10, -1).max(axis=1)
        assert np.all(err <= bound * d * (1 + 1e-3) + 1e-7), (mode, err / d)


def _exact_code(m, k, xi, b, orc):
    """floor(m' (2^b - 1) + 1/2 + xi) in exact rational arithmetic, with the
    range ends taken as the decimal values the paper prints (Sec. 5.3)."""
    lo = Fraction(str(orc.Q_LO[k]))
    hi = Fraction(str(orc.Q_HI[k]))
    v = (Fraction(m) - lo) / (hi - lo) * ((1 << b) - 1) + Fraction(1, 2) + Fraction(xi)
    return min(max(math.floor(v), 0), (1 << b) - 1)


def test_encode_is_the_printed_rule_in_exact_arithmetic(orc):
    """The encode decision is floor(m' (2^b - 1) + 1/2 + xi) (R15), checked
    against exact rational arithmetic on random values and dither levels:
    a decision taken in single precision, or with ties to even, or by
    truncation, disagrees on about one value in a hundred or more."""
    rng = np.random.default_rng(11)
    levels = (np.arange(64) + 0.5) / 64 - 0.5
    for k in range(10):
        lo, hi = orc.Q_LO[k], orc.Q_HI[k]
        ms = rng.uniform(lo - 0.01, hi + 0.01, 1500)
        xis = rng.choice(levels, ms.size)
        for m, xi in zip(ms, xis):
            assert orc.encode_one(float(m), k, float(xi)) == _exact_code(float(m), k, float(xi), 16, orc)
    # values a hair off a half-way point of the b-bit grids
    for k, b in [(0, 16), (1, 12), (4, 13), (9, 15)]:
        d = (Fraction(str(orc.Q_HI[k])) - Fraction(str(orc.Q_LO[k]))) / ((1 << b) - 1)
        for q in rng.integers(1, (1 << b) - 2, 200):
            for eps in (Fraction(1, 10**6), -Fraction(1, 10**6)):
                m = float(Fraction(str(orc.Q_LO[k])) + (int(q) + Fraction(1, 2) + eps) * d)
                got = orc.qb_encode_one(m, k, 0.0, b) if b != 16 else orc.encode_one(m, k)
                assert got == _exact_code(m, k, 0.0, b, orc) == (int(q) + 1 if eps > 0 else int(q))
