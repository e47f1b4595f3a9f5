"""GPU parity of the open x faces (inflow at x = 0 by the moment boundary of
Sec. 3.2, zero-gradient outflow at x = nx - 1) against the FP64 oracle.

The fluid pass takes the faces on itself: the column past the outflow face
is a copy of the last plane and the column before the inflow face sends
nothing.  Which lane plays that column depends on nx: with nx a multiple of
the 64-cell tile width it is the halo-column wavefront, otherwise a lane of
the last tile's row wavefronts.  Both are covered, with one tile and several
along x, with and without solids and a body force, in both storage formats.
With open faces the fluid pass also stores every solid cell as the rest state
(the oracle's solid cells hold it), interior solid cells included.
"""
import numpy as np
import pytest

from helpers import group_rel_err, unpack
from paper_2602_05295_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
U_IN = (0.06, 0.01, -0.02)

# (nx, ny, nz): ghost in the column wavefront (64, 128), in a row lane of a
# later tile (70, 131), and nx - 1 at the last lane of a tile (63)
SHAPES = [(64, 14, 9), (128, 11, 7), (70, 13, 8), (131, 9, 6), (63, 10, 7)]


def _note(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def H():
    from paper_2602_05295_amd import homelbm
    homelbm.lib()
    return homelbm


def _mask(dims, seed):
    mask = W.sphere_mask(*dims, phi=0.06, rmin=1.5, rmax=2.5, seed=seed)
    mask[:, :, :3] = 0  # solids stay two cells clear of the open faces
    mask[:, :, -3:] = 0
    return mask


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("force", [False, True])
def test_fp32_open_faces_steps(H, orc, dims, force):
    """Five FP32 steps with solids, every cell within 1e-5 per moment group."""
    _note("fp32 open faces", dims, "force", force)
    mask = _mask(dims, seed=dims[0])
    F = (2e-5, -1e-5, 5e-6) if force else (0.0, 0.0, 0.0)
    m = W.random_moments(*dims, seed=9).astype(np.float32)
    with H.HomeLBM(dims, 0.6, mask=mask) as s:
        s.set_options(inflow=True, u_in=U_IN, force=F)
        s.set_moments(m)
        m0 = s.get_moments()
        s.step(5)
        got = s.get_moments()
    P = orc.make_params(dims, 0.6, F=F, inflow=True, u_in=U_IN)
    ref = orc.run(P, m0.astype(np.float64), 5, mask)
    err = group_rel_err(got, ref)
    assert max(err.values()) <= TOL32, err


@pytest.mark.parametrize("dims", SHAPES)
def test_q16_open_faces_one_step(H, orc, dims):
    """One 16-bit step from identical codes (dither on): fluid codes within
    1 LSB of the oracle's, fewer than 1% differing, and the face planes as
    close as the rest."""
    _note("q16 open faces", dims)
    mask = _mask(dims, seed=dims[0] + 1)
    m = W.random_moments(*dims, seed=11, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, 0.58, mask=mask, fmt="q16") as s:
        s.set_options(dither_mode=1, seed=5, inflow=True, u_in=U_IN)
        s.set_moments(m)
        s.step_count = 4
        w0 = s.get_raw().copy()
        s.step(1)
        got = s.get_raw()
    P = orc.make_params(dims, 0.58, inflow=True, u_in=U_IN)
    ref = orc.q16_step(P, w0, mask, t=4, seed=5, mode=1)
    d = np.abs(unpack(got) - unpack(ref))
    fl = mask == 0
    assert d[:, fl].max() <= 1, d[:, fl].max()
    assert (d[:, fl] > 0).mean() < 0.01, (d[:, fl] > 0).mean()
    faces = d[:, :, :, [0, -1]]
    assert faces.max() <= 1 and (faces > 0).mean() < 0.02, (faces.max(), (faces > 0).mean())


def test_fp32_open_faces_without_solids(H, orc):
    """No mask: the boundary list is the two face planes, and the boundary
    pass visits the inflow plane alone.  Four FP32 steps against the oracle."""
    dims = (70, 9, 5)
    _note("fp32 open faces, no solids", dims)
    m = W.random_moments(*dims, seed=2).astype(np.float32)
    with H.HomeLBM(dims, 0.6) as s:
        s.set_options(inflow=True, u_in=U_IN)
        s.set_moments(m)
        m0 = s.get_moments()
        nfl, nso = s.boundary_counts()
        assert (nfl, nso) == (2 * dims[1] * dims[2], 0)
        s.step(4)
        got = s.get_moments()
    ref = orc.run(orc.make_params(dims, 0.6, inflow=True, u_in=U_IN), m0.astype(np.float64), 4)
    err = group_rel_err(got, ref)
    assert max(err.values()) <= TOL32, err


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
@pytest.mark.parametrize("dims", [(64, 14, 9), (70, 13, 8)])
def test_solid_cells_hold_the_rest_state(H, dims, fmt):
    """A box obstacle with interior cells and small spheres, three steps with
    open faces: every solid cell's stored words equal those of the rest state
    (what a context at rest, rho = 1 and u = 0, holds there)."""
    _note("solid cells at rest", dims, fmt)
    nx, ny, nz = dims
    mask = _mask(dims, seed=nx + 7)
    mask[2:6, 3:10, 20:30] = 1  # interior cells: z 3..4, y 4..8, x 21..28
    solid = mask == 1
    m = W.random_moments(*dims, seed=13, dj=0.02, dp=0.003).astype(np.float32)
    with H.HomeLBM(dims, 0.6, mask=mask, fmt=fmt) as s:
        s.set_options(inflow=True, u_in=U_IN, dither_mode=1 if fmt == "q16" else 0, seed=3)
        s.set_moments(m)
        s.step(3)
        got = s.get_raw().copy()
    with H.HomeLBM(dims, 0.6, mask=mask, fmt=fmt) as r:
        r.set_equilibrium(np.ones((nz, ny, nx), np.float32), np.zeros((3, nz, ny, nx), np.float32))
        rest = r.get_raw().copy()
    assert np.array_equal(got[:, solid], rest[:, solid])
