"""CPU checks of the batched step's host logic: the work split covers every
(domain, strip, plane) exactly once with balanced workgroups, strips fit the
workgroup, and bad batches are refused before the device is touched."""
import ctypes

import numpy as np
import pytest

from paper_2602_05295_amd import homelbm as H
from paper_2602_05295_amd import workloads as W

MIXED = [(20, 30, 7), (100, 37, 9), (3, 5, 2), (1, 1, 1), (64, 64, 5), (33, 17, 12)]


def _coverage(dims, plan):
    segs, strips = plan["segments"], plan["strips"]
    cover = {}
    for d, (nx, ny, nz) in enumerate(dims):
        rows, ty, span = (int(v) for v in strips[d])
        nstrips = 1 if span else -(-ny // ty)
        cover[d] = np.zeros((nstrips, nz), np.int32)
    for d, s, za, zb in segs.astype(int):
        assert 0 <= za < zb <= dims[d][2]
        cover[d][s, za:zb] += 1
    return all((c == 1).all() for c in cover.values())


@pytest.mark.parametrize("block", [512, 1024])
def test_split_covers_every_plane_once(block):
    for dims in (MIXED, [d["dims"] for d in W.batched_domains(128, seed=0)]):
        for nwg in (1, 7, 256):
            p = H.batch_plan(dims, block, nwg)
            assert _coverage(dims, p)
            first = p["wg_first"]
            assert first[0] == 0 and first[-1] == len(p["segments"]) and (np.diff(first.astype(int)) >= 0).all()


def test_strip_shapes():
    p = H.batch_plan(MIXED, 1024, 64)
    for (nx, ny, nz), (rows, ty, span) in zip(MIXED, p["strips"]):
        assert rows * nx <= 1024
        if nx * ny <= 1024:
            assert span == 1 and rows == ny == ty
        else:
            assert span == 0 and rows == ty + 2 and ty >= 1
            nstrips = -(-ny // ty)
            assert (nstrips - 1) * ty < ny <= nstrips * ty


def test_split_of_the_128_domain_workload_is_balanced():
    dims = [d["dims"] for d in W.batched_domains(128, seed=0)]
    assert 2.6e7 < sum(int(np.prod(d)) for d in dims) < 3.0e7
    for block in (512, 1024):
        assert H.batch_plan(dims, block, 256)["balance"] > 0.98


def test_too_wide_domains_are_refused():
    with pytest.raises(H.LBMError):
        H.batch_plan([(100, 37, 9)], 256, 8)


def test_create_rejects_bad_batches_without_a_device():
    L = H.lib()
    h = ctypes.c_void_p()

    def create(dims, taus, masks=None, fmt=1):
        flat = (ctypes.c_int * (3 * len(dims)))(*[v for d in dims for v in d])
        t = (ctypes.c_double * len(taus))(*taus)
        mp = None
        keep = []
        if masks is not None:
            mp = (ctypes.c_void_p * len(masks))()
            for k, m in enumerate(masks):
                a = np.ascontiguousarray(m, dtype=np.uint8)
                keep.append(a)
                mp[k] = a.ctypes.data_as(ctypes.c_void_p)
        return L.lbm_batch_create(len(dims), flat, t, mp, fmt, ctypes.byref(h))

    assert create([(8, 8, 8)], [0.5]) == H.ERR_INVALID_ARG
    assert b"tau" in L.lbm_batch_last_error(None)
    assert create([(400, 8, 8)], [0.6]) == H.ERR_INVALID_ARG
    assert create([(0, 8, 8)], [0.6]) == H.ERR_INVALID_ARG
    assert create([(4, 4, 4)], [0.6], masks=[np.full(64, 2)]) == H.ERR_INVALID_ARG
    assert create([(4, 4, 4)], [0.6], fmt=7) == H.ERR_INVALID_ARG
    assert L.lbm_batch_create(0, None, None, None, 1, ctypes.byref(h)) == H.ERR_INVALID_ARG
