"""CPU checks of the C ABI boundary: the library loads without a GPU and
exports every function include/homelbm.h declares; the header's option
struct matches the binding's."""
import ctypes

import numpy as np
import pytest
import os
import re

from paper_2602_05295_amd import homelbm


def test_library_exports_every_declared_symbol():
    L = homelbm.lib()
    names = homelbm.declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_options_struct_layout_matches_header():
    with open(homelbm.HEADER) as fh:
        text = fh.read()
    body = re.search(r"typedef struct lbm_options \{(.*?)\} lbm_options;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(\w+)\s+(\w+)(\[\d+\])?;", body)
    assert [f[1] for f in fields] == [f[0] for f in homelbm.Options._fields_]
    assert ctypes.sizeof(homelbm.Options) == 4 * 15


def test_default_options_without_gpu():
    o = homelbm.Options()
    assert homelbm.lib().lbm_default_options(ctypes.byref(o)) == 0
    assert o.dither_mode == homelbm.DITHER_PER_STEP and o.check_health == 1 and o.inflow == 0
    assert o.graph_steps == 256


def test_create_rejects_bad_arguments_before_touching_the_device():
    L = homelbm.lib()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int * 3)(0, 4, 4)
    assert L.lbm_create(dims, 0.6, None, 0, ctypes.byref(h)) == homelbm.ERR_INVALID_ARG
    assert b"dimension" in L.lbm_last_error(None)
    dims = (ctypes.c_int * 3)(4, 4, 4)
    assert L.lbm_create(dims, 0.5, None, 0, ctypes.byref(h)) == homelbm.ERR_INVALID_ARG
    assert L.lbm_create(dims, 0.6, None, 7, ctypes.byref(h)) == homelbm.ERR_INVALID_ARG
    # boundary-list entries hold y and z in 16 bits each: larger axes are refused
    for d in [(65536, 2, 2), (2, 65536, 2), (2, 2, 70000)]:
        dims = (ctypes.c_int * 3)(*d)
        assert L.lbm_create(dims, 0.6, None, 0, ctypes.byref(h)) == homelbm.ERR_INVALID_ARG
        assert b"65535" in L.lbm_last_error(None)
    assert h.value is None


def test_batch_create_rejects_bad_arguments_before_touching_the_device():
    """An empty batch, an empty or oversized domain, tau <= 1/2, a domain too
    wide for the strip kernel and more than 2^30 cells in all are refused with
    a message, before any device call."""
    L = homelbm.lib()
    h = ctypes.c_void_p()

    def create(dims_list, taus, fmt=homelbm.Q16):
        flat = (ctypes.c_int * (3 * max(1, len(dims_list))))(*[v for d in dims_list for v in d])
        tau = (ctypes.c_double * max(1, len(taus)))(*taus)
        return L.lbm_batch_create(len(dims_list), flat, tau, None, fmt, ctypes.byref(h))

    assert create([], []) == homelbm.ERR_INVALID_ARG
    assert b"count" in L.lbm_batch_last_error(None)
    assert create([(4, 0, 4)], [0.6]) == homelbm.ERR_INVALID_ARG
    assert b"dimensions" in L.lbm_batch_last_error(None)
    assert create([(4, 4, 4), (4, 4, 70000)], [0.6, 0.6]) == homelbm.ERR_INVALID_ARG
    assert create([(4, 4, 4)], [0.5]) == homelbm.ERR_INVALID_ARG
    assert b"tau" in L.lbm_batch_last_error(None)
    assert create([(342, 4, 4)], [0.6]) == homelbm.ERR_INVALID_ARG
    assert b"341" in L.lbm_batch_last_error(None)
    assert create([(256, 1024, 1024)] * 4 + [(1, 1, 1)], [0.6] * 5) == homelbm.ERR_INVALID_ARG
    assert b"2^30" in L.lbm_batch_last_error(None)
    assert h.value is None


def test_null_context_is_refused_by_the_newer_entry_points():
    """lbm_prepare, lbm_tile_rows and lbm_set_triangles check their arguments
    before any device call (a NULL context never reaches the GPU)."""
    L = homelbm.lib()
    rows = ctypes.c_int(-1)
    assert L.lbm_prepare(None, 4) == homelbm.ERR_INVALID_ARG
    assert L.lbm_tile_rows(None, ctypes.byref(rows)) == homelbm.ERR_INVALID_ARG
    assert rows.value == -1
    assert L.lbm_set_triangles(None, 0, None, None) == homelbm.ERR_INVALID_ARG


def test_no_oracle_in_product_path():
    pkg = os.path.dirname(homelbm.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                with open(os.path.join(root, f)) as fh:
                    src = fh.read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "homelbm_oracle" not in src, f


def _xcd_logical_block(b, n):
    x, k = b & 7, b >> 3
    return x * (n >> 3) + min(x, n & 7) + k


def _fluid_items(dims, p):
    """The (tile, za, zb) items of every workgroup, enumerated as the fluid
    kernel does from its launch arguments."""
    nz = dims[2]
    ntiles = p["ntx"] * p["nty"]
    items = ntiles * p["nseg"]
    nreg = p["nwg"] - p["ntail"]
    zt = nz - p["tail"]
    out = []
    for b in range(p["nwg"]):
        k = _xcd_logical_block(b, p["nwg"])
        if k < nreg:
            q = k
            while q < items:
                sg = q // ntiles
                out.append((q % ntiles, zt * sg // p["nseg"], zt * (sg + 1) // p["nseg"]))
                q += nreg
        else:
            j = k - nreg
            for t in range(ntiles * j // p["ntail"], ntiles * (j + 1) // p["ntail"]):
                out.append((t, zt, nz))
    return out


@pytest.mark.parametrize("cus", [256, 304, 80, 7])
def test_fluid_items_cover_every_plane_once(cus):
    """Every (tile, plane) of the grid belongs to exactly one work item, every
    item is in range and non-empty, and the logical workgroup numbering is a
    permutation."""
    shapes = [(256, 256, 256), (1000, 400, 400), (37, 29, 23), (64, 17, 9), (5, 3, 2), (1, 1, 1),
              (31, 45, 3), (2, 33, 4), (130, 53, 40), (128, 128, 128), (96, 24, 77), (64, 64, 1000)]
    for dims in shapes:
        for rows in (0, 8, 10, 12, 13):
            p = homelbm.fluid_plan(dims, tile_rows=rows, cus=cus)
            assert sorted(_xcd_logical_block(b, p["nwg"]) for b in range(p["nwg"])) == list(range(p["nwg"]))
            assert p["ntail"] <= p["ntx"] * p["nty"] and p["tail"] < dims[2]
            assert (p["tail"] == 0) == (p["ntail"] == 0)
            ntiles = p["ntx"] * p["nty"]
            seen = np.zeros((ntiles, dims[2]), dtype=np.int32)
            for t, za, zb in _fluid_items(dims, p):
                assert 0 <= t < ntiles and 0 <= za < zb <= dims[2], (dims, rows, p)
                seen[t, za:zb] += 1
            assert np.all(seen == 1), (dims, rows, p)


def test_fluid_plan_host_logic():
    """The fluid pass's work split: every item maps to a tile and a z segment,
    one wave of items fills the CUs when tiles are fewer than CUs, and the
    forced heights are honoured."""
    plan = homelbm.fluid_plan
    p = plan((256, 256, 256))
    tiles = p["ntx"] * p["nty"]
    assert p["ntx"] == 4 and p["nty"] == -(-256 // p["rows"])
    assert tiles * p["nseg"] <= 256 and p["nwg"] == tiles * p["nseg"] + p["ntail"]
    assert tiles * (p["nseg"] + 1) > 256  # no further split fits in one wave
    # the idle CUs share the top planes: both kinds of workgroup end together
    assert p["ntail"] == 256 - tiles * p["nseg"] and 0 < p["tail"] < 256
    per_tail = -(-tiles // p["ntail"])
    reg = -(-(256 - p["tail"]) // p["nseg"]) + 2
    assert max(reg, per_tail * (p["tail"] + 2)) < -(-256 // p["nseg"]) + 2
    q = plan((1000, 400, 400))
    assert q["ntx"] == 16 and q["nwg"] == 256
    for rows in (8, 10, 12, 13):
        r = plan((130, 53, 40), tile_rows=rows)
        assert r["rows"] == rows and r["ntx"] == 3 and r["nty"] == -(-53 // rows)
        assert 1 <= r["nwg"] <= 256 and r["nseg"] >= 1
    t = plan((1, 1, 1))
    assert t["nwg"] == 1 and t["nseg"] == 1 and t["tail"] == 0 and t["ntail"] == 0
    with pytest.raises(homelbm.LBMError):
        plan((8, 8, 8), tile_rows=7)


def test_default_options_have_no_force():
    o = homelbm.Options()
    assert homelbm.lib().lbm_default_options(ctypes.byref(o)) == 0
    assert list(o.force) == [0.0, 0.0, 0.0]


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before torch must not leave two HIP runtimes in the
    process: the binding loads torch's first, and this library binds to it."""
    import subprocess
    import sys
    code = ("from paper_2602_05295_amd import homelbm as H; H.lib(); "
            "import re; maps = open('/proc/self/maps').read(); "
            "paths = sorted(set(re.findall(r'\\S*libamdhip64\\S*', maps))); "
            "assert len(paths) == 1, paths; print(paths[0])")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
