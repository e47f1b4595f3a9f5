"""CPU checks of the C ABI boundary: the library loads without a GPU and
exports every function include/homelbm.h declares; the header's option
struct matches the binding's."""
import ctypes

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
    assert ctypes.sizeof(homelbm.Options) == 4 * 14


def test_default_options_without_gpu():
    o = homelbm.Options()
    assert homelbm.lib().lbm_default_options(ctypes.byref(o)) == 0
    assert o.dither_mode == homelbm.DITHER_PER_STEP and o.check_health == 1 and o.inflow == 0


def test_create_rejects_bad_arguments_before_touching_the_device():
    L = homelbm.lib()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int * 3)(0, 4, 4)
    assert L.lbm_create(dims, 0.6, None, 0, ctypes.byref(h)) == homelbm.ERR_INVALID_ARG
    assert b"dimension" in L.lbm_last_error(None)
    dims = (ctypes.c_int * 3)(4, 4, 4)
    assert L.lbm_create(dims, 0.5, None, 0, ctypes.byref(h)) == homelbm.ERR_INVALID_ARG
    assert L.lbm_create(dims, 0.6, None, 7, ctypes.byref(h)) == homelbm.ERR_INVALID_ARG
    assert h.value is None


def test_no_oracle_in_product_path():
    pkg = os.path.dirname(homelbm.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                with open(os.path.join(root, f)) as fh:
                    src = fh.read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "homelbm_oracle" not in src, f


def test_fluid_plan_host_logic():
    """The fluid pass's work split: every item maps to a tile and a z segment,
    one wave of items fills the CUs when tiles are fewer than CUs, and the
    forced heights are honoured."""
    plan = homelbm.fluid_plan
    p = plan((256, 256, 256))
    tiles = p["ntx"] * p["nty"]
    assert p["ntx"] == 4 and p["nty"] == -(-256 // p["rows"])
    assert tiles * p["nseg"] <= 256 and p["nwg"] == tiles * p["nseg"]
    assert tiles * (p["nseg"] + 1) > 256  # no further split fits in one wave
    q = plan((1000, 400, 400))
    assert q["ntx"] == 16 and q["nwg"] == 256
    for rows in (8, 10, 12, 13):
        r = plan((130, 53, 40), tile_rows=rows)
        assert r["rows"] == rows and r["ntx"] == 3 and r["nty"] == -(-53 // rows)
        assert 1 <= r["nwg"] <= 256 and r["nseg"] >= 1
    t = plan((1, 1, 1))
    assert t["nwg"] == 1 and t["nseg"] == 1
    with pytest.raises(homelbm.LBMError):
        plan((8, 8, 8), tile_rows=7)


def test_default_options_have_no_force():
    o = homelbm.Options()
    assert homelbm.lib().lbm_default_options(ctypes.byref(o)) == 0
    assert list(o.force) == [0.0, 0.0, 0.0]
