"""The C ABI library loads and exports every symbol include/legs.h declares;
host-only sizing calls behave as documented (no GPU work, no GPU needed)."""
import ctypes as ct
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(legs_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_2311_18482_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liblegs.so is not built (run __graft_entry__.build())")
    return _lib


def test_every_declared_symbol_is_exported(L):
    lib = ct.CDLL(L.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a prototype for each of them
    assert set(names) <= set(L.exported_names()), set(names) - set(L.exported_names())


def test_struct_sizes_match_header(L):
    assert ct.sizeof(L.Camera) == 8 + 4 * 8 + 9 * 8 + 3 * 8
    assert ct.sizeof(L.View) == ct.sizeof(L.Camera) + 8 + 16
    assert ct.sizeof(L.Opts) == 24 + 24
    assert ct.sizeof(L.Projected) == 7 * 8
    assert ct.sizeof(L.Bins) == 8 * 8


def test_views_build_and_sizes(L):
    lib = L.lib()
    o = L.Opts()
    lib.legs_opts_default(ct.byref(o))
    assert o.tile == 16 and o.lds_batch == 256 and abs(o.alpha_min - 1 / 255) < 1e-9
    from paper_2311_18482_amd.raster import to_camera
    cams = synth.cameras_sphere(3, 5, 8.0, synth.RESOLUTIONS_C3)
    arr = (L.Camera * 3)(*[to_camera(c) for c in cams])
    views = (L.View * 3)()
    tt, tp = ct.c_int64(), ct.c_int64()
    assert lib.legs_views_build(arr, 3, ct.byref(o), views, ct.byref(tt), ct.byref(tp)) == 0
    tiles = [((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams]
    assert tt.value == sum(tiles) and tp.value == sum(c.width * c.height for c in cams)
    assert [views[i].tile_offset for i in range(3)] == [0, tiles[0], tiles[0] + tiles[1]]
    o.tile = 12
    assert lib.legs_views_build(arr, 3, ct.byref(o), views, ct.byref(tt), ct.byref(tp)) == L.LEGS_ERR_ARG
    assert lib.legs_sort_passes(1) == 4
    assert lib.legs_sort_passes(8160) == 6       # 13 tile bits + 32 depth bits
    assert lib.legs_sort_passes(1 << 16) == 6
    assert lib.legs_sort_passes((1 << 16) + 1) == 7
    assert lib.legs_projected_blocks(1000, 3) == 4 * 3
    assert lib.legs_sort_scratch_bytes(10_000_000, 8160) > 0
    assert lib.legs_sort_scratch_bytes(-1, 1) == -1


def test_null_context_is_rejected(L):
    lib = L.lib()
    assert lib.legs_project(None, None, None, None, None, 0, None, 1, None, None, None) == L.LEGS_ERR_ARG
    assert lib.legs_create(0, None) == L.LEGS_ERR_ARG
