"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/omap.h, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2004_00540_amd as omap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "omap.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(omap_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("omap_plan_create", "omap_propagate", "omap_extract_paths", "omap_plan_destroy",
                     "omap_get_activity", "omap_batch_create", "omap_engine_submit"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = omap.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version():
    L = omap.lib()
    for code, name in omap.STATUS.items():
        assert L.omap_status_string(code).decode() == name
    assert L.omap_status_string(999).decode() == "OMAP_ERR_UNKNOWN"
    assert omap.version().startswith("omap-gfx950")


def _create(H, W, occ_ptr, src, tgt, opts=None, out=True):
    L = omap.lib()
    h = ctypes.c_void_p()
    s = np.ascontiguousarray(np.asarray(src, np.int32).reshape(-1, 2))
    t = np.ascontiguousarray(np.asarray(tgt, np.int32).reshape(-1, 2))
    return L.omap_plan_create(ctypes.byref(h) if out else None, H, W, occ_ptr,
                              s.ctypes.data if len(s) else None, len(s),
                              t.ctypes.data if len(t) else None, len(t),
                              ctypes.byref(opts) if opts is not None else None, None)


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


@pytest.mark.parametrize("args,status", [
    ((0, 5, FAKE, [[0, 0]], []), "OMAP_ERR_INVALID_ARG"),
    ((5, 0, FAKE, [[0, 0]], []), "OMAP_ERR_INVALID_ARG"),
    ((65536, 32768, FAKE, [[0, 0]], []), "OMAP_ERR_TOO_LARGE"),
    ((5, 5, None, [[0, 0]], []), "OMAP_ERR_INVALID_ARG"),
    ((5, 5, FAKE, [], []), "OMAP_ERR_NO_SOURCES"),
    ((5, 5, FAKE, [[5, 0]], []), "OMAP_ERR_SOURCE_OUT_OF_BOUNDS"),
    ((5, 5, FAKE, [[0, -1]], []), "OMAP_ERR_SOURCE_OUT_OF_BOUNDS"),
    ((5, 5, FAKE, [[0, 0]], [[2, 5]]), "OMAP_ERR_TARGET_OUT_OF_BOUNDS"),
    ((5, 5, FAKE, [[0, 0]], [[-1, 0]]), "OMAP_ERR_TARGET_OUT_OF_BOUNDS"),
])
def test_plan_create_validation(args, status):
    st = _create(*args)
    assert omap.STATUS[st] == status
    assert omap.lib().omap_last_error().decode().startswith(status)


def test_plan_create_null_out_and_bad_options():
    assert omap.STATUS[_create(5, 5, FAKE, [[0, 0]], [], out=False)] == "OMAP_ERR_INVALID_ARG"
    for bad in (omap.Options(3, 0, 0, 0, 0), omap.Options(0, 3, 0, 0, 0), omap.Options(0, 0, 7, 0, 0), omap.Options(0, 0, 0, 0, 0, 5), omap.Options(0, 0, 1, 0, 0, 2),
                omap.Options(16, 8, 0, 0, 0), omap.Options(0, 0, 0, -1, 0), omap.Options(0, 0, 0, 0, 3),
                omap.Options(24, 0, 0, 0, 4), omap.Options(32, 16, 0, 0, 2), omap.Options(24, 0, 0, 0, 1)):
        assert omap.STATUS[_create(5, 5, FAKE, [[0, 0]], [], opts=bad)] == "OMAP_ERR_INVALID_ARG"


def test_null_handles_are_rejected_or_ignored():
    L = omap.lib()
    assert L.omap_plan_destroy(None) == 0
    assert L.omap_batch_destroy(None) == 0
    assert L.omap_engine_destroy(None) == 0
    assert omap.STATUS[L.omap_propagate(None, -1, None)] == "OMAP_ERR_INVALID_ARG"
    assert omap.STATUS[L.omap_get_activity(None, None, 0)] == "OMAP_ERR_INVALID_ARG"
    assert omap.STATUS[L.omap_extract_paths(None, None, None, None, 0, None)] == "OMAP_ERR_INVALID_ARG"
    assert omap.STATUS[L.omap_batch_create(None, None, 0, None, None)] == "OMAP_ERR_INVALID_ARG"
    assert omap.STATUS[L.omap_engine_create(None, 1 << 30, 4, None, None)] == "OMAP_ERR_INVALID_ARG"
    h = ctypes.c_void_p()
    assert omap.STATUS[L.omap_engine_create(ctypes.byref(h), 100, 4, None, None)] == "OMAP_ERR_INVALID_ARG"
    assert omap.STATUS[L.omap_profile_enable(None, 0, 1)] == "OMAP_ERR_INVALID_ARG"


def test_batch_validation_names_the_maze():
    L = omap.lib()
    src = np.array([[0, 0]], np.int32)
    bad = np.array([[9, 9]], np.int32)
    descs = (omap.MazeDesc * 2)(
        omap.MazeDesc(4, 4, 0x1000, src.ctypes.data, 1, None, 0),
        omap.MazeDesc(4, 4, 0x1000, bad.ctypes.data, 1, None, 0))
    h = ctypes.c_void_p()
    st = L.omap_batch_create(ctypes.byref(h), descs, 2, None, None)
    assert omap.STATUS[st] == "OMAP_ERR_SOURCE_OUT_OF_BOUNDS"
    assert "(maze 1)" in L.omap_last_error().decode()


def test_resolve_options_fills_defaults():
    d = omap.resolve_options()
    assert d == {"temporal_depth": 16, "tile_rows": 16, "schedule": omap.SCHEDULE_ACTIVE,
                 "check_interval": 0, "lane_columns": 1, "round_launch": omap.LAUNCH_PER_ROUND}
    # the default schedule can also be asked for explicitly, and a plan's is the active one
    assert omap.resolve_options(schedule=omap.SCHEDULE_ACTIVE) == d
    assert omap.resolve_options(schedule=omap.SCHEDULE_DEFAULT) == d
    d = omap.resolve_options(schedule=omap.SCHEDULE_DENSE)
    assert (d["lane_columns"], d["tile_rows"], d["temporal_depth"]) == (4, 256, 16)
    d = omap.resolve_options(temporal_depth=32, round_launch=omap.LAUNCH_GRAPH)
    assert (d["tile_rows"], d["lane_columns"], d["round_launch"]) == (32, 2, omap.LAUNCH_GRAPH)
    d = omap.resolve_options(temporal_depth=16, lane_columns=2)
    assert (d["tile_rows"], d["lane_columns"]) == (16, 2)
    d = omap.resolve_options(lane_columns=2)
    assert (d["temporal_depth"], d["tile_rows"]) == (12, 16)
    d = omap.resolve_options(temporal_depth=12)
    assert (d["temporal_depth"], d["tile_rows"], d["lane_columns"]) == (12, 12, 1)
    for bad in (dict(temporal_depth=32, lane_columns=4), dict(round_launch=2), dict(schedule=4),
                dict(check_interval=-1), dict(tile_rows=7)):
        with pytest.raises(omap.OmapError):
            omap.resolve_options(**bad)
    d = omap.resolve_options(schedule=omap.SCHEDULE_BITS)
    assert (d["schedule"], d["temporal_depth"], d["tile_rows"], d["lane_columns"]) == (omap.SCHEDULE_BITS, 16, 16, 0)
    assert omap.resolve_options(schedule=omap.SCHEDULE_BITS, round_launch=omap.LAUNCH_GRAPH)["round_launch"] == 1
    for bad in (dict(temporal_depth=12), dict(lane_columns=2), dict(temporal_depth=16, tile_rows=8)):
        with pytest.raises(omap.OmapError):
            omap.resolve_options(schedule=omap.SCHEDULE_BITS, **bad)
    L = omap.lib()
    assert omap.STATUS[L.omap_resolve_options(None, None)] == "OMAP_ERR_INVALID_ARG"


def test_build_lists_every_sweep_variant_once():
    """The build compiles one object per sweep variant listed in the internal
    header; the list has no duplicates and covers the documented options."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "omap_build", os.path.join(ROOT, "paper_2004_00540_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    v = b.variants()
    assert len(v) == len(set(v))
    for T in (4, 8, 12, 16):
        for C in (1, 2, 4):
            assert (T, C) in v
    assert (24, 2) in v and (32, 2) in v
