"""Host-only checks of the C ABI: the library loads, exports every function the
headers declare, and validates plans without touching a device (CPU only)."""
import ctypes
import glob
import os
import re

import pytest

from paper_1904_06017_amd import _lib
from paper_1904_06017_amd.api import make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(stereo_[a-z0-9_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libstereo.so not built")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header(lib):
    assert _declared() <= set(_lib.SIGNATURES)


def test_struct_sizes_match_the_c_layout():
    assert ctypes.sizeof(_lib.StereoParams) == 96
    assert ctypes.sizeof(_lib.RoadFit) == 80


def _create(lib, p):
    h = ctypes.c_void_p()
    s = lib.stereo_plan_create(ctypes.byref(p), ctypes.byref(h))
    return s, h


def test_valid_plan_and_workspace(lib):
    p = make_params(1280, 720, 64, delta_p=32, plane=(24, 0, 0.1), ncc_radius=3,
                    bil_radius=7, sigma_s=5, sigma_r=12)
    s, h = _create(lib, p)
    assert s == 0 and h.value
    n = ctypes.c_size_t()
    assert lib.stereo_plan_workspace_bytes(h, ctypes.byref(n)) == 0
    cw = ((1280 + 63) + 3) & ~3
    assert n.value >= 4 * 64 * 720 * cw           # the cost volume dominates
    q = _lib.StereoParams()
    assert lib.stereo_plan_get_params(h, ctypes.byref(q)) == 0
    assert q.width == 1280 and q.num_disp == 64 and abs(q.plane[2] - 0.1) < 1e-15
    assert lib.stereo_plan_destroy(h) == 0
    assert lib.stereo_plan_destroy(None) == 0


@pytest.mark.parametrize("field,value,status", [
    ("width", 0, 1), ("height", -3, 1), ("num_disp", 2, 1), ("num_disp", 300, 2),
    ("ncc_radius", 0, 1), ("ncc_radius", 9, 2), ("bil_radius", 0, 1), ("bil_radius", 9, 2),
    ("sigma_s", 0.0, 1), ("sigma_r", -1.0, 1), ("pitch_ref", 10, 1), ("dtype", 7, 1),
    ("softargmin_T", 0.0, 1), ("perspective", 2, 1), ("lr_delta", -1.0, 1),
])
def test_invalid_parameters_are_rejected(lib, field, value, status):
    p = make_params(64, 48, 16, delta_p=8, plane=(4, 0, 0.1))
    setattr(p, field, value)
    s, h = _create(lib, p)
    assert s == status and not h.value
    assert lib.stereo_last_error().decode()


def test_delta_p_requires_the_perspective_step(lib):
    p = make_params(64, 48, 16, perspective=False)
    p.delta_p = 3.0
    assert _create(lib, p)[0] == 1


def test_null_arguments(lib):
    assert lib.stereo_plan_create(None, None) == 1
    p = make_params(64, 48, 16, delta_p=8, plane=(4, 0, 0.1))
    s, h = _create(lib, p)
    assert lib.stereo_plan_workspace_bytes(h, None) == 1
    # enqueue calls reject NULL buffers before touching a device
    assert lib.stereo_warp(h, None, None, None) == 1
    assert lib.stereo_match(h, None, None, None, None, None, None, None, None, 0, None) == 1
    assert lib.stereo_wta_subpixel(None, None, None, None, None) == 1
    lib.stereo_plan_destroy(h)


def test_workspace_checks(lib):
    p = make_params(64, 48, 16, delta_p=8, plane=(4, 0, 0.1))
    s, h = _create(lib, p)
    buf = ctypes.c_void_p(4096)   # never dereferenced: the size check fails first
    st = lib.stereo_match(h, buf, buf, buf, None, None, None, None, buf, 16, None)
    assert st == 3
    assert "workspace" in lib.stereo_last_error().decode()
    lib.stereo_plan_destroy(h)


def test_tuning_keys(lib):
    p = make_params(64, 48, 16, delta_p=8, plane=(4, 0, 0.1))
    s, h = _create(lib, p)
    v = ctypes.c_int32()
    assert lib.stereo_plan_get_tuning(h, b"agg_levels_u8", ctypes.byref(v)) == 0 and v.value == 8
    assert lib.stereo_plan_set_tuning(h, b"agg_levels_f32", 16) == 0
    assert lib.stereo_plan_get_tuning(h, b"agg_levels_f32", ctypes.byref(v)) == 0 and v.value == 16
    assert lib.stereo_plan_set_tuning(h, b"agg_levels_f32", 12) == 1
    assert lib.stereo_plan_get_tuning(h, b"ncc_levels", ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stereo_plan_set_tuning(h, b"ncc_levels", 64) == 0
    assert lib.stereo_plan_get_tuning(h, b"ncc_levels", ctypes.byref(v)) == 0 and v.value == 64
    assert lib.stereo_plan_set_tuning(h, b"ncc_levels", 48) == 1
    assert lib.stereo_plan_get_tuning(h, b"agg_engine", ctypes.byref(v)) == 0 and v.value == 2
    assert lib.stereo_plan_set_tuning(h, b"agg_engine", 0) == 0
    assert lib.stereo_plan_get_tuning(h, b"agg_engine", ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stereo_plan_set_tuning(h, b"agg_engine", 3) == 1
    assert lib.stereo_plan_set_tuning(h, b"no_such_key", 8) == 1
    lib.stereo_plan_destroy(h)


def test_batch_tuning_keys(lib):
    # batch creation is host only: the item pointers are stored, never read
    p = make_params(64, 48, 16, delta_p=8, plane=(4, 0, 0.1))
    s, h = _create(lib, p)
    items = (_lib.BatchItem * 1)()
    items[0].plan = h.value
    for f in ("ref", "tar", "dint_R", "valid", "disp"):
        setattr(items[0], f, 4096)
    b = ctypes.c_void_p()
    assert lib.stereo_batch_create(items, 1, ctypes.byref(b)) == 0
    v = ctypes.c_int32()
    assert lib.stereo_batch_get_tuning(b, b"ncc_levels", ctypes.byref(v)) == 0 and v.value == 0
    for nl in (16, 32, 64, 0):
        assert lib.stereo_batch_set_tuning(b, b"ncc_levels", nl) == 0
        assert lib.stereo_batch_get_tuning(b, b"ncc_levels", ctypes.byref(v)) == 0
        assert v.value == nl
    assert lib.stereo_batch_set_tuning(b, b"ncc_levels", 48) == 1
    assert lib.stereo_batch_get_tuning(b, b"group_overlap", ctypes.byref(v)) == 0 and v.value == 1
    assert lib.stereo_batch_set_tuning(b, b"group_overlap", 0) == 0
    assert lib.stereo_batch_get_tuning(b, b"group_overlap", ctypes.byref(v)) == 0 and v.value == 0
    assert lib.stereo_batch_set_tuning(b, b"group_overlap", 2) == 1
    assert lib.stereo_batch_get_tuning(b, b"tile_band", ctypes.byref(v)) == 0 and v.value == 4
    assert lib.stereo_batch_set_tuning(b, b"tile_band", 3) == 1
    assert lib.stereo_batch_set_tuning(b, b"no_such_key", 8) == 1
    lib.stereo_batch_destroy(b)
    lib.stereo_plan_destroy(h)


def test_volume_size_limit(lib):
    p = make_params(8192, 8192, 256, delta_p=8, plane=(4, 0, 0.1))
    assert _create(lib, p)[0] == 2


def test_status_strings(lib):
    for k, v in _lib.STATUS.items():
        assert lib.stereo_status_string(k).decode() == v
    assert b"gfx950" in lib.stereo_version()


def test_damage_mask_argument_checks(lib):
    p = make_params(64, 48, 16, delta_p=8, plane=(4, 0, 0.1))
    s, h = _create(lib, p)
    buf = ctypes.create_string_buffer(64)
    # NULL pointers and a non-positive threshold are rejected before any launch
    assert lib.stereo_damage_mask(h, None, ctypes.c_float(0.0), ctypes.c_float(0.5), buf,
                                  None) == 1
    assert lib.stereo_damage_mask(h, buf, ctypes.c_float(0.0), ctypes.c_float(0.0), buf,
                                  None) == 1
    assert lib.stereo_damage_mask(h, buf, ctypes.c_float(0.0), ctypes.c_float(float("nan")),
                                  buf, None) == 1
    lib.stereo_plan_destroy(h)


def test_homography_argument_checks(lib):
    p = make_params(64, 48, 16, delta_p=8, plane=(4, 0, 0.1))
    s, h = _create(lib, p)
    H = (ctypes.c_double * 9)(1, 0, -4, 0, 1, 0, 0, 0, 1)
    assert lib.stereo_plan_set_homography(h, H) == 0
    assert lib.stereo_plan_set_homography(h, None) == 0          # back to the row shift
    bad = (ctypes.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, float("nan"))
    assert lib.stereo_plan_set_homography(h, bad) == 1
    behind = (ctypes.c_double * 9)(1, 0, 0, 0, 1, 0, -0.1, 0, 1)  # z <= 0 at the far columns
    assert lib.stereo_plan_set_homography(h, behind) == 1
    lib.stereo_plan_destroy(h)
    raw = make_params(64, 48, 16, perspective=False)
    s, h = _create(lib, raw)
    assert lib.stereo_plan_set_homography(h, H) == 1              # needs perspective = 1
    lib.stereo_plan_destroy(h)


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library every entry point raises: there is no CPU
    fallback behind the Python layer."""
    from paper_1904_06017_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libstereo.so")
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        L.load()
    from paper_1904_06017_amd import api
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        api.Plan(api.make_params(64, 48, 16, delta_p=8, plane=(4, 0, 0.1)))
