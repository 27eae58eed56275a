"""The C-ABI library loads, exports every entry point of include/hyrf.h, and
rejects invalid arguments on the host before anything is launched (these
calls never reach the GPU, so they run on the CPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2509_17083_amd import _abi as A
    if not os.path.exists(A.LIB_PATH):
        pytest.fail("libhyrf.so is not built (run __graft_entry__.build())")
    return A, A.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "hyrf.h")).read()
    return sorted(set(re.findall(r"\b(hyrf_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    A, lib = _lib()
    names = _declared()
    assert "hyrf_query_fields" in names and "hyrf_render_backward" in names
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(names) <= set(A.EXPORTS), set(names) - set(A.EXPORTS)


def _fields(A, **kw):
    f = A.hyrf_fields()
    f.levels, f.features, f.log2_T_geo, f.log2_T_rad = 16, 2, 20, 21
    f.base_res, f.growth = 16.0, 1.5
    f.table_geo = f.table_rad = f.mlp_geo = f.mlp_col = 0x1000   # never dereferenced on the host
    f.hidden, f.n_hidden = 64, 2
    f.aabb_inv_half[:] = [1, 1, 1]
    f.bg_radius, f.tau_T = 100.0, 0.2
    for k, v in kw.items():
        setattr(f, k, v)
    return f


def _cam(A, **kw):
    c = (A.hyrf_camera * 1)()
    c[0].R[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
    c[0].fx = c[0].fy = 100.0
    c[0].cx, c[0].cy = 32.0, 32.0
    c[0].width = c[0].height = 64
    c[0].z_near, c[0].cull_tol = 0.2, 0.3
    for k, v in kw.items():
        setattr(c[0], k, v)
    return c


def _query(A, lib, f, cams=None, n_views=1, out=True, ws_bytes=1 << 20):
    g = A.hyrf_gaussians()
    g.n = 10
    g.pos = g.scale_e = g.opac_e = g.col_e = 0x2000
    o = A.hyrf_query_out()
    if out:
        o.vis_count = o.vis_idx = o.opacity = o.scale = o.quat = o.rgb = 0x3000
    cams = cams if cams is not None else _cam(A)
    st = lib.hyrf_query_fields(C.byref(f) if f is not None else None, C.byref(g), cams, n_views, C.byref(o),
                               C.c_void_p(0x4000), ws_bytes, None)
    return st, lib.hyrf_last_error().decode()


@pytest.mark.parametrize("kw,status", [
    (dict(levels=5), 1), (dict(features=4), 1), (dict(log2_T_rad=30), 1), (dict(hidden=100), 1),
    (dict(n_hidden=3), 1), (dict(table_dtype=7), 2), (dict(levels=12), 2), (dict(bg_radius=0.0), 1),
    (dict(scatter_merge=3), 1), (dict(scatter_merge=-1), 1),
])
def test_query_rejects_bad_fields(kw, status):
    A, lib = _lib()
    st, msg = _query(A, lib, _fields(A, **kw))
    assert st == status and msg


def test_query_rejects_null_and_bad_views():
    A, lib = _lib()
    st, msg = _query(A, lib, None)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT and "fields" in msg
    st, msg = _query(A, lib, _fields(A), n_views=0)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT
    st, msg = _query(A, lib, _fields(A), n_views=9)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT
    st, msg = _query(A, lib, _fields(A), cams=_cam(A, width=0))
    assert st == A.HYRF_ERR_INVALID_ARGUMENT and "width" in msg
    st, msg = _query(A, lib, _fields(A), out=False)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT
    st, msg = _query(A, lib, _fields(A), ws_bytes=8)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT and "workspace" in msg


def test_bin_sort_capacity_checked_on_host():
    A, lib = _lib()
    sp = A.hyrf_splats(10, 0x1000, 0x2000, 0x3000, 0x4000, 0x5000)
    st = lib.hyrf_bin_sort(C.byref(sp), _cam(A), 1, 100, 50, None, C.c_void_p(0x6000), C.c_void_p(0x7000),
                           C.c_void_p(0x8000), 1 << 30, None)
    assert st == A.HYRF_ERR_CAPACITY and "capacity" in lib.hyrf_last_error().decode()
    st = lib.hyrf_bin_sort(C.byref(sp), _cam(A), 1, 10, 50, None, None, C.c_void_p(0x7000),
                           C.c_void_p(0x8000), 1 << 30, None)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT


def test_composite_rejects_bad_mode_and_missing_train_outputs():
    A, lib = _lib()
    sp = A.hyrf_splats(10, 0x1000, 0x2000, 0x3000, 0x4000, 0x5000)
    args = [C.byref(sp), C.c_void_p(0x100), C.c_void_p(0x200), _cam(A), 1, None]
    st = lib.hyrf_composite(*args, 5, C.c_void_p(0x300), C.c_void_p(0x400), None, None, None, C.c_void_p(0x500),
                            1 << 30, None)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT and "mode" in lib.hyrf_last_error().decode()
    f = _fields(A)
    args[-1] = C.byref(f)
    st = lib.hyrf_composite(*args, A.HYRF_TRAIN, C.c_void_p(0x300), C.c_void_p(0x400), None, None, None,
                            C.c_void_p(0x500), 1 << 30, None)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT


def test_workspace_sizes_grow_with_problem():
    A, lib = _lib()
    assert lib.hyrf_query_workspace_bytes(1000) < lib.hyrf_query_workspace_bytes(1_000_000)
    a = lib.hyrf_bin_sort_workspace_bytes(1, 1000, 10000, 64, 64)
    b = lib.hyrf_bin_sort_workspace_bytes(1, 1000, 100000, 64, 64)
    assert 0 < a < b
    assert lib.hyrf_composite_workspace_bytes(2, 64, 64) > lib.hyrf_composite_workspace_bytes(1, 64, 64)


def test_l1_dssim_rejects_bad_arguments():
    A, lib = _lib()
    p = C.c_void_p
    ws = lib.hyrf_l1_dssim_workspace_bytes(3, 64, 64)
    assert ws > 0 and lib.hyrf_l1_dssim_workspace_bytes(3, 640, 640) > ws
    assert lib.hyrf_l1_dssim_workspace_bytes(0, 64, 64) == 0
    good = [p(0x100), p(0x200), 3, 64, 64, 0.2, p(0x300), p(0x400), p(0x500), ws, None]
    for i, bad in [(0, None), (2, 0), (3, -1), (5, 1.5), (5, -0.1), (9, ws - 1), (8, None)]:
        args = list(good)
        args[i] = bad
        assert lib.hyrf_l1_dssim_loss(*args) == A.HYRF_ERR_INVALID_ARGUMENT, (i, bad)


def test_background_entry_points_reject_bad_arguments():
    A, lib = _lib()
    f = _fields(A)
    assert lib.hyrf_background(C.byref(f), _cam(A), 1, None, None, None) == A.HYRF_ERR_INVALID_ARGUMENT
    assert lib.hyrf_background(None, _cam(A), 1, C.c_void_p(0x100), None, None) == A.HYRF_ERR_INVALID_ARGUMENT
    assert lib.hyrf_blend_background(None, C.c_void_p(0x100), C.c_void_p(0x200), 1, 4, 4, None) == \
        A.HYRF_ERR_INVALID_ARGUMENT
    assert lib.hyrf_blend_background(C.c_void_p(0x1), C.c_void_p(0x100), C.c_void_p(0x200), 1, 0, 4, None) == \
        A.HYRF_ERR_INVALID_ARGUMENT


def test_query_rejects_bad_position_dtype():
    A, lib = _lib()
    f = _fields(A)
    g = A.hyrf_gaussians()
    g.n = 10
    g.pos = g.scale_e = g.opac_e = g.col_e = 0x2000
    g.pos_dtype = 7
    o = A.hyrf_query_out()
    o.vis_count = o.vis_idx = o.opacity = o.scale = o.quat = o.rgb = 0x3000
    st = lib.hyrf_query_fields(C.byref(f), C.byref(g), _cam(A), 1, C.byref(o), C.c_void_p(0x4000), 1 << 20, None)
    assert st == A.HYRF_ERR_INVALID_ARGUMENT and b"pos_dtype" in lib.hyrf_last_error()
