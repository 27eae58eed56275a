"""hyrf_query_fields_noalloc (the query with the library's own scratch, for
callers that cannot allocate) against hyrf_query_fields on the same inputs:
outputs equal bit for bit, over two calls in a row, the second smaller."""
import ctypes as C

import numpy as np
import pytest
import torch

from _hyrf_testutil import device_scene, make

pytestmark = pytest.mark.gpu

KEYS = ("opacity", "scale", "quat", "rgb", "feat_geo", "feat_rad", "feat_jac", "dbg_index")


def _P():
    import paper_2509_17083_amd as P
    return P


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _P()._abi.load()


def _compare(P, cfg_name, over, mode):
    print("case", cfg_name, over, mode, flush=True)
    cfg, scene, cams = make(cfg_name, table_init=1.0, **over)
    ds = device_scene(scene)
    qa, _ = P.query_fields(ds, cams, mode, debug_index=True)
    qb, _ = P.query_fields_noalloc(ds, cams, mode, debug_index=True)
    torch.cuda.synchronize()
    cnt = int(qa["vis_count"].item())
    assert cnt > 0 and int(qb["vis_count"].item()) == cnt
    assert torch.equal(qa["vis_idx"][:cnt], qb["vis_idx"][:cnt])
    for k in KEYS:
        if k not in qa:
            continue
        a, b = qa[k], qb[k]
        a = a[..., :cnt] if k in ("opacity", "scale", "quat", "rgb") else a[:cnt]
        b = b[..., :cnt] if k in ("opacity", "scale", "quat", "rgb") else b[:cnt]
        assert torch.equal(a, b), k
    return cnt


def test_noalloc_query_equals_workspace_query_twice_second_smaller():
    P = _P()
    lib = P._abi.load()
    assert lib.hyrf_query_noalloc_scratch_bytes() >= 2 * 4 * P._abi.HYRF_QUERY_NOALLOC_MAX_GAUSSIANS
    # a c100k-shaped scene of 40k Gaussians with the train-mode outputs ...
    n1 = _compare(P, "c100k", {"n_gauss": 40000, "width": 320, "height": 240, "focal": 350.0}, P.TRAIN)
    # ... then the 1k-Gaussian scene: the scratch keeps the first call's
    # contents, which must not leak into the second call's result
    n2 = _compare(P, "tiny", {}, P.RENDER)
    assert n2 < n1


def test_noalloc_query_rejects_more_gaussians_than_its_scratch():
    P = _P()
    A = P._abi
    lib = A.load()
    cfg, scene, cams = make("tiny", table_init=1.0)
    ds = device_scene(scene)
    from paper_2509_17083_amd.render import _query_outputs
    q, out = _query_outputs(ds, 1, P.RENDER, False)
    g = ds.c_gauss()
    g.n = A.HYRF_QUERY_NOALLOC_MAX_GAUSSIANS + 1
    f, cc = ds.c_fields(), P.c_cameras(cams)
    st = lib.hyrf_query_fields_noalloc(C.byref(f), C.byref(g), cc, 1, C.byref(out), None)
    assert st == A.HYRF_ERR_CAPACITY and b"exceeds" in lib.hyrf_last_error()
