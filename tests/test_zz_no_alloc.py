"""qc_fit_noalloc, the entry point that allocates nothing (its recomputation list lives in
the library's fixed device scratch): through the C ABI, its outputs equal qc_fit's bit for
bit on two calls in a row, the second on a smaller frame, and a frame beyond the scratch
is refused before any work is enqueued."""
import numpy as np
import pytest

from paper_1707_00385_amd import scenes
from tests.helpers import log

pytestmark = pytest.mark.gpu


def _fit_both(ctx, depth, K, **kw):
    import torch
    from paper_1707_00385_amd.api import make_outputs, make_params
    p = make_params(**kw)
    h, w = depth.shape
    ref = ctx.fit(depth, K, params=p, normal=True, residual=True)
    torch.cuda.synchronize()
    n_ref = ctx.last_refit_count()
    got = make_outputs(h, w, depth.device, normal=True, residual=True)
    for name, t in got.items():   # stale contents the call must overwrite
        t.fill_(0xAB if t.dtype == torch.uint8 else 7.0)
    ctx.fit_noalloc(depth, K, got, params=p)
    torch.cuda.synchronize()
    n_got = ctx.last_refit_count()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    got = {k: v.cpu().numpy() for k, v in got.items()}
    return ref, got, n_ref, n_got


def test_noalloc_equals_qc_fit_on_two_calls_then_refuses_oversize():
    import torch
    from paper_1707_00385_amd import _lib
    from paper_1707_00385_amd.api import Context, make_outputs, upload_depth
    assert torch.cuda.is_available()
    ctx = Context(0)
    try:
        # first call: the headline frame (640x480 u16, r = 7, T = 5, MIXED)
        sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=5, config_index=1)
        cam = sc.camera
        K = (cam.fx, cam.fy, cam.cx, cam.cy)
        log("[case] noalloc 640x480 u16 r=7 T=5 mixed")
        ref, got, n_ref, n_got = _fit_both(ctx, upload_depth(sc.depth_u16(), "u16"), K, radius=7, iterations=5)
        assert n_ref > 0 and n_got == n_ref, (n_ref, n_got)
        for k in ref:
            assert np.array_equal(ref[k], got[k], equal_nan=True), k
        log(f"  640x480: {n_got} pixels recomputed in FP64, outputs bit-equal")
        # second call, smaller and ragged: 100x75 f32, r = 3, T = 3
        cam2 = scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0)
        sc2 = scenes.cluttered_scene(cam2, seed_frame=6, config_index=2)
        log("[case] noalloc 100x75 f32 r=3 T=3 mixed")
        ref, got, n_ref, n_got = _fit_both(ctx, upload_depth(sc2.depth_m.astype(np.float32), "f32"),
                                           (cam2.fx, cam2.fy, cam2.cx, cam2.cy), radius=3, iterations=3)
        assert n_got == n_ref, (n_ref, n_got)
        for k in ref:
            assert np.array_equal(ref[k], got[k], equal_nan=True), k
        log(f"  100x75: {n_got} pixels recomputed in FP64, outputs bit-equal")
        # a frame beyond the fixed scratch (4096 x 4096 at 256-pixel tiles) is refused
        big = torch.zeros((4096, 4096), dtype=torch.int16, device="cuda:0")
        out = make_outputs(4096, 4096, big.device)
        with pytest.raises(_lib.QcError) as err:
            ctx.fit_noalloc(big, K, out)
        assert err.value.status == _lib.QC_ERR_TOO_LARGE
    finally:
        ctx.close()
