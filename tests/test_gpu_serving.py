"""GPU tests of the serving loop: frames of mixed sizes and window radii submitted from
host memory are admitted by device memory, batched as they arrive and fitted; each result
must equal, bit for bit, the plain per-frame fit of the same frame alone."""
import threading
import time

import numpy as np
import pytest

from paper_1707_00385_amd import scenes
from tests.helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frames():
    specs = [
        (scenes.Camera(128, 96, 100.0, 100.0, 63.5, 47.5), 3, 5),
        (scenes.Camera(96, 72, 80.0, 80.0, 47.5, 35.5), 7, 5),
        (scenes.Camera(160, 120, 131.25, 131.25, 80.0, 60.0), 11, 3),
        (scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0), 5, 5),
    ]
    out = []
    for i, (cam, r, T) in enumerate(specs):
        sc = scenes.cluttered_scene(cam, seed_frame=60 + i, config_index=4)
        out.append((sc.depth_u16(), cam, r, T))
    return out


def _alone(ctx, depth, cam, r, T, precision="mixed"):
    import torch
    from paper_1707_00385_amd.api import make_outputs, make_params, upload_depth
    t = upload_depth(depth, "u16")
    o = make_outputs(t.shape[0], t.shape[1], t.device, normal=True, residual=True)
    ctx.fit(t, (cam.fx, cam.fy, cam.cx, cam.cy), params=make_params(radius=r, iterations=T, precision=precision),
            out=o)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def _served(c, tensor_of):
    import torch
    from paper_1707_00385_amd.api import device_view
    h, w = c.height, c.width
    res = {"k1": device_view(c.k1, (h, w), torch.float32).cpu().numpy(),
           "k2": device_view(c.k2, (h, w), torch.float32).cpu().numpy()}
    if c.normal:
        res["normal"] = device_view(c.normal, (h, w, 3), torch.float32).cpu().numpy()
    if c.residual:
        res["residual"] = device_view(c.residual, (h, w), torch.float32).cpu().numpy()
    if c.flags:
        res["flags"] = device_view(c.flags, (h, w), torch.uint8).cpu().numpy()
    return res


def _drain(srv, n, timeout_s=60.0):
    got, t0 = [], time.time()
    while len(got) < n:
        got += srv.poll(64, wait_us=20000)
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {n} completions"
    return got


def test_served_results_equal_alone(frames):
    from paper_1707_00385_amd import _lib
    from paper_1707_00385_amd.api import Context, Server, make_params
    ctx_alone = Context(0)
    ref = [_alone(ctx_alone, d, cam, r, T) for d, cam, r, T in frames]
    ctx = Context(0)
    srv = Server(ctx, memory_budget=64 << 20, max_batch=8, max_in_flight=2,
                 outputs=_lib.QC_OUT_NORMAL | _lib.QC_OUT_RESIDUAL | _lib.QC_OUT_FLAGS)
    try:
        tickets = {}
        order = [0, 1, 2, 3, 2, 0, 3, 1, 1, 2, 0, 3]   # every frame several times, interleaved
        for j, i in enumerate(order):
            d, cam, r, T = frames[i]
            t = srv.submit(d, "u16", (cam.fx, cam.fy, cam.cx, cam.cy),
                           make_params(radius=r, iterations=T), tag=i)
            assert t is not None
            tickets[t] = i
            if j % 3 == 2:
                time.sleep(0.002)   # let some batches start while more frames arrive
        done = _drain(srv, len(order))
        log("[case] served", len(done), "frames; stats", srv.stats())
        assert srv.stats()["batches"] >= 2
        for c in done:
            assert c.status == 0 and tickets[c.ticket] == c.tag
            assert c.t_done_ns >= c.t_submit_ns
            got = _served(c, None)
            for key, val in ref[c.tag].items():
                assert np.array_equal(got[key], val, equal_nan=True), (c.tag, key)
            srv.release(c.ticket)
        assert srv.stats()["device_bytes_in_use"] == 0
    finally:
        srv.close()
        ctx.close()
        ctx_alone.close()


def test_admission_waits_for_memory(frames):
    """A budget that holds about one frame at a time: every frame still completes, in
    submission order of admission, and the pool never exceeds the budget."""
    from paper_1707_00385_amd.api import Context, Server, make_params
    d, cam, r, T = frames[2]   # 160x120
    one = d.size * 2 + 2 * d.size * 4 + 3 * 256
    ctx = Context(0)
    srv = Server(ctx, memory_budget=one + 4096, max_batch=8)
    try:
        tickets = []
        for i in range(5):
            t = srv.submit(d, "u16", (cam.fx, cam.fy, cam.cx, cam.cy), make_params(radius=r, iterations=T))
            tickets.append(t)
        seen = []
        t0 = time.time()
        while len(seen) < 5:
            for c in srv.poll(8, wait_us=20000):
                assert c.status == 0
                assert srv.stats()["device_bytes_in_use"] <= one + 4096
                seen.append(c.ticket)
                srv.release(c.ticket)   # frees memory for the next admission
            assert time.time() - t0 < 60
        assert seen == tickets
    finally:
        srv.close()
        ctx.close()


def test_rejects_frames_that_can_never_fit(frames):
    from paper_1707_00385_amd import _lib
    from paper_1707_00385_amd.api import Context, Server, make_params
    d, cam, r, T = frames[2]
    ctx = Context(0)
    srv = Server(ctx, memory_budget=64 * 1024, staging_budget=1 << 20)
    try:
        with pytest.raises(_lib.QcError):
            srv.submit(d, "u16", (cam.fx, cam.fy, cam.cx, cam.cy), make_params(radius=r, iterations=T))
    finally:
        srv.close()
        ctx.close()


def test_mixed_and_fp32_requests_share_the_server(frames):
    """MIXED and FP32 requests interleaved in one server: a batch holds frames of one
    precision, so every request completes with status 0, and each result equals the same
    frame fitted alone at its own precision, bit for bit."""
    from paper_1707_00385_amd import _lib
    from paper_1707_00385_amd.api import Context, Server, make_params
    ctx_alone = Context(0)
    precs = ("mixed", "fp32")
    ref = {(i, p): _alone(ctx_alone, d, cam, r, T, precision=p)
           for i, (d, cam, r, T) in enumerate(frames) for p in precs}
    ctx = Context(0)
    srv = Server(ctx, memory_budget=64 << 20, max_batch=8, max_in_flight=2,
                 outputs=_lib.QC_OUT_NORMAL | _lib.QC_OUT_RESIDUAL | _lib.QC_OUT_FLAGS)
    try:
        jobs = [(i, precs[j % 2]) for j, i in enumerate([0, 1, 2, 3, 1, 0, 3, 2, 2, 3, 0, 1])]
        for j, (i, p) in enumerate(jobs):
            d, cam, r, T = frames[i]
            t = srv.submit(d, "u16", (cam.fx, cam.fy, cam.cx, cam.cy),
                           make_params(radius=r, iterations=T, precision=p), tag=j)
            assert t is not None
        done = _drain(srv, len(jobs))
        log("[case] served mixed precisions", len(done), "frames; stats", srv.stats())
        for c in done:
            assert c.status == 0, (c.tag, c.status)
            got = _served(c, None)
            for key, val in ref[jobs[c.tag]].items():
                assert np.array_equal(got[key], val, equal_nan=True), (jobs[c.tag], key)
            srv.release(c.ticket)
    finally:
        srv.close()
        ctx.close()
        ctx_alone.close()


def test_destroy_returns_with_frames_waiting_for_memory(frames):
    """A budget that holds one frame; three frames submitted and the first completion not
    released: the other two wait for memory that only a release could free.  Destroying
    the server returns (those frames complete as busy) instead of waiting for ever."""
    from paper_1707_00385_amd.api import Context, Server, make_params
    d, cam, r, T = frames[2]   # 160x120
    one = d.size * 2 + 2 * d.size * 4 + 3 * 256
    ctx = Context(0)
    srv = Server(ctx, memory_budget=one + 4096, max_batch=8)
    try:
        for _ in range(3):
            assert srv.submit(d, "u16", (cam.fx, cam.fy, cam.cx, cam.cy), make_params(radius=r, iterations=T))
        first = _drain(srv, 1)
        assert first[0].status == 0
        time.sleep(0.05)
        assert srv.stats()["queued"] == 2
        log("[case] destroy with two frames waiting for memory")
        th = threading.Thread(target=srv.close, daemon=True)
        th.start()
        th.join(30.0)
        assert not th.is_alive(), "qc_server_destroy did not return"
    finally:
        if not srv._h.value:
            ctx.close()
