"""GPU tests of the batched form (one persistent launch over many frames, replayed from a
captured HIP graph) and of tile-shape tuning: every frame's outputs must equal, bit for
bit, those of the plain per-frame call, and the plain call must not depend on the tile
shape.  The per-frame call is itself checked against the oracle in test_gpu_parity.py;
one batch is also compared with the oracle directly here."""
import os
import tempfile

import numpy as np
import pytest

from paper_1707_00385_amd import scenes
from tests.helpers import compare, log, oracle_pair

pytestmark = pytest.mark.gpu

KEYS = ("k1", "k2", "normal", "residual", "flags")


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1707_00385_amd.api import Context
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


def _jobs():
    """Uneven frames: sizes, formats, radii 1..18, iterations 0..5, tile widths."""
    specs = [
        (scenes.Camera(96, 72, 80.0, 80.0, 47.5, 35.5), "u16", 3, 3, 8),
        (scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0), "f32", 5, 5, 16),
        (scenes.Camera(64, 48, 60.0, 60.0, 31.5, 23.5), "f16", 7, 5, 32),
        (scenes.Camera(160, 120, 131.25, 131.25, 80.0, 60.0), "u16", 11, 3, 64),
        (scenes.Camera(33, 31, 40.0, 40.0, 16.0, 15.0), "f32", 18, 2, 16),
        (scenes.Camera(17, 16, 40.0, 40.0, 8.0, 7.5), "u16", 1, 4, 0),
        (scenes.Camera(40, 30, 40.0, 40.0, 19.5, 14.5), "f32", 4, 0, 0),
    ]
    out = []
    for i, (cam, fmt, r, T, tw) in enumerate(specs):
        sc = scenes.cluttered_scene(cam, seed_frame=40 + i, config_index=3)
        depth = sc.depth_u16() if fmt == "u16" else sc.depth_m
        out.append((sc, cam, fmt, depth, r, T, tw))
    return out


def _run_single(ctx, depth_t, cam, params):
    import torch
    from paper_1707_00385_amd.api import make_outputs
    o = make_outputs(depth_t.shape[0], depth_t.shape[1], depth_t.device, normal=True, residual=True)
    ctx.fit(depth_t, (cam.fx, cam.fy, cam.cx, cam.cy), params=params, out=o)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def _batch_jobs(jobs):
    from paper_1707_00385_amd.api import make_outputs, make_params, upload_depth
    bj, singles = [], []
    for sc, cam, fmt, depth, r, T, tw in jobs:
        t = upload_depth(depth, fmt)
        p = make_params(radius=r, iterations=T, tile_width=tw)
        o = make_outputs(t.shape[0], t.shape[1], t.device, normal=True, residual=True)
        bj.append((t, (cam.fx, cam.fy, cam.cx, cam.cy), p, o))
    return bj


def _equal(a, b, what):
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), f"{what}: {k} differs"


def test_tile_shape_does_not_change_results(ctx):
    from paper_1707_00385_amd.api import make_params, upload_depth
    sc = scenes.cluttered_scene(scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0), seed_frame=3,
                                config_index=8)
    t = upload_depth(sc.depth_u16(), "u16")
    ref = None
    for tw in (8, 16, 32, 64):
        log(f"[case] tile width {tw}")
        r = _run_single(ctx, t, sc.camera, make_params(radius=5, iterations=5, tile_width=tw))
        if ref is None:
            ref = r
        else:
            _equal(r, ref, f"tile width {tw}")


def test_batch_equals_per_frame_calls(ctx):
    import torch
    jobs = _jobs()
    bj = _batch_jobs(jobs)
    log(f"[case] batch of {len(bj)} uneven frames")
    outs = ctx.fit_batch(bj)
    torch.cuda.synchronize()
    for i, ((t, K, p, _), o) in enumerate(zip(bj, outs)):
        single = _run_single(ctx, t, jobs[i][1], p)
        _equal({k: v.cpu().numpy() for k, v in o.items()}, single, f"frame {i}")


def test_batch_with_rejection_equals_per_frame_calls(ctx):
    """Batches holding rejection-variant items run as per-frame launches: same outputs."""
    import torch
    jobs = _jobs()[:4]
    bj = _batch_jobs(jobs)
    for i, (_, _, p, _) in enumerate(bj):
        p.reject = i % 2
    log(f"[case] batch of {len(bj)} frames, alternate items with rejection")
    outs = ctx.fit_batch(bj)
    torch.cuda.synchronize()
    for i, ((t, K, p, _), o) in enumerate(zip(bj, outs)):
        single = _run_single(ctx, t, jobs[i][1], p)
        _equal({k: v.cpu().numpy() for k, v in o.items()}, single, f"frame {i}")


def test_batch_with_strided_items_equals_per_frame_calls(ctx):
    """Batches holding strided items run as per-frame launches: same outputs."""
    import torch
    jobs = _jobs()[:4]
    bj = _batch_jobs(jobs)
    for i, (_, _, p, _) in enumerate(bj):
        if i % 2 == 0 and p.radius >= 2:
            p.stride = 2
    log(f"[case] batch of {len(bj)} frames, some strided")
    outs = ctx.fit_batch(bj)
    torch.cuda.synchronize()
    for i, ((t, K, p, _), o) in enumerate(zip(bj, outs)):
        single = _run_single(ctx, t, jobs[i][1], p)
        _equal({k: v.cpu().numpy() for k, v in o.items()}, single, f"frame {i}")


def test_batch_graph_replays_match_eager(ctx):
    """The batch runs from a captured graph; replay it several times with the program's
    own GPU work and synchronisations in between, and check every replay."""
    import torch
    jobs = _jobs()[:4]
    bj = _batch_jobs(jobs)
    ref = [_run_single(ctx, t, jobs[i][1], p) for i, (t, K, p, _) in enumerate(bj)]
    for rep in range(4):
        log(f"[case] replay {rep}")
        for _, _, _, o in bj:
            for v in o.values():
                v.fill_(0)
        outs = ctx.fit_batch(bj)
        x = torch.randn(1024, device="cuda:0").sum()   # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(x)
        for i, o in enumerate(outs):
            _equal({k: v.cpu().numpy() for k, v in o.items()}, ref[i], f"replay {rep} frame {i}")


def test_two_batches_in_flight_on_two_streams(ctx):
    import torch
    jobs = _jobs()
    a, b = _batch_jobs(jobs[:3]), _batch_jobs(jobs[3:])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    oa = ctx.fit_batch(a, stream=s1)
    ob = ctx.fit_batch(b, stream=s2)
    torch.cuda.synchronize()
    for (t, K, p, _), o, j in zip(a + b, oa + ob, jobs):
        _equal({k: v.cpu().numpy() for k, v in o.items()}, _run_single(ctx, t, j[1], p), "2 streams")


def test_batch_against_oracle(ctx):
    import torch
    jobs = _jobs()[:3]
    bj = _batch_jobs(jobs)
    outs = ctx.fit_batch(bj)
    torch.cuda.synchronize()
    for (sc, cam, fmt, depth, r, T, tw), o in zip(jobs, outs):
        g = {k: v.cpu().numpy() for k, v in o.items()}
        ref, alt = oracle_pair(depth, fmt, cam, r, T, 1e-5)
        compare(g, ref, 1e-3, f"batch {cam.width}x{cam.height} r={r}", o_alt=alt)


def test_tune_records_and_round_trips(ctx):
    """qc_tune records a tile width and a schedule for the frame's configuration; the
    saved table has one line "width height radius iterations stride reject tile_width
    schedule", loads back, and the older five-field line loads too."""
    from paper_1707_00385_amd import _lib
    from paper_1707_00385_amd.api import make_params, upload_depth
    sc = scenes.cluttered_scene(scenes.Camera(128, 96, 100.0, 100.0, 63.5, 47.5), seed_frame=9,
                                config_index=8)
    t = upload_depth(sc.depth_u16(), "u16")
    K = (sc.camera.fx, sc.camera.fy, sc.camera.cx, sc.camera.cy)
    tw, sched = ctx.tune(t, K, make_params(radius=3, iterations=3), reps=2, with_schedule=True)
    assert tw in (8, 16, 32, 64) and sched in (_lib.QC_PREC_MIXED, _lib.QC_PREC_FP64)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        ctx.tune_save(path)
        line = open(path).read().split()
        assert line == ["128", "96", "3", "3", "1", "0", str(tw), str(sched)]
        ctx.tune_load(path)
        legacy = os.path.join(d, "legacy.txt")
        with open(legacy, "w") as f:
            f.write("64 48 5 5 32\n")
        ctx.tune_load(legacy)
        bad = os.path.join(d, "bad.txt")
        with open(bad, "w") as f:
            f.write("64 48 5 5 1 0 32 1\n")   # schedule FP32 is not a schedule
        with pytest.raises(_lib.QcError):
            ctx.tune_load(bad)


def test_tuned_fp64_schedule_runs_fp64_alone_and_in_batches():
    """A configuration whose recorded schedule is FP64 throughout: a MIXED request with
    tile_width 0 runs every pixel in FP64 (flags say so) and gives the FP64-precision
    request's results bit for bit; in a batch beside ordinary MIXED items each item
    equals its per-frame call."""
    import torch
    from paper_1707_00385_amd import _lib
    from paper_1707_00385_amd.api import Context, make_outputs, make_params, upload_depth
    c = Context(0)
    try:
        cam_a = scenes.Camera(96, 72, 80.0, 80.0, 47.5, 35.5)
        cam_b = scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0)
        ta = upload_depth(scenes.cluttered_scene(cam_a, seed_frame=70, config_index=3).depth_u16(), "u16")
        tb = upload_depth(scenes.cluttered_scene(cam_b, seed_frame=71, config_index=3).depth_u16(), "u16")
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, "tune.txt")
            with open(path, "w") as f:
                f.write("96 72 4 3 1 0 16 2\n")   # 96x72, r = 4, T = 3: FP64 throughout
            c.tune_load(path)
        log("[case] tuned FP64 schedule, per frame and in a batch")
        mixed = make_params(radius=4, iterations=3)
        got = _run_single(c, ta, cam_a, mixed)
        valid = (got["flags"] & _lib.QC_FLAG_VALID) != 0
        assert valid.any() and np.all((got["flags"][valid] & _lib.QC_FLAG_FP64) != 0)
        fp64 = _run_single(c, ta, cam_a, make_params(radius=4, iterations=3, precision="fp64"))
        for k in KEYS:
            assert np.array_equal(got[k], fp64[k], equal_nan=True), k
        jobs = [(ta, cam_a), (tb, cam_b), (ta, cam_a)]
        bj = [(t, (cam.fx, cam.fy, cam.cx, cam.cy), mixed,
               make_outputs(cam.height, cam.width, t.device, normal=True, residual=True)) for t, cam in jobs]
        outs = c.fit_batch(bj)
        torch.cuda.synchronize()
        for (t, cam), o in zip(jobs, outs):
            single = _run_single(c, t, cam, mixed)
            for k in KEYS:
                assert np.array_equal(o[k].cpu().numpy(), single[k], equal_nan=True), k
    finally:
        c.close()


def test_batches_needing_more_lds_recapture():
    """The batched FP64 pass stages each chunk's tile in LDS sized for the batch's largest
    region, fixed when the slot's graph is captured: a later batch with a larger region
    (r = 18, 64-wide tiles: 100 x 40 samples) must be captured again, and batches with
    small regions after it must still be right.  Every item equals its per-frame call."""
    import torch
    from paper_1707_00385_amd.api import Context, make_outputs, make_params, upload_depth
    c = Context(0)
    try:
        cams = [scenes.Camera(90, 70, 80.0, 80.0, 44.5, 34.5), scenes.Camera(130, 50, 90.0, 90.0, 64.5, 24.5)]
        frames = []
        for i, cam in enumerate(cams):
            sc = scenes.cluttered_scene(cam, seed_frame=60 + i, config_index=3)
            frames.append((cam, upload_depth(sc.depth_u16(), "u16")))
        for step, (r, tw) in enumerate(((2, 16), (18, 64), (3, 8), (18, 64), (2, 32))):
            bj = []
            for cam, t in frames:
                p = make_params(radius=r, iterations=3, tile_width=tw)
                bj.append((t, (cam.fx, cam.fy, cam.cx, cam.cy), p,
                           make_outputs(cam.height, cam.width, t.device, normal=True, residual=True)))
            log(f"[case] batch {step}: r={r} tile width {tw}")
            outs = c.fit_batch(bj)
            torch.cuda.synchronize()
            for i, ((t, K, p, _), o) in enumerate(zip(bj, outs)):
                single = _run_single(c, t, frames[i][0], p)
                _equal({k: v.cpu().numpy() for k, v in o.items()}, single, f"batch {step} frame {i}")
    finally:
        c.close()


@pytest.mark.parametrize("fmt", ["u16", "f16", "f32"])
def test_pitched_rows_equal_dense_rows(ctx, fmt):
    """A frame whose rows lie `pitch_bytes` apart, with padding between them, gives the
    outputs of the same frame stored densely: per frame in MIXED and FP64 precision, and
    inside a batch.  The padding (an odd number of samples, so the pitch is not a multiple
    of four bytes for u16) holds valid depth, so a read past the last column would change
    the right-hand border pixels."""
    import torch
    from paper_1707_00385_amd.api import make_params, upload_depth
    cam = scenes.Camera(90, 70, 80.0, 80.0, 44.5, 34.5)
    sc = scenes.cluttered_scene(cam, seed_frame=11, config_index=8)
    dense = upload_depth(sc.depth_u16() if fmt == "u16" else sc.depth_m, fmt)
    pad = 5
    padded = torch.empty((cam.height, cam.width + pad), dtype=dense.dtype, device=dense.device)
    padded.fill_(900 if fmt == "u16" else 0.9)
    padded[:, :cam.width].copy_(dense)
    view = padded[:, :cam.width]
    assert view.stride(0) == cam.width + pad and view.stride(1) == 1
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    for precision in ("mixed", "fp64"):
        log(f"[case] pitched rows {fmt} {precision}")
        p = make_params(radius=5, iterations=5, precision=precision)
        a = _run_single(ctx, dense, cam, p)
        b = _run_single(ctx, view, cam, p)
        assert (a["flags"] & 1).sum() > cam.width * cam.height // 2
        _equal(a, b, f"pitched {fmt} {precision}")
    log(f"[case] pitched rows {fmt} in a batch")
    ref = _run_single(ctx, dense, cam, make_params(radius=5, iterations=5))
    outs = ctx.fit_batch([(view, K, make_params(radius=5, iterations=5), None),
                          (dense, K, make_params(radius=3, iterations=3), None)])
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in outs[0].items()}
    for key in ("k1", "k2", "flags"):
        assert np.array_equal(got[key], ref[key], equal_nan=True), f"batched pitched {fmt}: {key}"


def test_two_contexts_on_two_host_threads(ctx):
    """Two contexts, each driven by its own host thread on its own stream, fitting
    different frames at the same time: every result equals the same fit run alone."""
    import threading
    import torch
    from paper_1707_00385_amd.api import Context, make_params, upload_depth
    cams = [scenes.Camera(120, 90, 100.0, 100.0, 59.5, 44.5), scenes.Camera(96, 80, 90.0, 90.0, 47.5, 39.5)]
    work = []
    for i, cam in enumerate(cams):
        sc = scenes.cluttered_scene(cam, seed_frame=30 + i, config_index=8)
        work.append((upload_depth(sc.depth_u16(), "u16"), cam, make_params(radius=4 + i, iterations=5)))
    alone = [_run_single(ctx, t, cam, p) for t, cam, p in work]
    log("[case] two contexts on two host threads")
    results = [[None] * 4 for _ in work]
    errors = []

    def worker(i):
        try:
            t, cam, p = work[i]
            c = Context(0)
            s = torch.cuda.Stream(device=t.device)
            from paper_1707_00385_amd.api import make_outputs
            for rep in range(4):
                o = make_outputs(t.shape[0], t.shape[1], t.device, normal=True, residual=True)
                with torch.cuda.stream(s):
                    c.fit(t, (cam.fx, cam.fy, cam.cx, cam.cy), params=p, out=o, stream=s)
                s.synchronize()
                results[i][rep] = {k: v.cpu().numpy() for k, v in o.items()}
            c.close()
        except Exception as e:  # reported on the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(work))]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not any(th.is_alive() for th in threads), "a worker thread did not finish"
    assert not errors, errors
    for i, reps in enumerate(results):
        for rep, r in enumerate(reps):
            _equal(r, alone[i], f"thread {i} call {rep}")


def test_caller_captured_fit_replays_match_eager(ctx):
    """Once a context holds the scratch a frame size needs, qc_fit only enqueues kernels
    (no allocation, no synchronisation, no memset node), so a caller can capture it in a
    HIP graph.  The graph is replayed over new depth contents, with eager work and
    synchronisations between replays, and every replay equals the eager fit."""
    import torch
    from paper_1707_00385_amd.api import make_outputs, make_params, upload_depth
    cam = scenes.Camera(128, 96, 110.0, 110.0, 63.5, 47.5)
    frames = [scenes.cluttered_scene(cam, seed_frame=40 + i, config_index=8).depth_u16() for i in range(4)]
    p = make_params(radius=5, iterations=5)
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    eager = [_run_single(ctx, upload_depth(f, "u16"), cam, p) for f in frames]
    depth = upload_depth(frames[0], "u16")
    out = make_outputs(cam.height, cam.width, depth.device, normal=True, residual=True)
    ctx.fit(depth, K, params=p, out=out)          # sizes the context's scratch outside the capture
    torch.cuda.synchronize()
    log("[case] caller-captured qc_fit, 3 replays per frame")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            ctx.fit(depth, K, params=p, out=out, stream=side)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        for rep in range(3):
            depth.copy_(upload_depth(f, "u16"))
            for t in out.values():
                t.fill_(3)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            _equal({k: v.cpu().numpy() for k, v in out.items()}, eager[i], f"frame {i} replay {rep}")
