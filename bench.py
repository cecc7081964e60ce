#!/usr/bin/env python3
"""Benchmark of the per-pixel quadric-patch curvature fit on one MI355X.

A step is one frame through the whole fit (qc_fit: FP32 tiled pass + FP64
recomputation of unreliable pixels) at the headline workload: 640x480 Kinect-like u16
depth of a seeded cluttered scene, window 15x15 (r = 7), 5 re-weighted Gauss-Newton
iterations, k = 1e-5 m^2.  Inputs are resident in HBM before timing starts.

Prints one JSON line: throughput in pixels/s, per-frame latency percentiles, the
roofline of the dominant kernel (the FP32 tiled pass, timed with HIP events on the
launch stream) and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WIDTH, HEIGHT, RADIUS, ITERS, NRAD, K_ROBUST = 640, 480, 7, 5, 3, 1e-5
N_FRAMES = 8                 # distinct seeded frames cycled through the timed steps
KERNEL_TIMING_LAUNCHES = 200 # launches of the kernel-timing pass (at least)
FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32 peak (256 CU x 2.4 GHz x 256 flop/clk)
PROFILE_JSON = os.path.join(ROOT, "profiles", "fit_tile_f32_r7_vga_u16_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1707_00385_amd", "csrc", f)
                  for f in ("fit_device.h", "fit_frame.h", "fit_frame.hip", "fit_internal.h")]


def _code_only(text: str) -> str:
    """C++ source without comments, blank lines and differences in spacing, so that a
    comment edit does not count as a change of the kernel."""
    out, i, n = [], 0, len(text)
    while i < n:
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif text[i] in "\"'":
            q, j = text[i], i + 1
            while j < n and text[j] != q:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(text[i])
            i += 1
    lines = [" ".join(line.split()) for line in "".join(out).split("\n")]
    return "\n".join(line for line in lines if line)


def kernel_source_hash() -> str:
    """Hash of the FP32 kernel's code (comments excluded): the stored HBM traffic is used
    only while it matches."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def box_count(valid: np.ndarray, r: int) -> np.ndarray:
    """Number of valid pixels in the (2r+1)^2 window of every pixel (clipped)."""
    v = np.pad(valid.astype(np.int64), r)
    c = np.cumsum(np.cumsum(v, 0), 1)
    c = np.pad(c, ((1, 0), (1, 0)))
    H, W = valid.shape
    n = 2 * r + 1
    return c[n:n + H, n:n + W] - c[0:H, n:n + W] - c[n:n + H, 0:W] + c[0:H, 0:W]


def algorithmic_flops(depth_u16: np.ndarray) -> float:
    """Algorithmic FP work of one frame: per valid pixel T (97 |S| + 250) + 14 |S_n| + 40
    flops, |S| and |S_n| the valid samples of its fit and normal windows (97 flops per
    neighbour and iteration: rotate, residual, weight, Jacobian, 27 accumulations)."""
    valid = depth_u16 > 0
    s = box_count(valid, RADIUS)
    sn = box_count(valid, NRAD)
    f = ITERS * (97.0 * s + 250.0) + 14.0 * sn + 40.0
    return float(f[valid].sum())


def make_frames():
    from paper_1707_00385_amd import scenes
    frames = []
    for i in range(N_FRAMES):
        sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=i, config_index=1)
        frames.append(sc.depth_u16())
    return frames, scenes.CAM_VGA


def cpu_baseline(frame: np.ndarray, cam, budget_s: float = 10.0, served_samples=None) -> dict:
    """The FP64 oracle (test infrastructure) on this host's cores: whole 640x480 frames of
    the same workload, repeated until `budget_s` of wall time has been spent; one thread on
    a band of the same frame; and the small workload (160x120 sphere on a plane, r = 3,
    T = 3) in full.  With `served_samples` (pixels of served frames, see measure_served),
    the oracle also fits those pixels and their error is reported."""
    import oracle
    from oracle.build import LIB
    from paper_1707_00385_amd import scenes
    if not os.path.exists(LIB):
        from oracle.build import build
        build()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    d = frame.astype(np.float64) * np.float64(np.float32(1e-3))
    runs, t0 = 0, time.perf_counter()
    while True:
        oracle.fit_image(d, cam.fx, cam.fy, cam.cx, cam.cy, radius=RADIUS, iterations=ITERS,
                         k=K_ROBUST, normal_radius=NRAD, threads=threads)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    valid = int(np.sum(frame > 0))
    # one thread on a band of the same frame (its rows plus the window's halo)
    r0, r1 = HEIGHT // 2 - 40, HEIGHT // 2 + 40
    band = np.ascontiguousarray(d[r0 - RADIUS:r1 + RADIUS])
    t1 = time.perf_counter()
    oracle.fit_image(band, cam.fx, cam.fy, cam.cx, cam.cy - (r0 - RADIUS), radius=RADIUS,
                     iterations=ITERS, k=K_ROBUST, normal_radius=NRAD, threads=1)
    el1 = time.perf_counter() - t1
    # the small workload: 160x120 FP64 metres, r = 3, T = 3, every pixel
    sm = scenes.sphere_on_plane(noise=True)
    c1 = sm.camera
    n1, t2 = 0, time.perf_counter()
    while True:
        oracle.fit_image(sm.depth_m, c1.fx, c1.fy, c1.cx, c1.cy, radius=3, iterations=3, k=K_ROBUST,
                         normal_radius=NRAD, threads=threads)
        n1 += 1
        el2 = time.perf_counter() - t2
        if el2 >= 1.0:
            break
    res = {"value": runs * valid / el, "unit": "valid pixels/s", "cores": threads, "kind": "oracle",
           "all_pixels_per_s": runs * WIDTH * HEIGHT / el,
           "sample": f"{runs} full 640x480 u16 frames (r=7, T=5), FP64 C + OpenMP, {el:.1f} s",
           "one_core": {"value": band.size / el1, "unit": "pixels/s",
                        "sample": f"rows {r0 - RADIUS}..{r1 + RADIUS - 1} of the first frame, "
                                  f"1 thread, {el1:.2f} s"},
           "small_workload": {"value": n1 * sm.depth_m.size / el2, "unit": "pixels/s",
                              "ms_per_frame": round(1e3 * el2 / n1, 3), "cores": threads,
                              "sample": f"{n1} full 160x120 FP64 frames (sphere r=0.1 m on a plane, "
                                        f"r=3, T=3), {el2:.2f} s"},
           "host_cpu": _cpu_model()}
    if served_samples:
        res["served_oracle_check"] = served_oracle_check(served_samples)
    return res


def served_oracle_check(samples, tol: float = 1e-3) -> dict:
    """The oracle at the sampled pixels of served frames (run by the CPU-baseline leg):
    error of k1/k2 relative to the curvature scale max(|k1|, |k2|, 1 m^-1) against the
    oracle on the same u16 input, over
    pixels the oracle itself gives to within tol/100 under a rounding-level perturbation
    of the depth (the parity tests' rule for pixels determined by their input)."""
    import oracle
    errs, n_nonunique, n_valid_mismatch, frames = [], 0, 0, 0
    for smp in samples:
        d, cam = smp["frame"]
        dm = d.astype(np.float64) * np.float64(np.float32(1e-3))
        kw = dict(radius=smp["radius"], iterations=5, k=float(np.float32(K_ROBUST)), normal_radius=NRAD)
        K = [float(np.float32(x)) for x in (cam.fx, cam.fy, cam.cx, cam.cy)]
        o = oracle.fit_pixels(dm, smp["pixels"], *K, **kw)
        sign = np.random.default_rng([20170703, 1]).choice([-1.0, 1.0], size=dm.shape)
        dp = np.where(dm > 0, dm * (1.0 + sign * 2.0 ** -44), 0.0)
        p = oracle.fit_pixels(dp, smp["pixels"], *K, **kw)
        ov, pv = o["flags"] == 1, p["flags"] == 1
        gv = np.isfinite(smp["k1"])
        def curv_err(a1, a2):
            # relative to the curvature scale max(|k1|, |k2|, 1 m^-1) of the oracle's result
            scale = np.maximum(np.maximum(np.abs(o["k1"]), np.abs(o["k2"])), 1.0)
            return np.maximum(np.abs(a1 - o["k1"]), np.abs(a2 - o["k2"])) / scale
        sens = curv_err(p["k1"], p["k2"])
        unique = ov & pv & (sens <= tol / 100)
        n_nonunique += int(np.sum(ov & ~unique))
        n_valid_mismatch += int(np.sum((gv != ov) & (ov == pv)))
        e = curv_err(smp["k1"].astype(np.float64), smp["k2"].astype(np.float64))
        errs.append(e[unique & gv])
        frames += 1
    e = np.concatenate(errs) if errs else np.zeros(0)
    return {"frames": frames, "pixels_compared": int(e.size), "tolerance": tol,
            "max_rel_err": float(e.max()) if e.size else 0.0,
            "rms_rel_err": float(np.sqrt(np.mean(e ** 2))) if e.size else 0.0,
            "over_tolerance": int(np.sum(e > tol)), "nonunique_skipped": n_nonunique,
            "validity_mismatch": n_valid_mismatch,
            "sampling": f"every 50th frame of the realtime served trace, {SERVED_SAMPLE_PIXELS} seeded pixels each"}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_POOL = {}


def sensor_pool(per_kind: int = 3) -> dict:
    """Rendered u16 frames per sensor kind (ToF 512x424, VGA, 720p), shared by the batched
    and served measurements."""
    from paper_1707_00385_amd import scenes
    if not _POOL:
        for kind in ("tof", "vga", "hd"):
            for j in range(per_kind):
                sc = scenes.sensor_frame(kind, seed_frame=j)
                _POOL[(kind, j)] = (sc.depth_u16(), sc.camera)
    return _POOL


SERVED_SAMPLE_PIXELS = 64   # pixels kept from each sampled served frame


def _served_sample(c, frame, radius) -> dict:
    """k1/k2 of a served frame at seeded pixels with depth, copied to the host before the
    frame's results are released (checked against the oracle in the CPU-baseline leg)."""
    import torch
    from paper_1707_00385_amd.api import device_view
    d, cam = frame
    idx = np.flatnonzero(d.reshape(-1) > 0)
    rng = np.random.default_rng([1707_00385, 50, int(c.tag)])
    px = np.sort(rng.choice(idx, size=min(SERVED_SAMPLE_PIXELS, idx.size), replace=False))
    h, w = c.height, c.width
    k1 = device_view(c.k1, (h * w,), torch.float32).cpu().numpy()[px]
    k2 = device_view(c.k2, (h * w,), torch.float32).cpu().numpy()[px]
    return {"tag": int(c.tag), "radius": int(radius), "pixels": px, "k1": k1, "k2": k2, "frame": frame}


def tune_for_sensors(ctx, reps: int = 3) -> list:
    """Records, on `ctx`, qc_tune's tile width and schedule for every (sensor kind, window
    radius 3..11, T = 5) configuration the served trace draws from, on the first rendered
    frame of each kind; returns the table.  The served and the plain path then share it."""
    from paper_1707_00385_amd.api import make_params, upload_depth
    table = []
    for (kind, j), (d, cam) in sorted(sensor_pool().items()):
        if j != 0:
            continue
        t = upload_depth(d, "u16")
        K = (cam.fx, cam.fy, cam.cx, cam.cy)
        for r in range(3, 12):
            tw, sched = ctx.tune(t, K, make_params(radius=r, iterations=5), reps=reps, with_schedule=True)
            table.append({"sensor": kind, "radius": r, "tile_width": tw,
                          "schedule": {0: "mixed", 2: "fp64"}.get(sched, str(sched))})
    return table


def measure_served(ctx, duration_s: float = 4.0, fps: float = 240.0, sensors: int = 6,
                   saturated: bool = True, warm_up: bool = True, sample_every: int = 0,
                   samples: list = None) -> dict:
    """The serving form on a seeded Poisson trace (sensors with fixed resolutions, per-frame
    window radius 3..11, T = 5) and in a saturating run (the whole trace queued at once),
    against the plain path (one qc_fit per frame in arrival order, one frame in flight).
    Latency is completion time minus the frame's scheduled arrival (the start of the run
    when saturated), on both paths.  With sample_every = n, every n-th frame of the
    realtime served run leaves a sample of its results in `samples`."""
    import threading
    import torch
    from paper_1707_00385_amd import scenes
    from paper_1707_00385_amd.api import Server, make_outputs, make_params, upload_depth
    pool = sensor_pool()
    trace = scenes.poisson_trace(sensors, fps, duration_s, seed=0)
    samples = samples if samples is not None else []
    params = {r: make_params(radius=r, iterations=5) for r in range(3, 12)}
    frames = [pool[(e["kind"], i % 3)] for i, e in enumerate(trace)]
    total_px = sum(d.size for d, _ in frames)

    def served(realtime: bool, sample_every: int = 0) -> dict:
        srv = Server(ctx, memory_budget=2 << 30, max_batch=32, max_in_flight=2)
        lat, t_first, t_last = [], None, 0.0
        arrivals = {}
        base = time.perf_counter()
        state = {"fed": 0}

        def feed():
            for i, e in enumerate(trace):
                if realtime:
                    delay = base + e["t"] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                d, cam = frames[i]
                # the frame's arrival is its scheduled time, as for the plain path: a
                # submission refused while the pinned staging is full waits on its clock
                arrivals[i] = base + e["t"] if realtime else base
                while True:
                    t = srv.submit(d, "u16", (cam.fx, cam.fy, cam.cx, cam.cy), params[e["radius"]], tag=i)
                    if t is not None:
                        break
                    time.sleep(0.0002)
                state["fed"] += 1

        th = threading.Thread(target=feed)
        th.start()
        done = 0
        while done < len(trace):
            for c in srv.poll(64, wait_us=2000):
                now = time.perf_counter()
                lat.append(1e3 * (now - arrivals[c.tag]))
                t_last = now
                if sample_every and c.tag % sample_every == 0 and c.status == 0:
                    samples.append(_served_sample(c, frames[c.tag], trace[c.tag]["radius"]))
                srv.release(c.ticket)
                done += 1
        th.join()
        st = srv.stats()
        srv.close()
        span = t_last - base
        return {"pixels_per_s": round(total_px / span, 1), "frames": len(trace),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "batches": st["batches"],
                "wall_s": round(span, 3)}

    def plain(realtime: bool) -> dict:
        lat = []
        outs = {}
        base = time.perf_counter()
        for i, e in enumerate(trace):
            if realtime:
                delay = base + e["t"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            arrival = base + e["t"] if realtime else base
            d, cam = frames[i]
            t = upload_depth(d, "u16")
            key = d.shape
            if key not in outs:
                outs[key] = make_outputs(d.shape[0], d.shape[1], t.device, flags=False)
            ctx.fit(t, (cam.fx, cam.fy, cam.cx, cam.cy), params=params[e["radius"]], out=outs[key])
            torch.cuda.synchronize()
            lat.append(1e3 * (time.perf_counter() - arrival))
        span = time.perf_counter() - base
        return {"pixels_per_s": round(total_px / span, 1), "frames": len(trace),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "wall_s": round(span, 3)}

    def progress(name, r):
        print(f"[served trace] {fps:.0f} frames/s, {duration_s:.0f} s: {name} done "
              f"(p50 {r['p50_ms']} ms, p99 {r['p99_ms']} ms)", file=sys.stderr, flush=True)
        return r

    if warm_up:
        plain(False)   # warm-up of every radius variant
    res = {"trace": f"{sensors} sensors, Poisson arrivals {fps:.0f} frames/s aggregate over "
                    f"{duration_s:.0f} s (seeded), 512x424 ToF / 640x480 / 1280x720 u16, "
                    f"r in 3..11, T=5, {len(trace)} frames",
           "served_realtime": progress("served realtime", served(True, sample_every)),
           "plain_realtime": progress("plain realtime", plain(True))}
    if saturated:
        res["served_saturated"] = progress("served saturated", served(False))
        res["plain_saturated"] = progress("plain saturated", plain(False))
    return res


def measure_batched(ctx, reps: int = 5, tune_reps: int = 3, tune: bool = True) -> dict:
    """The batched form: 64 frames in equal thirds of 512x424 ToF-like, 640x480 and
    1280x720 depth, window radius from {3, 5, 7, 11}, iterations from {3, 5} (seeded), fitted
    by one qc_fit_batch call (persistent launches replayed from a graph) and, for
    comparison, by 64 qc_fit calls; first with the default tile width (16) and schedule
    (MIXED), then on a second context after qc_tune has recorded a tile width and schedule
    for each (size, radius, iterations) of the mix (the table is saved with qc_tune_save
    and loaded back, as a deployment would).  Three rendered frames per sensor kind are
    shared by the 64 items; every item has its own outputs."""
    import tempfile
    import torch
    from paper_1707_00385_amd import scenes
    from paper_1707_00385_amd.api import Context, make_outputs, make_params, upload_depth
    mix = scenes.batch_mix(64, seed=0)
    pool = {k: (upload_depth(d, "u16"), cam) for k, (d, cam) in sensor_pool().items()}
    jobs, pixels = [], 0
    configs = {}
    for i, m in enumerate(mix):
        t, cam = pool[(m["kind"], i % 3)]
        p = make_params(radius=m["radius"], iterations=m["iterations"])
        o = make_outputs(t.shape[0], t.shape[1], t.device, flags=False)
        jobs.append((t, (cam.fx, cam.fy, cam.cx, cam.cy), p, o))
        pixels += t.shape[0] * t.shape[1]
        configs.setdefault((m["kind"], m["radius"], m["iterations"]), (t, (cam.fx, cam.fy, cam.cx, cam.cy), p))

    def timed(c):
        c.fit_batch(jobs)
        for t, K, p, o in jobs:
            c.fit(t, K, params=p, out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c.fit_batch(jobs)
        torch.cuda.synchronize()
        t_batch = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            for t, K, p, o in jobs:
                c.fit(t, K, params=p, out=o)
        torch.cuda.synchronize()
        t_single = (time.perf_counter() - t0) / reps
        return {"batched": {"ms_per_batch": round(1e3 * t_batch, 3), "pixels_per_s": round(pixels / t_batch, 1)},
                "per_frame_launches": {"ms_per_batch": round(1e3 * t_single, 3),
                                       "pixels_per_s": round(pixels / t_single, 1)},
                "speedup": round(t_single / t_batch, 3)}

    res = {"frames": len(jobs), "pixels_per_batch": pixels}
    res.update(timed(ctx))
    res["mix"] = ("64 frames: 1/3 each 512x424 ToF (sigma=1e-3 Z), 640x480 and 1280x720 "
                  "Kinect-like u16; r in {3,5,7,11}, T in {3,5}, seeded")
    if not tune:
        return res
    tuned_ctx = Context(0)
    try:
        t0 = time.perf_counter()
        table = []
        for (kind, r, T), (t, K, p) in sorted(configs.items()):
            tw, sched = tuned_ctx.tune(t, K, p, reps=tune_reps, with_schedule=True)
            table.append({"sensor": kind, "size": f"{t.shape[1]}x{t.shape[0]}", "radius": r, "iterations": T,
                          "tile_width": tw, "schedule": {0: "mixed", 2: "fp64"}.get(sched, str(sched))})
        tune_s = time.perf_counter() - t0
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, "tune.txt")
            tuned_ctx.tune_save(path)
            fresh = Context(0)
            try:
                fresh.tune_load(path)
                tuned = timed(fresh)
            finally:
                fresh.close()
    finally:
        tuned_ctx.close()
    res["tuned"] = dict(tuned, tuning_seconds=round(tune_s, 2), table=table,
                        speedup_over_untuned_batch=round(res["batched"]["ms_per_batch"] /
                                                         tuned["batched"]["ms_per_batch"], 3))
    return res


def measure_served_headline(ctx, frames, cam, n: int = 400) -> dict:
    """The headline workload through the serving loop: n host frames (the 8 headline frames
    cycled, 640x480 u16, r = 7, T = 5) submitted at once, batched by the server (up to 32
    per batch, two in flight), against n plain per-frame fits of the same device-resident
    frames one after another on one stream.  The served rate includes the uploads from
    pinned host staging; the plain rate does not."""
    import torch
    from paper_1707_00385_amd.api import Server, make_outputs, make_params, upload_depth
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    p = make_params(radius=RADIUS, iterations=ITERS, k=K_ROBUST, normal_radius=NRAD)
    valid = [int(np.sum(f > 0)) for f in frames]

    def served() -> float:
        srv = Server(ctx, memory_budget=2 << 30, max_batch=32, max_in_flight=2)
        try:
            t0 = time.perf_counter()
            submitted = done = failed = 0
            while done < n:
                while submitted < n:
                    if srv.submit(frames[submitted % N_FRAMES], "u16", K, p, tag=submitted) is None:
                        break
                    submitted += 1
                for c in srv.poll(64, wait_us=500):
                    failed += c.status != 0
                    srv.release(c.ticket)
                    done += 1
            return time.perf_counter() - t0, failed
        finally:
            srv.close()

    served()   # warm-up (graphs, staging)
    t_served, failed = served()
    dev = [upload_depth(f, "u16") for f in frames]
    out = make_outputs(cam.height, cam.width, dev[0].device, flags=False)
    for i in range(20):
        ctx.fit(dev[i % N_FRAMES], K, params=p, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n):
        ctx.fit(dev[i % N_FRAMES], K, params=p, out=out)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    px = sum(valid[i % N_FRAMES] for i in range(n))
    return {"frames": n, "failed": failed, "served": {"ms_per_frame": round(1e3 * t_served / n, 4),
                                                      "valid_pixels_per_s": round(px / t_served, 1)},
            "plain": {"ms_per_frame": round(1e3 * t_plain / n, 4), "valid_pixels_per_s": round(px / t_plain, 1)},
            "ratio": round(t_plain / t_served, 3)}


def measure_precision_modes(ctx, dev, K, steps: int = 100) -> dict:
    """The headline frames in the other two precision modes: FP64 throughout (every pixel
    fitted in double precision) and FP32 only (no recomputation, so unreliable pixels keep
    their FP32 fit and flag) -- the cost of the precision form's choices."""
    import torch
    from paper_1707_00385_amd.api import make_outputs, make_params
    out = make_outputs(HEIGHT, WIDTH, dev[0].device, flags=False)
    res = {}
    for prec in ("fp64", "fp32"):
        params = make_params(radius=RADIUS, iterations=ITERS, k=K_ROBUST, normal_radius=NRAD,
                             precision=prec)
        for i in range(10):
            ctx.fit(dev[i % N_FRAMES], K, params=params, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ctx.fit(dev[i % N_FRAMES], K, params=params, out=out)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[prec] = {"ms_per_frame": round(1e3 * wall / steps, 4),
                     "pixels_per_s": round(steps * WIDTH * HEIGHT / wall, 1)}
    return res


def measure_rejection(ctx, dev, K, precision: str, steps: int = 100) -> dict:
    """The rejection variant ("Ours+R": Eq. (11) with R = 2 MSE) on the headline frames:
    per-frame fits as in the headline measurement, plus its FP64 recomputation share."""
    import torch
    from paper_1707_00385_amd.api import make_outputs, make_params
    params = make_params(radius=RADIUS, iterations=ITERS, k=K_ROBUST, normal_radius=NRAD,
                         precision=precision, reject=1)
    out = make_outputs(HEIGHT, WIDTH, dev[0].device, flags=False)
    for i in range(10):
        ctx.fit(dev[i % N_FRAMES], K, params=params, out=out)
    torch.cuda.synchronize()
    ctx.get_timing(reset=True)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for i in range(steps):
        ctx.fit(dev[i % N_FRAMES], K, params=params, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_timing(False)
    timing = ctx.get_timing(reset=True)
    refits = []
    for i in range(N_FRAMES):
        ctx.fit(dev[i], K, params=params, out=out)
        refits.append(ctx.last_refit_count())
    calls = max(timing["calls"], 1)
    return {"ms_per_frame": round(1e3 * wall / steps, 4),
            "pixels_per_s": round(steps * WIDTH * HEIGHT / wall, 1),
            "kernels_ms": {"fit_fp32": round(timing["fit_ms"] / calls, 4),
                           "refit_fp64": round(timing["refit_ms"] / calls, 4)},
            "refit_fraction": round(float(np.mean(refits)) / (WIDTH * HEIGHT), 5),
            "workload": "headline frames, reject=1 (R = 2 x unweighted MSE of the window)"}


# The paper's timing table (Section 4, one Tesla K40c; iterations and k not given, 37x37
# "sparsely sampled" with the stride not given): ms per frame, quoted as context.
PAPER_GRID_MS = {(640, 480): (10.2, 16.1, 19.3), (512, 424): (6.7, 12.2, 13.2),
                 (320, 240): (2.5, 4.5, 5.0)}
PAPER_PATCHES = ((4, 1, "9x9"), (10, 1, "21x21"), (18, 3, "37x37 every 3rd pixel (13x13 samples)"))


def measure_paper_grid(ctx, steps: int = 50, tune: bool = True) -> list:
    """The paper's timing grid on this GPU: three image sizes x three patches (T = 5), one
    seeded cluttered u16 frame per size, per-frame launches: MIXED with the default tile
    width, FP64 throughout, and MIXED after qc_tune (on a context of its own) has recorded
    the cell's tile width and schedule."""
    import torch
    from paper_1707_00385_amd import scenes
    from paper_1707_00385_amd.api import Context, make_outputs, make_params, upload_depth
    cams = {(640, 480): scenes.CAM_VGA, (512, 424): scenes.CAM_TOF,
            (320, 240): scenes.Camera(320, 240, 262.5, 262.5, 159.5, 119.5)}
    rows = []
    tuned_ctx = Context(0)
    try:
        for (w, h), cam in cams.items():
            sc = scenes.cluttered_scene(cam, seed_frame=0, config_index=10)
            t = upload_depth(sc.depth_u16(), "u16")
            K = (cam.fx, cam.fy, cam.cx, cam.cy)
            out = make_outputs(h, w, t.device, flags=False)
            for j, (r, stride, label) in enumerate(PAPER_PATCHES):
                def timed(c, p):
                    for _ in range(5):
                        c.fit(t, K, params=p, out=out)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(steps):
                        c.fit(t, K, params=p, out=out)
                    torch.cuda.synchronize()
                    return 1e3 * (time.perf_counter() - t0) / steps
                p = make_params(radius=r, iterations=ITERS, k=K_ROBUST, stride=stride)
                ms = timed(ctx, p)
                ctx.fit(t, K, params=p, out=out)
                refit = ctx.last_refit_count() / (w * h)
                ms64 = timed(ctx, make_params(radius=r, iterations=ITERS, k=K_ROBUST, stride=stride,
                                              precision="fp64"))
                row = {"image": f"{w}x{h}", "patch": label, "radius": r, "stride": stride,
                       "ms_per_frame": round(ms, 4), "pixels_per_s": round(w * h / ms * 1e3, 1),
                       "refit_fraction": round(refit, 4), "fp64_mode_ms_per_frame": round(ms64, 4),
                       "paper_k40c_ms": PAPER_GRID_MS[(w, h)][j]}
                if tune:
                    tw, sched = tuned_ctx.tune(t, K, p, reps=5, with_schedule=True)
                    row["tuned"] = {"tile_width": tw, "schedule": {0: "mixed", 2: "fp64"}.get(sched, str(sched)),
                                    "ms_per_frame": round(timed(tuned_ctx, p), 4)}
                rows.append(row)
    finally:
        tuned_ctx.close()
    return rows


def _fit_gpu(ctx, depth_m, cam, radius, stride=1):
    import torch
    from paper_1707_00385_amd.api import upload_depth
    t = upload_depth(depth_m.astype(np.float32), "f32")
    out = ctx.fit(t, (cam.fx, cam.fy, cam.cx, cam.cy), radius=radius, iterations=ITERS,
                  k=K_ROBUST, stride=stride, normal=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _rms(x):
    return float(np.sqrt(np.mean(np.square(x)))) if x.size else float("nan")


def pca_normals(depth_m: np.ndarray, cam, r: int) -> np.ndarray:
    """Normal of the least-variance direction of the back-projected points in each
    (2r+1)^2 window (the usual PCA normal; missing depth skipped), facing away from the
    camera.  A comparison baseline, computed on the host."""
    dx, dy, _ = cam.rays()
    valid = depth_m > 0
    P = np.stack([dx * depth_m, dy * depth_m, depth_m], -1) * valid[..., None]
    def box(a):
        pad = np.pad(a, [(r + 1, r)] + [(r + 1, r)] + [(0, 0)] * (a.ndim - 2))
        c = pad.cumsum(0).cumsum(1)
        n = 2 * r + 1
        return c[n:, n:] - c[:-n, n:] - c[n:, :-n] + c[:-n, :-n]
    N = box(valid.astype(np.float64)[..., None])[..., 0]
    S1 = box(P)
    S2 = box(np.einsum("hwi,hwj->hwij", P, P).reshape(*P.shape[:2], 9)).reshape(*P.shape[:2], 3, 3)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = S1 / N[..., None]
        cov = S2 / N[..., None, None] - np.einsum("hwi,hwj->hwij", mean, mean)
    cov = np.where(np.isfinite(cov), cov, 0.0)
    _, vec = np.linalg.eigh(cov)
    n = vec[..., :, 0]
    ray = np.stack([dx, dy, np.ones_like(dx)], -1)
    return np.where((np.sum(n * ray, -1) < 0)[..., None], -n, n)


def _angle_deg(a, b):
    c = np.clip(np.sum(a * b, -1) / (np.linalg.norm(a, axis=-1) * np.linalg.norm(b, axis=-1)), -1, 1)
    return np.degrees(np.arccos(c))


def measure_accuracy(ctx) -> dict:
    """Error against the closed-form truth of the synthetic shapes (Section 4): the
    100 mm sphere under increasing noise, refined vs PCA normals on the headline frame,
    and the Table 1 torus (R = 100 mm, r = 30 mm).  MIXED precision, T = 5, k = 1e-5;
    dense 15x15 windows and the 37x37 patch sampled every third pixel."""
    from paper_1707_00385_amd import scenes
    out = {}
    # (1) sphere r = 0.1 m at 0.6 m, constant-sigma noise on Z
    cam = scenes.CAM_VGA
    sph = scenes.single_shape_scene("sphere", cam, 0.6, 0.1)
    rng = np.random.default_rng([1707_00385, 20, 0])
    hit = sph.depth_clean_m > 0
    rows = []
    for sigma_mm in (0.0, 0.25, 0.5, 1.0, 2.0):
        d = np.where(hit, sph.depth_clean_m + rng.standard_normal(hit.shape) * sigma_mm * 1e-3, 0.0)
        for radius, stride in ((7, 1), (18, 3)):
            g = _fit_gpu(ctx, d, cam, radius, stride)
            m = sph.eval_mask(radius) & ((g["flags"] & 1) == 1)
            err = np.concatenate([g["k1"][m] - 10.0, g["k2"][m] - 10.0])
            rows.append({"sigma_mm": sigma_mm, "window": f"{2 * radius + 1}x{2 * radius + 1}/{stride}",
                         "pixels": int(m.sum()), "rms_err_per_m": round(_rms(err), 5),
                         "mean_k_per_m": round(float(np.mean(np.concatenate([g["k1"][m], g["k2"][m]]))), 5)})
    out["sphere_100mm_noise_sweep"] = {"truth_per_m": 10.0, "distance_m": 0.6, "rows": rows,
                                       "paper_rms_per_m": 0.037}
    # (2) normals on the headline frame: refined (Section 3.2.4) vs initial vs PCA
    sc = scenes.cluttered_scene(cam, seed_frame=0, config_index=1)
    d = sc.depth_u16().astype(np.float64) * 1e-3
    g = _fit_gpu(ctx, d, cam, RADIUS)
    g0 = None
    import torch
    from paper_1707_00385_amd.api import upload_depth
    t = upload_depth(d.astype(np.float32), "f32")
    o0 = ctx.fit(t, (cam.fx, cam.fy, cam.cx, cam.cy), radius=RADIUS, iterations=0, normal=True)
    torch.cuda.synchronize()
    g0 = o0["normal"].cpu().numpy()
    m = sc.eval_mask(RADIUS) & ((g["flags"] & 1) == 1)
    nt = sc.normal_true
    ang = {"refined_15x15": _angle_deg(g["normal"], nt)[m],
           "initial_7x7_regression": _angle_deg(g0, nt)[m],
           "pca_7x7": _angle_deg(pca_normals(d, cam, 3), nt)[m],
           "pca_15x15": _angle_deg(pca_normals(d, cam, RADIUS), nt)[m]}
    out["normal_angle_deg_headline"] = {
        "pixels": int(m.sum()),
        **{k: {"median": round(float(np.median(v)), 4), "rms": round(_rms(v), 4)} for k, v in ang.items()}}
    # (3) torus R = 0.1 m, r = 0.03 m at 0.6 m, pixels seen within 60 degrees of head-on
    tor_rows = []
    for sigma_mm in (0.0, 1.0):
        tor = scenes.torus_scene(cam, 0.6, noise_sigma=sigma_mm * 1e-3)
        dx, dy, dz = cam.rays()
        ray = np.stack([dx, dy, dz], -1)
        ray /= np.linalg.norm(ray, axis=-1, keepdims=True)
        cos_t = np.abs(np.sum(ray * tor.normal_true, -1))
        for radius, stride in ((7, 1), (18, 3)):
            g = _fit_gpu(ctx, tor.depth_m, cam, radius, stride)
            m = tor.eval_mask(radius) & (cos_t >= 0.5) & ((g["flags"] & 1) == 1)
            err = np.concatenate([g["k1"][m] - tor.k1_true[m], g["k2"][m] - tor.k2_true[m]])
            tor_rows.append({"sigma_mm": sigma_mm, "window": f"{2 * radius + 1}x{2 * radius + 1}/{stride}",
                             "pixels": int(m.sum()), "rms_err_per_m": round(_rms(err), 4)})
    out["torus_100_30mm"] = {"rows": tor_rows, "paper_rms_per_m": 0.63}
    return out


def copy_calibration(nbytes: int) -> int:
    """Ten device-to-device copies of a known size: the HBM read/write counters of these
    dispatches give the scale factor between counter readings and bytes moved."""
    import torch
    n = nbytes // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "copies": 10}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-reject", action="store_true")
    ap.add_argument("--no-paper-grid", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-precision-modes", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip qc_tune in the timing grid, the batched form and the served trace "
                         "(their untuned figures only; for profiling runs)")
    ap.add_argument("--trace-seconds", type=float, default=0.0,
                    help="length of every served trace (default: 60 s at 240 frames/s, 10 s at "
                         "1000 frames/s, 3 s at the lower rates)")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run 10 plain device copies of BYTES bytes (calibrates the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the fit shards by frame with no inter-GPU traffic, "
              f"and several GPUs are not measured by this script (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        return 2

    import torch
    from paper_1707_00385_amd.api import Context, make_outputs, make_params, upload_depth

    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)

    frames, cam = make_frames()
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    dev = [upload_depth(f, "u16") for f in frames]
    flops = [algorithmic_flops(f) for f in frames]
    ctx = Context(0)
    params = make_params(radius=RADIUS, iterations=ITERS, k=K_ROBUST, normal_radius=NRAD,
                         precision=args.precision)
    out = make_outputs(HEIGHT, WIDTH, dev[0].device, flags=False)
    stream = torch.cuda.current_stream()

    # Untimed: 0.2 s of the same fits before the warm-up steps.  The GPU's clocks ramp over
    # the first ~25 ms of sustained load: with 5 warm-up steps alone, 20 timed steps read
    # 0.73 instead of 0.65 ms per step (40 or more warm-up steps: 0.65).
    t_prime = time.perf_counter() + 0.2
    while time.perf_counter() < t_prime:
        for i in range(N_FRAMES):
            ctx.fit(dev[i], K, params=params, out=out)
        torch.cuda.synchronize()
    for i in range(args.warmup):
        ctx.fit(dev[i % N_FRAMES], K, params=params, out=out)
    torch.cuda.synchronize()
    # the timed steps: plain per-frame fits, kernel timing off (nothing but the launches)
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.fit(dev[i % N_FRAMES], K, params=params, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    valid_px = [int(np.sum(f > 0)) for f in frames]
    value = sum(valid_px[i % N_FRAMES] for i in range(args.steps)) / wall
    flops_per_step = float(np.mean([flops[i % N_FRAMES] for i in range(args.steps)]))

    # kernel durations: a separate pass of the same fits with HIP events recorded around
    # the FP32 pass and the FP64 recomputation on the launch stream (events from a pool
    # created beforehand, so a call only records them)
    n_kt = max(args.steps, KERNEL_TIMING_LAUNCHES)
    ctx.set_timing(True)
    ctx.get_timing(reset=True)
    for i in range(n_kt):
        ctx.fit(dev[i % N_FRAMES], K, params=params, out=out)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    timing = ctx.get_timing(reset=True)

    # refit fraction over the distinct frames
    refits = []
    for i in range(N_FRAMES):
        ctx.fit(dev[i], K, params=params, out=out)
        refits.append(ctx.last_refit_count())

    # per-frame latency: enqueue to completion, one frame at a time
    lat = []
    for i in range(args.latency_frames):
        s = time.perf_counter()
        ctx.fit(dev[i % N_FRAMES], K, params=params, out=out)
        stream.synchronize()
        lat.append(1e3 * (time.perf_counter() - s))
    lat = np.array(lat)

    fit_ms = timing["fit_ms"] / max(timing["calls"], 1)
    refit_ms = timing["refit_ms"] / max(timing["calls"], 1)
    flops_per_launch = float(np.mean([flops[i % N_FRAMES] for i in range(n_kt)]))
    achieved = flops_per_launch / (fit_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(PROFILE_JSON):
        with open(PROFILE_JSON) as f:
            prof = json.load(f)
        if prof.get("kernel_source_hash") == kernel_source_hash():
            traffic = prof.get("hbm_bytes_per_launch")
    end_to_end = flops_per_step / (ms_per_step * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": traffic, "kernel": "fit_tile_f32<7, false, false>",
                "kernel_ms": round(fit_ms, 4), "kernel_launches_timed": int(timing["calls"]),
                "algorithmic_gflop_per_launch": round(flops_per_launch / 1e9, 3),
                "end_to_end_tflops": round(end_to_end, 3),
                "end_to_end_frac": round(end_to_end / FP32_PEAK_TFLOPS, 4)}

    result = {
        "metric": "curvature pixels/s @640x480 r=7, served vs plain; p50/p99 frame latency",
        "value": round(value, 1),
        "unit": "valid pixels/s",
        "all_pixels_per_s": round(args.steps * WIDTH * HEIGHT / wall, 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else args.precision.replace("fp", "f"),
        "data": "synthetic",
        "config": {"workload": "plain per-frame fit, 640x480 u16 Kinect-like cluttered scene "
                               "(sigma=1.425e-3 Z^2, 2% dropout), r=7 (15x15), T=5, k=1e-5, "
                               f"precision={args.precision}",
                   "width": WIDTH, "height": HEIGHT, "radius": RADIUS, "iterations": ITERS,
                   "frames_cycled": N_FRAMES},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "mode": "plain, one frame in flight"},
        "kernels_ms": {"fit_fp32": round(fit_ms, 4), "refit_fp64": round(refit_ms, 4)},
        "refit_fraction": round(float(np.mean(refits)) / (WIDTH * HEIGHT), 5),
        "roofline": roofline,
    }
    if args.precision == "mixed" and not args.no_precision_modes:
        result["precision_modes"] = measure_precision_modes(ctx, dev, K)
    if not args.no_reject:
        result["rejection_variant"] = measure_rejection(ctx, dev, K, args.precision)
    if not args.no_paper_grid and args.precision == "mixed":
        result["paper_timing_grid"] = measure_paper_grid(ctx, tune=not args.no_tune)
    if not args.no_accuracy and args.precision == "mixed":
        result["accuracy"] = measure_accuracy(ctx)
    if not args.no_batched and args.precision != "fp64":
        result["batched_form"] = measure_batched(ctx, tune=not args.no_tune)
    served_samples = []
    if not args.no_served and args.precision == "mixed":
        result["served_headline"] = measure_served_headline(ctx, frames, cam)
    if not args.no_served and args.precision != "fp64":
        # the serving configuration: tile widths and schedules tuned for every sensor kind
        # and radius of the trace (shared by the served and the plain path), a 60 s realtime
        # trace at 240 frames/s (every 50th served frame sampled for the oracle check of
        # the CPU-baseline leg), then the same trace queued at once (saturated)
        t_tune = time.perf_counter()
        tuned = tune_for_sensors(ctx) if not args.no_tune else []
        t_tune = time.perf_counter() - t_tune
        sv = measure_served(ctx, duration_s=args.trace_seconds or 60.0, sample_every=50,
                            samples=served_samples)
        if tuned:
            sv["tuned"] = {"seconds": round(t_tune, 2), "table": tuned}
        result["served_form"] = sv
        result["served_vs_plain"] = {
            "saturated_throughput_ratio": round(sv["served_saturated"]["pixels_per_s"] /
                                                sv["plain_saturated"]["pixels_per_s"], 3),
            "realtime_p99_ms": {"served": sv["served_realtime"]["p99_ms"],
                                "plain": sv["plain_realtime"]["p99_ms"]}}
        # latency against load: the same sensors at lower aggregate rates, and near the
        # plain path's saturation
        sweep = []
        for fps, dur in ((30.0, 3.0), (60.0, 3.0), (120.0, 3.0), (240.0, None), (1000.0, 10.0)):
            lv = sv if dur is None else measure_served(ctx, duration_s=args.trace_seconds or dur, fps=fps,
                                                       saturated=False, warm_up=False)
            sweep.append({"fps": fps, "seconds": round(args.trace_seconds or dur or 60.0, 1),
                          "frames": lv["served_realtime"]["frames"],
                          "served_p50_ms": lv["served_realtime"]["p50_ms"],
                          "served_p99_ms": lv["served_realtime"]["p99_ms"],
                          "served_pixels_per_s": lv["served_realtime"]["pixels_per_s"],
                          "plain_p50_ms": lv["plain_realtime"]["p50_ms"],
                          "plain_p99_ms": lv["plain_realtime"]["p99_ms"],
                          "plain_pixels_per_s": lv["plain_realtime"]["pixels_per_s"]})
        result["served_load_sweep"] = sweep
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(frames[0], cam, served_samples=served_samples)
    print(json.dumps(result), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
