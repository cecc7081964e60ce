"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the same
seeded inputs, element by element.

Tolerance (relative to the curvature scale max(|k1|, |k2|, 1 m^-1)): 1e-4 on noiseless input, 1e-3 on noisy
input, in k1 and k2 of every pixel whose oracle result is unique at that tolerance (see
tests/helpers.compare).  FP64 mode must agree to 2e-7: its outputs are stored as FP32,
whose rounding alone is up to 2^-24 relative.
"""
import numpy as np
import pytest

from paper_1707_00385_amd import scenes
from tests.helpers import compare, gpu_fit, log, oracle_pair, window_crosses_edge

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1707_00385_amd.api import Context
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


def _run(ctx, name, depth, fmt, cam, radius, iterations, tol, precision="mixed", k=1e-5,
         normal_radius=3, reject=False, stride=1, scene=None, **kw):
    log(f"[case] {name} fmt={fmt} {cam.width}x{cam.height} fx={cam.fx} fy={cam.fy} r={radius} "
        f"T={iterations} {precision}{' reject' if reject else ''}{f' stride={stride}' if stride > 1 else ''}")
    g = gpu_fit(ctx, depth, fmt, cam, radius=radius, iterations=iterations, k=k,
                normal_radius=normal_radius, precision=precision, reject=int(reject), stride=stride)
    o, oa = oracle_pair(depth, fmt, cam, radius, iterations, k, normal_radius=normal_radius,
                        reject=reject, stride=stride)
    edge = window_crosses_edge(scene.surface_id, radius) if scene is not None else None
    return compare(g, o, tol, name, o_alt=oa, edge=edge, **kw), g, o


def test_sphere_on_plane_160x120(ctx):
    """The small workload: sphere r = 0.10 m on a plane, r = 3, T = 3, FP32 metres."""
    for noise, tol in ((False, 1e-4), (True, 1e-3)):
        sc = scenes.sphere_on_plane(noise=noise)
        _run(ctx, f"sphere_on_plane noise={noise}", sc.depth_m, "f32", sc.camera, 3, 3, tol,
             normal_tol=1e-3, residual_tol=1e-2)


def test_fp64_mode_matches_oracle_tightly(ctx):
    """FP64 mode runs the oracle's steps in double precision on the GPU."""
    sc = scenes.cluttered_scene(scenes.Camera(96, 72, 80.0, 80.0, 47.5, 35.5), seed_frame=5,
                                config_index=7)
    _run(ctx, "fp64 clutter", sc.depth_u16(), "u16", sc.camera, 5, 5, 2e-7, precision="fp64",
         normal_tol=2e-7, residual_tol=2e-7)


@pytest.mark.parametrize("fmt", ["u16", "f16", "f32"])
def test_clutter_small_formats(ctx, fmt):
    """Spans several 16x16 tiles and a ragged tail (100x75); noisy input, r = 5, T = 5."""
    cam = scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0)
    sc = scenes.cluttered_scene(cam, seed_frame=3, config_index=8)
    depth = sc.depth_u16() if fmt == "u16" else sc.depth_m
    _run(ctx, f"clutter100x75 {fmt}", depth, fmt, cam, 5, 5, 1e-3)


def test_vga_headline_full_frame(ctx):
    """The headline frame: 640x480 Kinect-like u16, r = 7, T = 5, every pixel."""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=0, config_index=1)
    st, g, o = _run(ctx, "vga u16 noisy", sc.depth_u16(), "u16", sc.camera, 7, 5, 1e-3, scene=sc,
                    normal_tol=1e-3, residual_tol=1e-3)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_vga_headline_frame_at_r10(ctx):
    """The headline scene's first frame at r = 10 (21x21), every pixel.  With the update
    bound of 0.1 window units applied unscaled, one pixel of this frame (row 149, column
    328) was left to FP32 at 2.4 times the tolerance; the bound now tightens as (7/r)^2."""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=0, config_index=1)
    _run(ctx, "vga u16 noisy r=10", sc.depth_u16(), "u16", sc.camera, 10, 5, 1e-3, scene=sc)


def test_vga_noiseless_full_frame(ctx):
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=1, config_index=1, noise=False,
                                dropout=0.0)
    _run(ctx, "vga f32 noiseless", sc.depth_m, "f32", sc.camera, 7, 5, 1e-4, scene=sc,
         normal_tol=1e-4, residual_tol=1e-3)


def test_vga_noiseless_near_singular_initial_normal(ctx):
    """A noiseless frame with a cluster of pixels whose 7x7 normal regression is nearly
    singular (det M / (tr M)^2 = 0.002): FP32 and FP64 place the initial normal differently
    enough to end apart, so these must be recomputed (a determinant bound of 1e-3 left five
    of them at up to 4.6 times the tolerance)."""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=20, config_index=1, noise=False,
                                dropout=0.0)
    _run(ctx, "vga f32 noiseless seed 20", sc.depth_m, "f32", sc.camera, 7, 5, 1e-4, scene=sc)


def test_mixed_at_radius_one_is_fp64(ctx):
    """A 3x3 window (nine samples for six parameters) is fitted in FP64 throughout in MIXED
    (an FP32 fit of this noiseless frame left four pixels just beyond the tolerance that no
    recompute criterion caught): MIXED gives FP64 mode's outputs bit for bit, every valid
    pixel flagged FP64.  (Against the oracle the frame's last column, where a window holds
    as many samples as parameters and the fit interpolates, has no determined answer.)"""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=30, config_index=1, noise=False, dropout=0.0)
    log("[case] vga f32 noiseless r=1 T=3: mixed against fp64 mode")
    gm = gpu_fit(ctx, sc.depth_m, "f32", sc.camera, radius=1, iterations=3, precision="mixed")
    gf = gpu_fit(ctx, sc.depth_m, "f32", sc.camera, radius=1, iterations=3, precision="fp64")
    for k in ("k1", "k2", "normal", "residual", "flags"):
        assert np.array_equal(gm[k], gf[k], equal_nan=True), k
    v = (gm["flags"] & 1) != 0
    assert v.mean() > 0.9 and np.all((gm["flags"][v] & 2) != 0)


@pytest.mark.parametrize("kind", ["tof", "hd"])
def test_sensor_frames_whose_fit_moved_late(ctx, kind):
    """Noisy ToF and 720p frames, every pixel: each holds a pixel whose fit moved 0.2-0.6
    window units in the iteration before the last and that FP32 ends 2-7 times the
    tolerance away from FP64 (recomputed since the update before the last is bounded)."""
    sc = scenes.sensor_frame(kind, seed_frame=0)
    _run(ctx, f"{kind} u16 seed 0", sc.depth_u16(), "u16", sc.camera, 7, 5, 1e-3, scene=sc)


# A camera whose focal lengths differ (pixels 1.2 % taller than wide): back-projection
# divides the row offset by fy and the column offset by fx (Section 3.2, pinhole model).
CAM_VGA_ANISO = scenes.Camera(640, 480, 525.0, 518.9, 319.5, 239.5)


@pytest.mark.parametrize("noise", [False, True])
def test_vga_unequal_focal_lengths_full_frame(ctx, noise):
    """Every pixel of a 640x480 frame with fx != fy: noisy u16 at 1e-3, noiseless f32 at
    1e-4 (a kernel that used fx for the rows would be off by about 1 % in curvature)."""
    sc = scenes.cluttered_scene(CAM_VGA_ANISO, seed_frame=4, config_index=1, noise=noise,
                                dropout=0.02 if noise else 0.0)
    if noise:
        _run(ctx, "vga fx!=fy u16 noisy", sc.depth_u16(), "u16", sc.camera, 7, 5, 1e-3, scene=sc,
             normal_tol=1e-3, residual_tol=1e-3)
    else:
        _run(ctx, "vga fx!=fy f32 noiseless", sc.depth_m, "f32", sc.camera, 7, 5, 1e-4, scene=sc,
             normal_tol=1e-4, residual_tol=1e-3)


@pytest.mark.parametrize("w,h,r", [(1, 1, 1), (5, 3, 2), (17, 16, 3), (33, 31, 18), (1, 40, 3), (40, 1, 3),
                                   (257, 2, 4)])
def test_tiny_and_ragged_images(ctx, w, h, r):
    """Images smaller than a tile or a window, one pixel wide or high (no pixel has the three
    non-collinear neighbours of the initial normal), and 257x2 (17 tiles across, two rows:
    the patch's y curvature is set by two sample rows, so the oracle's own result is set by
    rounding at more pixels than the 1 % a full image allows; they are held to its
    envelope)."""
    cam = scenes.Camera(w, h, 40.0, 40.0, (w - 1) / 2, (h - 1) / 2)
    sc = scenes.cluttered_scene(cam, seed_frame=w * 100 + h, config_index=9, n_objects=3)
    _run(ctx, f"tiny {w}x{h}", sc.depth_m, "f32", cam, r, 4, 1e-3, max_nonunique=0.05 if h == 2 else 0.01)


@pytest.mark.parametrize("fmt", ["f32", "f16"])
def test_non_finite_and_negative_depth_is_missing(ctx, fmt):
    """Float depth samples that are NaN, +-inf, negative or -0 carry no depth (like 0): a
    100x75 clutter frame with 3 % of its samples replaced by such values, against the oracle
    on the same frame with those samples at 0."""
    cam = scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0)
    sc = scenes.cluttered_scene(cam, seed_frame=22, config_index=8)
    dt = np.float32 if fmt == "f32" else np.float16
    depth = sc.depth_m.astype(dt)
    rng = np.random.default_rng([1707_00385, 77])
    pick = rng.random(depth.shape) < 0.03
    bad = np.array([np.nan, np.inf, -np.inf, -1.0, -0.0], dtype=dt)
    depth[pick] = bad[rng.integers(0, bad.size, size=int(pick.sum()))]
    st, g, _ = _run(ctx, f"non-finite {fmt}", depth, fmt, cam, 5, 5, 1e-3, normal_tol=1e-3)
    assert np.all((g["flags"][pick] & 1) == 0)   # a pixel without depth is not fitted


def test_all_invalid_and_zero_iterations(ctx):
    cam = scenes.Camera(40, 30, 40.0, 40.0, 19.5, 14.5)
    z = np.zeros((30, 40), np.float32)
    g = gpu_fit(ctx, z, "f32", cam, radius=3, iterations=5)
    assert (g["flags"] == 0).all() and np.isnan(g["k1"]).all()
    sc = scenes.cluttered_scene(cam, seed_frame=4, config_index=9)
    _run(ctx, "T=0", sc.depth_m, "f32", cam, 3, 0, 1e-4, normal_tol=1e-4)


def test_deterministic_repeat(ctx):
    sc = scenes.cluttered_scene(scenes.Camera(64, 48, 60.0, 60.0, 31.5, 23.5), seed_frame=6,
                                config_index=9)
    a = gpu_fit(ctx, sc.depth_u16(), "u16", sc.camera, radius=4, iterations=5)
    b = gpu_fit(ctx, sc.depth_u16(), "u16", sc.camera, radius=4, iterations=5)
    for key in ("k1", "k2", "normal", "residual", "flags"):
        assert np.array_equal(a[key], b[key], equal_nan=True), key


# ---- rejection variant ("Ours+R": Eq. (11) with R = 2 MSE, Section 3.2.3) ----
# The decisions e^2 < R are discrete: a pixel whose oracle result moves under the
# rounding-level probe (a decision at the bound) counts as non-unique like any other.
# MIXED recomputes in FP64 every pixel with an FP32 decision near the bound.

@pytest.mark.parametrize("fmt", ["u16", "f32"])
def test_reject_clutter_small(ctx, fmt):
    cam = scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0)
    sc = scenes.cluttered_scene(cam, seed_frame=11, config_index=8)
    depth = sc.depth_u16() if fmt == "u16" else sc.depth_m
    st, g, _ = _run(ctx, f"reject clutter100x75 {fmt}", depth, fmt, cam, 5, 5, 1e-3, reject=True,
                    residual_tol=1e-2)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_reject_vga_headline(ctx):
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=2, config_index=1)
    st, g, _ = _run(ctx, "reject vga u16", sc.depth_u16(), "u16", sc.camera, 7, 5, 1e-3, reject=True)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_reject_vga_noiseless_float(ctx):
    """Rejection on a noiseless float frame, every pixel, at the noiseless tolerance.  The
    residuals of its flat regions are at the rounding level of the float depth, where the
    FP32 pass cannot decide e^2 < R as FP64 does: such pixels must be left to FP64 (an
    earlier margin, a fixed 2e-5 of R, left 3,088 of them beyond the tolerance here)."""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=29, config_index=1, noise=False, dropout=0.0)
    # two non-unique pixels at a 0.56 m / 2.63 m depth edge, where the FP64 fit with rejection
    # turns by tens of radians per step, end outside the oracle's envelope in FP64 on the GPU
    st, g, _ = _run(ctx, "reject vga noiseless f32", sc.depth_m, "f32", sc.camera, 7, 5, 1e-4,
                    reject=True, scene=sc, max_outside_at_edges=4)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_reject_hd_edge_on_surfaces(ctx):
    """Rejection on a noisy 1280x720 frame, every pixel: where surfaces are seen edge-on the
    FP64 fit moves far for several iterations while its rejected set changes, and an FP32
    fit that follows a different path must be left to FP64 (earlier criteria left three
    pixels of this frame at 21-408 times the tolerance)."""
    sc = scenes.sensor_frame("hd", seed_frame=0)
    st, g, _ = _run(ctx, "reject hd u16", sc.depth_u16(), "u16", sc.camera, 7, 5, 1e-3, reject=True,
                    scene=sc)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_reject_vga_small_window_few_iterations(ctx):
    """Rejection at r = 3, T = 3 on a noisy VGA frame, every pixel: one of its pixels has a
    first-iteration decision 1.6e-5 of R from the bound in FP64, which FP32 once saw on
    the other side (1,578 times the tolerance)."""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=23, config_index=1)
    st, g, _ = _run(ctx, "reject vga u16 r3 T3", sc.depth_u16(), "u16", sc.camera, 3, 3, 1e-3,
                    reject=True, scene=sc)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_reject_vga_half_precision_input(ctx):
    """Rejection on a noisy VGA frame stored as f16 metres (11-bit samples), every pixel."""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=16, config_index=1)
    st, g, _ = _run(ctx, "reject vga f16", sc.depth_m, "f16", sc.camera, 7, 5, 1e-3, reject=True, scene=sc)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_reject_fp64_mode_tight(ctx):
    sc = scenes.cluttered_scene(scenes.Camera(96, 72, 80.0, 80.0, 47.5, 35.5), seed_frame=12,
                                config_index=7)
    _run(ctx, "reject fp64", sc.depth_u16(), "u16", sc.camera, 5, 5, 2e-7, precision="fp64",
         reject=True, normal_tol=2e-7, residual_tol=2e-7)


def test_reject_changes_results_near_outliers(ctx):
    """The variant is not a no-op: on a noisy scene some fits change, and on pixels far
    from depth edges the two variants stay close (both estimate the same surface)."""
    cam = scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0)
    sc = scenes.cluttered_scene(cam, seed_frame=13, config_index=8)
    a = gpu_fit(ctx, sc.depth_u16(), "u16", cam, radius=5, iterations=5, reject=0)
    b = gpu_fit(ctx, sc.depth_u16(), "u16", cam, radius=5, iterations=5, reject=1)
    both = ((a["flags"] & 1) == 1) & ((b["flags"] & 1) == 1)
    diff = np.abs(a["k1"] - b["k1"])[both]
    assert (diff > 0).mean() > 0.5


# ---- strided ("sparsely sampled") fit window: offsets that are multiples of the stride ----

# (7, 7) is the sparsest window: 3x3 samples for six parameters.  Such a fit is barely
# determined, and a few percent of its pixels move under the rounding-level probe.
@pytest.mark.parametrize("radius,stride,nonunique", [(6, 2, 0.01), (18, 3, 0.01), (7, 7, 0.05)])
def test_strided_window_small(ctx, radius, stride, nonunique):
    cam = scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0)
    sc = scenes.cluttered_scene(cam, seed_frame=14, config_index=8)
    _run(ctx, f"stride clutter100x75 r={radius} s={stride}", sc.depth_u16(), "u16", cam, radius, 5,
         1e-3, stride=stride, residual_tol=1e-2, max_nonunique=nonunique, scene=sc)


def test_strided_paper_patch_vga(ctx):
    """The paper's largest patch, 37x37, sampled every third pixel (13x13 samples), on a
    full headline-like frame."""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=3, config_index=1)
    st, g, _ = _run(ctx, "stride vga 37x37/3", sc.depth_u16(), "u16", sc.camera, 18, 5, 1e-3, stride=3,
                    scene=sc)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_strided_paper_patch_vga_noiseless(ctx):
    """The 37x37 patch sampled every third pixel on a noiseless 640x480 frame, every pixel,
    at the noiseless tolerance 1e-4."""
    sc = scenes.cluttered_scene(scenes.CAM_VGA, seed_frame=1, config_index=1, noise=False,
                                dropout=0.0)
    st, g, _ = _run(ctx, "stride vga 37x37/3 noiseless", sc.depth_m, "f32", sc.camera, 18, 5, 1e-4,
                    stride=3, scene=sc)
    log("  refit fraction", st["refits"] / st["pixels"])


def test_strided_fp64_mode_tight(ctx):
    sc = scenes.cluttered_scene(scenes.Camera(96, 72, 80.0, 80.0, 47.5, 35.5), seed_frame=15,
                                config_index=7)
    _run(ctx, "stride fp64", sc.depth_u16(), "u16", sc.camera, 10, 5, 2e-7, precision="fp64",
         stride=2, normal_tol=2e-7, residual_tol=2e-7)


def test_strided_with_rejection(ctx):
    cam = scenes.Camera(100, 75, 90.0, 90.0, 49.5, 37.0)
    sc = scenes.cluttered_scene(cam, seed_frame=16, config_index=8)
    _run(ctx, "stride+reject", sc.depth_u16(), "u16", cam, 8, 5, 1e-3, stride=2, reject=True)


def test_invalid_arguments_rejected_before_any_launch(ctx):
    """qc_fit checks every argument before it enqueues anything: each malformed frame,
    parameter set or output set returns QC_ERR_INVALID_ARG and leaves the outputs as they
    were; the well-formed call then succeeds."""
    import ctypes
    import torch
    from paper_1707_00385_amd import _lib
    from paper_1707_00385_amd.api import make_frame, make_outputs, make_params, output_struct, upload_depth
    cam = scenes.Camera(48, 40, 50.0, 50.0, 23.5, 19.5)
    sc = scenes.cluttered_scene(cam, seed_frame=5, config_index=9)
    depth = upload_depth(sc.depth_u16(), "u16")
    out = make_outputs(cam.height, cam.width, depth.device, normal=True, residual=True)
    for t in out.values():
        t.fill_(7)
    torch.cuda.synchronize()
    before = {k: v.cpu().numpy().copy() for k, v in out.items()}
    good_f = make_frame(depth, (cam.fx, cam.fy, cam.cx, cam.cy))
    good_p = make_params(radius=3, iterations=3)
    good_o = output_struct(out)

    def call(f, p, o):
        st = torch.cuda.current_stream(depth.device).cuda_stream
        return ctx._lib.qc_fit(ctx._h, ctypes.byref(f), ctypes.byref(p), ctypes.byref(o),
                               ctypes.c_void_p(st))

    def variant(struct, **fields):
        c = type(struct).from_buffer_copy(struct)
        for name, value in fields.items():
            if name in ("fx", "fy", "cx", "cy"):
                setattr(c.K, name, value)
            else:
                setattr(c, name, value)
        return c

    nan, inf = float("nan"), float("inf")
    frames = [dict(pitch_bytes=cam.width * 2 - 2), dict(pitch_bytes=cam.width * 2 + 1),
              dict(width=0), dict(height=-1), dict(format=7), dict(depth=None),
              dict(fx=0.0), dict(fy=-1.0), dict(cx=nan), dict(fx=inf)]
    params = [dict(radius=0), dict(radius=_lib.QC_MAX_RADIUS + 1), dict(normal_radius=0),
              dict(iterations=-1), dict(iterations=65), dict(k=0.0), dict(k=nan),
              dict(depth_scale=0.0), dict(precision=3), dict(tile_width=12), dict(reject=2),
              dict(stride=0), dict(stride=4), dict(cond_max=nan)]
    outputs = [dict(k1=None), dict(k2=None)]
    for fields in frames:
        assert call(variant(good_f, **fields), good_p, good_o) == _lib.QC_ERR_INVALID_ARG, fields
    for fields in params:
        assert call(good_f, variant(good_p, **fields), good_o) == _lib.QC_ERR_INVALID_ARG, fields
    for fields in outputs:
        assert call(good_f, good_p, variant(good_o, **fields)) == _lib.QC_ERR_INVALID_ARG, fields
    torch.cuda.synchronize()
    for k, v in out.items():
        assert np.array_equal(v.cpu().numpy(), before[k]), f"{k} written by a rejected call"
    assert call(good_f, good_p, good_o) == _lib.QC_OK
    torch.cuda.synchronize()
    assert ((out["flags"].cpu().numpy() & 1) == 1).sum() > cam.width * cam.height // 2
