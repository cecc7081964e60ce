"""Seeded synthetic range images for the quadric-patch curvature path.

This module is the only code shared by the FP64 oracle's tests and the GPU path's
tests and benchmark.  It holds none of the fitting method's arithmetic: it ray-casts
analytic shapes through a pinhole camera (the inverse of back-projection), adds
sensor noise, quantises and drops pixels, and reports the closed-form principal
curvatures of every hit point so that results can be scored against ground truth.

The paper's own dataset (Section 4.1, Table 1) is not available, so these scenes
stand in for it and for real Kinect / ToF sensors (Section 1): spheres, cylinders
and hyperbolic paraboloids over a background plane, with the Kinect-style depth
noise sigma = 1.425e-3 * Z^2 m, millimetre quantisation and random dropout.

Sign convention for the truth (matching the method's normal, Eq. (7), which points
away from the camera): a surface that bulges toward the camera (the visible face of a
sphere or cylinder) has positive curvature.  k1 >= k2 always.

All geometry is FP64 NumPy.  Depth is returned as Z along the optical axis.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 1707_00385

SURF_NONE = -1          # no hit (depth 0)
CAP_BIT = 1 << 20       # surface ids of cylinder end caps carry this bit


@dataclasses.dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def rays(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """Ray directions scaled so that the ray parameter equals the depth Z."""
        u = np.arange(self.width, dtype=np.float64)[None, :]
        v = np.arange(self.height, dtype=np.float64)[:, None]
        dx = np.broadcast_to((u - self.cx) / self.fx, (self.height, self.width))
        dy = np.broadcast_to((v - self.cy) / self.fy, (self.height, self.width))
        dz = np.ones((self.height, self.width))
        return dx, dy, dz


# Camera presets used by the workloads.
CAM_SMALL = Camera(160, 120, 131.25, 131.25, 80.0, 60.0)
CAM_VGA = Camera(640, 480, 525.0, 525.0, 319.5, 239.5)
CAM_HD = Camera(1280, 720, 1050.0, 1050.0, 639.5, 359.5)
CAM_TOF = Camera(512, 424, 365.0, 365.0, 255.5, 211.5)


@dataclasses.dataclass
class Scene:
    """A rendered range image with its ground truth."""
    camera: Camera
    depth_m: np.ndarray          # (H, W) float64 metres after noise (0 = no depth)
    depth_clean_m: np.ndarray    # (H, W) float64 metres before noise (0 = no hit)
    k1_true: np.ndarray          # (H, W) float64, m^-1, NaN where no hit
    k2_true: np.ndarray
    normal_true: np.ndarray      # (H, W, 3) unit normal pointing away from the camera
    surface_id: np.ndarray       # (H, W) int32, SURF_NONE where no hit
    params: dict                 # generator parameters (written into result records)

    def depth_u16(self, scale: float = 1e-3) -> np.ndarray:
        """Depth quantised to integer units of `scale` metres (0 stays 0)."""
        q = np.rint(self.depth_m / scale)
        q = np.clip(q, 0, 65535)
        return q.astype(np.uint16)

    def eval_mask(self, radius: int) -> np.ndarray:
        """Pixels with depth whose whole (2r+1)^2 window lies on one non-cap surface.

        Edges, corners and pixels without depth are excluded from scoring
        (Section 4.1)."""
        sid = self.surface_id
        H, W = sid.shape
        ok = (sid >= 0) & ((sid & CAP_BIT) == 0)
        same = ok & (self.depth_m > 0)   # dropped neighbours are skipped, the centre is not
        pad = np.full((H + 2 * radius, W + 2 * radius), -2, dtype=np.int64)
        pad[radius:radius + H, radius:radius + W] = np.where(ok, sid, -2)
        for dv in range(-radius, radius + 1):
            for du in range(-radius, radius + 1):
                win = pad[radius + dv:radius + dv + H, radius + du:radius + du + W]
                same &= win == sid
        return same


def rng_for(config_index: int, frame_index: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, config_index, frame_index])


# ----------------------------------------------------------------------------
# analytic shapes: each returns (t, k1, k2, normal(3,H,W), is_cap) with t = inf on miss
# ----------------------------------------------------------------------------

def _orient(k1, k2, n, rays):
    """Flip normals to point away from the camera and curvatures to match."""
    dx, dy, dz = rays
    dot = n[0] * dx + n[1] * dy + n[2] * dz
    flip = dot < 0
    n = np.where(flip[None], -n, n)
    k1o = np.where(flip, -k2, k1)
    k2o = np.where(flip, -k1, k2)
    return k1o, k2o, n


def _plane(rays, point, normal):
    dx, dy, dz = rays
    nd = normal[0] * dx + normal[1] * dy + normal[2] * dz
    num = float(np.dot(normal, point))
    with np.errstate(divide="ignore", invalid="ignore"):
        t = num / nd
    t = np.where((t > 0) & np.isfinite(t), t, np.inf)
    shape = dx.shape
    n = np.broadcast_to(np.asarray(normal, dtype=np.float64)[:, None, None], (3,) + shape).copy()
    k = np.zeros(shape)
    k1, k2, n = _orient(k, k, n, rays)
    return t, k1, k2, n, np.zeros(shape, dtype=bool)


def _sphere(rays, centre, radius):
    dx, dy, dz = rays
    c = np.asarray(centre, dtype=np.float64)
    a = dx * dx + dy * dy + dz * dz
    b = -2.0 * (dx * c[0] + dy * c[1] + dz * c[2])
    cc = float(np.dot(c, c) - radius * radius)
    disc = b * b - 4 * a * cc
    with np.errstate(invalid="ignore"):
        sq = np.sqrt(np.maximum(disc, 0.0))
    t0 = (-b - sq) / (2 * a)
    t1 = (-b + sq) / (2 * a)
    t = np.where(t0 > 0, t0, np.where(t1 > 0, t1, np.inf))
    t = np.where(disc > 0, t, np.inf)
    px, py, pz = t * dx - c[0], t * dy - c[1], t * dz - c[2]
    n = np.stack([px, py, pz]) / radius
    # outward normal; seen from outside the visible face bulges toward the camera
    k = np.full(dx.shape, -1.0 / radius)   # curvature w.r.t. the outward normal
    k1, k2, n = _orient(k, k, n, rays)
    return t, k1, k2, n, np.zeros(dx.shape, dtype=bool)


def _cylinder(rays, centre, axis, radius, length):
    """Closed finite cylinder; the end caps are flagged."""
    dx, dy, dz = rays
    c = np.asarray(centre, dtype=np.float64)
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    m = -c
    ma = float(np.dot(m, a))
    da = dx * a[0] + dy * a[1] + dz * a[2]
    dpx, dpy, dpz = dx - da * a[0], dy - da * a[1], dz - da * a[2]
    mpx, mpy, mpz = m[0] - ma * a[0], m[1] - ma * a[1], m[2] - ma * a[2]
    qa = dpx * dpx + dpy * dpy + dpz * dpz
    qb = 2.0 * (dpx * mpx + dpy * mpy + dpz * mpz)
    qc = mpx * mpx + mpy * mpy + mpz * mpz - radius * radius
    disc = qb * qb - 4 * qa * qc
    sq = np.sqrt(np.maximum(disc, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (-qb - sq) / (2 * qa)
    half = 0.5 * length
    h0 = ma + t0 * da
    side_ok = (disc > 0) & (t0 > 0) & (np.abs(h0) <= half) & (qa > 1e-18)
    t_side = np.where(side_ok, t0, np.inf)
    # caps
    t_cap = np.full(dx.shape, np.inf)
    cap_n = np.zeros((3,) + dx.shape)
    for sgn in (-1.0, 1.0):
        with np.errstate(divide="ignore", invalid="ignore"):
            tc = (sgn * half - ma) / da
        px, py, pz = tc * dx - c[0], tc * dy - c[1], tc * dz - c[2]
        ax = px * a[0] + py * a[1] + pz * a[2]
        rx, ry, rz = px - ax * a[0], py - ax * a[1], pz - ax * a[2]
        inside = (rx * rx + ry * ry + rz * rz <= radius * radius) & (tc > 0) & np.isfinite(tc)
        better = inside & (tc < t_cap)
        t_cap = np.where(better, tc, t_cap)
        for i in range(3):
            cap_n[i] = np.where(better, sgn * a[i], cap_n[i])
    use_cap = t_cap < t_side
    t = np.minimum(t_side, t_cap)
    px, py, pz = t * dx - c[0], t * dy - c[1], t * dz - c[2]
    ax = px * a[0] + py * a[1] + pz * a[2]
    side_n = np.stack([px - ax * a[0], py - ax * a[1], pz - ax * a[2]]) / radius
    n = np.where(use_cap[None], cap_n, side_n)
    # outward normal: principal curvatures -1/r (around) and 0 (along the axis)
    k1 = np.where(use_cap, 0.0, 0.0)
    k2 = np.where(use_cap, 0.0, -1.0 / radius)
    k1, k2, n = _orient(k1, k2, n, rays)
    with np.errstate(invalid="ignore"):
        n = np.nan_to_num(n)
    return t, k1, k2, n, use_cap & np.isfinite(t)


def _torus(rays, centre, rot, R, r):
    """Torus with major radius R (centre circle) and minor radius r (tube) around the
    axis rot[:, 2] through `centre`.  The ray/torus intersection is the smallest positive
    real root of a quartic, found from the eigenvalues of its companion matrix and
    polished by Newton steps.  Principal curvatures w.r.t. the outward normal: -1/r across
    the tube and -cos(v)/(R + r cos(v)) along it, v the tube angle (0 on the outer
    equator)."""
    dx, dy, dz = rays
    shape = dx.shape
    c = np.asarray(centre, dtype=np.float64)
    Q = np.asarray(rot, dtype=np.float64)
    d = np.stack([dx.ravel(), dy.ravel(), dz.ravel()], axis=1) @ Q      # ray directions, torus frame
    o = -(Q.T @ c)                                                        # camera origin, torus frame
    t = np.full(d.shape[0], np.inf)
    # rays passing within R + r of the centre can hit
    dn = d / np.linalg.norm(d, axis=1, keepdims=True)
    closest = np.linalg.norm(o[None, :] - (dn @ o)[:, None] * dn, axis=1)
    cand = np.nonzero(closest < R + r)[0]
    if cand.size:
        dd = d[cand]
        a = np.sum(dd * dd, axis=1)
        B = 2.0 * (dd @ o)
        A = float(o @ o) + R * R - r * r
        rxy = dd[:, 0] ** 2 + dd[:, 1] ** 2
        oxy = dd[:, 0] * o[0] + dd[:, 1] * o[1]
        coef = np.stack([a * a, 2 * a * B, B * B + 2 * a * A - 4 * R * R * rxy,
                         2 * A * B - 8 * R * R * oxy,
                         np.full(a.shape, A * A - 4 * R * R * (o[0] ** 2 + o[1] ** 2))], axis=1)
        mon = coef[:, 1:] / coef[:, :1]
        comp = np.zeros((cand.size, 4, 4))
        comp[:, 0, :] = -mon
        comp[:, 1, 0] = comp[:, 2, 1] = comp[:, 3, 2] = 1.0
        roots = np.linalg.eigvals(comp)
        real = np.abs(roots.imag) <= 1e-7 * np.maximum(1.0, np.abs(roots.real))
        tr = np.where(real & (roots.real > 0), roots.real, np.inf)
        tt = tr.min(axis=1)
        ok = np.isfinite(tt)
        for _ in range(4):   # Newton on the quartic
            p4 = (((coef[:, 0] * tt + coef[:, 1]) * tt + coef[:, 2]) * tt + coef[:, 3]) * tt + coef[:, 4]
            dp = ((4 * coef[:, 0] * tt + 3 * coef[:, 1]) * tt + 2 * coef[:, 2]) * tt + coef[:, 3]
            step = np.where(ok & (dp != 0), p4 / np.where(dp != 0, dp, 1.0), 0.0)
            tt = np.where(ok, tt - step, tt)
        t[cand] = tt
    p = o[None, :] + t[:, None] * d
    rho = np.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2)
    ring = np.stack([p[:, 0] / rho * R, p[:, 1] / rho * R, np.zeros_like(rho)], axis=1)
    n_local = (p - ring) / np.linalg.norm(p - ring, axis=1, keepdims=True)
    cosv = (rho - R) / r
    n = (n_local @ Q.T).T.reshape(3, *shape)
    ka = np.full(rho.shape, -1.0 / r)
    kb = -cosv / (R + r * cosv)
    k1 = np.maximum(ka, kb).reshape(shape)
    k2 = np.minimum(ka, kb).reshape(shape)
    k1, k2, n = _orient(k1, k2, n, rays)
    return t.reshape(shape), k1, k2, n, np.zeros(shape, dtype=bool)


def monge_curvatures(fx, fy, fxx, fxy, fyy):
    """Principal curvatures of z = f(x, y) w.r.t. the normal (-f_x, -f_y, 1)/sqrt(W)."""
    Wm = 1.0 + fx * fx + fy * fy
    Hm = ((1 + fy * fy) * fxx - 2 * fx * fy * fxy + (1 + fx * fx) * fyy) / (2 * Wm ** 1.5)
    Km = (fxx * fyy - fxy * fxy) / (Wm * Wm)
    root = np.sqrt(np.maximum(Hm * Hm - Km, 0.0))
    return Hm + root, Hm - root


def _quadric_patch(rays, origin, rot, A, B, C, half_extent):
    """Patch z = A/2 x^2 + B x y + C/2 y^2 (|x|,|y| <= half_extent) in frame (rot, origin).

    rot's columns are the patch's local x, y, z axes in camera coordinates."""
    dx, dy, dz = rays
    Q = np.asarray(rot, dtype=np.float64)
    o = np.asarray(origin, dtype=np.float64)
    # local ray: y(t) = t d' + e'
    dl = [Q[0, i] * dx + Q[1, i] * dy + Q[2, i] * dz for i in range(3)]
    el = [-float(np.dot(Q[:, i], o)) for i in range(3)]
    # f(x, y) - z = 0  ->  alpha t^2 + beta t + gamma = 0
    def quad(x, y, xx, yy):
        return 0.5 * A * x * xx + B * 0.5 * (x * yy + y * xx) + 0.5 * C * y * yy
    alpha = quad(dl[0], dl[1], dl[0], dl[1])
    beta = 0.5 * A * 2 * dl[0] * el[0] + B * (dl[0] * el[1] + dl[1] * el[0]) + 0.5 * C * 2 * dl[1] * el[1] - dl[2]
    gamma = 0.5 * A * el[0] ** 2 + B * el[0] * el[1] + 0.5 * C * el[1] ** 2 - el[2]
    lin = np.abs(alpha) < 1e-14 * (np.abs(beta) + 1e-30)
    disc = beta * beta - 4 * alpha * gamma
    sq = np.sqrt(np.maximum(disc, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        # numerically stable roots
        qq = -0.5 * (beta + np.copysign(sq, beta))
        r0 = np.where(lin, -gamma / beta, qq / alpha)
        r1 = np.where(lin, np.inf, gamma / qq)
    ok_disc = lin | (disc >= 0)
    lo = np.minimum(r0, r1)
    hi = np.maximum(r0, r1)

    def inside(t):
        x = t * dl[0] + el[0]
        y = t * dl[1] + el[1]
        return (t > 0) & np.isfinite(t) & (np.abs(x) <= half_extent) & (np.abs(y) <= half_extent)

    t = np.where(ok_disc & inside(lo), lo, np.where(ok_disc & inside(hi), hi, np.inf))
    x = t * dl[0] + el[0]
    y = t * dl[1] + el[1]
    with np.errstate(invalid="ignore"):
        fx = A * x + B * y
        fy = B * x + C * y
    k1, k2 = monge_curvatures(fx, fy, A, B, C)
    nl = np.stack([-fx, -fy, np.ones_like(fx)]) / np.sqrt(1 + fx * fx + fy * fy)
    n = np.stack([Q[i, 0] * nl[0] + Q[i, 1] * nl[1] + Q[i, 2] * nl[2] for i in range(3)])
    # Monge curvatures are w.r.t. the local +z side; orient to "away from camera"
    k1, k2, n = _orient(k1, k2, n, rays)
    n = np.where(np.isfinite(t)[None], n, 0.0)
    return t, k1, k2, n, np.zeros(dx.shape, dtype=bool)


# ----------------------------------------------------------------------------
# compositing
# ----------------------------------------------------------------------------

def _composite(camera: Camera, shapes, max_depth: float = 10.0):
    rays = camera.rays()
    H, W = camera.height, camera.width
    depth = np.full((H, W), np.inf)
    k1 = np.full((H, W), np.nan)
    k2 = np.full((H, W), np.nan)
    nrm = np.zeros((H, W, 3))
    sid = np.full((H, W), SURF_NONE, dtype=np.int64)
    for idx, fn in enumerate(shapes):
        with np.errstate(all="ignore"):      # misses produce inf/NaN that are masked below
            t, a1, a2, n, cap = fn(rays)
        closer = t < depth
        depth = np.where(closer, t, depth)
        k1 = np.where(closer, a1, k1)
        k2 = np.where(closer, a2, k2)
        nrm = np.where(closer[..., None], np.moveaxis(n, 0, -1), nrm)
        sid = np.where(closer, np.where(cap, idx | CAP_BIT, idx), sid)
    miss = ~np.isfinite(depth) | (depth > max_depth)
    depth = np.where(miss, 0.0, depth)
    k1 = np.where(miss, np.nan, k1)
    k2 = np.where(miss, np.nan, k2)
    nrm = np.where(miss[..., None], 0.0, nrm)
    sid = np.where(miss, SURF_NONE, sid).astype(np.int32)
    return depth, k1, k2, nrm, sid


def _finish(camera, depth_clean, k1, k2, nrm, sid, rng, noise_coeff, noise_power,
            dropout, params) -> Scene:
    depth = depth_clean.copy()
    hit = depth > 0
    if noise_coeff > 0:
        sigma = noise_coeff * depth ** noise_power
        depth = np.where(hit, depth + rng.standard_normal(depth.shape) * sigma, 0.0)
        depth = np.where(depth > 0, depth, 0.0)
    if dropout > 0:
        drop = rng.random(depth.shape) < dropout
        depth = np.where(drop, 0.0, depth)
    return Scene(camera, depth, depth_clean, k1, k2, nrm, sid, params)


def random_rotation(rng) -> np.ndarray:
    """Uniformly random rotation matrix (QR of a Gaussian matrix)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def sphere_on_plane(noise: bool = True, seed_frame: int = 0) -> Scene:
    """160x120 sphere r = 0.10 m centred 0.8 m away on a fronto-parallel plane at 1.0 m.

    Truth k1 = k2 = 10 m^-1 on the sphere and 0 on the plane; Kinect noise on Z."""
    cam = CAM_SMALL
    shapes = [
        lambda r: _plane(r, (0.0, 0.0, 1.0), (0.0, 0.0, 1.0)),
        lambda r: _sphere(r, (0.0, 0.0, 0.8), 0.10),
    ]
    d, k1, k2, n, sid = _composite(cam, shapes)
    rng = rng_for(0, seed_frame)
    params = dict(kind="sphere_on_plane", width=cam.width, height=cam.height,
                  noise="1.425e-3*Z^2" if noise else "none", seed=[SEED_BASE, 0, seed_frame])
    return _finish(cam, d, k1, k2, n, sid, rng, 1.425e-3 if noise else 0.0, 2, 0.0, params)


def cluttered_scene(camera: Camera = CAM_VGA, seed_frame: int = 0, config_index: int = 1,
                    noise: bool = True, dropout: float = 0.02, noise_coeff: float = 1.425e-3,
                    noise_power: int = 2, n_objects: Optional[int] = None) -> Scene:
    """8-16 spheres / cylinders / saddles over a tilted background plane.

    Spheres r ~ U(0.03, 0.2); cylinders r ~ U(0.02, 0.15), random axis, length
    U(0.1, 0.5); saddles z = (x^2 - y^2) / (2R), R ~ U(0.1, 1), half-extent 0.15 m,
    random pose.  Background plane at Z ~ U(0.6, 3.0) with up to 15 degrees of tilt.
    Object centres at depth U(0.4, plane Z) inside the frustum."""
    rng = rng_for(config_index, seed_frame)
    cam = camera
    zp = rng.uniform(0.6, 3.0)
    tilt = math.radians(rng.uniform(-15.0, 15.0))
    az = rng.uniform(0, 2 * math.pi)
    axis = np.array([math.cos(az), math.sin(az), 0.0])
    # rotate e_z about the in-image-plane axis by `tilt`
    ez = np.array([0.0, 0.0, 1.0])
    pn = ez * math.cos(tilt) + np.cross(axis, ez) * math.sin(tilt)
    shapes = [lambda r, pn=pn, zp=zp: _plane(r, (0.0, 0.0, zp), pn)]
    n_obj = int(rng.integers(8, 17)) if n_objects is None else n_objects
    objs = []
    for _ in range(n_obj):
        kind = int(rng.integers(0, 3))
        u = rng.uniform(0, cam.width - 1)
        v = rng.uniform(0, cam.height - 1)
        z = rng.uniform(0.4, zp)
        c = np.array([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z])
        if kind == 0:
            rad = rng.uniform(0.03, 0.2)
            shapes.append(lambda r, c=c, rad=rad: _sphere(r, c, rad))
            objs.append(dict(kind="sphere", centre=c.tolist(), radius=rad))
        elif kind == 1:
            rad = rng.uniform(0.02, 0.15)
            ax = rng.standard_normal(3)
            ax /= np.linalg.norm(ax)
            ln = rng.uniform(0.1, 0.5)
            shapes.append(lambda r, c=c, ax=ax, rad=rad, ln=ln: _cylinder(r, c, ax, rad, ln))
            objs.append(dict(kind="cylinder", centre=c.tolist(), axis=ax.tolist(), radius=rad, length=ln))
        else:
            Rr = rng.uniform(0.1, 1.0)
            rot = random_rotation(rng)
            shapes.append(lambda r, c=c, rot=rot, Rr=Rr:
                          _quadric_patch(r, c, rot, 1.0 / Rr, 0.0, -1.0 / Rr, 0.15))
            objs.append(dict(kind="saddle", centre=c.tolist(), R=Rr))
    d, k1, k2, n, sid = _composite(cam, shapes)
    params = dict(kind="cluttered", width=cam.width, height=cam.height, fx=cam.fx, fy=cam.fy,
                  cx=cam.cx, cy=cam.cy, plane_z=zp, tilt_deg=math.degrees(tilt), objects=objs,
                  noise=f"{noise_coeff}*Z^{noise_power}" if noise else "none",
                  dropout=dropout, seed=[SEED_BASE, config_index, seed_frame])
    return _finish(cam, d, k1, k2, n, sid, rng, noise_coeff if noise else 0.0, noise_power,
                   dropout, params)


def quadric_vertex_scene(A: float, B: float, C: float, rot: np.ndarray, distance: float,
                         size: int = 41, f: float = 525.0, vertex_px: Tuple[float, float] = None,
                         half_extent: float = 0.1, fy: Optional[float] = None
                         ) -> Tuple[Scene, Tuple[int, int]]:
    """A parabolic patch whose vertex sits on a pixel ray, ray-cast exactly.

    `rot` columns give the patch's local axes; its local z axis must point away from
    the camera so that the curvature at the vertex is eig([[A, B], [B, C]]).  The camera
    has focal lengths f (x) and fy (y; default f)."""
    cx = cy = (size - 1) / 2.0
    fy = f if fy is None else fy
    cam = Camera(size, size, f, fy, cx, cy)
    if vertex_px is None:
        vertex_px = (size // 2, size // 2)
    u, v = vertex_px
    origin = np.array([(u - cx) / f * distance, (v - cy) / fy * distance, distance])
    shapes = [lambda r: _quadric_patch(r, origin, rot, A, B, C, half_extent)]
    d, k1, k2, n, sid = _composite(cam, shapes)
    params = dict(kind="quadric_vertex", A=A, B=B, C=C, distance=distance, size=size, f=f, fy=fy)
    sc = Scene(cam, d.copy(), d, k1, k2, n, sid, params)
    return sc, (int(u), int(v))


def plane_scene(normal: Sequence[float], distance: float, camera: Camera) -> Scene:
    """A single infinite plane through (0, 0, distance) with the given normal."""
    nn = np.asarray(normal, dtype=np.float64)
    nn = nn / np.linalg.norm(nn)
    d, k1, k2, n, sid = _composite(camera, [lambda r: _plane(r, (0.0, 0.0, distance), nn)])
    return Scene(camera, d.copy(), d, k1, k2, n, sid, dict(kind="plane", normal=nn.tolist()))


def single_shape_scene(kind: str, camera: Camera, distance: float, radius: float,
                       axis: Sequence[float] = (0.0, 1.0, 0.0), length: float = 10.0) -> Scene:
    """One sphere or cylinder centred on the optical axis (no background)."""
    c = (0.0, 0.0, distance)
    if kind == "sphere":
        fn = lambda r: _sphere(r, c, radius)
    elif kind == "cylinder":
        fn = lambda r: _cylinder(r, c, axis, radius, length)
    else:
        raise ValueError(kind)
    d, k1, k2, n, sid = _composite(camera, [fn])
    return Scene(camera, d.copy(), d, k1, k2, n, sid, dict(kind=kind, radius=radius))


def torus_scene(camera: Camera, distance: float, R: float = 0.10, r: float = 0.03,
                rot: Optional[np.ndarray] = None, noise_sigma: float = 0.0, seed_frame: int = 0,
                background: Optional[float] = None) -> Scene:
    """A torus (Table 1's synthetic torus: R = 100 mm, r = 30 mm) centred on the optical
    axis at `distance`, axis tilted by `rot` (default 60 degrees about x, so both the
    outer and the inner, saddle-shaped side face the camera); optional constant-sigma
    noise on Z and a fronto-parallel background plane."""
    if rot is None:
        a = np.deg2rad(60.0)
        rot = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(a), -np.sin(a)], [0.0, np.sin(a), np.cos(a)]])
    shapes = [lambda rays: _torus(rays, (0.0, 0.0, distance), rot, R, r)]
    if background is not None:
        shapes.append(lambda rays: _plane(rays, (0.0, 0.0, background), (0.0, 0.0, -1.0)))
    d, k1, k2, n, sid = _composite(camera, shapes)
    rng = rng_for(11, seed_frame)
    depth = d.copy()
    if noise_sigma > 0:
        depth = np.where(d > 0, d + rng.standard_normal(d.shape) * noise_sigma, 0.0)
        depth = np.where(depth > 0, depth, 0.0)
    return Scene(camera, depth, d, k1, k2, n, sid,
                 dict(kind="torus", R=R, r=r, distance=distance, noise_sigma=noise_sigma))


def saddle_scene(camera: Camera, distance: float, R: float, rot: np.ndarray,
                 half_extent: float = 0.2) -> Scene:
    """Hyperbolic paraboloid z = (x^2 - y^2) / (2R) with its vertex on the optical axis."""
    o = (0.0, 0.0, distance)
    fn = lambda r: _quadric_patch(r, o, rot, 1.0 / R, 0.0, -1.0 / R, half_extent)
    d, k1, k2, n, sid = _composite(camera, [fn])
    return Scene(camera, d.copy(), d, k1, k2, n, sid, dict(kind="saddle", R=R))


# ----------------------------------------------------------------------------
# frame mixes for the batched and served forms
# ----------------------------------------------------------------------------

SENSOR_KINDS = {
    "tof": (CAM_TOF, 1e-3, 1),       # ToF-like: sigma = 1e-3 * Z
    "vga": (CAM_VGA, 1.425e-3, 2),   # Kinect-like: sigma = 1.425e-3 * Z^2
    "hd": (CAM_HD, 1.425e-3, 2),
}


def sensor_frame(kind: str, seed_frame: int, config_index: int = 3) -> Scene:
    cam, coeff, power = SENSOR_KINDS[kind]
    return cluttered_scene(cam, seed_frame=seed_frame, config_index=config_index,
                           noise=True, noise_coeff=coeff, noise_power=power)


def batch_mix(n_frames: int = 64, seed: int = 0) -> List[dict]:
    """Frame descriptors for the batched form: equal thirds of ToF 512x424, VGA and
    720p frames, window radius from {3, 5, 7, 11}, iterations from {3, 5}."""
    rng = rng_for(3, seed)
    kinds = ["tof", "vga", "hd"]
    out = []
    for i in range(n_frames):
        out.append(dict(kind=kinds[i % 3], radius=int(rng.choice([3, 5, 7, 11])),
                        iterations=int(rng.choice([3, 5])), frame=i))
    return out


def poisson_trace(n_sensors: int, aggregate_fps: float, duration_s: float, seed: int = 0,
                  radius_range: Tuple[int, int] = (3, 11)) -> List[dict]:
    """Seeded Poisson arrivals from several sensors, each with a fixed resolution."""
    rng = rng_for(4, seed)
    kinds = ["tof", "vga", "hd"]
    sensors = [kinds[int(rng.integers(0, 3))] for _ in range(n_sensors)]
    rate = aggregate_fps / n_sensors
    events = []
    for s, kind in enumerate(sensors):
        t = 0.0
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= duration_s:
                break
            events.append(dict(t=t, sensor=s, kind=kind,
                               radius=int(rng.integers(radius_range[0], radius_range[1] + 1)),
                               iterations=5, noise_seed=int(rng.integers(0, 2**31))))
    events.sort(key=lambda e: e["t"])
    return events
