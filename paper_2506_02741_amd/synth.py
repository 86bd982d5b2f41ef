"""Seeded synthetic RGBD inputs shaped like indoor SLAM sequences.

This module is the one input generator shared by the CPU oracle and the HIP
path.  It holds none of the splatting arithmetic: it ray-casts analytic
scenes (an inward-facing room box, yaw-rotated boxes, spheres) in float64
with numpy and returns z-depth, RGB, world->camera poses and pinhole
intrinsics.  Every random number comes from ``numpy.random.default_rng(seed)``.

The scenes stand in for the indoor RGBD sequences the paper evaluates on
(Replica, TUM-RGBD, ScanNet, ScanNet++; Sec. 4): rooms of a few metres,
depth 0.3-6 m, 640x480 and 1200x680 frames, sections of consecutive
keyframes along a smooth camera path.  No dataset item is reproduced.

Conventions
-----------
* Pose: world->camera 3x4 float32 ``[R | t]``; camera x right, y down,
  z forward.  World is z-up.
* Pixel (u, v) = (column, row); its centre is at integer coordinates.
* Depth is z-depth (distance along the optical axis), 0 = invalid.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DEPTH_MIN = 0.3
DEPTH_MAX = 6.0


@dataclasses.dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def as_tuple(self):
        return (self.fx, self.fy, self.cx, self.cy, self.width, self.height)


def camera_for(width: int, height: int) -> Camera:
    """Intrinsics used for the synthetic frames: cx = W/2, cy = H/2 and a
    focal length that keeps the field of view fixed across resolutions
    (525 at 640x480, 262.5 at 320x240, 600 at 1200x680)."""
    f = {(640, 480): 525.0, (320, 240): 262.5, (1200, 680): 600.0}.get(
        (width, height), 525.0 * width / 640.0)
    return Camera(f, f, width / 2.0, height / 2.0, width, height)


# ----------------------------------------------------------------------------
# rigid-body helpers (float64)
# ----------------------------------------------------------------------------

def axis_angle(axis, angle) -> np.ndarray:
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * k + (1 - math.cos(angle)) * (k @ k)


def look_pose(center, forward, up=(0.0, 0.0, 1.0)):
    """Camera-to-world rotation (columns right, down, forward) and centre."""
    f = np.asarray(forward, np.float64)
    f = f / np.linalg.norm(f)
    right = np.cross(f, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    return np.stack([right, down, f], axis=1), np.asarray(center, np.float64)


def w2c_from_c2w(R_c2w, c):
    R = R_c2w.T
    t = -R @ c
    return np.concatenate([R, t[:, None]], axis=1)


def c2w_from_w2c(T):
    T = np.asarray(T, np.float64)
    R = T[:, :3].T
    return R, -R @ T[:, 3]


# ----------------------------------------------------------------------------
# scene description and ray casting
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    room_lo: np.ndarray
    room_hi: np.ndarray
    boxes: list      # (center[3], half[3], yaw)
    spheres: list    # (center[3], radius)
    planes: list     # (z) fronto-parallel planes in camera space (toy scene only)
    surf: np.ndarray  # per-surface texture parameters [n_surf, 8]


def _surface_params(rng, n):
    base = rng.uniform(0.15, 0.95, size=(n, 3))
    cell = rng.uniform(0.2, 0.5, size=(n, 1))
    k = rng.normal(size=(n, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    lam = rng.uniform(0.15, 0.6, size=(n, 1))
    return np.concatenate([base, cell, k, lam], axis=1)


def _hash3(ix, iy, iz, salt):
    h = (ix * 73856093) ^ (iy * 19349663) ^ (iz * 83492791) ^ (salt * 2654435761)
    h = (h ^ (h >> 13)) * 1274126177
    h = h ^ (h >> 16)
    return (h & 0xFFFF).astype(np.float64) / 65535.0


def _value_noise(p, salt, scale=0.1):
    q = p / scale
    i = np.floor(q).astype(np.int64)
    f = q - i
    w = f * f * (3 - 2 * f)
    out = 0.0
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                v = _hash3(i[..., 0] + dx, i[..., 1] + dy, i[..., 2] + dz, salt)
                wx = w[..., 0] if dx else 1 - w[..., 0]
                wy = w[..., 1] if dy else 1 - w[..., 1]
                wz = w[..., 2] if dz else 1 - w[..., 2]
                out = out + v * wx * wy * wz
    return out


def _texture(p, sid, surf):
    """Procedural colour of surface ``sid`` at world points ``p`` [n,3]."""
    prm = surf[sid]
    base, cell, k, lam = prm[:, 0:3], prm[:, 3], prm[:, 4:7], prm[:, 7]
    chk = (np.floor(p[:, 0] / cell) + np.floor(p[:, 1] / cell)
           + np.floor(p[:, 2] / cell)) % 2
    stripes = 0.5 + 0.5 * np.sin(2 * np.pi * np.sum(p * k, axis=1) / lam)
    noise = _value_noise(p, sid.astype(np.int64) + 1)
    col = base * (0.55 + 0.3 * chk[:, None] + 0.15 * stripes[:, None])
    col = col + 0.15 * (noise[:, None] - 0.5)
    return np.clip(col, 0.0, 1.0)


def make_room(seed: int, n_boxes=10, n_spheres=10, size=(5.0, 4.0, 3.0)) -> Scene:
    """A room box of ``size`` metres with yaw-rotated boxes (0.2-1.0 m) on the
    floor and spheres (radius 0.1-0.5 m) at random heights."""
    rng = np.random.default_rng(seed)
    lo = np.zeros(3)
    hi = np.asarray(size, np.float64)
    boxes, spheres = [], []
    for _ in range(n_boxes):
        half = rng.uniform(0.1, 0.5, size=3)
        c = np.array([rng.uniform(lo[0] + 0.6, hi[0] - 0.6),
                      rng.uniform(lo[1] + 0.6, hi[1] - 0.6), half[2]])
        boxes.append((c, half, rng.uniform(0, np.pi)))
    for _ in range(n_spheres):
        r = rng.uniform(0.1, 0.5)
        c = np.array([rng.uniform(lo[0] + 0.6, hi[0] - 0.6),
                      rng.uniform(lo[1] + 0.6, hi[1] - 0.6),
                      rng.uniform(r, hi[2] - r)])
        spheres.append((c, r))
    n_surf = 6 + n_boxes + n_spheres
    return Scene(lo, hi, boxes, spheres, [], _surface_params(rng, n_surf))


def _rows_times(x, M):
    """x[n,3] @ M[3,3] as explicit sums in a fixed order (no BLAS, so the
    result does not depend on library threading)."""
    return np.stack([(x[:, 0] * M[0, j] + x[:, 1] * M[1, j]) + x[:, 2] * M[2, j] for j in range(3)],
                    axis=1)


def ray_cast(scene: Scene, cam: Camera, pose_w2c, with_color=True):
    """Return (depth[H,W] float32 z-depth, rgb[3,H,W] float32 or None, hit_pts)."""
    W, H = cam.width, cam.height
    R_c2w, c = c2w_from_w2c(pose_w2c)
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    d_cam = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones_like(u)], -1)
    d = _rows_times(d_cam.reshape(-1, 3), R_c2w.T)  # world direction, camera-z component 1
    o = np.broadcast_to(c, d.shape)
    n = d.shape[0]
    t_best = np.full(n, np.inf)
    sid = np.full(n, -1, np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        # room box from inside: nearest exit face
        for ax in range(3):
            for face, bound in ((0, scene.room_lo[ax]), (1, scene.room_hi[ax])):
                t = (bound - o[:, ax]) / d[:, ax]
                ok = (t > 0) & np.isfinite(t)
                other = [a for a in range(3) if a != ax]
                p = o + t[:, None] * d
                for a in other:
                    ok &= (p[:, a] >= scene.room_lo[a] - 1e-9) & (p[:, a] <= scene.room_hi[a] + 1e-9)
                better = ok & (t < t_best)
                t_best = np.where(better, t, t_best)
                sid = np.where(better, 2 * ax + face, sid)
        base = 6
        for bi, (bc, half, yaw) in enumerate(scene.boxes):
            Rb = axis_angle((0, 0, 1), yaw)
            ol = _rows_times(o - bc, Rb)
            dl = _rows_times(d, Rb)
            t1 = (-half - ol) / dl
            t2 = (half - ol) / dl
            tmin = np.max(np.minimum(t1, t2), axis=1)
            tmax = np.min(np.maximum(t1, t2), axis=1)
            ok = (tmax >= tmin) & (tmin > 0)
            better = ok & (tmin < t_best)
            t_best = np.where(better, tmin, t_best)
            sid = np.where(better, base + bi, sid)
        base += len(scene.boxes)
        for si, (sc, rad) in enumerate(scene.spheres):
            oc = o - sc
            a = np.sum(d * d, axis=1)
            b = 2 * np.sum(d * oc, axis=1)
            cc = np.sum(oc * oc, axis=1) - rad * rad
            disc = b * b - 4 * a * cc
            t = (-b - np.sqrt(np.maximum(disc, 0))) / (2 * a)
            ok = (disc >= 0) & (t > 0)
            better = ok & (t < t_best)
            t_best = np.where(better, t, t_best)
            sid = np.where(better, base + si, sid)
    hit = np.isfinite(t_best)
    depth = np.where(hit, t_best, 0.0)   # d has camera-z component 1 => t is z-depth
    depth = np.where((depth >= DEPTH_MIN) & (depth <= DEPTH_MAX), depth, 0.0)
    if not with_color:
        return depth.reshape(H, W).astype(np.float32), None, None
    p = o + np.where(hit, t_best, 0)[:, None] * d
    col = np.zeros((n, 3))
    col[hit] = _texture(p[hit], sid[hit], scene.surf)
    return (depth.reshape(H, W).astype(np.float32),
            col.reshape(H, W, 3).transpose(2, 0, 1).astype(np.float32).copy(), p)


def _all_valid(scene, cam, pose, stride=1):
    depth, _, _ = ray_cast(scene, Camera(cam.fx / stride, cam.fy / stride,
                                         cam.cx / stride, cam.cy / stride,
                                         max(cam.width // stride, 1),
                                         max(cam.height // stride, 1)), pose,
                               with_color=False)
    return bool(np.all(depth > 0))


def random_room_pose(scene: Scene, cam: Camera, rng, max_tries=4000):
    """Rejection-sample a camera pose whose every pixel has depth in range
    (checked on a 8x-decimated grid first, then at full resolution)."""
    for _ in range(max_tries):
        c = np.array([rng.uniform(scene.room_lo[0] + 0.5, scene.room_hi[0] - 0.5),
                      rng.uniform(scene.room_lo[1] + 0.5, scene.room_hi[1] - 0.5),
                      rng.uniform(0.9, min(2.0, scene.room_hi[2] - 0.4))])
        yaw = rng.uniform(0, 2 * np.pi)
        pitch = rng.uniform(-0.35, 0.15)
        fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch),
                        math.sin(pitch)])
        T = w2c_from_c2w(*look_pose(c, fwd))
        if not _all_valid(scene, cam, T, stride=8):
            continue
        if _all_valid(scene, cam, T, stride=1):
            return T
    raise RuntimeError("no valid pose found")


def perturb_pose(T, rng, trans=0.01, rot_deg=0.5):
    """Move the camera centre by exactly ``trans`` metres along a random
    direction and rotate it by exactly ``rot_deg`` degrees about a random axis."""
    R_c2w, c = c2w_from_w2c(T)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    ax = rng.normal(size=3)
    dR = axis_angle(ax, math.radians(rot_deg))
    return w2c_from_c2w(dR @ R_c2w, c + trans * d)


def random_walk(scene: Scene, cam: Camera, rng, n, step=0.10, rot_deg=5.0,
                max_tries=400):
    """``n`` poses along a smooth walk: each step translates ``step`` metres
    along a persistent heading and rotates by ``rot_deg`` degrees; steps are
    rejection-sampled so every pixel of every frame stays valid."""
    poses = [random_room_pose(scene, cam, rng)]
    heading = rng.normal(size=3)
    heading[2] *= 0.2
    heading /= np.linalg.norm(heading)
    while len(poses) < n:
        R_c2w, c = c2w_from_w2c(poses[-1])
        for _ in range(max_tries):
            h = heading + 0.3 * rng.normal(size=3) * np.array([1, 1, 0.3])
            h /= np.linalg.norm(h)
            ax = np.array([0, 0, 1.0]) + 0.3 * rng.normal(size=3)
            dR = axis_angle(ax, math.radians(rot_deg) * rng.choice([-1.0, 1.0]))
            T = w2c_from_c2w(dR @ R_c2w, c + step * h)
            if _all_valid(scene, cam, T, 8) and _all_valid(scene, cam, T, 1):
                poses.append(T)
                heading = h
                break
        else:
            raise RuntimeError("random walk stuck")
    return poses


# ----------------------------------------------------------------------------
# frames and workload builders
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Frame:
    cam: Camera
    pose: np.ndarray     # [3,4] float32 world->camera
    depth: np.ndarray    # [H,W] float32
    rgb: np.ndarray      # [3,H,W] float32


def frame(scene, cam, pose) -> Frame:
    d, rgb, _ = ray_cast(scene, cam, pose)
    return Frame(cam, np.asarray(pose, np.float32), d, rgb)


def _frames(scene, jobs, workers=8):
    """frame() over (camera, pose) pairs on a thread pool (same arrays as a
    sequential loop: the ray caster has no BLAS products)."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max(1, workers)) as ex:
        return list(ex.map(lambda a: frame(scene, a[0], a[1]), jobs))


def toy_scene(seed=0, width=64, height=48, f=60.0, n_spheres=3):
    """Toy single view: back plane at 3.5 m plus spheres at 1-2.5 m whose
    projected centres lie in the central 60% of the image; identity pose.
    Returns (Frame, colors[3,H,W]) with per-pixel colours U[0,1]^3."""
    rng = np.random.default_rng(seed)
    cam = Camera(f, f, width / 2.0, height / 2.0, width, height)
    u, v = np.meshgrid(np.arange(width, dtype=np.float64), np.arange(height, dtype=np.float64))
    d = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones_like(u)], -1).reshape(-1, 3)
    t_best = np.full(d.shape[0], 3.5)
    for _ in range(n_spheres):
        z = rng.uniform(1.0, 2.5)
        rad = rng.uniform(0.15, 0.4)
        pu = rng.uniform(0.2 * width, 0.8 * width)
        pv = rng.uniform(0.2 * height, 0.8 * height)
        c = np.array([(pu - cam.cx) / cam.fx * z, (pv - cam.cy) / cam.fy * z, z])
        a = np.sum(d * d, 1)
        b = -2 * ((d[:, 0] * c[0] + d[:, 1] * c[1]) + d[:, 2] * c[2])
        cc = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2] - rad * rad
        disc = b * b - 4 * a * cc
        t = (-b - np.sqrt(np.maximum(disc, 0))) / (2 * a)
        ok = (disc >= 0) & (t > 0) & (t < t_best)
        t_best = np.where(ok, t, t_best)
    depth = t_best.reshape(height, width).astype(np.float32)
    colors = rng.uniform(0, 1, size=(3, height, width)).astype(np.float32)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
    return Frame(cam, pose, depth, colors.copy()), colors


def tracking_workload(seed=1, width=640, height=480, n_boxes=10, n_spheres=10):
    """One keyframe of a synthetic room (every pixel valid) and a new frame
    observed at the keyframe pose, whose initial pose estimate is the true
    pose perturbed by exactly 1 cm and 0.5 degrees."""
    rng = np.random.default_rng(seed)
    scene = make_room(seed, n_boxes, n_spheres)
    cam = camera_for(width, height)
    T = random_room_pose(scene, cam, rng)
    kf = frame(scene, cam, T)
    init = perturb_pose(T, rng).astype(np.float32)
    return dict(scene=scene, keyframe=kf, observed=kf, true_pose=kf.pose, init_pose=init)


def section_workload(seed=2, n_kf=8, width=640, height=480):
    """``n_kf`` keyframes along a smooth random walk in one synthetic room."""
    rng = np.random.default_rng(seed)
    scene = make_room(seed)
    cam = camera_for(width, height)
    poses = random_walk(scene, cam, rng, n_kf)
    return dict(scene=scene, keyframes=_frames(scene, [(cam, T) for T in poses]))


def draw_views(seed, n_total, n_pick, iters):
    """Per iteration, ``n_pick`` distinct keyframe indices drawn uniformly."""
    rng = np.random.default_rng(seed)
    return [sorted(rng.choice(n_total, size=n_pick, replace=False).tolist()) for _ in range(iters)]


RESOLUTIONS = ((320, 240), (640, 480), (1200, 680))


def uneven_workload(seed=3, n_sections=3, kf_per_section=8, n_views=16, workers=8):
    """Sections of keyframes whose resolutions are drawn uniformly from
    320x240 / 640x480 / 1200x680, and views drawn from the keyframes.  The
    frames are ray-cast on `workers` threads (same arrays for any count)."""
    rng = np.random.default_rng(seed)
    scene = make_room(seed)
    jobs = []
    for _ in range(n_sections):
        res = [RESOLUTIONS[i] for i in rng.integers(0, 3, size=kf_per_section)]
        poses = random_walk(scene, camera_for(320, 240), rng, kf_per_section)
        jobs.append(list(zip(res, poses)))
    sections = [_frames(scene, [(camera_for(*wh), T) for wh, T in sec], workers) for sec in jobs]
    views = [int(x) for x in rng.integers(0, n_sections * kf_per_section, size=n_views)]
    return dict(scene=scene, sections=sections, views=views)


def strided_frame(scene, cam: Camera, pose, stride):
    """A full-resolution frame whose depth/RGB are ray-cast only at the
    stride grid (the only pixels a stride-s keyframe ties Gaussians to);
    other pixels hold depth 0."""
    sub = Camera(cam.fx / stride, cam.fy / stride, cam.cx / stride, cam.cy / stride,
                 (cam.width + stride - 1) // stride, (cam.height + stride - 1) // stride)
    d, rgb, _ = ray_cast(scene, sub, pose)
    depth = np.zeros((cam.height, cam.width), np.float32)
    col = np.zeros((3, cam.height, cam.width), np.float32)
    depth[::stride, ::stride] = d[:(cam.height + stride - 1) // stride, :(cam.width + stride - 1) // stride]
    col[:, ::stride, ::stride] = rgb
    return Frame(cam, np.asarray(pose, np.float32), depth, col)


def serving_sections(seed=4, n_unique=3, kf_per_section=10, width=1200, height=680, stride=2):
    """Sections of keyframes at width x height for a stride-s map, each along
    a random walk (validity checked on the stride grid)."""
    rng = np.random.default_rng(seed)
    scene = make_room(seed)
    cam = camera_for(width, height)
    sub = Camera(cam.fx / stride, cam.fy / stride, cam.cx / stride, cam.cy / stride,
                 width // stride, height // stride)
    walks = [random_walk(scene, sub, rng, kf_per_section) for _ in range(n_unique)]
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(8) as ex:
        sections = [list(ex.map(lambda T: strided_frame(scene, cam, T, stride), poses))
                    for poses in walks]
    return dict(scene=scene, sections=sections, cam=cam, stride=stride)
