"""ctypes wrapper around ``liboracle.so`` (plain single-threaded C).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  Each function
cites the part of the paper it follows; the arithmetic lives in
``oracle.c``.  Arrays are numpy; the wrapper only marshals them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")

# Renderer constants (readings of what the paper leaves open):
# alpha_min 1/255, alpha_max 0.99, t_min 1e-4, Q_CUT = 2 ln 255 rounded up,
# near plane 0.01 m, low-pass 0.3 px^2, black background, tile 16.
DEFAULTS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, q_cut=11.0826,
                z_near=0.01, lowpass=0.3, bg=(0.0, 0.0, 0.0), tile=16)


SO_OMP = os.path.join(HERE, "liboracle_omp.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall"]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc -O2 -ffp-contract=off (no fast-math): the
    single-threaded reference, and the same source with OpenMP for the
    all-cores timing."""
    src = os.path.join(HERE, "oracle.c")
    hdr = os.path.join(HERE, "oracle.h")
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    for so, extra in ((SO, []), (SO_OMP, ["-fopenmp"])):
        if force or not os.path.exists(so) or os.path.getmtime(so) < newest:
            tmp = so + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc"] + CFLAGS + extra + ["-shared", "-fPIC", "-o", tmp, src,
                                                               "-lm"])
            os.replace(tmp, so)
    return SO


class Cam(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class KF(C.Structure):
    _fields_ = [("n", C.c_int32), ("pix", C.c_void_p), ("depth", C.c_void_p),
                ("color", C.c_void_p), ("opacity", C.c_void_p), ("radius", C.c_void_p),
                ("pose", C.c_void_p), ("cam", Cam)]


class View(C.Structure):
    _fields_ = [("cam", Cam), ("pose", C.c_void_p), ("kf_first", C.c_int32),
                ("kf_count", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("q_cut", C.c_float), ("z_near", C.c_float), ("lowpass", C.c_float),
                ("bg", C.c_float * 3), ("tile", C.c_int32)]


class Rec(C.Structure):
    _fields_ = [("px", C.c_float), ("py", C.c_float), ("pz", C.c_float),
                ("mx", C.c_float), ("my", C.c_float),
                ("qa", C.c_float), ("qb", C.c_float), ("qc", C.c_float),
                ("ext", C.c_float), ("rect", C.c_int32 * 4), ("count", C.c_int32)]


REC_DTYPE = np.dtype([("px", "<f4"), ("py", "<f4"), ("pz", "<f4"), ("mx", "<f4"),
                      ("my", "<f4"), ("qa", "<f4"), ("qb", "<f4"), ("qc", "<f4"),
                      ("ext", "<f4"), ("rect", "<i4", (4,)), ("count", "<i4")])


class Values(C.Structure):
    _fields_ = [("color", C.c_void_p), ("opacity", C.c_void_p), ("radius", C.c_void_p),
                ("twist", C.c_double * 6), ("geometry64", C.c_int32), ("depth", C.c_void_p),
                ("kf_twist", C.c_void_p)]


_libs = {}
_threads = [1]


class threads:
    """Within ``with oracle.threads(n):`` (n > 1) the oracle runs its OpenMP
    build on n threads; otherwise the single-threaded reference."""

    def __init__(self, n):
        self.n = int(n)

    def __enter__(self):
        self.prev = _threads[0]
        _threads[0] = self.n
        if self.n > 1:
            lib().omp_set_num_threads(self.n)
        return self

    def __exit__(self, *exc):
        _threads[0] = self.prev


def lib():
    key = "omp" if _threads[0] > 1 else "serial"
    if key not in _libs:
        build()
        L = C.CDLL(SO_OMP if key == "omp" else SO)
        if key == "omp":
            L.omp_set_num_threads.argtypes = [C.c_int]
        P = C.c_void_p
        L.orc_ingest_count.restype = C.c_int32
        L.orc_ingest_count.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32]
        L.orc_ingest_fill.restype = C.c_int32
        L.orc_ingest_fill.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float,
                                      C.c_float, C.c_int32, P, P, P, P, P]
        L.orc_relpose32.argtypes = [P, P, P]
        L.orc_slice_size.restype = C.c_int32
        L.orc_slice_size.argtypes = [P, P]
        L.orc_preprocess32.restype = C.c_int32
        L.orc_preprocess32.argtypes = [P, P, P, P]
        L.orc_tile_lists.restype = C.c_int64
        L.orc_tile_lists.argtypes = [P, P, P, P, P, P, C.c_int64]
        L.orc_render_fwd.restype = C.c_int
        L.orc_render_fwd.argtypes = [P, P, P, P, C.c_float, C.c_int32, P, P, P, P, P, P, P]
        L.orc_visibility.restype = C.c_int
        L.orc_visibility.argtypes = [P, P, P, C.c_int32, P, P, P, C.c_float, C.c_float, P, P]
        L.orc_render_alt.restype = C.c_int
        L.orc_render_alt.argtypes = [P, P, P, P, C.c_float, C.c_int32, P, C.c_int32, P, P, P, P]
        L.orc_render_bwd.restype = C.c_int
        L.orc_render_bwd.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_track_loss.restype = C.c_double
        L.orc_track_loss.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_double, C.c_double,
                                     C.c_double, P, P]
        L.orc_ssim.restype = C.c_double
        L.orc_ssim.argtypes = [C.c_int32, C.c_int32, P, P, P]
        L.orc_map_loss.restype = C.c_double
        L.orc_map_loss.argtypes = [C.c_int32, C.c_int32, P, P, P, P, C.c_double, C.c_double,
                                   C.c_double, P, P]
        L.orc_se3_exp.argtypes = [P, P]
        L.orc_adam.argtypes = [C.c_int64, P, P, P, P, C.c_int64, C.c_double, C.c_double,
                               C.c_double, C.c_double]
        _libs[key] = L
    return _libs[key]


def _p(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# plain Python containers for keyframes and views
# ----------------------------------------------------------------------------

class Keyframe:
    """Compact view-tied Gaussians of one keyframe (Sec. 3.2)."""

    def __init__(self, cam, pose, pix, depth, color, opacity, radius):
        self.cam = tuple(cam)
        self.pose = _f32(np.asarray(pose).reshape(12))
        self.pix = np.ascontiguousarray(pix, dtype=np.uint32)
        self.depth = _f32(depth)
        self.color = _f32(np.asarray(color).reshape(3, -1))
        self.opacity = _f32(opacity)
        self.radius = _f32(radius)
        self.n = int(self.pix.shape[0])

    def cstruct(self):
        fx, fy, cx, cy, w, h = self.cam
        return KF(self.n, _p(self.pix), _p(self.depth), _p(self.color), _p(self.opacity),
                  _p(self.radius), _p(self.pose), Cam(fx, fy, cx, cy, int(w), int(h)))


class ViewSpec:
    def __init__(self, cam, pose, kf_first=0, kf_count=1):
        self.cam = tuple(cam)
        self.pose = _f32(np.asarray(pose).reshape(12))
        self.kf_first = int(kf_first)
        self.kf_count = int(kf_count)

    @property
    def P(self):
        return int(self.cam[4]) * int(self.cam[5])

    def cstruct(self):
        fx, fy, cx, cy, w, h = self.cam
        return View(Cam(fx, fy, cx, cy, int(w), int(h)), _p(self.pose), self.kf_first,
                    self.kf_count)


def params(**kw):
    d = dict(DEFAULTS)
    d.update(kw)
    return Params(d["alpha_min"], d["alpha_max"], d["t_min"], d["q_cut"], d["z_near"],
                  d["lowpass"], (C.c_float * 3)(*d["bg"]), int(d["tile"]))


def _kf_array(kfs):
    arr = (KF * max(len(kfs), 1))()
    for i, k in enumerate(kfs):
        arr[i] = k.cstruct()
    return arr


def _values(n, color=None, opacity=None, radius=None, twist=None, geometry64=False, depth=None,
            kf_twist=None):
    keep = []
    c = o = r = d = kt = None
    if color is not None:
        c = _f64(np.asarray(color).reshape(3, n)); keep.append(c)
    if opacity is not None:
        o = _f64(opacity); keep.append(o)
    if radius is not None:
        r = _f64(radius); keep.append(r)
    if depth is not None:
        d = _f64(depth); keep.append(d)
    if kf_twist is not None:
        kt = _f64(np.asarray(kf_twist).reshape(-1, 6)); keep.append(kt)
    tw = (C.c_double * 6)(*(twist if twist is not None else (0.0,) * 6))
    return Values(_p(c), _p(o), _p(r), tw, 1 if geometry64 else 0, _p(d), _p(kt)), keep


# ----------------------------------------------------------------------------
# API
# ----------------------------------------------------------------------------

def ingest(depth_img, rgb_img=None, mask=None, stride=1, fx=None, o_init=0.99, cam=None, pose=None):
    """Valid depth pixels on the stride grid -> compact Gaussians; colour from
    the observed RGB, opacity o_init, radius r = stride * D / f (App. A)."""
    L = lib()
    d = _f32(depth_img)
    H, W = d.shape
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    rgb = None if rgb_img is None else _f32(np.asarray(rgb_img).reshape(3, H, W))
    n = L.orc_ingest_count(_p(d), _p(m), H, W, stride)
    pix = np.zeros(n, np.uint32)
    dep = np.zeros(n, np.float32)
    col = np.zeros((3, n), np.float32)
    opa = np.zeros(n, np.float32)
    rad = np.zeros(n, np.float32)
    got = L.orc_ingest_fill(_p(d), _p(rgb), _p(m), H, W, stride, float(fx), float(o_init), n,
                            _p(pix), _p(dep), _p(col), _p(opa), _p(rad))
    assert got == n
    if cam is None:
        return dict(pix=pix, depth=dep, color=col, opacity=opa, radius=rad)
    return Keyframe(cam, pose, pix, dep, col, opa, rad)


def relpose32(Tv, Tk):
    M = np.zeros(12, np.float32)
    lib().orc_relpose32(_p(_f32(np.asarray(Tv).reshape(12))), _p(_f32(np.asarray(Tk).reshape(12))), _p(M))
    return M.reshape(3, 4)


def preprocess32(view, kfs, prm=None):
    """FP32 records of every Gaussian of the view's slice (local-id order)."""
    L = lib()
    prm = prm or params()
    ka = _kf_array(kfs)
    vs = view.cstruct()
    n = L.orc_slice_size(C.byref(vs), ka)
    out = np.zeros(max(n, 1), REC_DTYPE)
    L.orc_preprocess32(C.byref(vs), ka, C.byref(prm), _p(out))
    return out[:n]


def tile_lists(view, kfs, prm=None):
    """Sorted (tile, depth bits) keys, view-local ids and per-tile ranges."""
    L = lib()
    prm = prm or params()
    ka = _kf_array(kfs)
    vs = view.cstruct()
    B = prm.tile
    nt = ((view.cam[4] + B - 1) // B) * ((view.cam[5] + B - 1) // B)
    ranges = np.zeros((nt, 2), np.uint32)
    K = L.orc_tile_lists(C.byref(vs), ka, C.byref(prm), None, None, _p(ranges), 0)
    keys = np.zeros(max(K, 1), np.uint64)
    vals = np.zeros(max(K, 1), np.uint32)
    K2 = L.orc_tile_lists(C.byref(vs), ka, C.byref(prm), _p(keys), _p(vals), _p(ranges), K)
    assert K2 == K
    return keys[:K], vals[:K], ranges


def slice_size(view, kfs):
    return int(sum(k.n for k in kfs[view.kf_first:view.kf_first + view.kf_count]))


def render(view, kfs, prm=None, margin=2e-6, pixels=None, color=None, opacity=None,
           radius=None, twist=None, geometry64=False, depth=None, kf_twist=None):
    """splat({g}, p) -> RGB [3,P], depth [P], silhouette [P]: FP64
    compositing on the FP32 contributor decisions (Sec. 3.3, Eq. 1 / Sec.
    3.4, Eq. 2 inputs).  By default the composited mean, conic and depth are
    those of the pinned FP32 records; geometry64=True recomputes them in FP64
    (a smooth function of the inputs, for finite differences).  ``depth``
    [N] overrides the tied depths and ``kf_twist`` [kf_count, 6] left-twists
    the slice's keyframe poses, both in FP64 (values only: the decisions
    stay those of the keyframes' float data).
    ``pixels`` selects row-major pixel indices (brute force per pixel)."""
    L = lib()
    prm = prm or params()
    ka = _kf_array(kfs)
    vs = view.cstruct()
    N = slice_size(view, kfs)
    val, keep = _values(N, color, opacity, radius, twist, geometry64, depth, kf_twist)
    if pixels is None:
        P, npx, idx = view.P, -1, None
    else:
        idx = np.ascontiguousarray(pixels, dtype=np.int32)
        P, npx = int(idx.shape[0]), int(idx.shape[0])
    rgb = np.zeros((3, P)); dep = np.zeros(P); sil = np.zeros(P); tf = np.zeros(P)
    nc = np.zeros(P, np.int32); mg = np.zeros(P, np.uint8)
    rc = L.orc_render_fwd(C.byref(vs), ka, C.byref(prm), C.byref(val), float(margin), npx,
                          _p(idx), _p(rgb), _p(dep), _p(sil), _p(tf), _p(nc), _p(mg))
    if rc < 0:
        raise MemoryError("oracle render failed")
    return dict(rgb=rgb, depth=dep, sil=sil, t_final=tf, n_contrib=nc, marginal=mg.astype(bool),
                marginal_kind=mg, superset_violations=int(rc))


def render_alternatives(view, kfs, pixels, prm=None, margin=2e-6, max_alt=4, color=None,
                        opacity=None, radius=None, twist=None):
    """The other outcomes of the near-tie decisions of the listed pixels
    (Sec. 3.3 splat; the tie reading of the stop and cut-off rules): for
    pixel i, variant j takes its j-th near-tie decision (candidate tests in
    slice order, then stop decisions front to back) the other way.  Returns
    n_dec [n], rgb [n, max_alt, 3], depth and sil [n, max_alt] (variants
    j >= n_dec[i] are NaN)."""
    L = lib()
    prm = prm or params()
    ka = _kf_array(kfs)
    vs = view.cstruct()
    N = slice_size(view, kfs)
    val, keep = _values(N, color, opacity, radius, twist, False)
    idx = np.ascontiguousarray(pixels, dtype=np.int32)
    n = int(idx.shape[0])
    rgb = np.full((max(n, 1), max_alt, 3), np.nan); dep = np.full((max(n, 1), max_alt), np.nan)
    sil = np.full((max(n, 1), max_alt), np.nan); nd = np.zeros(max(n, 1), np.int32)
    rc = L.orc_render_alt(C.byref(vs), ka, C.byref(prm), C.byref(val), float(margin), n, _p(idx),
                          int(max_alt), _p(rgb), _p(dep), _p(sil), _p(nd))
    if rc < 0:
        raise MemoryError("oracle alternatives failed")
    return dict(n_dec=nd[:n], rgb=rgb[:n], depth=dep[:n], sil=sil[:n])


def render_bwd(view, kfs, g_rgb, g_depth=None, g_sil=None, prm=None, color=None,
               opacity=None, radius=None, twist=None, geometry64=False, depth=None,
               kf_twist=None):
    """Exact derivative of ``render`` (contributor sets fixed) w.r.t. colour,
    opacity, radius of every Gaussian of the slice and the view twist, plus
    (Sec. 3.5 bundle adjustment; the supplementary's Gaussians movable along
    the ray) each Gaussian's tied depth and each slice keyframe's pose twist."""
    L = lib()
    prm = prm or params()
    ka = _kf_array(kfs)
    vs = view.cstruct()
    N = slice_size(view, kfs)
    val, keep = _values(N, color, opacity, radius, twist, geometry64, depth, kf_twist)
    P = view.P
    gr = _f64(np.asarray(g_rgb).reshape(3, P))
    gd = None if g_depth is None else _f64(g_depth)
    gs = None if g_sil is None else _f64(g_sil)
    gc = np.zeros((3, max(N, 1))); go = np.zeros(max(N, 1)); grd = np.zeros(max(N, 1))
    tw = np.zeros(6)
    gkd = np.zeros(max(N, 1)); gkp = np.zeros((max(view.kf_count, 1), 6))
    gkm = np.zeros(N + 6 * max(view.kf_count, 1))
    mag = np.zeros(5 * N + 6)
    rc = L.orc_render_bwd(C.byref(vs), ka, C.byref(prm), C.byref(val), _p(gr), _p(gd), _p(gs),
                          _p(gc), _p(go), _p(grd), _p(tw), _p(mag), _p(gkd),
                          _p(gkp), _p(gkm))
    if rc < 0:
        raise MemoryError("oracle backward failed")
    mags = dict(color=mag[:3 * N].reshape(3, N), opacity=mag[3 * N:4 * N],
                radius=mag[4 * N:5 * N], twist=mag[5 * N:5 * N + 6], depth=gkm[:N],
                kf_pose=gkm[N:N + 6 * view.kf_count].reshape(view.kf_count, 6))
    return dict(color=gc[:, :N], opacity=go[:N], radius=grd[:N], twist=tw, mag=mags,
                depth=gkd[:N], kf_pose=gkp[:view.kf_count])


def visibility(src_depth, src_cam, src_pose, targets, rel_tol=0.01, z_near=0.01):
    """Sec. 3.3 visibility check of a source frame's depth points in target
    views: targets = [(depth [H, W], cam tuple, pose [3, 4])].  Returns
    vis [n_tgt, H*W] bool and counts [n_tgt]."""
    L = lib()
    sd = _f32(np.ravel(src_depth))
    sc = Cam(*src_cam)
    sp = _f32(np.ravel(src_pose))
    n = len(targets)
    depths = [_f32(np.ravel(t[0])) for t in targets]
    poses = [_f32(np.ravel(t[2])) for t in targets]
    dptr = (C.c_void_p * max(n, 1))(*[d.ctypes.data for d in depths])
    pptr = (C.c_void_p * max(n, 1))(*[q.ctypes.data for q in poses])
    cams = (Cam * max(n, 1))(*[Cam(*t[1]) for t in targets])
    P = sd.size
    vis = np.zeros((max(n, 1), P), np.uint8)
    counts = np.zeros(max(n, 1), np.int64)
    L.orc_visibility(_p(sd), C.byref(sc), _p(sp), n, dptr, cams, pptr, float(rel_tol),
                     float(z_near), _p(vis), _p(counts))
    return vis[:n].astype(bool), counts[:n]


def select_overlap(counts, n_valid, candidate_sections, gamma, n_front=3):
    """Sec. 3.3 overlap selection, first stage: the candidate views whose
    visible-point fraction exceeds gamma, then the n_front most front
    (earliest) sections holding at least one of them."""
    keep = [s for c, s in zip(counts, candidate_sections) if c > gamma * n_valid]
    return sorted(set(keep))[:n_front]


def track_loss(rgb, depth, sil, obs_rgb, obs_depth, vis=None, alpha=0.5, beta=1.0,
               sil_thr=0.5):
    """Eq. 1 with the mask W = vis & (D > 0) & (S' > sil_thr)."""
    P = int(np.asarray(depth).size)
    rgb = _f64(np.asarray(rgb).reshape(3, P)); depth = _f64(np.ravel(depth)); sil = _f64(np.ravel(sil))
    orgb = _f32(np.asarray(obs_rgb).reshape(3, P)); od = _f32(np.ravel(obs_depth))
    v = None if vis is None else np.ascontiguousarray(np.ravel(vis), dtype=np.uint8)
    g_rgb = np.zeros((3, P)); g_d = np.zeros(P)
    L = lib().orc_track_loss(P, _p(rgb), _p(depth), _p(sil), _p(orgb), _p(od), _p(v),
                             alpha, beta, sil_thr, _p(g_rgb), _p(g_d))
    return L, g_rgb, g_d


def ssim(x, y, grad=False):
    """Mean SSIM (11x11 Gaussian window, sigma 1.5, zero padding)."""
    x = _f64(x); y = _f64(y)
    H, W = x.shape
    g = np.zeros((H, W)) if grad else None
    s = lib().orc_ssim(H, W, _p(x), _p(y), _p(g))
    return (s, g) if grad else s


def map_loss(H, W, rgb, depth, obs_rgb, obs_depth, rho=0.8, tau=0.2, sigma=1.0):
    """Eq. 2 with means and U = (D > 0)."""
    P = H * W
    rgb = _f64(np.asarray(rgb).reshape(3, P)); depth = _f64(np.ravel(depth))
    orgb = _f32(np.asarray(obs_rgb).reshape(3, P)); od = _f32(np.ravel(obs_depth))
    g_rgb = np.zeros((3, P)); g_d = np.zeros(P)
    L = lib().orc_map_loss(H, W, _p(rgb), _p(depth), _p(orgb), _p(od), rho, tau, sigma,
                           _p(g_rgb), _p(g_d))
    return L, g_rgb, g_d


def se3_exp(xi):
    T = np.zeros(12)
    lib().orc_se3_exp(_p(_f64(xi)), _p(T))
    return T.reshape(3, 4)


def adam(param, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    lib().orc_adam(int(param.size), _p(param), _p(_f64(grad)), _p(m), _p(v), int(t), lr, b1, b2,
                   eps)


def compose(A, B):
    """3x4 rigid A * B."""
    A = np.asarray(A, np.float64).reshape(3, 4); B = np.asarray(B, np.float64).reshape(3, 4)
    return np.concatenate([A[:, :3] @ B[:, :3], (A[:, :3] @ B[:, 3] + A[:, 3])[:, None]], 1)


def track_iteration(view, kfs, obs_rgb, obs_depth, state, alpha=0.5, beta=1.0, lr_rot=0.002,
                    lr_trans=0.002, sil_thr=0.5, vis=None, prm=None):
    """One tracking iteration (Sec. 3.3, Eq. 1): render at the pose, loss,
    gradient to the twist at zero, Adam on the twist (lr_trans on rho,
    lr_rot on phi; App. A), pose <- exp(step^) * pose.  ``state`` holds
    m[6], v[6], t; returns (loss, new_pose[3,4] float64, new_state)."""
    out = render(view, kfs, prm)
    L, g_rgb, g_d = track_loss(out["rgb"], out["depth"], out["sil"], obs_rgb, obs_depth, vis,
                               alpha, beta, sil_thr)
    g = render_bwd(view, kfs, g_rgb, g_d, None, prm)["twist"]
    m = np.array(state["m"], np.float64); v = np.array(state["v"], np.float64)
    t = int(state["t"]) + 1
    xi = np.zeros(6)
    lr = np.array([lr_trans] * 3 + [lr_rot] * 3)
    for i in range(6):
        pi, mi, vi = xi[i:i + 1].copy(), m[i:i + 1], v[i:i + 1]
        adam(pi, g[i:i + 1], mi, vi, t, lr[i])
        xi[i] = pi[0]
    new_pose = compose(se3_exp(xi), np.asarray(view.pose, np.float64).reshape(3, 4))
    return L, new_pose, dict(m=m, v=v, t=t), g, out


__all__ = ["DEFAULTS", "threads", "Keyframe", "ViewSpec", "params", "ingest", "relpose32", "preprocess32",
           "tile_lists", "slice_size", "render", "render_alternatives", "render_bwd", "track_loss", "ssim", "map_loss",
           "se3_exp", "adam", "compose", "track_iteration", "REC_DTYPE", "visibility",
           "select_overlap"]
