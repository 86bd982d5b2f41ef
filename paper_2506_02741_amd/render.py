"""Torch-facing wrapper of the HIP renderer.

PyTorch provides device memory and streams only; the arithmetic of every
step runs in ``libvtgs.so``.  Objects:

* :class:`Keyframe` -- one keyframe's view-tied Gaussians (Sec. 3.2 of the
  paper) in compact device arrays, created by GPU ingestion of a depth map.
* :class:`View` -- a camera (intrinsics, world->camera pose tensor) that
  renders a slice of keyframes, with optional observations for tracking and
  mapping.
* :class:`Plan` -- a batch of views bound to a workspace; exposes
  ``render_fwd``, ``render_bwd``, ``track_step``, ``map_step``.
* :func:`render` -- differentiable splat through ``torch.autograd``.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _lib
from ._lib import check, load


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev(device=None):
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


@dataclasses.dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @classmethod
    def of(cls, c):
        if isinstance(c, Camera):
            return c
        if hasattr(c, "as_tuple"):
            c = c.as_tuple()
        return cls(*[float(x) for x in c[:4]], int(c[4]), int(c[5]))

    def cstruct(self):
        return _lib.vtgs_camera(self.fx, self.fy, self.cx, self.cy, self.width, self.height)

    @property
    def P(self):
        return self.width * self.height


def _f32(x, device):
    return torch.as_tensor(x, dtype=torch.float32).to(device).contiguous()


class Keyframe:
    """View-tied Gaussians of one keyframe: pixel index, depth, colour [3,n],
    opacity, radius (device tensors) and the keyframe camera and pose."""

    def __init__(self, cam, pose, pix, depth, color, opacity, radius, learnable=False,
                 device=None):
        dev = _dev(device)
        self.cam = Camera.of(cam)
        self.pose = _f32(pose, dev).reshape(12)
        self.pix = torch.as_tensor(pix).to(dev).to(torch.int32).contiguous()
        self.depth = _f32(depth, dev)
        self.color = _f32(color, dev).reshape(3, -1)
        self.opacity = _f32(opacity, dev)
        self.radius = _f32(radius, dev)
        self.n = int(self.pix.numel())
        self.learnable = bool(learnable)
        self.g_color = self.g_opacity = self.g_radius = None
        self.adam = None
        # geometry: depth along the pixel rays and the keyframe pose
        self.g_depth = self.g_pose = self.depth_adam = self.pose_adam = None
        self.depth_map = None

    @classmethod
    def ingest(cls, depth_img, rgb_img, cam, pose, stride=1, o_init=0.99, mask=None,
               learnable=False, device=None, stream=None):
        """GPU ingestion: a Gaussian at every valid depth pixel of the stride
        grid, colour from the RGB image, opacity o_init, radius stride*D/f."""
        L = load()
        dev = _dev(device)
        cam = Camera.of(cam)
        d = _f32(depth_img, dev)
        H, W = d.shape[-2], d.shape[-1]
        rgb = None if rgb_img is None else _f32(rgb_img, dev).reshape(3, H, W)
        m = None if mask is None else torch.as_tensor(mask).to(dev).to(torch.uint8).contiguous()
        nbytes = L.vtgs_ingest_scratch_bytes(H, W, stride)
        scratch = torch.empty(max(nbytes, 4), dtype=torch.uint8, device=dev)
        count = torch.zeros(1, dtype=torch.int32, device=dev)
        st = _stream(stream)
        check(L.vtgs_ingest_count(_ptr(d), _ptr(m), H, W, stride, _ptr(scratch), nbytes,
                                  _ptr(count), st))
        n = int(count.item())
        pix = torch.empty(n, dtype=torch.int32, device=dev)
        dep = torch.empty(n, dtype=torch.float32, device=dev)
        col = torch.zeros(3, n, dtype=torch.float32, device=dev)
        opa = torch.empty(n, dtype=torch.float32, device=dev)
        rad = torch.empty(n, dtype=torch.float32, device=dev)
        check(L.vtgs_ingest_fill(_ptr(d), _ptr(rgb), _ptr(m), H, W, stride, float(cam.fx),
                                 float(o_init), _ptr(scratch), nbytes, n, _ptr(pix), _ptr(dep),
                                 _ptr(col), _ptr(opa), _ptr(rad), st))
        k = cls(cam, pose, pix, dep, col, opa, rad, learnable, dev)
        k.depth_map = d.reshape(-1)  # the frame's depth map (visibility tests)
        return k

    def with_grad_buffers(self):
        dev = self.depth.device
        self.g_color = torch.zeros(3, self.n, device=dev)
        self.g_opacity = torch.zeros(self.n, device=dev)
        self.g_radius = torch.zeros(self.n, device=dev)
        return self

    def with_adam(self):
        self.adam = torch.zeros(10, self.n, device=self.depth.device)
        return self

    def with_geometry_grads(self):
        """Gradient buffers of the tied depths [n] and the pose twist [6]
        (render_bwd adds into them; a learnable keyframe only)."""
        dev = self.depth.device
        self.g_depth = torch.zeros(self.n, device=dev)
        self.g_pose = torch.zeros(6, device=dev)
        return self

    def with_geometry_adam(self, depth=True, pose=True):
        """Adam states that let map_step move the Gaussians along their rays
        (depth) and adjust the keyframe pose (bundle adjustment)."""
        dev = self.depth.device
        self.depth_adam = torch.zeros(2, self.n, device=dev) if depth else None
        self.pose_adam = torch.zeros(13, device=dev) if pose else None
        return self

    def cstruct(self):
        return _lib.vtgs_keyframe(self.n, _ptr(self.pix), _ptr(self.depth), _ptr(self.color),
                                  _ptr(self.opacity), _ptr(self.radius), _ptr(self.pose),
                                  self.cam.cstruct(), 1 if self.learnable else 0,
                                  _ptr(self.g_color), _ptr(self.g_opacity), _ptr(self.g_radius),
                                  _ptr(self.adam), _ptr(self.g_depth), _ptr(self.g_pose),
                                  _ptr(self.depth_adam), _ptr(self.pose_adam))


class View:
    """A camera rendering keyframes [kf_first, kf_first + kf_count)."""

    def __init__(self, cam, pose, kf_first=0, kf_count=1, obs_rgb=None, obs_depth=None, vis=None,
                 pose_adam=None, device=None):
        dev = _dev(device)
        self.cam = Camera.of(cam)
        self.pose = pose if isinstance(pose, torch.Tensor) and pose.device == dev and \
            pose.dtype == torch.float32 and pose.is_contiguous() and pose.numel() == 12 \
            else _f32(pose, dev).reshape(12).clone()
        self.kf_first = int(kf_first)
        self.kf_count = int(kf_count)
        self.obs_rgb = None if obs_rgb is None else _f32(obs_rgb, dev).reshape(3, -1)
        self.obs_depth = None if obs_depth is None else _f32(obs_depth, dev).reshape(-1)
        self.vis = None if vis is None else torch.as_tensor(vis).to(dev).to(torch.uint8).reshape(-1).contiguous()
        self.pose_adam = pose_adam

    def with_pose_adam(self):
        self.pose_adam = torch.zeros(13, device=self.pose.device)
        return self

    def cstruct(self):
        return _lib.vtgs_view(self.cam.cstruct(), _ptr(self.pose), self.kf_first, self.kf_count,
                              _ptr(self.obs_rgb), _ptr(self.obs_depth), _ptr(self.vis),
                              _ptr(self.pose_adam))


def params(**kw):
    """Renderer parameters (defaults: alpha_min 1/255, alpha_max 0.99, t_min
    1e-4, q_cut 11.0826, z_near 0.01, lowpass 0.3, black bg, tile 16, batch
    256)."""
    return _lib.default_params(**kw)


def track_cfg(alpha=0.5, beta=1.0, lr_rot=0.002, lr_trans=0.002, sil_thr=0.5):
    return _lib.vtgs_track_cfg(alpha, beta, lr_rot, lr_trans, sil_thr)


def map_cfg(rho=0.8, tau=0.2, sigma=1.0, lr_color=0.0025, lr_opacity=0.05, lr_radius=0.005,
            lr_depth=0.001, lr_trans=0.002, lr_rot=0.002):
    """Eq. 2 weights and App. A's learning rates; lr_depth (tied depths of
    movable keyframes) and lr_trans / lr_rot (poses under bundle adjustment)
    are readings (the paper gives none for them: the pose rates are its
    tracking rates)."""
    return _lib.vtgs_map_cfg(rho, tau, sigma, lr_color, lr_opacity, lr_radius, lr_depth,
                             lr_trans, lr_rot)


def keyframe_array(keyframes):
    """The C descriptors of a keyframe list (vtgs_keyframe[n])."""
    return (_lib.vtgs_keyframe * max(len(keyframes), 1))(*[k.cstruct() for k in keyframes])


class Plan:
    """A batch of views over keyframes, bound to a device workspace."""

    def __init__(self, keyframes, views, prm=None, pair_capacity=0, device=None, stream=None,
                 workspace=None, bind=True, kf_array=None):
        self.L = load()
        self.keyframes = list(keyframes)
        # the descriptors capture the gradient buffers: create them first
        for k in self.keyframes:
            if k.learnable and k.g_color is None:
                k.with_grad_buffers()
        self.views = list(views)
        self.prm = prm if prm is not None else params()
        self.device = _dev(device)
        # kf_array: the keyframes' descriptors built once by a caller that
        # plans over the same keyframes many times (their buffers unchanged)
        kfa = kf_array if kf_array is not None else keyframe_array(self.keyframes)
        va = (_lib.vtgs_view * len(self.views))(*[v.cstruct() for v in self.views])
        h = C.c_void_p()
        check(self.L.vtgs_plan_create(kfa, len(self.keyframes), va, len(self.views),
                                      C.byref(self.prm), int(pair_capacity), C.byref(h)))
        self.h = h
        self.ws_bytes = int(self.L.vtgs_plan_workspace_bytes(h))
        self.P = int(self.L.vtgs_plan_pixels(h))
        self.n_rec = int(self.L.vtgs_plan_records(h))
        self.n_tiles = int(self.L.vtgs_plan_tiles(h))
        self.cap = int(self.L.vtgs_plan_pair_capacity(h))
        self.offsets = [int(self.L.vtgs_plan_view_offset(h, v)) for v in range(len(self.views))]
        self.generation = 0
        if isinstance(workspace, str) and workspace == "static":
            # state in the library's static scratch (render_fwd_static binds it)
            self.ws = None
            return
        if workspace is not None and workspace.numel() >= self.ws_bytes:
            self.ws = workspace
        else:
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        if bind:
            self.bind(stream)

    def bind(self, stream=None):
        """Upload the descriptors into the workspace (again); needed before use
        when several plans share one workspace."""
        check(self.L.vtgs_plan_bind(self.h, _ptr(self.ws), self.ws.numel(), _stream(stream)))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.L.vtgs_plan_destroy(h)
            self.h = None

    # -- images -----------------------------------------------------------
    def empty_images(self):
        d = self.device
        return (torch.empty(3, self.P, device=d), torch.empty(self.P, device=d),
                torch.empty(self.P, device=d))

    def view_image(self, plane, v):
        """Slice view v out of a packed [..., P] plane as [..., H, W]."""
        c = self.views[v].cam
        o = self.offsets[v]
        return plane[..., o:o + c.P].reshape(*plane.shape[:-1], c.height, c.width)

    # -- ABI calls --------------------------------------------------------
    def render_fwd(self, rgb=None, depth=None, sil=None, stream=None):
        if rgb is None and depth is None and sil is None:
            rgb, depth, sil = self.empty_images()
        check(self.L.vtgs_render_fwd(self.h, _ptr(rgb), _ptr(depth), _ptr(sil), _stream(stream)))
        self.generation += 1
        return rgb, depth, sil

    def render_fwd_static(self, rgb, depth, sil, stream=None):
        """render_fwd with the plan's state in the library's static scratch
        (no device allocation by the library; the caller passes the outputs)."""
        check(self.L.vtgs_render_fwd_static(self.h, _ptr(rgb), _ptr(depth), _ptr(sil),
                                            _stream(stream)))
        self.generation += 1
        return rgb, depth, sil

    def render_bwd(self, g_rgb=None, g_depth=None, g_sil=None, twist=True, stream=None):
        g_tw = torch.zeros(len(self.views), 6, device=self.device) if twist else None
        c = lambda t: None if t is None else t.contiguous().float()
        g_rgb, g_depth, g_sil = c(g_rgb), c(g_depth), c(g_sil)
        check(self.L.vtgs_render_bwd(self.h, _ptr(g_rgb), _ptr(g_depth), _ptr(g_sil), _ptr(g_tw),
                                     _stream(stream)))
        return g_tw

    def track_step(self, cfg=None, iters=1, loss=None, stream=None):
        cfg = cfg if cfg is not None else track_cfg()
        if loss is None:
            loss = torch.zeros(iters, len(self.views), device=self.device)
        check(self.L.vtgs_track_step(self.h, C.byref(cfg), int(iters), _ptr(loss), _stream(stream)))
        self.generation += 1
        return loss

    def map_step(self, step, cfg=None, loss=None, stream=None):
        cfg = cfg if cfg is not None else map_cfg()
        if loss is None:
            loss = torch.zeros(len(self.views), device=self.device)
        check(self.L.vtgs_map_step(self.h, C.byref(cfg), _ptr(step), _ptr(loss), _stream(stream)))
        self.generation += 1
        return loss

    def status(self, clear=True, stream=None):
        need = C.c_int64(0)
        rc = self.L.vtgs_plan_status(self.h, C.byref(need), 1 if clear else 0, _stream(stream))
        return rc, int(need.value)

    def timing(self, enable, repeat=1):
        """Start (enable=True) or stop per-stage HIP-event timing; stopping
        returns {stage: (total_ms, launches)}.  `repeat` > 1 launches each
        compositing stage that many times between its events."""
        import numpy as np
        if enable:
            check(self.L.vtgs_plan_timing(self.h, max(1, int(repeat)), None, None))
            return None
        ms = np.zeros(_lib.VTGS_N_STAGES, np.float64)
        cnt = np.zeros(_lib.VTGS_N_STAGES, np.int64)
        check(self.L.vtgs_plan_timing(self.h, 0, ms.ctypes.data, cnt.ctypes.data))
        return {self.L.vtgs_stage_name(i).decode(): (float(ms[i]), int(cnt[i]))
                for i in range(_lib.VTGS_N_STAGES) if cnt[i] > 0}

    def debug_state(self, stream=None):
        d = self.device
        rec = torch.empty(max(self.n_rec, 1), 12, device=d)
        rect = torch.empty(max(self.n_rec, 1), 4, dtype=torch.int32, device=d)
        ranges = torch.empty(self.n_tiles, 2, dtype=torch.int32, device=d)
        ids = torch.empty(self.cap, dtype=torch.int32, device=d)
        npairs = torch.zeros(1, dtype=torch.int64, device=d)
        check(self.L.vtgs_debug_state(self.h, _ptr(rec), _ptr(rect), _ptr(ranges), _ptr(ids),
                                      _ptr(npairs), _stream(stream)))
        return dict(records=rec[:self.n_rec], rect=rect[:self.n_rec], ranges=ranges, ids=ids,
                    n_pairs=npairs)


    def debug_images(self, stream=None):
        """(img [5, P], gimg [5, P]): the internal RGB/depth/silhouette of the
        last fused step and the upstream gradients map_step formed."""
        img = torch.empty(5, self.P, device=self.device)
        gimg = torch.empty(5, self.P, device=self.device)
        check(self.L.vtgs_debug_images(self.h, _ptr(img), _ptr(gimg), _stream(stream)))
        return img, gimg

    def debug_gather(self, stream=None):
        """Add the per-Gaussian gradients of the last backward to colour,
        opacity and radius (those map_step's Adam step used) into the
        learnable keyframes' g_color / g_opacity / g_radius."""
        check(self.L.vtgs_debug_gather(self.h, _stream(stream)))


def plan_checked(keyframes, views, prm=None, pair_capacity=0, device=None, run=None):
    """Create a plan, run ``run(plan)`` and, if the (Gaussian, tile) pairs
    overflowed the capacity, re-plan with room for what was needed."""
    plan = Plan(keyframes, views, prm, pair_capacity, device)
    if run is None:
        return plan
    out = run(plan)
    rc, need = plan.status()
    if rc == _lib.VTGS_E_CAPACITY:
        plan = Plan(keyframes, views, prm, int(need * 1.25) + 1024, device)
        out = run(plan)
        rc, need = plan.status()
    if rc != _lib.VTGS_OK:
        raise _lib.VtgsError(rc, _lib.last_error())
    return plan, out


class _RenderFn(torch.autograd.Function):
    """Differentiable splat: inputs are the view twists [n_views, 6] (taken at
    zero; the gradient is that of a left perturbation of each pose) and the
    colour, opacity, radius tensors of the plan's learnable keyframes."""

    @staticmethod
    def forward(ctx, plan, twist, *kf_params):
        rgb, depth, sil = plan.render_fwd()
        ctx.plan = plan
        ctx.gen = plan.generation
        return rgb, depth, sil

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_sil):
        plan = ctx.plan
        if plan.generation != ctx.gen:
            raise RuntimeError("the plan rendered again before this backward; one outstanding "
                               "forward per plan")
        # a forward whose (Gaussian, tile) pairs overflowed the plan's capacity
        # rendered from truncated tile lists: refuse to differentiate it
        rc, need = plan.status(clear=False)
        if rc != _lib.VTGS_OK:
            raise _lib.VtgsError(rc, _lib.last_error())
        learn = [k for k in plan.keyframes if k.learnable]
        for k in learn:
            k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
        g_tw = plan.render_bwd(g_rgb, g_depth, g_sil, twist=ctx.needs_input_grad[1])
        grads = []
        for k in learn:
            grads += [k.g_color.clone(), k.g_opacity.clone(), k.g_radius.clone()]
        return (None, g_tw) + tuple(grads)


def render(plan, twist=None):
    """(rgb [3,P], depth [P], sil [P]) with gradients to ``twist`` and to the
    learnable keyframes' colour/opacity/radius tensors."""
    learn = [k for k in plan.keyframes if k.learnable]
    for k in learn:
        if k.g_color is None:
            k.with_grad_buffers()
    if twist is None:
        twist = torch.zeros(len(plan.views), 6, device=plan.device)
    flat = []
    for k in learn:
        flat += [k.color, k.opacity, k.radius]
    return _RenderFn.apply(plan, twist, *flat)
