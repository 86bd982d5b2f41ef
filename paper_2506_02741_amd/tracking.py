"""Per-frame tracking driver (Sec. 3.3 and the supplementary implementation
details): the pose of each new frame starts from the constant-speed
prediction, is optimised by ``track_step`` against the current section, and
the final Eq. 1 loss is checked for divergence -- a loss more than `factor`
(50) times the mean final loss of the frames tracked before it.  On
divergence a caller-supplied hook may give another initial pose (the paper
uses RGB-D odometry there, which is not part of this library), and the frame
is tracked again from it.

Host-side orchestration only: every per-pixel step runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from .render import Plan, View, _dev, track_cfg


def _h(T):
    """3x4 (or 4x4) pose -> 4x4 float64."""
    M = np.eye(4)
    M[:3, :4] = np.asarray(T, dtype=np.float64).reshape(-1, 4)[:3]
    return M


def constant_speed(T_prev, T_prev2):
    """Constant-speed prediction of the next world->camera pose from the two
    before it: the motion between them, T_prev T_prev2^-1, applied once more
    to T_prev.  Returns a 3x4 float64 array."""
    A, B = _h(T_prev), _h(T_prev2)
    return (A @ np.linalg.inv(B) @ A)[:3]


class DivergenceCheck:
    """Final tracking losses of the frames accepted so far; a loss diverges
    when it exceeds `factor` times their mean (never for the first frame)."""

    def __init__(self, factor=50.0):
        self.factor = float(factor)
        self.losses = []

    def mean(self):
        return float(np.mean(self.losses)) if self.losses else None

    def diverged(self, loss):
        m = self.mean()
        return m is not None and float(loss) > self.factor * m

    def record(self, loss):
        self.losses.append(float(loss))


class FrameTracker:
    """Tracks a sequence of frames against the keyframes of the current
    section (one single-view track plan per frame).

    `on_divergence(frame_index, init_pose, loss, mean_loss)` is called when a
    frame's final loss diverges; it returns another initial pose (3x4) to
    track the frame again from, or None to keep the result.  Either way the
    frame's final loss joins the history that later frames are checked
    against."""

    def __init__(self, cam, iters=40, cfg=None, prm=None, factor=50.0, on_divergence=None,
                 device=None, stream=None):
        self.cam = cam
        self.iters = int(iters)
        self.cfg = cfg if cfg is not None else track_cfg()
        self.prm = prm
        self.check = DivergenceCheck(factor)
        self.on_divergence = on_divergence
        self.device = _dev(device)
        self.stream = stream
        self.poses = []       # tracked world->camera poses (3x4 float64)
        self.events = []      # (frame index, loss, mean loss, re-tracked)

    def predict(self):
        """Initial pose of the next frame: constant speed from the last two
        tracked poses (the last pose when fewer are known)."""
        if len(self.poses) >= 2:
            return constant_speed(self.poses[-1], self.poses[-2])
        return None if not self.poses else self.poses[-1].copy()

    def _run(self, keyframes, init_pose, obs_rgb, obs_depth, vis):
        pose = torch.as_tensor(np.asarray(init_pose, np.float32).reshape(12), device=self.device).clone()
        view = View(self.cam, pose, 0, len(keyframes), obs_rgb, obs_depth, vis,
                    device=self.device).with_pose_adam()
        plan = Plan(keyframes, [view], self.prm, device=self.device, stream=self.stream)
        loss = plan.track_step(self.cfg, iters=self.iters, stream=self.stream)
        rc, _ = plan.status(stream=self.stream)
        if rc != _lib.VTGS_OK:
            raise _lib.VtgsError(rc, _lib.last_error())
        final = float(loss[-1, 0].item())
        return view.pose.detach().cpu().numpy().astype(np.float64).reshape(3, 4), final

    def track(self, keyframes, obs_rgb, obs_depth, init_pose=None, vis=None):
        """Track one frame; returns (pose 3x4, final loss, diverged)."""
        if init_pose is None:
            init_pose = self.predict()
        if init_pose is None:
            raise ValueError("the first frame needs an initial pose")
        pose, loss = self._run(keyframes, init_pose, obs_rgb, obs_depth, vis)
        diverged = self.check.diverged(loss)
        if diverged:
            idx, mean = len(self.poses), self.check.mean()
            alt = self.on_divergence(idx, np.asarray(init_pose), loss, mean) if self.on_divergence else None
            self.events.append((idx, loss, mean, alt is not None))
            if alt is not None:
                pose, loss = self._run(keyframes, alt, obs_rgb, obs_depth, vis)
        self.check.record(loss)
        self.poses.append(pose)
        return pose, loss, diverged
