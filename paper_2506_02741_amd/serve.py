"""Continuous-batching request server over a device-resident map.

Requests against a map of sections (consecutive keyframes, Sec. 3.2):

* render(section, camera, pose)            -> RGB, depth, silhouette
* track(section, camera, init pose, RGBD, n)  -> pose after n iterations of
  Eq. 1 tracking (Sec. 3.3) and its loss curve

The scheduler works in ticks.  Each tick admits queued requests while a
slot is free and their workspace fits the memory budget, then launches one
batched plan over every active render request (forward) and one over every
active track request (one tracking iteration each), on two streams so the
two batches overlap on the device.  A render request finishes in the tick
it was admitted; a track request stays active for n ticks.  Requests that
arrive while a tick runs join at the next tick.  Each view's result depends
only on its own view (per-view tile lists, per-view twist reductions, no
atomics on the pose path), so a request's result is the same alone or in
any mix.

With ``pipeline=True`` the host does not wait for a tick: it builds and
launches the next tick while the device runs the previous one (two
workspaces per kind, used by alternate ticks; a tick's track iterations
follow the previous tick's on the same stream, so poses and Adam states
carry over on the device).  A tick is retired -- its requests completed,
their memory released, losses read from pinned host copies -- once its
events have completed; at most two ticks are in flight.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import _lib
from . import render as R


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                      # "render" | "track"
    section: int
    cam: tuple
    pose: np.ndarray               # [3,4] world->camera (initial pose for track)
    obs_rgb: object = None         # track only: [3,H,W] observed colour
    obs_depth: object = None       # track only: [H,W] observed depth
    iters: int = 20
    arrival: float = 0.0
    # filled by the server
    admitted: float = 0.0
    done: float = 0.0
    ws_bytes: int = 0
    result: dict = dataclasses.field(default_factory=dict)
    _view: object = None
    _left: int = 0
    _losses: list = dataclasses.field(default_factory=list)


class Server:
    """Continuous batching of render / track requests over one GPU."""

    def __init__(self, keyframes, sections, budget_bytes=16 << 30, max_active=64, prm=None,
                 track_cfg=None, device="cuda", pipeline=False):
        self.keyframes = keyframes
        self.sections = sections          # list of (kf_first, kf_count)
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.prm = prm if prm is not None else R.params()
        self.cfg = track_cfg if track_cfg is not None else R.track_cfg()
        self.device = torch.device(device)
        self.peak_mem = 0
        self.queue = collections.deque()
        self.active = []
        self.finished = []
        self.mem_used = 0
        self.s_render = self.s_track = None
        if self.device.type == "cuda":
            self.s_render = torch.cuda.Stream(device=self.device)
            self.s_track = torch.cuda.Stream(device=self.device)
        self.ticks = 0
        self.batch_sizes = []
        self._ws = {}       # per kind, one workspace reused by every tick (grown on demand)
        self._kfa = None    # keyframe descriptors, built once
        self._est = {}      # workspace estimate per (section, camera, kind)
        self.host_s = 0.0   # building plans and launching, per tick, summed
        self.wait_s = 0.0   # waiting for the device after launching
        self.pipeline = bool(pipeline)
        self.inflight = collections.deque()  # launched, not yet retired ticks

    # -- admission ---------------------------------------------------------
    def _view_for(self, req):
        first, count = self.sections[req.section]
        v = R.View(req.cam, req.pose, first, count, req.obs_rgb, req.obs_depth, device=self.device)
        if req.kind == "track":
            v.with_pose_adam()
        return v

    def _kf_array(self):
        if self._kfa is None:
            self._kfa = R.keyframe_array(self.keyframes)
        return self._kfa

    def estimate_bytes(self, req):
        """Workspace of a one-view plan for this request (host-only sizing)
        plus its output/observation buffers; cached per section, camera and
        kind."""
        key = (req.section, tuple(req.cam), req.kind)
        if key in self._est:
            return self._est[key]
        L = _lib.load()
        first, count = self.sections[req.section]
        ka = self._kf_array()
        cam = R.Camera.of(req.cam)
        va = (_lib.vtgs_view * 1)(_lib.vtgs_view(cam.cstruct(), 1, first, count, None, None, None, None))
        import ctypes as C
        h = C.c_void_p()
        _lib.check(L.vtgs_plan_create(ka, len(self.keyframes), va, 1, C.byref(self.prm), 0,
                                      C.byref(h)))
        b = int(L.vtgs_plan_workspace_bytes(h))
        L.vtgs_plan_destroy(h)
        self._est[key] = b + 5 * 4 * cam.P
        return self._est[key]

    def submit(self, req):
        req.ws_bytes = self.estimate_bytes(req)
        if req.ws_bytes > self.budget:
            raise ValueError("request %d needs %d bytes, more than the budget" % (req.rid, req.ws_bytes))
        self.queue.append(req)

    def _admit(self, now):
        while self.queue and len(self.active) < self.max_active and \
                self.mem_used + self.queue[0].ws_bytes <= self.budget:
            req = self.queue.popleft()
            req.admitted = now
            req._view = self._view_for(req)
            req._left = req.iters if req.kind == "track" else 1
            self.mem_used += req.ws_bytes
            self.peak_mem = max(self.peak_mem, self.mem_used)
            self.active.append(req)

    def _plan(self, kind, views):
        """A plan over this tick's views in the kind's reused workspace (the
        previous tick on that stream has finished: ticks wait for both)."""
        plan = R.Plan(self.keyframes, views, self.prm, device=self.device,
                      workspace=self._ws.get(kind), kf_array=self._kf_array())
        self._ws[kind] = plan.ws
        return plan

    def drain(self, now_fn=time.perf_counter):
        """Retire every tick still in flight (pipelined mode)."""
        if self.pipeline:
            self._retire_done(now_fn, block=True, keep=0)

    # -- one tick ----------------------------------------------------------
    def tick(self, now_fn=time.perf_counter):
        if self.pipeline:
            return self._tick_pipelined(now_fn)
        self._admit(now_fn())
        if not self.active:
            return False
        rend = [r for r in self.active if r.kind == "render"]
        trk = [r for r in self.active if r.kind == "track"]
        self.batch_sizes.append((len(rend), len(trk)))
        self._execute(rend, trk)
        t = now_fn()
        keep = []
        for r in self.active:
            if r._left == 0:
                r.done = t
                self.mem_used -= r.ws_bytes
                self.finished.append(r)
            else:
                keep.append(r)
        self.active = keep
        self.ticks += 1
        return True

    def _execute(self, rend, trk):
        """One batched forward over the render requests and one tracking
        iteration over the track requests, on two streams; waits for both."""
        t0 = time.perf_counter()
        main = torch.cuda.current_stream(self.device)
        ev = []
        out = plan_r = plan_t = loss = None
        if rend:
            self.s_render.wait_stream(main)
            with torch.cuda.stream(self.s_render):
                plan_r = self._plan("render", [r._view for r in rend])
                out = plan_r.render_fwd()
                e = torch.cuda.Event()
                e.record(self.s_render)
                ev.append(e)
        if trk:
            self.s_track.wait_stream(main)
            with torch.cuda.stream(self.s_track):
                plan_t = self._plan("track", [r._view for r in trk])
                loss = plan_t.track_step(self.cfg, 1)
                e = torch.cuda.Event()
                e.record(self.s_track)
                ev.append(e)
        t1 = time.perf_counter()
        for e in ev:
            e.synchronize()
        self.host_s += t1 - t0
        self.wait_s += time.perf_counter() - t1
        if rend:
            rc, need = plan_r.status(clear=True, stream=self.s_render)
            if rc != 0:
                raise _lib.VtgsError(rc, _lib.last_error())
            rgb, depth, sil = out
            for i, r in enumerate(rend):
                r.result = dict(rgb=plan_r.view_image(rgb, i).clone(),
                                depth=plan_r.view_image(depth, i).clone(),
                                sil=plan_r.view_image(sil, i).clone())
                r._left = 0
        if trk:
            rc, need = plan_t.status(clear=True, stream=self.s_track)
            if rc != 0:
                raise _lib.VtgsError(rc, _lib.last_error())
            lv = loss[0].cpu().numpy()
            for i, r in enumerate(trk):
                r._losses.append(float(lv[i]))
                r._left -= 1
                if r._left == 0:
                    r.result = dict(pose=r._view.pose.detach().cpu().numpy().reshape(3, 4),
                                    loss=np.array(r._losses))

    # -- pipelined ticks ------------------------------------------------------
    def _tick_pipelined(self, now_fn):
        """Launch a tick over the requests with work left, without waiting
        for the device; retire completed ticks.  Returns False when nothing
        was launched and nothing is in flight."""
        self._retire_done(now_fn, block=False)
        self._admit(now_fn())
        rend = [r for r in self.active if r.kind == "render" and r._left > 0]
        trk = [r for r in self.active if r.kind == "track" and r._left > 0]
        if not rend and not trk:
            if self.inflight:
                self._retire_done(now_fn, block=True, keep=0)
                return True
            return False
        # the workspaces of the tick before last are reused by this one
        self._retire_done(now_fn, block=True, keep=1)
        self.batch_sizes.append((len(rend), len(trk)))
        self.inflight.append(self._launch(rend, trk))
        self.ticks += 1
        return True

    def _launch(self, rend, trk):
        t0 = time.perf_counter()
        main = torch.cuda.current_stream(self.device)
        rec = dict(rend=rend, trk=trk, events=[], finishing=[])
        par = self.ticks % 2
        if rend:
            self.s_render.wait_stream(main)
            with torch.cuda.stream(self.s_render):
                plan = self._plan(("render", par), [r._view for r in rend])
                rec["plan_r"] = plan
                rec["out"] = plan.render_fwd()
                e = torch.cuda.Event()
                e.record(self.s_render)
                rec["events"].append(e)
            for r in rend:
                r._left = 0
                rec["finishing"].append(r)
        if trk:
            self.s_track.wait_stream(main)
            with torch.cuda.stream(self.s_track):
                plan = self._plan(("track", par), [r._view for r in trk])
                rec["plan_t"] = plan
                loss = plan.track_step(self.cfg, 1)
                host = torch.empty(loss.shape, dtype=loss.dtype, pin_memory=True)
                host.copy_(loss, non_blocking=True)
                rec["loss"] = (loss, host)
                e = torch.cuda.Event()
                e.record(self.s_track)
                rec["events"].append(e)
            for r in trk:
                r._left -= 1
                if r._left == 0:
                    rec["finishing"].append(r)
        self.host_s += time.perf_counter() - t0
        return rec

    def _retire_done(self, now_fn, block, keep=None):
        """Retire the oldest in-flight ticks: those whose events completed
        (block=False), or as many as needed to leave `keep` in flight."""
        while self.inflight:
            rec = self.inflight[0]
            ready = all(e.query() for e in rec["events"])
            if not ready:
                if not block or keep is None or len(self.inflight) <= keep:
                    return
                t1 = time.perf_counter()
                for e in rec["events"]:
                    e.synchronize()
                self.wait_s += time.perf_counter() - t1
            self.inflight.popleft()
            self._finish(rec, now_fn())

    def _finish(self, rec, t):
        if rec["rend"]:
            plan = rec["plan_r"]
            rc, need = plan.status(clear=True, stream=self.s_render)
            if rc != 0:
                raise _lib.VtgsError(rc, _lib.last_error())
            rgb, depth, sil = rec["out"]
            for i, r in enumerate(rec["rend"]):
                r.result = dict(rgb=plan.view_image(rgb, i), depth=plan.view_image(depth, i),
                                sil=plan.view_image(sil, i))
        if rec["trk"]:
            plan = rec["plan_t"]
            rc, need = plan.status(clear=True, stream=self.s_track)
            if rc != 0:
                raise _lib.VtgsError(rc, _lib.last_error())
            lv = rec["loss"][1][0].numpy()
            for i, r in enumerate(rec["trk"]):
                r._losses.append(float(lv[i]))
        for r in rec["finishing"]:
            if r.kind == "track":
                r.result = dict(pose=r._view.pose.detach().cpu().numpy().reshape(3, 4),
                                loss=np.array(r._losses))
            r.done = t
            self.mem_used -= r.ws_bytes
            self.finished.append(r)
            self.active.remove(r)

    # -- driving a trace -----------------------------------------------------
    def run_trace(self, requests, realtime=True, max_seconds=None):
        """Serve requests whose ``arrival`` times (seconds from start) are set;
        with realtime=True arrivals follow the wall clock."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while pending or self.queue or self.active or self.inflight:
            tnow = now()
            while pending and (pending[0].arrival <= tnow or not realtime):
                r = pending.popleft()
                if not realtime:
                    r.arrival = tnow
                self.submit(r)
            if not self.tick(now) and pending:
                time.sleep(max(0.0, min(0.001, pending[0].arrival - now())))
            if max_seconds is not None and now() > max_seconds:
                break
        return self.report()

    def report(self):
        lat = np.array([r.done - r.arrival for r in self.finished])
        rl = np.array([r.done - r.arrival for r in self.finished if r.kind == "render"])
        tl = np.array([r.done - r.arrival for r in self.finished if r.kind == "track"])
        span = max((r.done for r in self.finished), default=0.0) - \
            min((r.arrival for r in self.finished), default=0.0)
        px = sum(R.Camera.of(r.cam).P * (r.iters if r.kind == "track" else 1) for r in self.finished)

        def pct(a, q):
            return float(np.percentile(a, q) * 1e3) if a.size else None
        return dict(requests=len(self.finished), seconds=span,
                    req_per_s=len(self.finished) / span if span > 0 else None,
                    mpix_per_s=px / span / 1e6 if span > 0 else None,
                    p50_ms=pct(lat, 50), p99_ms=pct(lat, 99),
                    render_p50_ms=pct(rl, 50), render_p99_ms=pct(rl, 99),
                    track_p50_ms=pct(tl, 50), track_p99_ms=pct(tl, 99),
                    ticks=self.ticks, host_s=self.host_s, device_wait_s=self.wait_s,
                    mean_batch=[float(np.mean([b[0] for b in self.batch_sizes])) if self.batch_sizes else 0,
                                float(np.mean([b[1] for b in self.batch_sizes])) if self.batch_sizes else 0])


def poisson_trace(rng, rate, seconds, n_sections, cams, poses_for, obs_for=None, p_render=0.6,
                  track_iters=20):
    """Requests with exponential inter-arrival times (rate per second); kind
    render with probability p_render, section and camera uniform."""
    t = 0.0
    out = []
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        kind = "render" if rng.uniform() < p_render else "track"
        sec = int(rng.integers(0, n_sections))
        cam = cams[int(rng.integers(0, len(cams)))]
        pose, true_pose = poses_for(rng, sec, cam)
        req = Request(rid, kind, sec, cam, pose, arrival=t, iters=track_iters)
        if kind == "track" and obs_for is not None:
            req.obs_rgb, req.obs_depth = obs_for(sec, cam, true_pose)
        out.append(req)
        rid += 1
    return out
