#!/usr/bin/env python3
"""Benchmark of the view-tied splatting renderer on one MI355X.

Metric: forward+backward Mpix/s at 640x480.  Workload (the tracking
configuration): one 640x480 keyframe of a synthetic room tied to 307,200
Gaussians, a new frame observed at the keyframe pose whose initial estimate
is off by 1 cm / 0.5 degrees; each frame runs 40 tracking iterations of
splat forward -> Eq. 1 loss -> backward to the SE(3) twist -> Adam step and
retraction.  A step is one such iteration; value = 640*480*steps / seconds.

Also reported on the same JSON line:
  roofline      the dominant kernel's algorithmic FP32 lane-ops per second
                (its contributing (pixel, Gaussian) pairs; with every list
                entry stepped through as a secondary figure) vs the VALU
                issue peak, its time from HIP events on the stream the
                kernels run on
  cpu_baseline  the CPU oracle on a bounded sample of the same workload,
                single-threaded and on all the host's cores, with the host's
                CPU model; plus bounded samples of the other workloads
  batched       mapping-section batch (5 of 8 keyframes per iteration,
                gradients to colour/opacity/radius) in one plan vs one view
                per launch with a host sync in between, with the mapping
                compositors' roofline
  uneven        16 views of mixed resolution in one captured graph (tuned
                tile shape) vs one view per launch
  serving       continuous batching of Poisson render/track requests
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)



args = None  # the command line, set by main()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tracking_setup():
    import numpy as np
    import torch
    from paper_2506_02741_amd import render as R
    from paper_2506_02741_amd import synth
    w = synth.tracking_workload(1)
    kf = w["keyframe"]
    cam = kf.cam.as_tuple()
    k = R.Keyframe.ingest(kf.depth, kf.rgb, cam, kf.pose)
    init = torch.tensor(np.asarray(w["init_pose"], np.float32).reshape(12), device="cuda")
    view = R.View(cam, init.clone(), obs_rgb=kf.rgb, obs_depth=kf.depth).with_pose_adam()
    plan = R.Plan([k], [view])
    return w, k, view, plan, init


def run_frames(plan, view, init, cfg, iters, loss, frame=40):
    """iters tracking iterations in frames of `frame` (the last one possibly
    shorter), each from the initial pose."""
    done = 0
    while done < iters:
        n = min(frame, iters - done)
        view.pose.copy_(init)
        view.pose_adam.zero_()
        plan.track_step(cfg, n, loss[:n])
        done += n


def frame_lengths(steps, frame):
    """The frame lengths a run of `steps` iterations in frames of `frame` uses."""
    return sorted({min(frame, steps - d) for d in range(0, steps, frame)}, reverse=True)


def host_info():
    """The host's CPU model and core counts (os.cpu_count, and the cores this
    process may run on)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return dict(cpu_model=model, nproc=os.cpu_count(), cores_available=avail)


# Lane-ops per unit of the compositing kernels' algorithmic work: one FP32
# VALU operation per lane, an exp counted as 4 (quarter rate).  Forward: an
# entry a pixel steps past costs d (2), q (5) and the cut test (1) = 8; a
# contributor adds exp, alpha, transmittance, the stop test and the colour
# and depth accumulation, 22 in all.  Backward: 10 per entry stepped past;
# 90 per contributor (alpha and T recovery, dL/dalpha against the behind
# accumulators, dL/dq, dL/dmu and the twist chain).
LANE_OPS = dict(fwd_skip=8, fwd_contrib=22, bwd_skip=10, bwd_contrib=90)
# FP32 VALU issue rate without packed operations: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (one lane-op per lane per clock)
PEAK_LANE_OPS_T = 256 * 4 * 16 * 2.4e9 / 1e12


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "%s_tracking_640x480_traffic.txt")
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2506_02741_amd", "csrc", f)
                   for f in ("k_composite.hip", "vtgs_internal.h")]


def measured_traffic(stage="composite_bwd"):
    """HBM bytes per launch of a tracking compositing kernel from the
    committed counter summary, or None when the kernel sources changed since
    the counters were taken (the summary records their SHA-256)."""
    import hashlib
    path = TRAFFIC_FILE % stage if "%s" in TRAFFIC_FILE else TRAFFIC_FILE
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for p in TRAFFIC_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    if kv.get("sources_sha256") != h.hexdigest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def plan_layout(plan):
    """(width, height, first record, first tile) of every view of a plan."""
    layout = getattr(plan, "layout", None)
    if layout is not None:
        return layout
    B = int(plan.prm.tile)
    out, rec, tile = [], 0, 0
    for v in plan.views:
        w, h = v.cam.width, v.cam.height
        out.append((w, h, rec, tile))
        rec += sum(k.n for k in plan.keyframes[v.kf_first:v.kf_first + v.kf_count])
        tile += ((w + B - 1) // B) * ((h + B - 1) // B)
    return out


def scan_counts(plan, chunk_elems=1 << 23):
    """Units the compositing launches of a plan process, counted on the host
    from the plan's own sorted tile lists and records (the state the kernels
    read after a render): per pixel, the forward steps through its tile's
    list front to back up to and including the entry that stops it (the
    whole list when none does), and composites its contributors; the
    backward steps from the pixel's last contributor back to the front.
    alpha is taken in FP32 with exp2 and q without fused multiply-adds, and
    the transmittance is a sequential FP32 product, so a decision within an
    ulp of a threshold may count one entry differently from the kernel."""
    import numpy as np
    import torch
    st = plan.debug_state()
    rec = st["records"].detach().cpu()[:, :6].contiguous()
    ranges = st["ranges"].detach().cpu().to(torch.int64)
    ids = st["ids"].detach().cpu().to(torch.int64) & 0xFFFFFFFF
    prm = plan.prm
    B = int(prm.tile)
    f32 = torch.float32
    amin, amax = float(np.float32(prm.alpha_min)), float(np.float32(prm.alpha_max))
    tmin, qcut = float(np.float32(prm.t_min)), float(np.float32(prm.q_cut))
    k = float(np.float32(-0.5 * np.log2(np.e)))
    yy, xx = torch.meshgrid(torch.arange(B), torch.arange(B), indexing="ij")
    xx, yy = xx.reshape(-1), yy.reshape(-1)
    tot = dict(fwd_scanned=0, contrib=0, bwd_scanned=0)
    for (W, H, rb, tb) in plan_layout(plan):
        tiles_x, tiles_y = (W + B - 1) // B, (H + B - 1) // B
        nt_view = tiles_x * tiles_y
        lens = (ranges[tb:tb + nt_view, 1] - ranges[tb:tb + nt_view, 0]).clamp(min=0)
        order = torch.argsort(lens, stable=True)   # similar lengths share a chunk
        i = 0
        while i < nt_view:
            L = max(int(lens[order[min(nt_view - 1, i)]]), 1)
            j = i + 1
            while j < nt_view and int(lens[order[j]]) <= L * 2 and (j - i + 1) * B * B * max(
                    int(lens[order[j]]), 1) <= chunk_elems:
                j += 1
            t = order[i:j]
            L = max(int(lens[t].max()), 1)
            i = j
            s0 = ranges[tb + t, 0]
            n = lens[t]
            pos = s0[:, None] + torch.arange(L)[None, :]
            valid = torch.arange(L)[None, :] < n[:, None]
            rows = rb + ids[torch.where(valid, pos, s0[:, None]).clamp(max=ids.numel() - 1)]
            r = rec[rows]                                    # [nt, L, 6]
            px = ((t % tiles_x) * B)[:, None] + xx[None, :]  # [nt, B*B]
            py = ((t // tiles_x) * B)[:, None] + yy[None, :]
            inside = (px < W) & (py < H)
            dx = px.to(f32)[:, :, None] - r[:, None, :, 0]
            dy = py.to(f32)[:, :, None] - r[:, None, :, 1]
            q = (r[:, None, :, 2] * dx) * dx + ((2.0 * r[:, None, :, 3]) * dx) * dy \
                + (r[:, None, :, 4] * dy) * dy
            a = torch.clamp(r[:, None, :, 5] * torch.exp2(q * k), max=amax)
            cover = (q <= qcut) & (a >= amin) & valid[:, None, :]
            del dx, dy, q
            Tn = torch.cumprod(torch.where(cover, 1.0 - a, torch.ones_like(a)), dim=2)
            stops = cover & (Tn < tmin)
            stopped = stops.any(dim=2)
            nn = n[:, None].expand_as(stopped)
            first = torch.where(stopped, stops.to(torch.int8).argmax(dim=2), nn)
            tot["fwd_scanned"] += int(torch.where(stopped, first + 1, nn)[inside].sum())
            took = cover & (torch.arange(L)[None, None, :] < first[:, :, None])
            nc = took.sum(dim=2)
            tot["contrib"] += int(nc[inside].sum())
            lastpos = torch.where(nc > 0, L - 1 - took.flip(2).to(torch.int8).argmax(dim=2),
                                  torch.full_like(nc, -1))
            tot["bwd_scanned"] += int((lastpos + 1)[inside].sum())
    return tot


def lane_op_work(c):
    """Algorithmic lane-ops of one forward and one backward launch."""
    fwd = LANE_OPS["fwd_skip"] * (c["fwd_scanned"] - c["contrib"]) + LANE_OPS["fwd_contrib"] * c["contrib"]
    bwd = LANE_OPS["bwd_skip"] * (c["bwd_scanned"] - c["contrib"]) + LANE_OPS["bwd_contrib"] * c["contrib"]
    return {"composite_fwd": fwd, "composite_bwd": bwd}


def compositing_roofline(cnt, stage_ms):
    """Per compositing kernel: the contributors' lane-ops per second (the
    method's necessary work, the headline) and the lane-ops of every list
    entry the pixels step through, each against the VALU issue peak."""
    work = lane_op_work(cnt)
    out = {}
    for stage, key in (("composite_fwd", "fwd_contrib"), ("composite_bwd", "bwd_contrib")):
        ms = stage_ms.get(stage)
        if not ms:
            continue
        nec = cnt["contrib"] * LANE_OPS[key]
        out[stage] = dict(avg_ms=ms, contrib_lane_ops=nec,
                          achieved=nec / (ms * 1e-3) / 1e12,
                          frac=nec / (ms * 1e-3) / 1e12 / PEAK_LANE_OPS_T,
                          with_list_steps=dict(lane_ops=work[stage],
                                               achieved=work[stage] / (ms * 1e-3) / 1e12,
                                               frac=work[stage] / (ms * 1e-3) / 1e12 / PEAK_LANE_OPS_T))
    return out


def cpu_tracking_iterations(w, seconds, threads):
    """Oracle tracking iterations of the 640x480 frame for about `seconds`."""
    import numpy as np
    import oracle
    kf = w["keyframe"]
    okf = oracle.ingest(kf.depth, kf.rgb, fx=kf.cam.fx, cam=kf.cam.as_tuple(), pose=kf.pose)
    pose = np.asarray(w["init_pose"], np.float32)
    st = dict(m=np.zeros(6), v=np.zeros(6), t=0)
    n = 0
    with oracle.threads(threads):
        t0 = time.perf_counter()
        while True:
            view = oracle.ViewSpec(kf.cam.as_tuple(), pose)
            L, new_pose, st, g, _ = oracle.track_iteration(view, [okf], kf.rgb, kf.depth, st)
            pose = new_pose.astype(np.float32)
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
    return n, dt


def cpu_baseline(w, seconds, all_seconds):
    """The oracle on the host: single-threaded (the parity reference) and its
    OpenMP build on every available core, on the tracking workload."""
    info = host_info()
    n, dt = cpu_tracking_iterations(w, seconds, 1)
    out = dict(value=640 * 480 * n / dt / 1e6, unit="Mpix/s", cores=1, kind="oracle",
               sample="%d tracking iterations (fwd + Eq.1 + bwd to twist + Adam/retraction) of "
                      "the 640x480 frame, single-threaded, %.1f s" % (n, dt), **info)
    if all_seconds > 0 and info["cores_available"] > 1:
        c = info["cores_available"]
        n2, dt2 = cpu_tracking_iterations(w, all_seconds, c)
        out["all_cores"] = dict(value=640 * 480 * n2 / dt2 / 1e6, unit="Mpix/s", cores=c,
                                sample="%d tracking iterations, OpenMP on %d threads, %.1f s"
                                       % (n2, c, dt2))
    return out


def cpu_configs(section, uneven_frames, uneven_views, threads):
    """Oracle fwd+bwd timings beside the other workloads (bounded samples):
    the 64x48 toy view whole (L1 colour + L1 depth against a jittered-colour
    target); one view of the mapping section (Eq. 2, 8 keyframes); one view
    of each resolution of the uneven batch (over its 8-keyframe section)."""
    import numpy as np
    import oracle
    from paper_2506_02741_amd import synth
    res = {}

    def fwd_bwd(view, kfs, target, eq2):
        t0 = time.perf_counter()
        out = oracle.render(view, kfs)
        H, W = int(view.cam[5]), int(view.cam[4])
        if eq2:
            L, g_rgb, g_d = oracle.map_loss(H, W, out["rgb"], out["depth"], target[0], target[1])
        else:
            g_rgb = -np.sign(target[0].reshape(3, -1) - out["rgb"])
            g_d = -np.sign(target[1].reshape(-1) - out["depth"])
        oracle.render_bwd(view, kfs, g_rgb, g_d, None)
        return time.perf_counter() - t0

    f, colors = synth.toy_scene(0)
    cam = f.cam.as_tuple()
    okf = oracle.ingest(f.depth, colors, fx=f.cam.fx, cam=cam, pose=f.pose)
    rng = np.random.default_rng(0)
    tgt = np.clip(colors + rng.uniform(-0.1, 0.1, colors.shape), 0, 1).astype(np.float32)
    ov = oracle.ViewSpec(cam, f.pose)
    for th in (1, threads):
        with oracle.threads(th):
            dt = min(fwd_bwd(ov, [okf], (tgt, f.depth), False) for _ in range(3))
        res["toy_64x48_threads%d" % th] = dict(mpix_s=64 * 48 / dt / 1e6, seconds=dt)
    if section is not None:
        frames = section
        okfs = [oracle.ingest(fr.depth, fr.rgb, fx=fr.cam.fx, cam=fr.cam.as_tuple(), pose=fr.pose)
                for fr in frames]
        fr = frames[3]
        v = oracle.ViewSpec(fr.cam.as_tuple(), fr.pose, 0, len(frames))
        with oracle.threads(threads):
            dt = fwd_bwd(v, okfs, (fr.rgb, fr.depth), True)
        res["mapping_view_640x480_8kf_threads%d" % threads] = dict(
            mpix_s=640 * 480 / dt / 1e6, seconds=dt,
            sample="one view of the 5-view mapping iteration (fwd + Eq. 2 + bwd)")
    if uneven_frames is not None:
        done = set()
        for vi in uneven_views:
            fr = uneven_frames[vi]
            wh = (fr.cam.width, fr.cam.height)
            if wh in done:
                continue
            done.add(wh)
            first = 8 * (vi // 8)
            sec = uneven_frames[first:first + 8]
            okfs = [oracle.ingest(x.depth, x.rgb, fx=x.cam.fx, cam=x.cam.as_tuple(), pose=x.pose)
                    for x in sec]
            v = oracle.ViewSpec(fr.cam.as_tuple(), fr.pose, 0, 8)
            with oracle.threads(threads):
                dt = fwd_bwd(v, okfs, (fr.rgb, fr.depth), True)
            res["uneven_view_%dx%d_threads%d" % (wh[0], wh[1], threads)] = dict(
                mpix_s=wh[0] * wh[1] / dt / 1e6, seconds=dt)
    return res


def batched_vs_single(iters):
    """5 of 8 section keyframes per mapping iteration: one plan vs one view per
    launch (render_fwd, host sync to size the pair list, render_bwd)."""
    import numpy as np
    import torch
    from paper_2506_02741_amd import render as R
    from paper_2506_02741_amd import synth
    sec = synth.section_workload(2, 8)
    frames = sec["keyframes"]
    cam = frames[0].cam.as_tuple()
    ks = [R.Keyframe.ingest(f.depth, f.rgb, cam, f.pose, learnable=True).with_grad_buffers()
          for f in frames]
    picks = synth.draw_views(2, 8, 5, iters + 2)
    ones = None

    def views_of(sel):
        return [R.View(cam, frames[i].pose, 0, 8) for i in sel]
    # batched: one plan per draw of 5 views, all sharing one workspace and
    # re-binding their descriptors before use
    first = R.Plan(ks, views_of(picks[0]))
    plans = [first] + [R.Plan(ks, views_of(sel), workspace=first.ws, bind=False) for sel in picks[1:]]
    g = torch.ones(3, first.P, device="cuda") * 1e-3
    for p in plans[:2]:
        p.bind(); p.render_fwd(); p.render_bwd(g, None, None, twist=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in plans[2:]:
        p.bind()
        p.render_fwd()
        p.render_bwd(g, None, None, twist=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    assert plans[-1].status()[0] == 0
    p = plans[-1]
    p.timing(True)
    p.render_fwd()
    p.render_bwd(g, None, None, twist=False)
    bstages = {s: v[0] for s, v in p.timing(False).items()}
    pairs = int(p.debug_state()["n_pairs"].item())
    # the units of that last batch's compositing launches and their rates
    cnt = scan_counts(p)
    roof = compositing_roofline(cnt, bstages)
    del plans, first, p
    # one view per launch
    singles = {i: R.Plan(ks, views_of([i])) for i in range(8)}
    g1 = torch.ones(3, singles[0].P, device="cuda") * 1e-3
    for i in picks[0]:
        singles[i].render_fwd(); singles[i].render_bwd(g1, None, None, twist=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sel in picks[2:]:
        for i in sel:
            p = singles[i]
            p.render_fwd()
            rc, need = p.status(clear=False)   # host sync sizing the pair list
            p.render_bwd(g1, None, None, twist=False)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    px = 5 * 640 * 480 * iters
    return dict(workload="mapping section: 8 keyframes 640x480 (2,457,600 Gaussians), 5 views "
                         "per iteration, fwd+bwd to colour/opacity/radius",
                iters=iters, batched_mpix_s=px / tb / 1e6, one_view_per_launch_mpix_s=px / ts / 1e6,
                speedup=ts / tb, batched_stages_ms=bstages, pairs=pairs, roofline=roof,
                counts=cnt), frames


def uneven_run(reps):
    """16 views of mixed resolution (320x240 / 640x480 / 1200x680) drawn from a
    3-section map of 24 keyframes; each view renders its section (8
    keyframes) and back-propagates to colour/opacity/radius.  The tile/batch
    shape comes from the autotuner's sweep; the batch runs as one captured
    graph of forward + backward, against one view per launch."""
    import tempfile
    import numpy as np
    import torch
    from paper_2506_02741_amd import autotune
    from paper_2506_02741_amd import render as R
    from paper_2506_02741_amd import synth
    t0 = time.perf_counter()
    w = synth.uneven_workload(3)
    frames = [f for sec in w["sections"] for f in sec]
    gen_s = time.perf_counter() - t0
    ks = [R.Keyframe.ingest(f.depth, f.rgb, f.cam.as_tuple(), f.pose, learnable=True).with_grad_buffers()
          for f in frames]
    views = [R.View(frames[v].cam.as_tuple(), frames[v].pose, 8 * (v // 8), 8) for v in w["views"]]
    px = sum(v.cam.width * v.cam.height for v in views)
    os.environ["VTGS_AUTOTUNE_CACHE"] = os.path.join(tempfile.mkdtemp(), "autotune.json")
    prm, entry = autotune.tune(ks, views, mode="map", reps=3, force=True)

    def timed_graph(prm):
        plan, _ = R.plan_checked(ks, views, prm, run=lambda p: (
            p.render_fwd(), p.render_bwd(gw(p), None, None, twist=False)))
        g = gw(plan)
        plan.render_fwd(); plan.render_bwd(g, None, None, twist=False)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            plan.render_fwd()
            plan.render_bwd(g, None, None, twist=False)
        graph.replay()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            graph.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / reps
        assert plan.status()[0] == 0
        return dt, plan.cap

    def gw(plan):
        return torch.ones(3, plan.P, device="cuda") * 1e-3
    tuned_s, cap = timed_graph(prm)
    default_s, _ = timed_graph(R.params())
    # one view per launch: forward, host sync sizing the pair list, backward
    singles = [R.plan_checked(ks, [v], prm, run=lambda p: (
        p.render_fwd(), p.render_bwd(gw(p), None, None, twist=False)))[0] for v in views]
    gs = [gw(p) for p in singles]
    for p, g in zip(singles, gs):
        p.render_fwd(); p.render_bwd(g, None, None, twist=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(max(1, reps // 2)):
        for p, g in zip(singles, gs):
            p.render_fwd()
            p.status(clear=False)
            p.render_bwd(g, None, None, twist=False)
    torch.cuda.synchronize()
    single_s = (time.perf_counter() - t) / max(1, reps // 2)
    n_gauss = sum(k.n for k in ks)
    return dict(workload="16 views (320x240/640x480/1200x680 uniform) of a 3-section map of 24 "
                         "keyframes, each view over its 8-keyframe section, fwd+bwd to "
                         "colour/opacity/radius, one captured graph",
                map_gaussians=n_gauss, pixels=px, tuned=dict(tile=entry["tile"], batch=entry["batch"]),
                sweep_ms=entry["sweep"], graph_mpix_s=px / tuned_s / 1e6,
                default_shape_mpix_s=px / default_s / 1e6, one_view_per_launch_mpix_s=px / single_s / 1e6,
                speedup=single_s / tuned_s, generation_s=gen_s), frames, list(w["views"])


def serving_run(seconds, rate, n_sections, budget_gib, seed=4, low_rate=0.0):
    """Poisson render/track requests against a device-resident map of
    n_sections x 10 keyframes at 1200x680, stride 2.  The map is built from
    3 ray-cast sections replicated on the device up to n_sections (a stand-in
    that keeps generation short; every section is its own copy in HBM)."""
    import numpy as np
    import torch
    from paper_2506_02741_amd import render as R
    from paper_2506_02741_amd import serve
    from paper_2506_02741_amd import synth
    t0 = time.perf_counter()
    m = synth.serving_sections(seed)
    base = []
    for sec in m["sections"]:
        base.append([R.Keyframe.ingest(f.depth, f.rgb, f.cam.as_tuple(), f.pose, stride=2)
                     for f in sec])
    kfs, sections = [], []
    for s in range(n_sections):
        src = base[s % len(base)]
        sections.append((len(kfs), len(src)))
        for k in src:
            kfs.append(R.Keyframe(k.cam, k.pose, k.pix, k.depth, k.color.clone(), k.opacity.clone(),
                                  k.radius.clone()))
    n_gauss = sum(k.n for k in kfs)
    # observations for track requests: a few frames per resolution per unique section
    rng = np.random.default_rng(seed)
    cams = [synth.camera_for(*wh).as_tuple() for wh in synth.RESOLUTIONS]
    obs = {}
    for u, sec in enumerate(m["sections"]):
        for ci, c in enumerate(cams):
            fr = sec[int(rng.integers(0, len(sec)))]
            cam = synth.Camera(*c)
            o = synth.frame(m["scene"], cam, fr.pose)
            obs[(u, ci)] = (o.pose, torch.tensor(o.rgb, device="cuda"),
                            torch.tensor(o.depth, device="cuda"))
    gen_s = time.perf_counter() - t0

    def poses_for(rng, sec, cam):
        ci = cams.index(cam)
        true = obs[(sec % len(base), ci)][0]
        return synth.perturb_pose(true, rng, 0.01, 0.5).astype(np.float32), (sec % len(base), ci)

    def obs_for(sec, cam, key):
        _, rgb, depth = obs[key]
        return rgb, depth
    budget = int(budget_gib * (1 << 30))

    def run(r, sd, warm_first, secs=seconds, pipeline=True):
        """One server on a fresh allocator state; freed before returning."""
        if warm_first:   # kernels and allocator warmed on a short prefix
            w = serve.Server(kfs, sections, budget_bytes=budget, max_active=64, pipeline=pipeline)
            w.run_trace(serve.poisson_trace(np.random.default_rng(seed + 2), r, 0.3, n_sections,
                                            cams, poses_for, obs_for), realtime=False)
            del w
        srv = serve.Server(kfs, sections, budget_bytes=budget, max_active=64, pipeline=pipeline)
        out = srv.run_trace(serve.poisson_trace(np.random.default_rng(sd), r, secs, n_sections,
                                                cams, poses_for, obs_for), realtime=True)
        out["peak_admitted_gib"] = srv.peak_mem / (1 << 30)
        del srv
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return out

    def drain(n_req, batched):
        """The same n_req requests, all queued at once: served in batched,
        pipelined ticks, or one request per launch (a single active request,
        each tick waited for)."""
        trace = serve.poisson_trace(np.random.default_rng(seed + 7), 1000.0, n_req / 1000.0,
                                    n_sections, cams, poses_for, obs_for)
        srv = serve.Server(kfs, sections, budget_bytes=budget, max_active=64 if batched else 1,
                           pipeline=batched)
        out = srv.run_trace(trace, realtime=False)
        del srv
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return out

    # served form against one request per launch, on the same requests
    log("bench: serving, %d queued requests batched vs one per launch" % args.serve_drain)
    drain(20, True); drain(5, False)   # warm both paths
    d_b, d_1 = drain(args.serve_drain, True), drain(args.serve_drain, False)
    served = dict(requests=d_b["requests"], batched_req_per_s=d_b["req_per_s"],
                  batched_mpix_per_s=d_b["mpix_per_s"],
                  one_per_launch_req_per_s=d_1["req_per_s"],
                  one_per_launch_mpix_per_s=d_1["mpix_per_s"],
                  speedup=d_b["mpix_per_s"] / d_1["mpix_per_s"])
    # sustainable rate: the highest offered rate whose p99 meets the objective
    sweep = []
    for r in args.serve_sweep:
        log("bench: serving sweep, %g req/s for %g s" % (r, args.serve_sweep_seconds))
        o = run(r, seed + 11, False, args.serve_sweep_seconds)
        sweep.append(dict(offered=r, served=o["req_per_s"], p50_ms=o["p50_ms"], p99_ms=o["p99_ms"]))
    ok = [x["offered"] for x in sweep if x["p99_ms"] is not None and x["p99_ms"] <= args.serve_p99_ms]
    if low_rate > 0:
        log("bench: serving %g req/s for %g s" % (low_rate, seconds))
    low = run(low_rate, seed + 3, True) if low_rate > 0 else None
    log("bench: serving %g req/s for %g s" % (rate, seconds))
    rep = run(rate, seed + 1, low is None)
    rep["served_vs_one_request_per_launch"] = served
    rep["rate_sweep"] = dict(p99_objective_ms=args.serve_p99_ms, seconds=args.serve_sweep_seconds,
                             runs=sweep, sustainable_req_per_s=max(ok) if ok else None)
    if low is not None:
        rep["at_lower_rate"] = dict(offered_req_per_s=low_rate, **{
            k: low[k] for k in ("requests", "req_per_s", "mpix_per_s", "p50_ms", "p99_ms",
                                "render_p50_ms", "render_p99_ms", "track_p50_ms", "track_p99_ms",
                                "mean_batch", "host_s", "device_wait_s", "seconds")})
    rep.update(offered_req_per_s=rate, map_gaussians=n_gauss, sections=n_sections,
               keyframes=len(kfs), budget_gib=budget_gib,
               generation_s=gen_s,
               workload="Poisson %g req/s for %g s, 60%% render / 40%% 20-iteration track, "
                        "resolutions 320x240/640x480/1200x680, map of %d sections x 10 keyframes "
                        "1200x680 stride 2" % (rate, seconds, n_sections))
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-all-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-configs", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-iters", type=int, default=20)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--uneven-reps", type=int, default=6)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one elementwise kernel that reads and writes 256 MiB (known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-drain", type=int, default=120,
                    help="requests of the batched vs one-request-per-launch comparison")
    ap.add_argument("--serve-sweep", type=float, nargs="*", default=[60.0, 100.0, 140.0])
    ap.add_argument("--serve-sweep-seconds", type=float, default=6.0)
    ap.add_argument("--serve-p99-ms", type=float, default=250.0,
                    help="p99 latency objective of the sustainable-rate sweep")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-rate-low", type=float, default=60.0,
                    help="a second, lower offered rate (0: skip)")
    ap.add_argument("--serve-sections", type=int, default=30)
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    global args
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the path has no multi-GPU "
              "collective); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_02741_amd import render as R
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    log("bench: building tracking workload (640x480, 307,200 Gaussians)")
    w, k, view, plan, init = tracking_setup()
    cfg = R.track_cfg(alpha=0.5, beta=1.0, lr_rot=0.002, lr_trans=0.002)
    # frames of up to 40 iterations; a non-default stream, so that each frame
    # length is one replay of a captured graph of the iteration's kernels.
    # The warmup runs every frame length the timed region uses (at least one
    # frame each, at least `warmup` iterations), so no graph is captured
    # while timing.
    frame = max(1, min(40, args.steps))
    loss = torch.zeros(frame, 1, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    lens = frame_lengths(args.steps, frame)
    warm = 0
    with torch.cuda.stream(stream):
        for n in lens:
            run_frames(plan, view, init, cfg, n, loss, frame)
            warm += n
        while warm < args.warmup:
            run_frames(plan, view, init, cfg, frame, loss, frame)
            warm += frame
    log("bench: warmup %d iterations (frames of %s)" % (warm, lens))
    torch.cuda.synchronize()
    rc, need = plan.status(stream=stream)
    if rc != 0:
        raise SystemExit("plan status %d (pairs needed %d)" % (rc, need))

    log("bench: timing %d iterations" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        run_frames(plan, view, init, cfg, args.steps, loss, frame)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rc, need = plan.status(stream=stream)
    assert rc == 0, rc
    value = 640 * 480 * args.steps / dt / 1e6

    # per-stage durations from HIP events on the launch stream (eager
    # launches while timing is on; each compositing stage is launched 10
    # times back to back between its events, so that its per-launch time
    # leaves out the events' own overhead)
    log("bench: stage timing")
    plan.timing(True, repeat=10)
    with torch.cuda.stream(stream):
        run_frames(plan, view, init, cfg, 2 * frame, loss, frame)
    stages = plan.timing(False)
    avg = {s: ms / n for s, (ms, n) in stages.items()}
    dom = max(stages, key=lambda s: stages[s][0])

    if args.calib_copy:
        # an elementwise kernel that reads 256 MiB and writes 256 MiB
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b

    # units per launch: counted at the initial pose of the frame and at the
    # pose the timed frames end on, averaged
    counts = []
    for pose in (init, view.pose.clone()):
        view.pose.copy_(pose)
        with torch.cuda.stream(stream):
            plan.render_fwd(stream=stream)
        torch.cuda.synchronize()
        counts.append(scan_counts(plan))
    cnt = {key: sum(c[key] for c in counts) / len(counts) for key in counts[0]}
    comp = compositing_roofline(cnt, avg)
    roof = None
    if dom in comp:
        d = comp[dom]
        per = LANE_OPS["fwd_contrib" if dom == "composite_fwd" else "bwd_contrib"]
        roof = dict(kernel=dom, bound="alu", achieved=d["achieved"], peak=PEAK_LANE_OPS_T,
                    unit="Tlane-op/s", frac=d["frac"], traffic=measured_traffic(dom),
                    avg_ms=d["avg_ms"], lane_ops_per_launch=d["contrib_lane_ops"],
                    units="%.0f contributing (pixel, Gaussian) pairs per launch (%.1f per pixel), "
                          "%d lane-ops each" % (cnt["contrib"], cnt["contrib"] / (640 * 480), per),
                    with_list_steps=dict(d["with_list_steps"], units=(
                        "%.0f pixel-entry steps (%.1f per pixel) of which %.0f contributing; "
                        "%d lane-ops per entry stepped past, %d per contributor"
                        % ((cnt["fwd_scanned"], cnt["fwd_scanned"] / (640 * 480), cnt["contrib"],
                            LANE_OPS["fwd_skip"], LANE_OPS["fwd_contrib"])
                           if dom == "composite_fwd" else
                           (cnt["bwd_scanned"], cnt["bwd_scanned"] / (640 * 480), cnt["contrib"],
                            LANE_OPS["bwd_skip"], LANE_OPS["bwd_contrib"])))))
        other = "composite_bwd" if dom == "composite_fwd" else "composite_fwd"
        if other in comp:
            roof[other] = dict(comp[other], traffic=measured_traffic(other))
        roof["counts"] = cnt

    batched = section_frames = None
    if not args.no_batched:
        log("bench: batched vs one view per launch")
        batched, section_frames = batched_vs_single(args.batched_iters)

    uneven = uneven_frames = uneven_views = None
    if not args.no_uneven:
        log("bench: uneven 16-view batch with autotuned tiles")
        uneven, uneven_frames, uneven_views = uneven_run(args.uneven_reps)

    serving = None
    if not args.no_serving:
        log("bench: serving %g s at %g req/s" % (args.serve_seconds, args.serve_rate))
        serving = serving_run(args.serve_seconds, args.serve_rate, args.serve_sections,
                              args.serve_budget_gib, low_rate=args.serve_rate_low)

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (~%.0f s single-threaded, ~%.0f s all cores)"
            % (args.cpu_seconds, args.cpu_all_seconds))
        cpu = cpu_baseline(w, args.cpu_seconds, args.cpu_all_seconds)
        if not args.no_cpu_configs:
            log("bench: CPU oracle on the other workloads (bounded samples)")
            cpu["other_workloads"] = cpu_configs(section_frames, uneven_frames, uneven_views,
                                                 cpu["cores_available"])

    out = dict(metric="fwd+bwd Mpix/s at 640x480 vs 1-view/launch; p50/p99 render-request latency",
               value=value, unit="Mpix/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=dt * 1e3 / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload="tracking 640x480: 1 keyframe, 307,200 view-tied Gaussians, "
                                    "%d-iteration frames of fwd + Eq.1 + bwd to twist + pose step"
                                    % frame,
                           global_batch=1, seq_len=0, parallelism="none"),
               roofline=roof, cpu_baseline=cpu, stages_ms=avg, batched=batched, uneven=uneven,
               serving=serving)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
