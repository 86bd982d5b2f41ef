#!/usr/bin/env python3
"""Benchmark of the view-tied splatting renderer on one MI355X.

Metric: forward+backward Mpix/s at 640x480.  Workload (the tracking
configuration): one 640x480 keyframe of a synthetic room tied to 307,200
Gaussians, a new frame observed at the keyframe pose whose initial estimate
is off by 1 cm / 0.5 degrees; each frame runs 40 tracking iterations of
splat forward -> Eq. 1 loss -> backward to the SE(3) twist -> Adam step and
retraction.  A step is one such iteration; value = 640*480*steps / seconds.

Also reported on the same JSON line:
  roofline      the dominant kernel's achieved rate vs the MI355X peak,
                from HIP events on the stream the kernels run on
  cpu_baseline  the CPU oracle (single thread) on a bounded sample of the
                same workload
  batched       mapping-section batch (5 of 8 keyframes per iteration,
                gradients to colour/opacity/radius) in one plan vs one view
                per launch with a host sync in between
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0


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


def run_frames(plan, view, init, cfg, iters, loss):
    """iters tracking iterations in frames of 40 from the initial pose."""
    done = 0
    while done < iters:
        n = min(40, iters - done)
        view.pose.copy_(init)
        view.pose_adam.zero_()
        plan.track_step(cfg, n, loss[:n])
        done += n


def flops_per_pair():
    """FP32 operations per contributing (pixel, Gaussian) pair, counted from
    the compositing arithmetic (add, mul, min = 1; fma = 2; exp2, rcp = 1;
    compares and selects not counted).  Forward: d (2), q (8), G (2), alpha
    (2), transmittance (2), weight (1), colour and depth accumulation (8) =
    25.  Backward to the twist: d and q (10), G (2), alpha (2), o G and
    1 - alpha (2), T recovery (2), weight (1), dL/dalpha (15), the behind
    accumulators (15), dL/dq (2), w = Q d and t = J^T w (11), dL/dp (16),
    rho and phi sums (15) = 99.  Pairs that cover a pixel without
    contributing are not counted (a lower bound on the work)."""
    return dict(fwd_contrib=25, bwd_contrib=99)


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


def pair_counts(w):
    """Per-frame counts of tested / covering / contributing pairs from the
    oracle's per-pixel lists (the workload's own numbers)."""
    import numpy as np
    import oracle
    kf = w["keyframe"]
    okf = oracle.ingest(kf.depth, kf.rgb, fx=kf.cam.fx, cam=kf.cam.as_tuple(), pose=kf.pose)
    out = oracle.render(oracle.ViewSpec(kf.cam.as_tuple(), w["init_pose"]), [okf])
    contrib = int(out["n_contrib"].sum())
    return contrib, out


def cpu_baseline(w, seconds):
    import numpy as np
    import oracle
    kf = w["keyframe"]
    okf = oracle.ingest(kf.depth, kf.rgb, fx=kf.cam.fx, cam=kf.cam.as_tuple(), pose=kf.pose)
    pose = np.asarray(w["init_pose"], np.float32)
    st = dict(m=np.zeros(6), v=np.zeros(6), t=0)
    n = 0
    t0 = time.perf_counter()
    while True:
        view = oracle.ViewSpec(kf.cam.as_tuple(), pose)
        L, new_pose, st, g, _ = oracle.track_iteration(view, [okf], kf.rgb, kf.depth, st)
        pose = new_pose.astype(np.float32)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return dict(value=640 * 480 * n / dt / 1e6, unit="Mpix/s", cores=1, kind="oracle",
                sample="%d tracking iterations (fwd + Eq.1 + bwd to twist + Adam/retraction) of "
                       "the 640x480 frame, single-threaded, %.1f s" % (n, dt))


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
                speedup=ts / tb, batched_stages_ms=bstages, pairs=pairs)


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
                speedup=single_s / tuned_s, generation_s=gen_s)


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

    def run(r, sd, warm_first):
        """One server on a fresh allocator state; freed before returning."""
        if warm_first:   # kernels and allocator warmed on a short prefix
            w = serve.Server(kfs, sections, budget_bytes=budget, max_active=64)
            w.run_trace(serve.poisson_trace(np.random.default_rng(seed + 2), r, 0.3, n_sections,
                                            cams, poses_for, obs_for), realtime=False)
            del w
        srv = serve.Server(kfs, sections, budget_bytes=budget, max_active=64)
        out = srv.run_trace(serve.poisson_trace(np.random.default_rng(sd), r, seconds, n_sections,
                                                cams, poses_for, obs_for), realtime=True)
        out["peak_admitted_gib"] = srv.peak_mem / (1 << 30)
        del srv
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return out
    low = run(low_rate, seed + 3, True) if low_rate > 0 else None
    rep = run(rate, seed + 1, low is None)
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-iters", type=int, default=20)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--uneven-reps", type=int, default=6)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one elementwise kernel that reads and writes 256 MiB (known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-rate-low", type=float, default=60.0,
                    help="a second, lower offered rate (0: skip)")
    ap.add_argument("--serve-sections", type=int, default=30)
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
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
    loss = torch.zeros(40, 1, device="cuda")
    # a non-default stream: each 40-iteration frame is one replay of a
    # captured graph of the iteration's kernels
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    log("bench: warmup %d iterations" % args.warmup)
    with torch.cuda.stream(stream):
        run_frames(plan, view, init, cfg, args.warmup, loss)
    torch.cuda.synchronize()
    rc, need = plan.status(stream=stream)
    if rc != 0:
        raise SystemExit("plan status %d (pairs needed %d)" % (rc, need))

    log("bench: timing %d iterations" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        run_frames(plan, view, init, cfg, args.steps, loss)
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
        run_frames(plan, view, init, cfg, 80, loss)
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

    contrib, _ = pair_counts(w)
    fl = flops_per_pair()
    roof = None
    per = {"composite_bwd": fl["bwd_contrib"], "composite_fwd": fl["fwd_contrib"]}.get(dom)
    if per is not None:
        work = contrib * per
        achieved = work / (avg[dom] * 1e-3) / 1e12
        roof = dict(kernel=dom, bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS,
                    unit="TFLOP/s", frac=achieved / PEAK_FP32_TFLOPS,
                    traffic=measured_traffic(dom),
                    avg_ms=avg[dom], flops_per_launch=work,
                    units="%d contributing (pixel, Gaussian) pairs x %d FLOP" % (contrib, per))
        # the other compositing kernel, same accounting
        other = "composite_bwd" if dom == "composite_fwd" else "composite_fwd"
        if avg.get(other):
            op = fl["bwd_contrib"] if other == "composite_bwd" else fl["fwd_contrib"]
            a2 = contrib * op / (avg[other] * 1e-3) / 1e12
            roof[other] = dict(avg_ms=avg[other], achieved=a2, frac=a2 / PEAK_FP32_TFLOPS,
                               traffic=measured_traffic(other))

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (~%.0f s)" % args.cpu_seconds)
        cpu = cpu_baseline(w, args.cpu_seconds)

    batched = None
    if not args.no_batched:
        log("bench: batched vs one view per launch")
        batched = batched_vs_single(args.batched_iters)

    uneven = None
    if not args.no_uneven:
        log("bench: uneven 16-view batch with autotuned tiles")
        uneven = uneven_run(args.uneven_reps)

    serving = None
    if not args.no_serving:
        log("bench: serving %g s at %g req/s" % (args.serve_seconds, args.serve_rate))
        serving = serving_run(args.serve_seconds, args.serve_rate, args.serve_sections,
                              args.serve_budget_gib, low_rate=args.serve_rate_low)

    out = dict(metric="fwd+bwd Mpix/s at 640x480 vs 1-view/launch; p50/p99 render-request latency",
               value=value, unit="Mpix/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=dt * 1e3 / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload="tracking 640x480: 1 keyframe, 307,200 view-tied Gaussians, "
                                    "40-iteration frames of fwd + Eq.1 + bwd to twist + pose step",
                           global_batch=1, seq_len=0, parallelism="none"),
               roofline=roof, cpu_baseline=cpu, stages_ms=avg, batched=batched, uneven=uneven,
               serving=serving)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
