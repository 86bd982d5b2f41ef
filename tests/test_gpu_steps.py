"""track_step and map_step through the C ABI against the oracle, one
iteration from identical state, plus the behavioural tracking check.

A first Adam step is -lr * m_hat / (sqrt(v_hat) + eps) = -lr g / (|g| + eps),
i.e. about -lr sign(g): updates are compared where |g| is clearly above eps
and the sign is therefore decided identically."""
import math

import numpy as np
import pytest

from scenes import oracle_kf, room_frames

pytestmark = pytest.mark.gpu
MARGIN = 2e-6


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2506_02741_amd import render
    return render


def np_(t):
    return t.detach().cpu().numpy()


def pose_error(T, Tref):
    T = np.asarray(T, np.float64).reshape(3, 4); Tref = np.asarray(Tref, np.float64).reshape(3, 4)
    Rc = T[:, :3].T; c = -Rc @ T[:, 3]
    Rr = Tref[:, :3].T; cr = -Rr @ Tref[:, 3]
    dR = Rc.T @ Rr
    ang = math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(dR) - 1) / 2))))
    return float(np.linalg.norm(c - cr)), ang


def test_track_one_iteration(R, orc):
    from paper_2506_02741_amd import synth
    w = synth.tracking_workload(1, 160, 120)
    kf = w["keyframe"]
    cam = kf.cam.as_tuple()
    k = R.Keyframe.ingest(kf.depth, kf.rgb, cam, kf.pose)
    view = R.View(cam, w["init_pose"], obs_rgb=kf.rgb, obs_depth=kf.depth).with_pose_adam()
    plan = R.Plan([k], [view])
    cfg = R.track_cfg(alpha=0.5, beta=1.0, lr_rot=0.002, lr_trans=0.002)
    loss = plan.track_step(cfg, iters=1)
    assert plan.status()[0] == 0
    L_ref, pose_ref, st, g_ref, _ = orc.track_iteration(
        orc.ViewSpec(cam, w["init_pose"]), [oracle_kf(orc, kf)], kf.rgb, kf.depth,
        dict(m=np.zeros(6), v=np.zeros(6), t=0))
    assert abs(float(np_(loss)[0, 0]) - L_ref) <= 1e-4 * abs(L_ref)
    assert np.all(np.abs(g_ref) > 1e-3 * np.abs(g_ref).max())
    assert np.allclose(np_(view.pose).reshape(3, 4), pose_ref, atol=2e-6), (np_(view.pose), pose_ref)
    ad = np_(view.pose_adam)
    assert ad[12] == 1.0
    assert np.allclose(ad[:6], 0.1 * g_ref, rtol=2e-3, atol=1e-6 * np.abs(g_ref).max())


def test_map_then_track_converges(R, orc):
    """Behavioural (the exact trajectory is not pinned): map the keyframe's
    Gaussians against its own RGBD (Eq. 2), then track a new frame observed
    at the keyframe pose from a 1 cm / 0.5 degree perturbation (Eq. 1).  The
    mapping loss falls, and 40 tracking iterations reduce the loss and the
    pose error.  Raw ingested Gaussians (o = 0.99, one-pixel footprint) blur
    slanted surfaces in depth order, which moves the tracking optimum; the
    paper tracks against mapped Gaussians."""
    import torch
    from paper_2506_02741_amd import synth
    w = synth.tracking_workload(1, 320, 240)
    kf = w["keyframe"]
    cam = kf.cam.as_tuple()
    k = R.Keyframe.ingest(kf.depth, kf.rgb, cam, kf.pose, learnable=True).with_adam()
    mp = R.Plan([k], [R.View(cam, kf.pose, obs_rgb=kf.rgb, obs_depth=kf.depth)])
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    ml = [float(mp.map_step(step)[0]) for _ in range(150)]
    assert mp.status()[0] == 0
    assert np.mean(ml[-10:]) < 0.7 * np.mean(ml[:3]), (ml[:3], ml[-10:])
    view = R.View(cam, w["init_pose"], obs_rgb=kf.rgb, obs_depth=kf.depth).with_pose_adam()
    plan = R.Plan([k], [view])
    e0 = pose_error(w["init_pose"], w["true_pose"])
    loss = np_(plan.track_step(R.track_cfg(), iters=40))[:, 0]
    assert plan.status()[0] == 0
    e1 = pose_error(np_(view.pose), w["true_pose"])
    assert loss[-5:].mean() < loss[:3].mean(), loss
    assert e1[0] < e0[0] and e1[1] < e0[1], (e0, e1)


def test_track_batched_views_match_single(R):
    """Two tracking requests in one plan follow the same trajectory as each
    alone (the pose path has no atomics, so bit-identical)."""
    from paper_2506_02741_amd import synth
    ws = [synth.tracking_workload(s, 96, 72) for s in (1, 2)]
    ks = [R.Keyframe.ingest(w["keyframe"].depth, w["keyframe"].rgb, w["keyframe"].cam.as_tuple(),
                            w["keyframe"].pose) for w in ws]

    def views():
        return [R.View(w["keyframe"].cam.as_tuple(), w["init_pose"], i, 1, w["keyframe"].rgb,
                       w["keyframe"].depth).with_pose_adam() for i, w in enumerate(ws)]
    vb = views()
    R.Plan(ks, vb).track_step(R.track_cfg(), iters=5)
    for i in range(2):
        vs = views()[i]
        R.Plan(ks, [vs]).track_step(R.track_cfg(), iters=5)
        assert np.array_equal(np_(vs.pose), np_(vb[i].pose))


def _oracle_map_iteration(orc, cams, poses, okfs, obs, cfg):
    """Eq. 2 per view, gradients summed over views, one Adam step."""
    N = sum(k.n for k in okfs)
    gc = np.zeros((3, N)); go = np.zeros(N); gr = np.zeros(N)
    losses = []
    for cam, pose, (orgb, odep) in zip(cams, poses, obs):
        v = orc.ViewSpec(cam, pose, 0, len(okfs))
        out = orc.render(v, okfs, margin=MARGIN)
        L, g_rgb, g_d = orc.map_loss(cam[5], cam[4], out["rgb"], out["depth"], orgb, odep,
                                     cfg["rho"], cfg["tau"], cfg["sigma"])
        losses.append(L)
        g = orc.render_bwd(v, okfs, g_rgb, g_d, None)
        gc += g["color"]; go += g["opacity"]; gr += g["radius"]
    return np.array(losses), gc, go, gr


def _section_inputs(frames, seed=0):
    """Gaussians at every pixel of each frame (all depths are valid in the
    generated rooms) with seeded colour, opacity and radius: the same arrays
    go to the oracle and to the GPU."""
    rng = np.random.default_rng(seed)
    out = []
    for f in frames:
        n = f.depth.size
        out.append(dict(pix=np.arange(n, dtype=np.uint32), depth=f.depth.ravel().copy(),
                        color=np.clip(f.rgb.reshape(3, -1) + rng.uniform(-0.1, 0.1, (3, n)), 0, 1).astype(np.float32),
                        opacity=rng.uniform(0.6, 0.95, n).astype(np.float32),
                        radius=rng.uniform(0.002, 0.012, n).astype(np.float32)))
    return out


def test_map_one_iteration(R, orc):
    import torch
    cam, frames, _ = room_frames(9, 64, 48, n_kf=2)
    assert all(np.all(f.depth > 0) for f in frames)
    inp = _section_inputs(frames)
    ks = [R.Keyframe(cam.as_tuple(), f.pose, d["pix"].astype(np.int32), d["depth"], d["color"], d["opacity"],
                     d["radius"], learnable=True).with_adam() for f, d in zip(frames, inp)]
    okfs = [orc.Keyframe(cam.as_tuple(), f.pose, d["pix"], d["depth"], d["color"], d["opacity"], d["radius"])
            for f, d in zip(frames, inp)]
    views = [R.View(cam.as_tuple(), f.pose, 0, 2, f.rgb, f.depth) for f in frames]
    plan = R.Plan(ks, views)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    cfg = dict(rho=0.8, tau=0.2, sigma=1.0)
    loss = np_(plan.map_step(step, R.map_cfg(**cfg)))
    assert plan.status()[0] == 0 and int(step.item()) == 1
    L_ref, gc, go, gr = _oracle_map_iteration(orc, [cam.as_tuple()] * 2, [f.pose for f in frames], okfs,
                                              [(f.rgb, f.depth) for f in frames], cfg)
    assert np.allclose(loss, L_ref, rtol=1e-4), (loss, L_ref)
    n0 = ks[0].n
    lrs = dict(color=0.0025, opacity=0.05, radius=0.005)
    for i, (k, d) in enumerate(zip(ks, inp)):
        sl = slice(0, n0) if i == 0 else slice(n0, n0 + k.n)
        c0, o0, r0 = d["color"].astype(np.float64), d["opacity"].astype(np.float64), d["radius"].astype(np.float64)
        g_logit = go[sl] * o0 * (1 - o0)
        g_log = gr[sl] * r0
        new_c, new_o, new_r = (np_(k.color).astype(np.float64), np_(k.opacity).astype(np.float64),
                               np_(k.radius).astype(np.float64))
        for got, old, g, lr, name in (
                (new_c, c0, gc[:, sl], lrs["color"], "color"),
                (np.log(new_o / (1 - new_o)), np.log(o0 / (1 - o0)), g_logit, lrs["opacity"], "opacity"),
                (np.log(new_r), np.log(r0), g_log, lrs["radius"], "radius")):
            step_ref = -lr * g / (np.abs(g) + 1e-8)
            sure = np.abs(g) > 1e-6
            assert sure.mean() > 0.5, name
            d_ = (got - old)[sure]
            assert np.all(np.abs(d_ - step_ref[sure]) <= 2e-3 * lr + 2e-6), name
            assert np.all(np.abs(got - old) <= lr * 1.001 + 2e-6), name


def test_track_graph_replay_equals_eager(R):
    """track_step replays a captured graph on a non-default stream; several
    replays, with eager work and synchronisation between them, give the same
    poses and losses bit for bit as eager launches."""
    import os
    import torch
    from paper_2506_02741_amd import synth
    w = synth.tracking_workload(1, 160, 120)
    kf = w["keyframe"]
    cam = kf.cam.as_tuple()
    k = R.Keyframe.ingest(kf.depth, kf.rgb, cam, kf.pose)
    init = torch.tensor(np.asarray(w["init_pose"], np.float32).reshape(12), device="cuda")
    cfg = R.track_cfg()
    out = {}
    for mode in ("eager", "graph"):
        view = R.View(cam, init.clone(), obs_rgb=kf.rgb, obs_depth=kf.depth).with_pose_adam()
        plan = R.Plan([k], [view])
        torch.cuda.synchronize()
        loss = torch.zeros(8, 1, device="cuda")
        s = torch.cuda.Stream()
        res = []
        with torch.cuda.stream(s):
            for rep in range(3):
                view.pose.copy_(init)
                view.pose_adam.zero_()
                if mode == "eager":
                    os.environ["VTGS_NO_GRAPH"] = "1"
                try:
                    plan.track_step(cfg, 8, loss)
                finally:
                    os.environ.pop("VTGS_NO_GRAPH", None)
                s.synchronize()
                res.append((np_(view.pose).copy(), np_(loss).copy()))
                _ = (view.pose * 2).sum().item()   # unrelated eager work between replays
        assert plan.status()[0] == 0
        out[mode] = res
    for (pe, le), (pg, lg) in zip(out["eager"], out["graph"]):
        assert np.array_equal(pe, pg) and np.array_equal(le, lg)
    assert np.array_equal(out["graph"][0][0], out["graph"][2][0])


def test_map_graph_replay_equals_eager(R):
    """map_step replays its captured iteration on a non-default stream: four
    iterations, with eager work and synchronisation between them, give the
    same parameters, Adam states and losses bit for bit as eager launches
    (the step counter advances on the device)."""
    import os
    import torch
    cam, frames, _ = room_frames(9, 64, 48, n_kf=2)
    inp = _section_inputs(frames)
    out = {}
    for mode in ("eager", "graph"):
        ks = [R.Keyframe(cam.as_tuple(), f.pose, d["pix"].astype(np.int32), d["depth"], d["color"],
                         d["opacity"], d["radius"], learnable=True).with_adam() for f, d in zip(frames, inp)]
        views = [R.View(cam.as_tuple(), f.pose, 0, 2, f.rgb, f.depth) for f in frames]
        plan = R.Plan(ks, views)
        step = torch.zeros(1, dtype=torch.int32, device="cuda")
        loss = torch.zeros(2, device="cuda")
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        res = []
        with torch.cuda.stream(s):
            for it in range(4):
                if mode == "eager":
                    os.environ["VTGS_NO_GRAPH"] = "1"
                try:
                    plan.map_step(step, R.map_cfg(), loss)
                finally:
                    os.environ.pop("VTGS_NO_GRAPH", None)
                s.synchronize()
                res.append(np_(loss).copy())
                _ = (ks[0].color * 2).sum().item()   # unrelated eager work between replays
        assert plan.status()[0] == 0 and int(step.item()) == 4
        out[mode] = (res, [(np_(k.color), np_(k.opacity), np_(k.radius), np_(k.adam)) for k in ks])
    for a, b in zip(out["eager"][0], out["graph"][0]):
        assert np.array_equal(a, b)
    for ka, kb in zip(out["eager"][1], out["graph"][1]):
        for a, b in zip(ka, kb):
            assert np.array_equal(a, b)
    assert not np.array_equal(out["graph"][0][0], out["graph"][0][3])  # it did learn


def test_batched_fwd_bwd_graph_replay_equals_eager(R):
    """Forward + backward of a multi-view mapping plan captured once in a
    graph: every replay (with eager work and syncs between replays) gives
    the eager images and gradients bit for bit."""
    import numpy as np
    import torch
    from scenes import room_frames
    cam, frames, _ = room_frames(9, 96, 72, n_kf=3)
    ks = [R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose, learnable=True).with_grad_buffers()
          for f in frames]
    views = [R.View(cam.as_tuple(), f.pose, 0, 3) for f in frames]
    plan = R.Plan(ks, views)
    rng = np.random.default_rng(7)
    g = torch.tensor(rng.normal(size=(3, plan.P)), dtype=torch.float32, device="cuda")
    gd = torch.tensor(rng.normal(size=plan.P), dtype=torch.float32, device="cuda")

    def zero():
        for k in ks:
            k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()

    def grads():
        return [t.clone() for k in ks for t in (k.g_color, k.g_opacity, k.g_radius)]
    zero()
    ref_img = [x.clone() for x in plan.render_fwd()]
    plan.render_bwd(g, gd, None, twist=False)
    ref_g = grads()
    assert plan.status()[0] == 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        img = plan.render_fwd()
        plan.render_bwd(g, gd, None, twist=False)
    torch.cuda.synchronize()
    for rep in range(3):
        zero()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(img, ref_img):
            assert torch.equal(a, b), rep
        for a, b in zip(grads(), ref_g):
            assert torch.equal(a, b), rep
        plan.render_fwd()          # eager work between replays
        torch.cuda.synchronize()


def test_stage_timing_with_repeats_changes_nothing(R):
    """Stage timing that launches each compositing stage several times
    counts every launch and leaves the images and gradients bit for bit as
    without timing (the compositing stages overwrite what they write)."""
    import numpy as np
    import torch
    from scenes import room_frames
    cam, frames, _ = room_frames(11, 96, 72, n_kf=2)
    ks = [R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose, learnable=True).with_grad_buffers()
          for f in frames]
    plan = R.Plan(ks, [R.View(cam.as_tuple(), f.pose, 0, 2) for f in frames])
    rng = np.random.default_rng(3)
    g = torch.tensor(rng.normal(size=(3, plan.P)), dtype=torch.float32, device="cuda")

    def run():
        for k in ks:
            k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
        img = [x.clone() for x in plan.render_fwd()]
        plan.render_bwd(g, None, None, twist=False)
        torch.cuda.synchronize()
        return img + [t.clone() for k in ks for t in (k.g_color, k.g_opacity, k.g_radius)]
    ref = run()
    plan.timing(True, repeat=3)
    got = run()
    stages = plan.timing(False)
    assert plan.status()[0] == 0
    assert stages["composite_fwd"][1] == 3 and stages["composite_bwd"][1] == 3, stages
    assert stages["preprocess"][1] == 1, stages
    for a, b in zip(got, ref):
        assert torch.equal(a, b)


# ----------------------------------------------------------------------------
# map_step and track_step in magnitude, two optimiser steps each
# ----------------------------------------------------------------------------

def _near_flagged(orc, ov, okfs, flagged_px, W):
    """Local ids of the Gaussians whose extent box (mu +- R, one pixel wider)
    holds a flagged pixel: their gradients may follow either outcome."""
    rec = orc.preprocess32(ov, okfs)
    near = np.zeros(rec.shape[0], bool)
    for p in flagged_px:
        x, y = p % W, p // W
        near |= (rec["count"] > 0) & (np.abs(rec["mx"] - x) <= rec["ext"] + 1) & \
            (np.abs(rec["my"] - y) <= rec["ext"] + 1)
    return near


def _map_state(k):
    n = k.n
    ad = np_(k.adam).astype(np.float64)
    return dict(color=np_(k.color).astype(np.float64), opacity=np_(k.opacity).astype(np.float64),
                radius=np_(k.radius).astype(np.float64), m=ad[:5], v=ad[5:])


def test_map_step_gradients_and_adam_two_steps(R, orc):
    """Two map_step iterations over a two-keyframe section seen by two views
    (Sec. 3.4, Eq. 2; App. A learning rates), each checked stage by stage
    against the oracle from the GPU's own state at that step:
    - the rendered images (1e-5, every pixel, near-ties by their outcomes);
    - the upstream gradient images Eq. 2 forms from them (L1 and SSIM terms)
      and the per-view loss, against the oracle's Eq. 2 on the same images;
    - the per-Gaussian gradients the Adam step used (slots summed over both
      views), against the oracle's backward of those upstream images summed
      over views, at the 1e-3 relative bar;
    - the Adam moments and the new (c, o, r) against an FP64 Adam step on
      (c, logit o, log r) from the GPU's gradient and previous state."""
    import torch
    from test_gpu_parity import check_images, grad_close, oracle_ref
    cam, frames, _ = room_frames(9, 64, 48, n_kf=2)
    c = cam.as_tuple()
    W, H = c[4], c[5]
    P = W * H
    inp = _section_inputs(frames)
    ks = [R.Keyframe(c, f.pose, d["pix"].astype(np.int32), d["depth"], d["color"], d["opacity"],
                     d["radius"], learnable=True).with_adam().with_grad_buffers()
          for f, d in zip(frames, inp)]
    views = [R.View(c, f.pose, 0, 2, f.rgb, f.depth) for f in frames]
    plan = R.Plan(ks, views)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    cfg = dict(rho=0.8, tau=0.2, sigma=1.0)
    lrs = [0.0025, 0.0025, 0.0025, 0.05, 0.005]
    n0 = ks[0].n
    before = [_map_state(k) for k in ks]
    for t in (1, 2):
        okfs = [orc.Keyframe(c, f.pose, d["pix"], d["depth"], s["color"].astype(np.float32),
                             s["opacity"].astype(np.float32), s["radius"].astype(np.float32))
                for f, d, s in zip(frames, inp, before)]
        for k in ks:
            k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
        loss = np_(plan.map_step(step, R.map_cfg(**cfg)))
        img, gimg = (np_(x).astype(np.float64) for x in plan.debug_images())
        plan.debug_gather()
        assert plan.status()[0] == 0 and int(step.item()) == t
        gc = np.zeros((3, sum(k.n for k in ks))); go = np.zeros(gc.shape[1]); gr = np.zeros(gc.shape[1])
        mc = np.zeros_like(gc); mo = np.zeros_like(go); mr = np.zeros_like(gr)
        skip = np.zeros(gc.shape[1], bool)
        for v, f in enumerate(frames):
            sl = slice(v * P, (v + 1) * P)
            ov = orc.ViewSpec(c, f.pose, 0, 2)
            ref = oracle_ref(orc, ov, okfs)
            check_images(img[:3, sl], img[3, sl], img[4, sl], ref)
            # Eq. 2 on the GPU's own images: the upstream gradients exactly
            L, g_rgb, g_d = orc.map_loss(H, W, img[:3, sl], img[3, sl], f.rgb, f.depth,
                                         cfg["rho"], cfg["tau"], cfg["sigma"])
            assert abs(loss[v] - L) <= 1e-5 * abs(L), (t, v, loss[v], L)
            ok, worst = grad_close(gimg[:3, sl], g_rgb, "d Eq.2 / d rgb (t=%d)" % t)
            assert ok, worst
            ok, worst = grad_close(gimg[3, sl], g_d, "d Eq.2 / d depth (t=%d)" % t)
            assert ok, worst
            assert not gimg[4, sl].any()
            g = orc.render_bwd(ov, okfs, gimg[:3, sl], gimg[3, sl], None)
            gc += g["color"]; go += g["opacity"]; gr += g["radius"]
            mc += g["mag"]["color"]; mo += g["mag"]["opacity"]; mr += g["mag"]["radius"]
            skip |= _near_flagged(orc, ov, okfs, np.nonzero(ref["marginal"])[0], W)
        got = [np.concatenate([np_(k.g_color) for k in ks], 1), np.concatenate([np_(k.g_opacity) for k in ks]),
               np.concatenate([np_(k.g_radius) for k in ks])]
        assert skip.mean() < 0.05
        for a, b, m, name in zip(got, (gc, go, gr), (mc, mo, mr), ("colour", "opacity", "radius")):
            ok, worst = grad_close(a[..., ~skip], b[..., ~skip], "map %s (t=%d)" % (name, t),
                                   m[..., ~skip])
            assert ok, worst
        # Adam on (c, logit o, log r) in FP64 from the GPU's gradient and state
        after = [_map_state(k) for k in ks]
        for i, (k, b0, a1) in enumerate(zip(ks, before, after)):
            sl = slice(0, n0) if i == 0 else slice(n0, n0 + k.n)
            o0, r0 = b0["opacity"], b0["radius"]
            x = np.concatenate([b0["color"], np.log(o0 / (1 - o0))[None], np.log(r0)[None]], 0)
            gx = np.concatenate([got[0][:, sl], (got[1][sl] * o0 * (1 - o0))[None],
                                 (got[2][sl] * r0)[None]], 0).astype(np.float64)
            m, vv = b0["m"].copy(), b0["v"].copy()
            for ch in range(5):
                xc, mc, vc = x[ch].copy(), m[ch].copy(), vv[ch].copy()
                orc.adam(xc, gx[ch], mc, vc, t, lrs[ch])
                x[ch], m[ch], vv[ch] = xc, mc, vc
            assert np.allclose(a1["m"], m, rtol=2e-6, atol=1e-12), (t, i)
            assert np.allclose(a1["v"], vv, rtol=5e-6, atol=1e-18), (t, i)
            assert np.allclose(a1["color"], x[:3], rtol=0, atol=2e-6)
            assert np.allclose(a1["opacity"], 1 / (1 + np.exp(-x[3])), rtol=2e-6, atol=0)
            assert np.allclose(a1["radius"], np.exp(x[4]), rtol=2e-6, atol=0)
        before = after


def test_track_two_iterations(R, orc):
    """Two tracking iterations (Sec. 3.3, Eq. 1; Adam on the twist with App.
    A's rates, then the retraction): the second starts from the GPU's pose
    and moments after the first, and its loss, gradient-driven moments and
    new pose match the oracle's iteration from that state."""
    from paper_2506_02741_amd import synth
    w = synth.tracking_workload(1, 160, 120)
    kf = w["keyframe"]
    cam = kf.cam.as_tuple()
    k = R.Keyframe.ingest(kf.depth, kf.rgb, cam, kf.pose)
    view = R.View(cam, w["init_pose"], obs_rgb=kf.rgb, obs_depth=kf.depth).with_pose_adam()
    plan = R.Plan([k], [view])
    cfg = R.track_cfg(alpha=0.5, beta=1.0, lr_rot=0.002, lr_trans=0.002)
    okfs = [oracle_kf(orc, kf)]
    pose = np.asarray(w["init_pose"], np.float32)
    state = dict(m=np.zeros(6), v=np.zeros(6), t=0)
    for t in (1, 2):
        loss = np_(plan.track_step(cfg, iters=1))[0, 0]
        assert plan.status()[0] == 0
        L_ref, pose_ref, st, g_ref, _ = orc.track_iteration(orc.ViewSpec(cam, pose), okfs, kf.rgb,
                                                            kf.depth, state)
        assert abs(loss - L_ref) <= 1e-5 * abs(L_ref), (t, loss, L_ref)
        ad = np_(view.pose_adam).astype(np.float64)
        assert ad[12] == t
        gmax = np.abs(g_ref).max()
        # m = b1 m + (1 - b1) g: the gradient's 1e-3 bar scaled by (1 - b1)
        assert np.all(np.abs(ad[:6] - st["m"]) <= 1e-4 * np.maximum(np.abs(g_ref), 1e-4 * gmax) + 1e-7 * np.abs(st["m"])), (t, ad[:6], st["m"])
        # v = b2 v + (1 - b2) g^2: twice the gradient's relative bar on the new term
        assert np.allclose(ad[6:12], st["v"], rtol=2e-3, atol=0), (t, ad[6:12], st["v"])
        newp = np_(view.pose).astype(np.float64).reshape(3, 4)
        assert np.allclose(newp, pose_ref, atol=4e-6), (t, newp, pose_ref)
        # the next iteration starts from the GPU's state
        pose = np_(view.pose).reshape(3, 4).copy()
        state = dict(m=ad[:6].copy(), v=ad[6:12].copy(), t=t)


def test_nonfinite_loss_is_reported(R):
    """A NaN in a learnable Gaussian's colour makes map_step's Eq. 2 loss
    non-finite and a NaN in a tracked frame's observed colour makes Eq. 1's:
    the plan's status reports VTGS_E_NONFINITE, and a cleared flag stays
    clear on the next clean step."""
    import torch
    from paper_2506_02741_amd import _lib
    cam, frames, _ = room_frames(9, 64, 48, n_kf=2)
    f = frames[0]
    k = R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose, learnable=True).with_adam()
    k.color[1, 1000] = float("nan")
    plan = R.Plan([k], [R.View(cam.as_tuple(), f.pose, 0, 1, f.rgb, f.depth)])
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.map_step(step)
    rc, _ = plan.status()
    assert rc == _lib.VTGS_E_NONFINITE
    k2 = R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose)
    obs = f.rgb.copy()
    obs[0, 24, 32] = np.nan
    view = R.View(cam.as_tuple(), frames[1].pose, 0, 1, obs, f.depth).with_pose_adam()
    tp = R.Plan([k2], [view])
    tp.track_step(R.track_cfg(), 1)
    assert tp.status()[0] == _lib.VTGS_E_NONFINITE
    assert tp.status()[0] == _lib.VTGS_OK            # cleared by the first status
    clean = R.View(cam.as_tuple(), frames[1].pose, 0, 1, f.rgb, f.depth).with_pose_adam()
    cp = R.Plan([k2], [clean])
    cp.track_step(R.track_cfg(), 2)
    assert cp.status()[0] == _lib.VTGS_OK
