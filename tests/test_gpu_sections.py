"""Sections around the splat through the C ABI against the oracle: the
visibility check and the overlapping-section selection with batched
pre-tracking (Sec. 3.3).

Visibility masks and counts are integer results decided in FP32 in the same
operation order on both sides: bit-exact.  The selection is host logic over
those counts; the pre-tracking batch equals one plan per section bit for bit
(tracking has no atomics) and picks the section with the smallest loss."""
import numpy as np
import pytest

from scenes import oracle_kf

pytestmark = pytest.mark.gpu


def np_(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    torch.cuda.set_device(0)
    from paper_2506_02741_amd import render
    return render


@pytest.fixture(scope="module")
def walk():
    """A 16-frame walk through a room at 96x72 in four sections of four
    keyframes, and a head frame further on (the next section's head)."""
    from paper_2506_02741_amd import synth
    rng = np.random.default_rng(51)
    w, h = 96, 72
    scene = synth.make_room(51)
    cam = synth.Camera(w * 525.0 / 640, w * 525.0 / 640, w / 2, h / 2, w, h)
    poses = synth.random_walk(scene, cam, rng, 17, step=0.10, rot_deg=5.0)
    frames = [synth.frame(scene, cam, T) for T in poses]
    return cam, frames


def test_visibility_bitwise(R, orc, walk):
    """Masks (union over targets) and per-target counts of the last frame's
    points in every earlier frame, including targets at other resolutions."""
    import torch
    from paper_2506_02741_amd import sections as S
    from paper_2506_02741_amd import synth
    cam, frames = walk
    src = frames[-1]
    ks = [R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose) for f in frames[:-1]]
    sd = torch.as_tensor(src.depth.ravel(), device="cuda")
    sp = torch.as_tensor(src.pose.ravel(), device="cuda")
    # a target at half resolution (its own depth map and intrinsics)
    half = synth.Camera(cam.fx / 2, cam.fy / 2, cam.cx / 2, cam.cy / 2, cam.width // 2, cam.height // 2)
    hf = synth.frame(synth.make_room(51), half, frames[3].pose)
    hd = torch.as_tensor(hf.depth.ravel(), device="cuda")
    hp = torch.as_tensor(hf.pose.ravel(), device="cuda")
    refs = [S.keyframe_ref(k) for k in ks] + [S.frame_ref(hd, half.as_tuple(), hp)]
    mask, counts = S.visibility(sd, cam.as_tuple(), sp, refs)
    tgts = [(f.depth, cam.as_tuple(), f.pose) for f in frames[:-1]] + [(hf.depth, half.as_tuple(), hf.pose)]
    vis, cref = orc.visibility(src.depth, cam.as_tuple(), src.pose, tgts)
    assert np.array_equal(np_(counts).astype(np.int64), cref), (np_(counts), cref)
    assert np.array_equal(np_(mask).astype(bool), vis.any(0))
    assert 0 < cref.min() and cref.max() < src.depth.size
    # one target at a time (more than one launch's targets above) gives the same
    m1, c1 = S.visibility(sd, cam.as_tuple(), sp, refs[:1])
    assert np.array_equal(np_(m1).astype(bool), vis[0]) and int(np_(c1)[0]) == cref[0]


def test_overlap_selection_and_batched_pretracking(R, orc, walk):
    """The head frame of a fifth section against four earlier ones: the
    candidates (every 5th keyframe) and their counts from the initial pose,
    the three most front sections above gamma (the oracle's rule on the
    oracle's counts gives the same ones), each section's mask (union over its
    head / middle / last keyframes) bit-exact, and the batched pre-tracking
    equal to one plan per section, the chosen section the one with the
    smallest final loss."""
    import torch
    from paper_2506_02741_amd import sections as S
    from paper_2506_02741_amd import synth
    cam, frames = walk
    head = frames[-1]
    secs = []
    for i in range(4):
        ks = [R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose) for f in frames[4 * i:4 * i + 4]]
        secs.append(S.Section(i, ks))
    init = synth.perturb_pose(head.pose, np.random.default_rng(3), 0.01, 0.5).astype(np.float32)
    hd = torch.as_tensor(head.depth.ravel(), device="cuda")
    hr = torch.as_tensor(head.rgb.reshape(3, -1), device="cuda")
    gamma = 0.24
    chosen, pose, info = S.choose_overlap_section(hd, hr, cam.as_tuple(), init, secs, gamma, n1=5,
                                                  iters=8)
    # the oracle's counts and rule
    cands = S.overlap_candidates(secs, 5)
    tgt_frames = [frames[4 * s.index + s.keyframes.index(k)] for s, k in
                  [(next(x for x in secs if x.index == si), k) for si, k in cands]]
    _, cref = orc.visibility(head.depth, cam.as_tuple(), init, [(f.depth, cam.as_tuple(), f.pose) for f in tgt_frames])
    assert np.array_equal(info["counts"].numpy().astype(np.int64), cref)
    picked = orc.select_overlap(cref, int((head.depth > 0).sum()), [si for si, _ in cands], gamma)
    assert picked == info["picked"] and len(picked) >= 2, (picked, cref)
    # each section's W mask: union over its head, middle and last keyframes
    for si, m in zip(picked, info["masks"]):
        fs = frames[4 * si:4 * si + 4]
        vis, _ = orc.visibility(head.depth, cam.as_tuple(), init,
                                [(fs[j].depth, cam.as_tuple(), fs[j].pose) for j in (0, 2, 3)])
        assert np.array_equal(np_(m).astype(bool), vis.any(0))
    # batched pre-tracking == one plan per section
    losses = info["losses"].numpy()
    for j, si in enumerate(picked):
        s = next(x for x in secs if x.index == si)
        b, L1, v1 = S.pretrack([s], cam.as_tuple(), init, hr, hd, 8, masks=[info["masks"][j]])
        assert np.array_equal(L1.numpy()[:, 0], losses[:, j])
    assert chosen.index == picked[int(np.argmin(losses[-1]))]
    assert np.isfinite(losses).all()


def test_complement_initialisation(R, orc, walk):
    """Sec. 3.4: a section of one keyframe rendered at a later frame's pose;
    the uncovered mask (silhouette < 0.5, valid depth) is the rule applied to
    the GPU's own silhouette (bit-exact), agrees with the oracle's rendering
    away from silhouettes within 1e-5 of 0.5, and the complement keyframe
    equals the oracle's ingestion with that mask; after it joins, every
    valid pixel of the frame is covered."""
    import torch
    from paper_2506_02741_amd import sections as S
    cam, frames = walk
    head, reg = frames[0], frames[6]
    k0 = R.Keyframe.ingest(head.depth, head.rgb, cam.as_tuple(), head.pose, 1, 0.99, None, True)
    sec = S.Section(0, [k0])
    kn, mask = S.complement_keyframe(sec, reg.depth, reg.rgb, cam.as_tuple(), reg.pose)
    # the rule on the GPU's own silhouette
    plan = R.Plan([k0], [R.View(cam.as_tuple(), reg.pose)])
    _, _, sil = plan.render_fwd()
    s = np_(sil)
    rule = (s < 0.5) & (reg.depth.ravel() > 0)
    assert np.array_equal(np_(mask).astype(bool), rule)
    assert 0 < rule.sum() < rule.size
    ref = orc.render(orc.ViewSpec(cam.as_tuple(), reg.pose), [oracle_kf(orc, head)])
    clear = np.abs(ref["sil"] - 0.5) > 1e-5
    assert np.array_equal(rule[clear], ((ref["sil"] < 0.5) & (reg.depth.ravel() > 0))[clear])
    okn = orc.ingest(reg.depth, reg.rgb, np_(mask).reshape(reg.depth.shape), 1, fx=cam.fx, o_init=0.99)
    assert kn.n == okn["pix"].shape[0]
    assert np.array_equal(np_(kn.pix).astype(np.uint32), okn["pix"])
    assert np.array_equal(np_(kn.depth), okn["depth"]) and np.array_equal(np_(kn.radius), okn["radius"])
    sec.keyframes.append(kn)
    p2 = R.Plan(sec.keyframes, [R.View(cam.as_tuple(), reg.pose, 0, 2)])
    _, _, sil2 = p2.render_fwd()
    assert (np_(sil2)[reg.depth.ravel() > 0] >= 0.5).all()


def test_section_store_offload_and_prefetch(R, walk):
    """Sec. 3.2 / 3.3 lifecycle: sections started by head frames, complement
    keyframes joining the current one, the finished ones frozen and offloaded
    to host memory, one prefetched back when needed: its rendering is bit
    for bit what it was before the offload, and the resident Gaussians stay
    below the total (Tab. 9's max-at-a-time against total)."""
    import torch
    from paper_2506_02741_amd import sections as S
    cam, frames = walk
    store = S.SectionStore()
    view_pose = frames[5].pose
    before = None
    for i in range(3):
        f = frames[5 * i]
        head = R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose, 1, 0.99, None, True)
        store.start_section(head)
        for j in (2, 4):
            g = frames[5 * i + j]
            kn, _ = S.complement_keyframe(store.current, g.depth, g.rgb, cam.as_tuple(), g.pose)
            if kn is not None:
                store.add_keyframe(kn)
        if i == 0:
            sec0 = store.current
            before = [np_(x) for x in R.Plan(sec0.keyframes, [R.View(cam.as_tuple(), view_pose, 0,
                                                                     len(sec0.keyframes))]).render_fwd()]
        if i < 2:
            store.freeze(store.current)
            store.offload(store.current)
    assert not sec0.resident and sec0.frozen
    assert store.resident_gaussians() < store.total_gaussians
    assert store.peak_resident <= store.total_gaussians
    ev = store.prefetch(sec0)
    torch.cuda.current_stream().wait_event(ev)
    assert sec0.resident
    after = [np_(x) for x in R.Plan(sec0.keyframes, [R.View(cam.as_tuple(), view_pose, 0,
                                                            len(sec0.keyframes))]).render_fwd()]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert all(not k.learnable for k in sec0.keyframes)
