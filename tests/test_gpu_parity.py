"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: ingestion, preprocessing records and tile lists bit-exact; images
within 1e-5 absolute on every pixel; gradients per element
|g - g_ref| <= 1e-3 max(|g_ref|, 1e-4 max|g_ref|) + 8 u m against the FP64
oracle gradient, m being the oracle's sum of the absolute values of that
element's summands and u = 2^-24 (the FP32 evaluation floor, which decides
only where the summands cancel by about 10^4 or more), with the upstream
gradient zeroed at flagged pixels.

Flagged pixels: q is evaluated in the same FP32 operation order on both
sides (bit identical), but exp is not: the GPU's exp2 with a rounded argument
is within about 5e-7 relative of the correctly rounded value for q <= q_cut.
The oracle flags a pixel when an alpha lies within MARGIN = 2e-6 (relative)
of alpha_min, q within MARGIN of q_cut, or a stop decision closer to t_min
than the transmittance uncertainty that such alpha errors accumulate
(amplified by alpha / (1 - alpha) near the 0.99 clamp).  A flagged pixel
must match the oracle's result or one of the other outcomes of its near-tie
decisions, which the oracle evaluates one flipped decision at a time.
"""
import numpy as np
import pytest

from scenes import oracle_kf, room_frames

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5
MARGIN = 2e-6
MAX_ALT = 4


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    torch.cuda.set_device(0)
    from paper_2506_02741_amd import render
    return render


def T(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def np_(t):
    return t if isinstance(t, np.ndarray) else t.detach().cpu().numpy()


def gpu_kf(R, fr, stride=1, mask=None, learnable=False):
    return R.Keyframe.ingest(fr.depth, fr.rgb, fr.cam.as_tuple(), fr.pose, stride, 0.99, mask,
                             learnable)


U32 = 2.0 ** -24  # FP32 unit roundoff
FP32_FLOOR = 8.0


def grad_close(g, ref, name="", mag=None, rel=1e-3, floor=1e-4):
    """Per element |g - ref| <= rel * max(|ref|, floor * max|ref|) against the
    FP64 oracle gradient (the twist per component, with the max over its six
    components), plus, when the oracle's sum of absolute summands `mag` is
    given, the FP32 evaluation floor FP32_FLOOR * u * mag (u = 2^-24): a sum
    whose terms cancel far below their magnitudes cannot be evaluated in FP32
    to a bar relative to the result.  Prints the worst error against the
    bound, and how many elements rest on the floor."""
    g, ref = (np.asarray(x, np.float64) for x in (g, ref))
    if not ref.size:
        return True, 0.0
    stated = rel * np.maximum(np.abs(ref), floor * np.abs(ref).max())
    err = np.abs(g - ref)
    bound = stated if mag is None else stated + FP32_FLOOR * U32 * np.asarray(mag, np.float64)
    ratio = err / np.maximum(bound, 1e-300)
    worst = float(ratio.max())
    on_floor = int((err > stated).sum())
    msg = "grad %s: worst |g - ref| / bound = %.3g (n = %d" % (name, worst, ref.size)
    if mag is not None:
        msg += ", %d on the FP32 floor, max err / (u mag) = %.2f" % (
            on_floor, float((err / np.maximum(U32 * np.asarray(mag, np.float64), 1e-300)).max()))
    print(msg + ")")
    return worst <= 1.0, worst


def same_ranges(got, ref):
    """Tile ranges agree: same length everywhere, same start where the tile is
    not empty (an empty range's start is arbitrary)."""
    got = np.asarray(got).astype(np.int64); ref = np.asarray(ref).astype(np.int64)
    lg, lr = got[:, 1] - got[:, 0], ref[:, 1] - ref[:, 0]
    return np.array_equal(lg, lr) and np.array_equal(got[lr > 0, 0], ref[lr > 0, 0])


def oracle_ref(orc, ov, okfs, prm=None):
    """The oracle's images, with a function that gives the other outcomes of
    the near-tie decisions of flagged pixels."""
    ref = orc.render(ov, okfs, prm, margin=MARGIN)
    ref["alt"] = lambda px: orc.render_alternatives(ov, okfs, px, prm, margin=MARGIN, max_alt=MAX_ALT)
    return ref


def check_images(rgb, depth, sil, ref, max_marginal=1e-3):
    """Every pixel within IMG_TOL of the oracle on RGB, depth and silhouette:
    unflagged pixels against its result, flagged ones against its result or
    one of the other outcomes of their near-tie decisions (each variant takes
    one decision the other way), so no pixel goes unchecked.  Flagged pixels
    may be at most `max_marginal` of the image.  Returns the unflagged mask."""
    flagged = ref["marginal"]
    frac = float(flagged.mean()) if flagged.size else 0.0
    assert frac <= max_marginal, frac
    got = np.concatenate([np_(rgb).reshape(3, -1), np_(depth).reshape(1, -1),
                          np_(sil).reshape(1, -1)], 0).astype(np.float64)
    want = np.concatenate([ref["rgb"], ref["depth"][None], ref["sil"][None]], 0)
    err = np.abs(got - want).max(0) if got.size else np.zeros(0)
    assert not (err[~flagged] > IMG_TOL).any(), float(err[~flagged].max())
    other = np.nonzero(flagged & (err > IMG_TOL))[0]
    if other.size:
        alt = ref["alt"](other)
        for i, p in enumerate(other):
            n = int(alt["n_dec"][i])
            assert 0 < n <= MAX_ALT, (int(p), n)
            va = np.concatenate([alt["rgb"][i, :n].T, alt["depth"][i, :n][None],
                                 alt["sil"][i, :n][None]], 0)
            assert (np.abs(va - got[:, p][:, None]).max(0) <= IMG_TOL).any(), (int(p), got[:, p], want[:, p], va)
    return ~flagged


# ----------------------------------------------------------------------------
# a0 ingestion
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("stride", [1, 2, 3])
@pytest.mark.parametrize("masked", [False, True])
def test_ingest_bitwise(R, orc, stride, masked):
    cam, frames, _ = room_frames(21, 83, 61)
    fr = frames[0]
    depth = fr.depth.copy()
    depth[::7, ::5] = 0.0   # holes
    rng = np.random.default_rng(stride)
    mask = (rng.uniform(size=depth.shape) < 0.7).astype(np.uint8) if masked else None
    k = R.Keyframe.ingest(depth, fr.rgb, cam.as_tuple(), fr.pose, stride, 0.8, mask)
    ref = orc.ingest(depth, fr.rgb, mask, stride, fx=cam.fx, o_init=0.8)
    assert k.n == ref["pix"].shape[0]
    assert np.array_equal(np_(k.pix).astype(np.uint32), ref["pix"])
    for a, b in ((k.depth, ref["depth"]), (k.color, ref["color"]), (k.opacity, ref["opacity"]),
                 (k.radius, ref["radius"])):
        assert np.array_equal(np_(a), b)


# ----------------------------------------------------------------------------
# a1-a5 preprocessing records and tile lists
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("tile", [8, 16, 32])
def test_records_and_tile_lists_bitwise(R, orc, tile):
    cam, frames, vpose = room_frames(5, 80, 60)
    fr = frames[0]
    k = gpu_kf(R, fr)
    plan = R.Plan([k], [R.View(cam.as_tuple(), vpose)], R.params(tile=tile))
    plan.render_fwd()
    st = plan.debug_state()
    rc, need = plan.status()
    assert rc == 0
    okf = oracle_kf(orc, fr)
    ov = orc.ViewSpec(cam.as_tuple(), vpose)
    prm = orc.params(tile=tile)
    rec = orc.preprocess32(ov, [okf], prm)
    g = np_(st["records"])
    rect = np_(st["rect"])
    valid = rec["count"] > 0
    assert np.array_equal(rect[:, 0] <= rect[:, 2], valid)
    assert np.array_equal(rect[valid], rec["rect"][valid])
    for col, name in ((0, "mx"), (1, "my"), (2, "qa"), (3, "qb"), (4, "qc"), (6, "pz"), (7, "ext")):
        assert np.array_equal(g[valid, col], rec[name][valid]), name
    keys, vals, ranges = orc.tile_lists(ov, [okf], prm)
    assert int(np_(st["n_pairs"])[0]) == len(vals) == need
    assert same_ranges(np_(st["ranges"]), ranges)
    assert np.array_equal(np_(st["ids"])[:len(vals)].astype(np.uint32), vals)


# ----------------------------------------------------------------------------
# a6 forward
# ----------------------------------------------------------------------------

def test_forward_toy_scene(R, orc):
    from paper_2506_02741_amd import synth
    f, colors = synth.toy_scene(0)
    cam = f.cam.as_tuple()
    k = R.Keyframe.ingest(f.depth, colors, cam, f.pose)
    plan = R.Plan([k], [R.View(cam, f.pose)])
    rgb, depth, sil = plan.render_fwd()
    okf = orc.ingest(f.depth, colors, fx=f.cam.fx, cam=cam, pose=f.pose)
    ref = oracle_ref(orc, orc.ViewSpec(cam, f.pose), [okf])
    check_images(rgb, depth, sil, ref)


@pytest.mark.parametrize("tile,batch", [(16, 256), (8, 128), (8, 512), (16, 128), (16, 512),
                                        (32, 128), (32, 256), (32, 512), (8, 256)])
def test_forward_room_all_configs_bitwise_equal(R, orc, tile, batch):
    cam, frames, vpose = room_frames(5, 80, 60)
    fr = frames[0]
    k = gpu_kf(R, fr)
    view = R.View(cam.as_tuple(), vpose)
    imgs = R.Plan([k], [view], R.params(tile=tile, batch=batch)).render_fwd()
    base = R.Plan([k], [view], R.params(tile=16, batch=256)).render_fwd()
    for a, b in zip(imgs, base):
        assert np.array_equal(np_(a), np_(b))
    ref = oracle_ref(orc, orc.ViewSpec(cam.as_tuple(), vpose), [oracle_kf(orc, fr)])
    check_images(*imgs, ref)


def test_forward_section_multi_keyframe(R, orc):
    cam, frames, vpose = room_frames(9, 96, 72, n_kf=3)
    ks = [gpu_kf(R, fr) for fr in frames]
    plan = R.Plan(ks, [R.View(cam.as_tuple(), vpose, 0, 3)])
    imgs = plan.render_fwd()
    ref = oracle_ref(orc, orc.ViewSpec(cam.as_tuple(), vpose, 0, 3),
                     [oracle_kf(orc, f) for f in frames])
    check_images(*imgs, ref)


def test_forward_full_size_tracking_frame(R, orc):
    """640x480, 307,200 Gaussians, perturbed pose: every pixel vs the oracle."""
    from paper_2506_02741_amd import synth
    w = synth.tracking_workload(1)
    kf = w["keyframe"]
    k = R.Keyframe.ingest(kf.depth, kf.rgb, kf.cam.as_tuple(), kf.pose)
    assert k.n == 640 * 480
    plan = R.Plan([k], [R.View(kf.cam.as_tuple(), w["init_pose"])])
    imgs = plan.render_fwd()
    assert plan.status()[0] == 0
    ref = oracle_ref(orc, orc.ViewSpec(kf.cam.as_tuple(), w["init_pose"]), [oracle_kf(orc, kf)])
    check_images(*imgs, ref)


# ----------------------------------------------------------------------------
# a9/a10 backward
# ----------------------------------------------------------------------------

def _random_upstream(P, marginal, seed=0):
    rng = np.random.default_rng(seed)
    g_rgb = rng.normal(size=(3, P)); g_d = rng.normal(size=P); g_s = rng.normal(size=P)
    g_rgb[:, marginal] = 0; g_d[marginal] = 0; g_s[marginal] = 0
    return g_rgb, g_d, g_s


@pytest.mark.parametrize("tile,batch", [(16, 256), (8, 128), (32, 512)])
def test_backward_parity(R, orc, tile, batch):
    cam, frames, vpose = room_frames(5, 80, 60)
    fr = frames[0]
    k = gpu_kf(R, fr, learnable=True).with_grad_buffers()
    plan = R.Plan([k], [R.View(cam.as_tuple(), vpose)], R.params(tile=tile, batch=batch))
    plan.render_fwd()
    okf = oracle_kf(orc, fr)
    ov = orc.ViewSpec(cam.as_tuple(), vpose)
    ref = orc.render(ov, [okf], margin=MARGIN)
    g_rgb, g_d, g_s = _random_upstream(plan.P, ref["marginal"])
    tw = plan.render_bwd(T(g_rgb), T(g_d), T(g_s))
    gref = orc.render_bwd(ov, [okf], g_rgb, g_d, g_s)
    for got, name in ((k.g_color, "color"), (k.g_opacity, "opacity"), (k.g_radius, "radius")):
        ok, worst = grad_close(np_(got), gref[name], name, gref["mag"][name])
        assert ok, (name, worst)
    ok, worst = grad_close(np_(tw)[0], gref["twist"], "twist", gref["mag"]["twist"])
    assert ok, ("twist", worst, np_(tw)[0], gref["twist"])


def test_backward_full_size_twist(R, orc):
    from paper_2506_02741_amd import synth
    w = synth.tracking_workload(1)
    kf = w["keyframe"]
    k = R.Keyframe.ingest(kf.depth, kf.rgb, kf.cam.as_tuple(), kf.pose)
    plan = R.Plan([k], [R.View(kf.cam.as_tuple(), w["init_pose"])])
    plan.render_fwd()
    ov = orc.ViewSpec(kf.cam.as_tuple(), w["init_pose"])
    okf = oracle_kf(orc, kf)
    ref = orc.render(ov, [okf], margin=MARGIN)
    L, g_rgb, g_d = orc.track_loss(ref["rgb"], ref["depth"], ref["sil"], kf.rgb, kf.depth)
    g_rgb[:, ref["marginal"]] = 0; g_d[ref["marginal"]] = 0
    tw = plan.render_bwd(T(g_rgb), T(g_d), None)
    gref = orc.render_bwd(ov, [okf], g_rgb, g_d, None)
    ok, worst = grad_close(np_(tw)[0], gref["twist"], "twist", gref["mag"]["twist"])
    assert ok, (worst, np_(tw)[0], gref["twist"])


# seed -> (width, height, keyframes, tile, batch): ragged tiles on both axes
RANDOM_SCENES = {0: (88, 60, 1, 16, 256), 1: (72, 88, 2, 16, 256), 2: (104, 56, 3, 8, 128),
                 3: (60, 100, 2, 32, 512), 4: (96, 72, 3, 16, 128), 5: (50, 66, 1, 8, 256)}


@pytest.mark.parametrize("seed", sorted(RANDOM_SCENES))
def test_random_attributes_forward_backward(R, orc, seed):
    """Seeded scenes with random colours, opacities over (0.05, 1) -- so the
    alpha_max clamp engages and its branch of dL/do is taken -- and radii
    scaled 0.5-3x (longer, overlapping lists): images, per-Gaussian gradients
    and the twist against the oracle at several tile/batch shapes."""
    w, h, n_kf, tile, batch = RANDOM_SCENES[seed]
    cam, frames, vpose = room_frames(100 + seed, w, h, n_kf=n_kf)
    rng = np.random.default_rng(seed)
    okfs, gks = [], []
    for fr in frames:
        base = oracle_kf(orc, fr)
        n = base.n
        color = rng.uniform(0.0, 1.0, (3, n)).astype(np.float32)
        opa = rng.uniform(0.05, 1.0, n).astype(np.float32)
        rad = (base.radius * rng.uniform(0.5, 3.0, n)).astype(np.float32)
        okfs.append(orc.Keyframe(base.cam, base.pose, base.pix, base.depth, color, opa, rad))
        gks.append(R.Keyframe(base.cam, base.pose, base.pix.astype(np.int64), base.depth, color, opa,
                              rad, learnable=True).with_grad_buffers())
    view = R.View(cam.as_tuple(), vpose, 0, n_kf)
    plan = R.Plan(gks, [view], R.params(tile=tile, batch=batch))
    imgs = plan.render_fwd()
    assert plan.status()[0] == 0
    ov = orc.ViewSpec(cam.as_tuple(), vpose, 0, n_kf)
    ref = oracle_ref(orc, ov, okfs)
    check_images(*imgs, ref, max_marginal=2e-3)
    g_rgb, g_d, g_s = _random_upstream(plan.P, ref["marginal"], seed)
    tw = plan.render_bwd(T(g_rgb), T(g_d), T(g_s))
    gref = orc.render_bwd(ov, okfs, g_rgb, g_d, g_s)
    off = 0
    for k in gks:
        for got, name in ((k.g_color, "color"), (k.g_opacity, "opacity"), (k.g_radius, "radius")):
            ok, worst = grad_close(np_(got), gref[name][..., off:off + k.n], name,
                                   gref["mag"][name][..., off:off + k.n])
            assert ok, (name, worst)
        off += k.n
    ok, worst = grad_close(np_(tw)[0], gref["twist"], "twist", gref["mag"]["twist"])
    assert ok, ("twist", worst, np_(tw)[0], gref["twist"])


def test_backward_frozen_keyframe_gets_nothing(R, orc):
    cam, frames, vpose = room_frames(9, 64, 48, n_kf=2)
    a = gpu_kf(R, frames[0], learnable=True).with_grad_buffers()
    b = gpu_kf(R, frames[1], learnable=False).with_grad_buffers()
    plan = R.Plan([a, b], [R.View(cam.as_tuple(), vpose, 0, 2)])
    plan.render_fwd()
    P = plan.P
    ref = orc.render(orc.ViewSpec(cam.as_tuple(), vpose, 0, 2),
                     [oracle_kf(orc, f) for f in frames], margin=MARGIN)
    g_rgb, g_d, g_s = _random_upstream(P, ref["marginal"], 3)
    plan.render_bwd(T(g_rgb), T(g_d), T(g_s), twist=False)
    assert float(b.g_color.abs().max()) == 0.0 and float(b.g_radius.abs().max()) == 0.0
    gref = orc.render_bwd(orc.ViewSpec(cam.as_tuple(), vpose, 0, 2),
                          [oracle_kf(orc, f) for f in frames], g_rgb, g_d, g_s)
    n = a.n
    for got, name in ((a.g_color, "color"), (a.g_opacity, "opacity"), (a.g_radius, "radius")):
        ok, worst = grad_close(np_(got), gref[name][..., :n], name, gref["mag"][name][..., :n])
        assert ok, (name, worst)


# ----------------------------------------------------------------------------
# batching: one plan over several views == one plan per view
# ----------------------------------------------------------------------------

def test_batched_views_equal_single(R, orc):
    cam, frames, vpose = room_frames(9, 64, 48, n_kf=3)
    ks = [gpu_kf(R, fr, learnable=True).with_grad_buffers() for fr in frames]
    poses = [fr.pose for fr in frames]
    views = [R.View(cam.as_tuple(), p, 0, 3) for p in poses]
    batch = R.Plan(ks, views)
    rgb, depth, sil = batch.render_fwd()
    rng = np.random.default_rng(1)
    g_rgb = rng.normal(size=(3, batch.P)); g_d = rng.normal(size=batch.P)
    tw_b = np_(batch.render_bwd(T(g_rgb), T(g_d), None))
    gb = [np_(k.g_color).copy() for k in ks]
    for k in ks:
        k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
    for v, view in enumerate(views):
        single = R.Plan(ks, [view])
        r1, d1, s1 = single.render_fwd()
        o = batch.offsets[v]
        sl = slice(o, o + single.P)
        assert np.array_equal(np_(r1), np_(rgb)[:, sl])
        assert np.array_equal(np_(d1), np_(depth)[sl])
        assert np.array_equal(np_(s1), np_(sil)[sl])
        tw1 = np_(single.render_bwd(T(g_rgb[:, sl]), T(g_d[sl]), None))
        assert np.array_equal(tw1[0], tw_b[v])
    for k, g in zip(ks, gb):
        assert np.allclose(np_(k.g_color), g, rtol=1e-5, atol=1e-7)


def test_many_views_and_segments_equal_single(R, orc):
    """300 small views over 4 keyframes in one plan: more views than the key
    fill keeps in LDS and more (view, keyframe) segments than the
    preprocess keeps in LDS, so both search their descriptors in global
    memory.  Every view's images and tile lists equal those of the view
    planned alone (bitwise), and a few views equal the oracle."""
    from paper_2506_02741_amd import synth
    cam, frames, vpose = room_frames(21, 40, 30, n_kf=4)
    ks = [gpu_kf(R, fr) for fr in frames]
    rng = np.random.default_rng(5)
    vcam = synth.Camera(30.0, 30.0, 12.0, 9.0, 24, 18)
    poses = [synth.perturb_pose(frames[i % 4].pose, rng, 0.05, 3.0).astype(np.float32)
             for i in range(300)]
    views = [R.View(vcam.as_tuple(), p, 0, 4) for p in poses]
    batch = R.Plan(ks, views)
    rgb, depth, sil = batch.render_fwd()
    assert batch.status()[0] == 0
    for v in range(0, 300, 7):
        single = R.Plan(ks, [views[v]])
        r1, d1, s1 = single.render_fwd()
        o = batch.offsets[v]
        sl = slice(o, o + single.P)
        assert np.array_equal(np_(r1), np_(rgb)[:, sl]), v
        assert np.array_equal(np_(d1), np_(depth)[sl]), v
        assert np.array_equal(np_(s1), np_(sil)[sl]), v
    okfs = [oracle_kf(orc, fr) for fr in frames]
    for v in (0, 151, 299):
        o = batch.offsets[v]
        sl = slice(o, o + vcam.width * vcam.height)
        ref = oracle_ref(orc, orc.ViewSpec(vcam.as_tuple(), poses[v], 0, 4), okfs)
        check_images(np_(rgb)[:, sl], np_(depth)[sl], np_(sil)[sl], ref, max_marginal=1e-2)


def test_uneven_resolutions_batch(R, orc):
    """Views of different sizes in one plan, each vs the oracle."""
    cam, frames, vpose = room_frames(9, 64, 48, n_kf=3)
    ks = [gpu_kf(R, fr) for fr in frames]
    from paper_2506_02741_amd import synth
    sizes = [(64, 48), (37, 23), (100, 75)]
    views, oviews = [], []
    for (w, h), fr in zip(sizes, frames):
        c = synth.Camera(w * 525 / 640, w * 525 / 640, w / 2, h / 2, w, h)
        views.append(R.View(c.as_tuple(), fr.pose, 0, 3))
        oviews.append(orc.ViewSpec(c.as_tuple(), fr.pose, 0, 3))
    plan = R.Plan(ks, views)
    rgb, depth, sil = plan.render_fwd()
    okfs = [oracle_kf(orc, f) for f in frames]
    for v, ov in enumerate(oviews):
        ref = oracle_ref(orc, ov, okfs)
        o = plan.offsets[v]
        sl = slice(o, o + ov.P)
        check_images(rgb[:, sl], depth[sl], sil[sl], ref)


# ----------------------------------------------------------------------------
# determinism, capacity, edge cases
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n_kf", [1, 3])
def test_deterministic(R, n_kf):
    """Repeated passes give bit-identical images, twists and per-Gaussian
    gradients (the gradient sums run in a fixed order)."""
    cam, frames, vpose = room_frames(5 if n_kf == 1 else 9, 80, 60, n_kf=n_kf)
    ks = [gpu_kf(R, f, learnable=True).with_grad_buffers() for f in frames]
    plan = R.Plan(ks, [R.View(cam.as_tuple(), vpose, 0, n_kf)])
    rng = np.random.default_rng(2)
    g = T(rng.normal(size=(3, plan.P)))
    gd = T(rng.normal(size=plan.P))
    out = []
    for _ in range(4):
        for k in ks:
            k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
        imgs = [np_(x) for x in plan.render_fwd()]
        tw = np_(plan.render_bwd(g, gd, None))
        out.append((imgs, tw, [np_(k.g_color) for k in ks], [np_(k.g_opacity) for k in ks],
                    [np_(k.g_radius) for k in ks]))
    for o in out[1:]:
        for a, b in zip(out[0][0], o[0]):
            assert np.array_equal(a, b)
        assert np.array_equal(out[0][1], o[1])
        for i in (2, 3, 4):
            for a, b in zip(out[0][i], o[i]):
                assert np.array_equal(a, b)


def test_capacity_overflow_is_reported_and_recoverable(R, orc):
    from paper_2506_02741_amd import _lib
    cam, frames, vpose = room_frames(5, 80, 60)
    fr = frames[0]
    k = gpu_kf(R, fr)
    view = R.View(cam.as_tuple(), vpose)
    keys, vals, ranges = orc.tile_lists(orc.ViewSpec(cam.as_tuple(), vpose), [oracle_kf(orc, fr)])
    small = R.Plan([k], [view], pair_capacity=len(vals) // 3)
    small.render_fwd()
    rc, need = small.status(clear=True)
    assert rc == _lib.VTGS_E_CAPACITY and need == len(vals)
    plan, imgs = R.plan_checked([k], [view], pair_capacity=100, run=lambda p: p.render_fwd())
    ref = oracle_ref(orc, orc.ViewSpec(cam.as_tuple(), vpose), [oracle_kf(orc, fr)])
    check_images(*imgs, ref)


def test_edge_cases(R, orc):
    import torch
    cam, frames, vpose = room_frames(5, 80, 60)
    fr = frames[0]
    k = gpu_kf(R, fr)
    empty = R.Keyframe(cam.as_tuple(), fr.pose, np.zeros(0, np.int32), np.zeros(0), np.zeros((3, 0)),
                       np.zeros(0), np.zeros(0))
    # empty keyframe in the slice changes nothing
    a = R.Plan([empty, k], [R.View(cam.as_tuple(), vpose, 0, 2)]).render_fwd()
    b = R.Plan([k], [R.View(cam.as_tuple(), vpose)]).render_fwd()
    for x, y in zip(a, b):
        assert np.array_equal(np_(x), np_(y))
    # camera turned around: everything culled -> background, silhouette 0
    back = fr.pose.copy()
    back[:, :3] = -back[:, :3]
    back[:, 3] = -back[:, 3]
    rgb, depth, sil = R.Plan([k], [R.View(cam.as_tuple(), back)], R.params(bg=(0.1, 0.2, 0.3))).render_fwd()
    assert float(sil.abs().max()) == 0.0 and float(depth.abs().max()) == 0.0
    assert np.allclose(np_(rgb)[:, 0], [0.1, 0.2, 0.3])
    # 1x1 and ragged views vs the oracle
    okf = oracle_kf(orc, fr)
    for (w, h) in ((1, 1), (17, 9), (33, 47)):
        c = (cam.fx, cam.fy, w / 2.0, h / 2.0, w, h)
        imgs = R.Plan([k], [R.View(c, vpose)]).render_fwd()
        ref = oracle_ref(orc, orc.ViewSpec(c, vpose), [okf])
        check_images(*imgs, ref, max_marginal=1.0)


def test_degenerate_views_backward_and_steps(R):
    """Views with nothing to render: a view over no keyframes beside a normal
    one (its twist is zero, the normal view's equals that view alone) and a
    camera turned away from everything, tracked for two iterations (zero
    loss, the pose unchanged bit for bit, no flags)."""
    import torch
    cam, frames, vpose = room_frames(5, 80, 60)
    fr = frames[0]
    k = gpu_kf(R, fr, learnable=True).with_grad_buffers()
    views = [R.View(cam.as_tuple(), vpose, 0, 0), R.View(cam.as_tuple(), vpose, 0, 1)]
    plan = R.Plan([k], views)
    rgb, depth, sil = plan.render_fwd()
    assert float(sil[:plan.offsets[1]].abs().max()) == 0.0
    rng = np.random.default_rng(2)
    g = T(rng.normal(size=(3, plan.P)))
    tw = np_(plan.render_bwd(g, None, None))
    assert plan.status()[0] == 0
    assert not tw[0].any()
    gc = np_(k.g_color).copy()
    k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
    alone = R.Plan([k], [views[1]])
    alone.render_fwd()
    o = plan.offsets[1]
    tw1 = np_(alone.render_bwd(g[:, o:o + alone.P].contiguous(), None, None))
    assert np.array_equal(tw1[0], tw[1])
    assert np.array_equal(np_(k.g_color), gc)
    # a camera turned away from every Gaussian, tracked
    back = fr.pose.copy()
    back[:, :3] = -back[:, :3]
    back[:, 3] = -back[:, 3]
    kt = gpu_kf(R, fr)
    v = R.View(cam.as_tuple(), back, 0, 1, fr.rgb, fr.depth).with_pose_adam()
    p0 = np_(v.pose).copy()
    tp = R.Plan([kt], [v])
    loss = np_(tp.track_step(R.track_cfg(), iters=2))
    assert tp.status()[0] == 0
    assert not loss.any()
    assert np.array_equal(np_(v.pose), p0)


# ----------------------------------------------------------------------------
# autograd wrapper
# ----------------------------------------------------------------------------

def test_autograd_matches_oracle_and_fd(R, orc):
    import torch
    cam, frames, vpose = room_frames(11, 24, 18)
    fr = frames[0]
    # smooth setting: no alpha_min skip, a wide cut-off and opacity 0.3 so
    # transmittance stays far above t_min (no stop decisions)
    prm = dict(alpha_min=0.0, q_cut=60.0)
    k = gpu_kf(R, fr, learnable=True)
    k.opacity.fill_(0.3)
    plan = R.Plan([k], [R.View(cam.as_tuple(), vpose)], R.params(**prm))
    rng = np.random.default_rng(4)
    w_rgb = T(rng.normal(size=(3, plan.P))); w_d = T(rng.normal(size=plan.P))
    tw = torch.zeros(1, 6, device="cuda", requires_grad=True)
    k.color.requires_grad_(True); k.opacity.requires_grad_(True); k.radius.requires_grad_(True)
    rgb, depth, sil = R.render(plan, tw)
    loss = (rgb * w_rgb).sum() + (depth * w_d).sum()
    loss.backward()
    okf = oracle_kf(orc, fr)
    okf.opacity[:] = 0.3
    gref = orc.render_bwd(orc.ViewSpec(cam.as_tuple(), vpose), [okf], np_(w_rgb).astype(np.float64),
                          np_(w_d).astype(np.float64), None, orc.params(**prm))
    for got, name in ((k.color.grad, "color"), (k.opacity.grad, "opacity"), (k.radius.grad, "radius")):
        ok, worst = grad_close(np_(got), gref[name], name, gref["mag"][name])
        assert ok, (name, worst)
    ok, worst = grad_close(np_(tw.grad)[0], gref["twist"], "twist", gref["mag"]["twist"])
    assert ok, worst
    # FP32 central differences on a few opacities (smooth: thresholds off)
    with torch.no_grad():
        for i in rng.choice(k.n, 4, replace=False):
            eps = 1e-2
            vals = []
            for s in (1, -1):
                k.opacity[i] += s * eps
                r2, d2, _ = plan.render_fwd()
                vals.append(float((r2 * w_rgb).sum() + (d2 * w_d).sum()))
                k.opacity[i] -= s * eps
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert abs(fd - float(k.opacity.grad[i])) <= 2e-2 * max(1.0, abs(fd)), (fd, float(k.opacity.grad[i]))


@pytest.mark.parametrize("zoom,tile,n_kf", [(2.5, 16, 3), (4.0, 32, 3), (8.0, 32, 3), (8.0, 16, 5),
                                             (12.0, 32, 5)])
def test_long_tile_lists_bitwise(R, orc, zoom, tile, n_kf):
    """A zoomed-out view puts several keyframes' Gaussians into few tiles, so
    tile lists exceed the short-list sort (768) and, from zoom 8, the LDS
    capacity (8192: runs of 8192 sorted in LDS, then merged in rounds).  The
    zoom-8 cases hold lists of 1 to 3 runs (up to 23,902 entries), the
    zoom-12 one a list of 34,560 (5 runs: three rounds, an odd run copied)."""
    cam, frames, vpose = room_frames(9, 96, 72, n_kf=n_kf)
    ks = [gpu_kf(R, fr) for fr in frames]
    c = (cam.fx / zoom, cam.fy / zoom, cam.cx, cam.cy, cam.width, cam.height)
    plan = R.Plan(ks, [R.View(c, vpose, 0, n_kf)], R.params(tile=tile))
    imgs = plan.render_fwd()
    st = plan.debug_state()
    assert plan.status()[0] == 0
    okfs = [oracle_kf(orc, f) for f in frames]
    ov = orc.ViewSpec(c, vpose, 0, n_kf)
    prm = orc.params(tile=tile)
    keys, vals, ranges = orc.tile_lists(ov, okfs, prm)
    lens = ranges[:, 1] - ranges[:, 0]
    assert lens.max() > 2048
    assert same_ranges(np_(st["ranges"]), ranges)
    assert np.array_equal(np_(st["ids"])[:len(vals)].astype(np.uint32), vals)
    check_images(*imgs, oracle_ref(orc, ov, okfs, prm))


@pytest.mark.parametrize("zoom", [4.0, 16.0])
def test_odd_long_lists_in_a_sparse_plan_bitwise(R, orc, zoom):
    """A 640x480 view (1,200 tiles) of one 96x72 keyframe seen from far away:
    long lists are not the rule (6,912 records), so one wave per tile sorts
    every list, the four long ones (2,668-3,117 entries at zoom 4, 5,149-5,892
    at zoom 16) as runs of 768 merged in rounds."""
    cam, frames, vpose = room_frames(9, 96, 72, n_kf=1)
    ks = [gpu_kf(R, frames[0])]
    c = (cam.fx / zoom, cam.fy / zoom, 320.0, 240.0, 640, 480)
    plan = R.Plan(ks, [R.View(c, vpose, 0, 1)])
    imgs = plan.render_fwd()
    st = plan.debug_state()
    assert plan.status()[0] == 0
    okfs = [oracle_kf(orc, frames[0])]
    ov = orc.ViewSpec(c, vpose, 0, 1)
    keys, vals, ranges = orc.tile_lists(ov, okfs)
    lens = ranges[:, 1] - ranges[:, 0]
    assert (lens > 768).sum() == 4 and lens.max() > 2600
    assert same_ranges(np_(st["ranges"]), ranges)
    assert np.array_equal(np_(st["ids"])[:len(vals)].astype(np.uint32), vals)
    check_images(*imgs, oracle_ref(orc, ov, okfs))


@pytest.mark.parametrize("case,tile", [("long_runs", 16), ("short_runs", 16), ("long_runs", 32)])
def test_tile_lists_with_depth_ties(R, orc, case, tile):
    """Equal depths are ordered by id: a constant-depth back plane seen from
    its own keyframe (runs of equal depth longer than 64 entries) and a
    keyframe whose column pairs share depths (runs of two).  At tile 32 the
    back plane's lists exceed 768 entries (up to 1311, runs up to 983), so
    the long-list sort takes them."""
    from paper_2506_02741_amd import synth
    if case == "long_runs":
        f, colors = synth.toy_scene(0)
        depth, rgb, cam, pose = f.depth, colors, f.cam.as_tuple(), f.pose
    else:
        cam_, frames, _ = room_frames(5, 80, 60)
        fr = frames[0]
        depth = fr.depth.copy()
        depth[:, 1::2] = depth[:, 0::2]
        rgb, cam, pose = fr.rgb, cam_.as_tuple(), fr.pose
    k = R.Keyframe.ingest(depth, rgb, cam, pose)
    plan = R.Plan([k], [R.View(cam, pose)], R.params(tile=tile))
    imgs = plan.render_fwd()
    st = plan.debug_state()
    assert plan.status()[0] == 0
    okf = orc.ingest(depth, rgb, fx=cam[0], cam=cam, pose=pose)
    ov = orc.ViewSpec(cam, pose)
    keys, vals, ranges = orc.tile_lists(ov, [okf], orc.params(tile=tile))
    z = keys & np.uint64(0xFFFFFFFF)
    ties = sum(int(np.any(z[s + 1:e] == z[s:e - 1])) for s, e in ranges if e - s > 1)
    assert ties > 0
    assert same_ranges(np_(st["ranges"]), ranges)
    assert np.array_equal(np_(st["ids"])[:len(vals)].astype(np.uint32), vals)
    check_images(*imgs, oracle_ref(orc, ov, [okf]))


# ----------------------------------------------------------------------------
# the work counter behind the benchmark's roofline figure, on the GPU state
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("tile", [16, 32])
def test_bench_work_counter_on_gpu_state(R, orc, tile):
    """bench.py counts the compositing units from the plan's own records and
    sorted lists; on the GPU state (bitwise equal to the oracle's, above) it
    gives the counts it gives on the oracle's state, and its contributor
    count agrees with the oracle's within the marginal pixels."""
    import bench
    from test_bench_counts import _OraclePlan
    cam, frames, vpose = room_frames(5, 80, 60)
    fr = frames[0]
    plan = R.Plan([gpu_kf(R, fr)], [R.View(cam.as_tuple(), vpose)], R.params(tile=tile))
    plan.render_fwd()
    assert plan.status()[0] == 0
    got = bench.scan_counts(plan)
    okf = oracle_kf(orc, fr)
    ov = orc.ViewSpec(cam.as_tuple(), vpose)
    prm = orc.params(tile=tile)
    assert got == bench.scan_counts(_OraclePlan(orc, ov, okf, prm))
    out = orc.render(ov, [okf], prm)
    assert abs(got["contrib"] - int(out["n_contrib"].sum())) <= int(out["marginal"].sum())


@pytest.mark.parametrize("case", ["one_wave", "long_list"])
def test_tile_sort_key_with_all_varying_nibbles_15(R, orc, case):
    """A tile whose keys differ only in nibbles where one real key holds 15
    everywhere (depths 1.0 and 1.9999999, bits 0x3F800000 and 0x3FFFFFFF):
    the padding of the sort must still end after that key.  'one_wave': two
    Gaussians in one 16-pixel tile; 'long_list': a plane of 832 Gaussians at
    depth 1.0 and one at 1.9999999 in one 32-pixel tile (a list for the
    long-list sort).  833 records also leave the last wave of the binning
    with one record whose rectangle spans two tile rows, counted and placed
    by lanes that hold no record."""
    W, H = 64, 48
    cam = (60.0, 60.0, 32.0, 24.0, W, H)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
    near_two = np.array([0x3FFFFFFF], np.uint32).view(np.float32)[0]
    depth = np.zeros((H, W), np.float32)
    if case == "one_wave":
        depth[10, 10] = 1.0
        depth[10, 11] = near_two
        tile = 16
    else:
        depth[0:26, 0:32] = 1.0
        depth[28, 20] = near_two
        tile = 32
    rng = np.random.default_rng(7)
    rgb = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    k = R.Keyframe.ingest(depth, rgb, cam, pose)
    plan = R.Plan([k], [R.View(cam, pose)], R.params(tile=tile))
    imgs = plan.render_fwd()
    st = plan.debug_state()
    assert plan.status()[0] == 0
    okf = orc.ingest(depth, rgb, fx=cam[0], cam=cam, pose=pose)
    ov = orc.ViewSpec(cam, pose)
    keys, vals, ranges = orc.tile_lists(ov, [okf], orc.params(tile=tile))
    z = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)  # (tile << 32 | depth bits)
    assert np.any(z == 0x3FFFFFFF)
    if case == "long_list":
        assert int((ranges[:, 1].astype(int) - ranges[:, 0].astype(int)).max()) > 768
    assert same_ranges(np_(st["ranges"]), ranges)
    assert np.array_equal(np_(st["ids"])[:len(vals)].astype(np.uint32), vals)
    check_images(*imgs, oracle_ref(orc, ov, [okf]))


def test_binning_wave_across_views_with_culled_owner_lanes(R, orc):
    """Two views of one 833-Gaussian keyframe in one plan, the second turned
    half way round (every record culled): the binning wave that holds the
    first view's last record and the second view's first 63 shares its box
    with lanes of the other view, which must still count and place the first
    view's pairs in that view's tiles."""
    W, H = 64, 48
    cam = (60.0, 60.0, 32.0, 24.0, W, H)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
    away = np.concatenate([np.diag([-1.0, 1.0, -1.0]), np.zeros((3, 1))], 1).astype(np.float32)
    depth = np.zeros((H, W), np.float32)
    depth[0:26, 0:32] = 1.0
    depth[28, 20] = 1.5
    rgb = np.random.default_rng(8).uniform(0, 1, (3, H, W)).astype(np.float32)
    k = R.Keyframe.ingest(depth, rgb, cam, pose)
    plan = R.Plan([k], [R.View(cam, pose), R.View(cam, away)], R.params(tile=32))
    rgb_o, dep_o, sil_o = plan.render_fwd()
    st = plan.debug_state()
    assert plan.status()[0] == 0
    okf = orc.ingest(depth, rgb, fx=cam[0], cam=cam, pose=pose)
    ov = orc.ViewSpec(cam, pose)
    keys, vals, ranges = orc.tile_lists(ov, [okf], orc.params(tile=32))
    nt = ranges.shape[0]
    assert same_ranges(np_(st["ranges"])[:nt], ranges)
    assert int(np_(st["n_pairs"])[0]) == len(vals)
    assert np.array_equal(np_(st["ids"])[:len(vals)].astype(np.uint32), vals)
    P = W * H
    check_images(rgb_o[:, :P], dep_o[:P], sil_o[:P], oracle_ref(orc, ov, [okf]))
    assert float(sil_o[P:].abs().max()) == 0.0


# ----------------------------------------------------------------------------
# the workloads' full shapes: a mapping section, an uneven pair of views
# ----------------------------------------------------------------------------

def _view_lists_match(st, v_tile_base, n_tiles_v, keys_ref, vals_ref, ranges_ref):
    """The GPU's sorted ids and ranges of one view of a multi-view plan equal
    the oracle's for that view alone (the view's lists are contiguous, in
    tile order, from the first position of its first tile)."""
    rg = np_(st["ranges"])[v_tile_base:v_tile_base + n_tiles_v].astype(np.int64)
    lens = rg[:, 1] - rg[:, 0]
    lens_ref = (ranges_ref[:, 1].astype(np.int64) - ranges_ref[:, 0])
    assert np.array_equal(lens, lens_ref)
    first = int(rg[lens > 0, 0].min()) if (lens > 0).any() else 0
    ids = np_(st["ids"])[first:first + len(vals_ref)].astype(np.uint32)
    assert np.array_equal(ids, vals_ref)
    assert np.array_equal(rg[lens > 0, 0] - first, ranges_ref[lens_ref > 0, 0].astype(np.int64))


def _check_plan_against_oracle(R, orc, plan, ks, okfs, oviews, seed, n_threads=16):
    """Records and tile lists (bitwise), images (1e-5) and the slot-mode
    backward to colour/opacity/radius summed over the plan's views plus each
    view's twist (1e-3 relative) of a multi-view plan against the oracle."""
    rgb, depth, sil = plan.render_fwd()
    st = plan.debug_state()
    assert plan.status()[0] == 0
    recs, rects = np_(st["records"]), np_(st["rect"])
    rng = np.random.default_rng(seed)
    P = plan.P
    g_rgb = rng.normal(size=(3, P)); g_d = rng.normal(size=P); g_s = rng.normal(size=P)
    gsum = None
    tw_ref = []
    rec0 = tile0 = 0
    with orc.threads(n_threads):
        for v, ov in enumerate(oviews):
            o = plan.offsets[v]
            sl = slice(o, o + ov.P)
            rec = orc.preprocess32(ov, okfs)
            n = rec.shape[0]
            valid = rec["count"] > 0
            g, rect = recs[rec0:rec0 + n], rects[rec0:rec0 + n]
            assert np.array_equal(rect[:, 0] <= rect[:, 2], valid)
            assert np.array_equal(rect[valid], rec["rect"][valid])
            for col, name in ((0, "mx"), (1, "my"), (2, "qa"), (3, "qb"), (4, "qc"), (6, "pz"),
                              (7, "ext")):
                assert np.array_equal(g[valid, col], rec[name][valid]), (v, name)
            keys, vals, ranges = orc.tile_lists(ov, okfs)
            _view_lists_match(st, tile0, ranges.shape[0], keys, vals, ranges)
            print("view %d: %d pairs, longest list %d" % (v, len(vals), int((ranges[:, 1] - ranges[:, 0]).max())))
            ref = oracle_ref(orc, ov, okfs)
            check_images(rgb[:, sl], depth[sl], sil[sl], ref)
            m = ref["marginal"]
            g_rgb[:, o:o + ov.P][:, m] = 0; g_d[o:o + ov.P][m] = 0; g_s[o:o + ov.P][m] = 0
            gr = orc.render_bwd(ov, okfs, g_rgb[:, sl], g_d[sl], g_s[sl])
            if gsum is None:
                gsum = {k: gr[k].copy() for k in ("color", "opacity", "radius")}
                msum = {k: gr["mag"][k].copy() for k in ("color", "opacity", "radius")}
            else:
                for k in gsum:
                    gsum[k] += gr[k]
                    msum[k] += gr["mag"][k]
            tw_ref.append((gr["twist"], gr["mag"]["twist"]))
            rec0 += n
            tile0 += ranges.shape[0]
    for k in ks:
        k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
    tw = np_(plan.render_bwd(T(g_rgb), T(g_d), T(g_s)))
    assert plan.status()[0] == 0
    got = dict(color=np.concatenate([np_(k.g_color) for k in ks], 1),
               opacity=np.concatenate([np_(k.g_opacity) for k in ks]),
               radius=np.concatenate([np_(k.g_radius) for k in ks]))
    for name in ("color", "opacity", "radius"):
        ok, worst = grad_close(got[name], gsum[name], name, msum[name])
        assert ok, (name, worst)
    for v, (t_ref, t_mag) in enumerate(tw_ref):
        ok, worst = grad_close(tw[v], t_ref, "twist of view %d" % v, t_mag)
        assert ok, (v, worst, tw[v], t_ref)


def test_mapping_section_full_size(R, orc):
    """The mapping workload's shape (Sec. 3.4: a section's keyframe views
    rendered and back-propagated together): 8 keyframes at 640x480 along a
    10 cm / 5 degree walk (2,457,600 Gaussians, ~90 contributors per pixel)
    seen from two of its keyframes in one plan, whose tile lists run to
    ~15K entries (so the long-list sorts run).  Records, lists, images and
    the summed slot-mode backward against the oracle."""
    from paper_2506_02741_amd import synth
    frames = synth.section_workload(2)["keyframes"]
    cam = frames[0].cam.as_tuple()
    ks = [R.Keyframe.ingest(f.depth, f.rgb, cam, f.pose, 1, 0.99, None, True).with_grad_buffers()
          for f in frames]
    assert sum(k.n for k in ks) == 8 * 640 * 480
    vids = (0, 5)
    plan = R.Plan(ks, [R.View(cam, frames[v].pose, 0, 8) for v in vids])
    okfs = [oracle_kf(orc, f) for f in frames]
    _check_plan_against_oracle(R, orc, plan, ks, okfs,
                               [orc.ViewSpec(cam, frames[v].pose, 0, 8) for v in vids], 11)


def test_uneven_pair_full_size(R, orc):
    """The uneven batch's extreme resolutions in one plan: a 1200x680 and a
    320x240 view (f = 600 and 262.5) of one two-keyframe section whose
    keyframes are 1200x680 and 320x240, each view at its keyframe's pose.
    Records, lists, images and the summed backward against the oracle."""
    from paper_2506_02741_amd import synth
    rng = np.random.default_rng(3)
    scene = synth.make_room(3)
    big, small = synth.camera_for(1200, 680), synth.camera_for(320, 240)
    poses = synth.random_walk(scene, small, rng, 2)
    frames = [synth.frame(scene, big, poses[0]), synth.frame(scene, small, poses[1])]
    ks = [R.Keyframe.ingest(f.depth, f.rgb, f.cam.as_tuple(), f.pose, 1, 0.99, None, True).with_grad_buffers()
          for f in frames]
    views = [R.View(f.cam.as_tuple(), f.pose, 0, 2) for f in frames]
    plan = R.Plan(ks, views)
    okfs = [oracle_kf(orc, f) for f in frames]
    _check_plan_against_oracle(R, orc, plan, ks, okfs,
                               [orc.ViewSpec(f.cam.as_tuple(), f.pose, 0, 2) for f in frames], 12)
