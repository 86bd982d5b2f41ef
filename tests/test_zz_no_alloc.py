"""vtgs_render_fwd_static, the forward for callers that cannot allocate,
against vtgs_render_fwd on a caller workspace: the same kernels, so the
images must be bitwise equal, and the backward through the static scratch
must equal the backward through the workspace.  Two calls in a row, the
second with a smaller input (fewer keyframes, a smaller view), so the
scratch's leftover contents from the first must not leak into the second."""
import numpy as np
import pytest

from scenes import room_frames

pytestmark = pytest.mark.gpu


def np_(t):
    return t.detach().cpu().numpy()


def test_static_forward_equals_workspace_forward_twice():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2506_02741_amd import _lib
    from paper_2506_02741_amd import render as R
    cam, frames, vpose = room_frames(9, 96, 72, n_kf=3)
    ks = [R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose, 1, 0.99, None, True).with_grad_buffers()
          for f in frames]
    small = (cam.fx / 2, cam.fy / 2, 24.0, 18.0, 48, 36)
    cases = [("3 keyframes, 96x72", ks, [R.View(cam.as_tuple(), vpose, 0, 3)]),
             ("1 keyframe, 48x36", ks[:1], [R.View(small, vpose, 0, 1)])]
    rng = np.random.default_rng(5)
    for name, kfs, views in cases:
        print("case:", name, flush=True)
        ref_plan = R.Plan(kfs, views)
        ref = [np_(x) for x in ref_plan.render_fwd()]
        for k in kfs:
            k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
        g_rgb = torch.tensor(rng.normal(size=(3, ref_plan.P)), dtype=torch.float32, device="cuda")
        g_d = torch.tensor(rng.normal(size=ref_plan.P), dtype=torch.float32, device="cuda")
        tw_ref = np_(ref_plan.render_bwd(g_rgb, g_d, None))
        gref = [(np_(k.g_color).copy(), np_(k.g_opacity).copy(), np_(k.g_radius).copy()) for k in kfs]
        assert ref_plan.status()[0] == 0
        sp = R.Plan(kfs, views, workspace="static")
        assert sp.ws_bytes <= _lib.VTGS_STATIC_SCRATCH_BYTES
        out = sp.empty_images()
        for _ in range(2):  # the second call reuses the uploaded descriptors
            got = [np_(x) for x in sp.render_fwd_static(*out)]
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), name
            for o in out:
                o.fill_(-1.0)
        for k in kfs:
            k.g_color.zero_(); k.g_opacity.zero_(); k.g_radius.zero_()
        sp.render_fwd_static(*out)
        tw = np_(sp.render_bwd(g_rgb, g_d, None))
        assert np.array_equal(tw, tw_ref), name
        for k, (c, o, r) in zip(kfs, gref):
            assert np.array_equal(np_(k.g_color), c) and np.array_equal(np_(k.g_opacity), o)
            assert np.array_equal(np_(k.g_radius), r)
        assert sp.status()[0] == 0
        del sp, ref_plan
    torch.cuda.synchronize()


def test_static_forward_rejects_a_plan_larger_than_the_scratch():
    import torch
    torch.cuda.set_device(0)
    from paper_2506_02741_amd import _lib
    from paper_2506_02741_amd import render as R
    cam, frames, vpose = room_frames(9, 96, 72, n_kf=3)
    k = R.Keyframe.ingest(frames[0].depth, frames[0].rgb, cam.as_tuple(), frames[0].pose)
    plan = R.Plan([k], [R.View(cam.as_tuple(), vpose)], pair_capacity=(1 << 31) - 1,
                  workspace="static")
    assert plan.ws_bytes > _lib.VTGS_STATIC_SCRATCH_BYTES
    with pytest.raises(_lib.VtgsError) as e:
        plan.render_fwd_static(*plan.empty_images())
    assert e.value.code == _lib.VTGS_E_WORKSPACE
