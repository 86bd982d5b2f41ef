"""The per-frame tracking driver on the GPU: frames of a walk tracked against
the first frame's keyframe from constant-speed predictions, then a frame
whose observation is replaced by noise, which diverges (its final Eq. 1 loss
above 50 times the mean of the frames before it): the hook is called once,
and the frame is tracked again from the pose the hook gives, with the same
result as a track run from that pose alone."""
import numpy as np
import pytest

from scenes import room_frames

pytestmark = pytest.mark.gpu


def test_frame_tracker_divergence_hook():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    from paper_2506_02741_amd import render as R
    from paper_2506_02741_amd import tracking
    cam, frames, _ = room_frames(21, 96, 72, n_kf=5, step=0.02)
    kf = frames[0]
    ks = [R.Keyframe.ingest(kf.depth, kf.rgb, cam.as_tuple(), kf.pose)]
    calls = []
    good = np.asarray(frames[4].pose, np.float64).reshape(3, 4)

    def hook(idx, init, loss, mean):
        calls.append((idx, loss, mean))
        return good

    tr = tracking.FrameTracker(cam.as_tuple(), iters=20, on_divergence=hook)
    for i in range(1, 4):
        init = frames[0].pose if i == 1 else None
        if i == 2:
            init = frames[1].pose     # two known poses before the prediction starts
        pose, loss, div = tr.track(ks, frames[i].rgb, frames[i].depth, init_pose=init)
        print("frame %d: loss %.4g" % (i, loss), flush=True)
        assert not div and np.isfinite(pose).all() and loss > 0
    rng = np.random.default_rng(3)
    noise_rgb = rng.uniform(0, 1, size=frames[4].rgb.shape).astype(np.float32)
    noise_d = (frames[4].depth * rng.uniform(0.1, 10.0, size=frames[4].depth.shape)).astype(np.float32)
    pose, loss, div = tr.track(ks, noise_rgb, noise_d)
    print("noise frame: loss %.4g, mean before %.4g" % (loss, calls[0][2] if calls else -1), flush=True)
    assert div and len(calls) == 1 and calls[0][0] == 3
    assert calls[0][1] > 50 * calls[0][2]
    ref_pose, ref_loss = tr._run(ks, good, noise_rgb, noise_d, None)
    assert np.array_equal(pose, ref_pose) and loss == ref_loss
    assert tr.events[-1][3] is True
