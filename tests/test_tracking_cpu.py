"""Host logic of the per-frame tracking driver: the constant-speed pose
prediction and the divergence check with its hook (a frame whose final
loss exceeds 50 times the mean of the frames before it).  The track runs
themselves are scripted here; the GPU test drives real ones."""
import numpy as np
import pytest

from paper_2506_02741_amd import tracking


def se3(rng, rot=0.05, trans=0.1):
    w = rng.normal(size=3) * rot
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]) / th
    R = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K   # Rodrigues
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = rng.normal(size=3) * trans
    return T


def test_constant_speed_continues_a_constant_motion():
    rng = np.random.default_rng(0)
    D, T0 = se3(rng), se3(rng, 1.0, 1.0)
    Ts = [np.linalg.matrix_power(D, k) @ T0 for k in range(4)]
    for k in range(2, 4):
        got = tracking.constant_speed(Ts[k - 1][:3], Ts[k - 2][:3])
        assert np.allclose(got, Ts[k][:3], atol=1e-12)
    # no motion: the same pose
    assert np.allclose(tracking.constant_speed(T0[:3], T0[:3]), T0[:3], atol=1e-12)


def test_divergence_threshold():
    c = tracking.DivergenceCheck(50.0)
    assert not c.diverged(1e9)            # nothing to compare with yet
    c.record(1.0); c.record(3.0)           # mean 2
    assert not c.diverged(100.0)           # exactly 50x: not above
    assert c.diverged(100.0 + 1e-9)
    assert c.mean() == 2.0


class Scripted(tracking.FrameTracker):
    """Track runs replaced by a script: init pose -> (pose, loss)."""

    def __init__(self, script, **kw):
        super().__init__(cam=None, device="cpu", **kw)
        self.script = script
        self.runs = []

    def _run(self, keyframes, init_pose, obs_rgb, obs_depth, vis):
        self.runs.append(np.asarray(init_pose, np.float64).copy())
        return self.script(len(self.runs) - 1, np.asarray(init_pose, np.float64))


def test_hook_retracks_a_diverged_frame_and_keeps_the_history():
    losses = iter([2.0, 2.0, 2.0, 500.0, 1.5, 2.5])
    calls = []
    good = np.hstack([np.eye(3), np.array([[0.0], [0.0], [9.0]])])

    def hook(idx, init, loss, mean):
        calls.append((idx, loss, mean))
        return good

    tr = Scripted(lambda i, init: (init + 0.01 * i, next(losses)), on_divergence=hook)
    P0 = np.hstack([np.eye(3), np.zeros((3, 1))])
    for k in range(3):
        pose, loss, div = tr.track([], None, None, init_pose=P0 if k == 0 else None)
        assert not div
    # frame 3 diverges (500 > 50 * 2): the hook's pose is tracked again
    pose, loss, div = tr.track([], None, None)
    assert div and calls == [(3, 500.0, 2.0)]
    assert np.array_equal(tr.runs[-1], good) and loss == 1.5
    assert tr.check.losses == [2.0, 2.0, 2.0, 1.5]
    # frame 4: predicted by constant speed from frames 3 and 2
    pred = tracking.constant_speed(tr.poses[-1], tr.poses[-2])
    tr.track([], None, None)
    assert np.allclose(tr.runs[-1], pred)
    assert tr.events == [(3, 500.0, 2.0, True)]


def test_hook_may_decline():
    losses = iter([1.0, 100.0])
    tr = Scripted(lambda i, init: (init, next(losses)), on_divergence=lambda *a: None)
    P0 = np.hstack([np.eye(3), np.zeros((3, 1))])
    tr.track([], None, None, init_pose=P0)
    pose, loss, div = tr.track([], None, None)
    assert div and loss == 100.0 and len(tr.runs) == 2
    assert tr.events == [(1, 100.0, 1.0, False)]


def test_first_frame_needs_a_pose():
    tr = Scripted(lambda i, init: (init, 1.0))
    with pytest.raises(ValueError):
        tr.track([], None, None)
