"""Checkpoint / resume of the map: a section store with a frozen, offloaded
section and a learnable one (with optimiser states) written by save_map and
read back by load_map gives the same structure, counters and tensors."""
import numpy as np
import torch

from paper_2506_02741_amd import render as R
from paper_2506_02741_amd import sections as S


def kf(rng, n, learnable):
    cam = (50.0, 50.0, 16.0, 12.0, 32, 24)
    pose = np.hstack([np.eye(3), rng.normal(size=(3, 1))]).astype(np.float32)
    k = R.Keyframe(cam, pose, rng.choice(32 * 24, size=n, replace=False), rng.uniform(0.5, 4, n),
                   rng.uniform(0, 1, (3, n)), np.full(n, 0.99), rng.uniform(0.01, 0.05, n),
                   learnable=learnable, device="cpu")
    k.depth_map = torch.tensor(rng.uniform(0.5, 4, (24, 32)), dtype=torch.float32)
    return k


def test_save_and_load_round_trip(tmp_path):
    rng = np.random.default_rng(3)
    store = S.SectionStore(device="cpu")
    store.start_section(kf(rng, 40, True))
    store.add_keyframe(kf(rng, 25, True))
    store.start_section(kf(rng, 30, True))      # freezes the first section
    store.offload(store.sections[0])
    cur = store.current.keyframes[0].with_adam().with_geometry_adam()
    cur.adam.uniform_(); cur.depth_adam.uniform_(); cur.pose_adam.uniform_()
    path = tmp_path / "map.safetensors"
    S.save_map(store, path)
    back = S.load_map(path, device="cpu")
    assert back.total_gaussians == store.total_gaussians == 95
    assert back.peak_resident == store.peak_resident
    assert [s.index for s in back.sections] == [0, 1]
    assert back.sections[0].frozen and not back.sections[1].frozen
    assert all(s.resident for s in back.sections)
    for s0, s1 in zip(store.sections, back.sections):
        for j, (a, b) in enumerate(zip(s0.keyframes, s1.keyframes)):
            src = s0.host[j] if not s0.resident else {n: getattr(a, n) for n in S._KF_TENSORS}
            for n in S._KF_TENSORS:
                assert torch.equal(src[n], getattr(b, n)), n
            assert b.cam == a.cam
            assert b.learnable == a.learnable
    nk = back.current.keyframes[0]
    for n in ("adam", "depth_adam", "pose_adam"):
        assert torch.equal(getattr(nk, n), getattr(cur, n)), n
    assert nk.g_color is not None and nk.g_depth is not None
