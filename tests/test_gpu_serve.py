"""Serving on the GPU: requests that share ticks give the same results as
each request served alone (render bit-identical, track pose bit-identical),
admission respects the memory budget, and every request completes."""
import numpy as np
import pytest

from scenes import room_frames

pytestmark = pytest.mark.gpu


def _requests(serve, cam, frames, n=10, seed=0):
    from paper_2506_02741_amd import synth
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        sec = i % 2
        base = frames[2 * sec + (i // 2) % 2]
        pose = synth.perturb_pose(base.pose, rng, 0.01, 0.5).astype(np.float32)
        if i % 3 == 2:
            reqs.append(serve.Request(i, "track", sec, cam.as_tuple(), pose, base.rgb, base.depth,
                                      iters=4 + i % 3, arrival=0.002 * i))
        else:
            reqs.append(serve.Request(i, "render", sec, cam.as_tuple(), pose, arrival=0.002 * i))
    return reqs


def test_serving_alone_equals_mix():
    import torch
    from paper_2506_02741_amd import render as R
    from paper_2506_02741_amd import serve
    torch.cuda.set_device(0)
    cam, frames, _ = room_frames(9, 96, 72, n_kf=4)
    ks = [R.Keyframe.ingest(f.depth, f.rgb, cam.as_tuple(), f.pose) for f in frames]
    sections = [(0, 2), (2, 2)]
    mix = serve.Server(ks, sections, budget_bytes=3 * 40 << 20, max_active=6)
    rep = mix.run_trace(_requests(serve, cam, frames), realtime=False)
    assert rep["requests"] == 10 and mix.peak_mem <= mix.budget
    assert max(a + b for a, b in mix.batch_sizes) > 1   # requests did share ticks
    got = {r.rid: r for r in mix.finished}
    for r in _requests(serve, cam, frames):
        alone = serve.Server(ks, sections, budget_bytes=1 << 34, max_active=1)
        alone.run_trace([r], realtime=False)
        a = alone.finished[0]
        m = got[r.rid]
        if r.kind == "render":
            for k in ("rgb", "depth", "sil"):
                assert torch.equal(a.result[k], m.result[k]), (r.rid, k)
        else:
            assert np.array_equal(a.result["pose"], m.result["pose"]), r.rid
            assert np.array_equal(a.result["loss"], m.result["loss"]), r.rid
