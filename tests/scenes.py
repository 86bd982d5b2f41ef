"""Seeded test scenes built once and handed to both the oracle and the HIP
path (the generator holds none of the renderer's arithmetic)."""
import functools

import numpy as np

from paper_2506_02741_amd import synth


@functools.lru_cache(maxsize=None)
def room_frames(seed, w, h, n_kf=1, step=0.10):
    """n_kf frames of a synthetic room along a walk; plus a perturbed view."""
    rng = np.random.default_rng(seed)
    scene = synth.make_room(seed)
    f = w * 525.0 / 640.0
    cam = synth.Camera(f, f, w / 2.0, h / 2.0, w, h)
    if n_kf == 1:
        poses = [synth.random_room_pose(scene, cam, rng)]
    else:
        poses = synth.random_walk(scene, cam, rng, n_kf, step=step)
    frames = [synth.frame(scene, cam, T) for T in poses]
    view_pose = synth.perturb_pose(poses[0], rng, 0.03, 2.0).astype(np.float32)
    return cam, frames, view_pose


def oracle_kf(orc, fr, stride=1, mask=None, o_init=0.99):
    return orc.ingest(fr.depth, fr.rgb, mask, stride, fx=fr.cam.fx, o_init=o_init,
                      cam=fr.cam.as_tuple(), pose=fr.pose)
