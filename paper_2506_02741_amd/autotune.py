"""Autotuner of the compositing launch shape.

For a workload (keyframes, views, mode) the tuner sweeps tile size
{8, 16, 32} x LDS batch {128, 256, 512}, times the forward + backward of
each configuration with the library's per-stage HIP events, and keeps the
fastest.  Results are cached per shape bucket in a JSON file keyed by the
GPU architecture:

    bucket = (arch, mode, number of views, sorted distinct resolutions,
              Gaussians per view rounded to a power of two)

Every configuration renders the same image bit for bit (each pixel walks
its Gaussians in the same depth order whatever the tile), so the choice
never changes results -- only time.
"""
from __future__ import annotations

import json
import math
import os
import threading

import torch

from . import render as R

TILES = (8, 16, 32)
BATCHES = (128, 256, 512)
_lock = threading.Lock()


def cache_path():
    return os.environ.get("VTGS_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "vtgs", "autotune.json"))


def _arch():
    try:
        return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    except Exception:
        return "unknown"


def bucket(keyframes, views, mode):
    res = sorted({(v.cam.width, v.cam.height) for v in views})
    per_view = [sum(k.n for k in keyframes[v.kf_first:v.kf_first + v.kf_count]) for v in views]
    g = max(per_view) if per_view else 0
    gb = 0 if g == 0 else 1 << int(math.ceil(math.log2(g)))
    return "%s|%s|v%d|%s|g%d" % (_arch(), mode, len(views),
                                  ",".join("%dx%d" % r for r in res), gb)


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _time_config(keyframes, views, mode, tile, batch, reps):
    prm = R.params(tile=tile, batch=batch)
    plan = R.Plan(keyframes, views, prm)
    g = torch.ones(3, plan.P, device=plan.device) * 1e-3
    gd = torch.ones(plan.P, device=plan.device) * 1e-3

    def once():
        plan.render_fwd()
        if mode == "render":
            return
        plan.render_bwd(g, gd, None, twist=(mode == "track"))

    once()
    rc, need = plan.status()
    if rc != 0:
        plan = R.Plan(keyframes, views, prm, pair_capacity=int(need * 1.25) + 1024)
        once()
        rc, _ = plan.status()
        if rc != 0:
            return float("inf"), 0
    plan.timing(True)
    for _ in range(reps):
        once()
    st = plan.timing(False)
    ms = sum(v[0] for v in st.values()) / reps
    return ms, plan.cap


def tune(keyframes, views, mode="track", reps=5, tiles=TILES, batches=BATCHES, force=False):
    """Best (tile, batch) for this workload bucket; returns (params, report).

    mode: "render" (forward only), "track" (forward + backward to the
    twist), "map" (forward + backward to colour/opacity/radius of the
    learnable keyframes).  Keyframe gradient buffers must exist for "map".
    """
    key = bucket(keyframes, views, mode)
    with _lock:
        cache = _load()
    if key in cache and not force:
        e = cache[key]
        return R.params(tile=e["tile"], batch=e["batch"]), e
    results = []
    for t in tiles:
        for b in batches:
            ms, cap = _time_config(keyframes, views, mode, t, b, reps)
            results.append(dict(tile=t, batch=b, ms=ms, cap=cap))
    best = min(results, key=lambda r: r["ms"])
    entry = dict(tile=best["tile"], batch=best["batch"], ms=best["ms"],
                 sweep=[(r["tile"], r["batch"], round(r["ms"], 4)) for r in results])
    with _lock:
        cache = _load()
        cache[key] = entry
        _save(cache)
    return R.params(tile=best["tile"], batch=best["batch"]), entry
