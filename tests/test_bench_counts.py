"""The work counter behind bench.py's roofline figure (host code, no GPU).

bench.py counts the units a compositing launch processes from the plan's
sorted tile lists and records.  Here the same counter runs on the oracle's
FP32 records and tile lists of a small room (80x60, a ragged tile row) and
is checked against the oracle's own contributor counts (Sec. 3.3 front-to-
back compositing with the alpha_min skip and the t_min stop) and, on every
pixel, against a plain per-entry walk of its tile list.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


class _OraclePlan:
    """A stand-in for a one-view plan whose state comes from the oracle."""

    def __init__(self, orc, view, kf, prm):
        import torch
        rec = orc.preprocess32(view, [kf], prm)
        keys, vals, ranges = orc.tile_lists(view, [kf], prm)
        n = rec.shape[0]
        r = np.zeros((n, 12), np.float32)
        for j, name in enumerate(("mx", "my", "qa", "qb", "qc")):
            r[:, j] = rec[name]
        r[:, 5] = kf.opacity
        self.prm = prm
        self.n_tiles = ranges.shape[0]
        self.layout = [(int(view.cam[4]), int(view.cam[5]), 0, 0)]
        self._state = dict(records=torch.from_numpy(r),
                           ranges=torch.from_numpy(ranges.astype(np.int64)),
                           ids=torch.from_numpy(vals.astype(np.int64)))

    def debug_state(self):
        return self._state


def _walk(plan, width, height):
    """Per pixel, step through the tile list one entry at a time."""
    st = plan.debug_state()
    rec = st["records"].numpy()
    ranges = st["ranges"].numpy()
    ids = st["ids"].numpy()
    prm = plan.prm
    B = prm.tile
    tiles_x = (width + B - 1) // B
    f32 = np.float32
    k = f32(-0.5 * np.log2(np.e))
    scanned = contrib = back = 0
    for y in range(height):
        for x in range(width):
            t = (y // B) * tiles_x + x // B
            s, e = int(ranges[t, 0]), int(ranges[t, 1])
            T = f32(1)
            nc, last, steps = 0, -1, 0
            for j in range(s, e):
                steps += 1
                r = rec[ids[j]]
                dx, dy = f32(x) - r[0], f32(y) - r[1]
                q = (r[2] * dx) * dx + (f32(2) * r[3] * dx) * dy + (r[4] * dy) * dy
                if q > f32(prm.q_cut):
                    continue
                a = min(f32(prm.alpha_max), r[5] * np.exp2(q * k))
                if a < f32(prm.alpha_min):
                    continue
                Tn = T * (f32(1) - a)
                if Tn < f32(prm.t_min):
                    break
                T = Tn
                nc += 1
                last = j - s
            scanned += steps
            contrib += nc
            back += last + 1
    return dict(fwd_scanned=scanned, contrib=contrib, bwd_scanned=back)


def test_scan_counts_match_walk_and_oracle(orc):
    import bench
    from test_oracle_pins import small_room
    fr, kf, view = small_room(orc)
    prm = orc.params()
    plan = _OraclePlan(orc, view, kf, prm)
    W, H = int(view.cam[4]), int(view.cam[5])
    got = bench.scan_counts(plan)
    assert got == _walk(plan, W, H)
    out = orc.render(view, [kf], prm)
    ref = int(out["n_contrib"].sum())
    # a pixel whose FP32 decision the oracle marks marginal may differ by one
    assert abs(got["contrib"] - ref) <= int(out["marginal"].sum())
    assert got["contrib"] <= got["bwd_scanned"] <= got["fwd_scanned"]
    # the figure reported with it: lane-ops per launch
    work = bench.lane_op_work(got)
    assert work["composite_fwd"] == 8 * (got["fwd_scanned"] - got["contrib"]) + 22 * got["contrib"]
    assert work["composite_bwd"] == 10 * (got["bwd_scanned"] - got["contrib"]) + 90 * got["contrib"]
