"""The compositing kernels skip, per wave, the entries whose cut-off ellipse
cannot reach the wave's pixel block, using a circle around mu of squared
radius 1.0201 q_cut lambda_max / det (lambda_max, det of the conic Q): every
offset d with d^T Q d <= q_cut has |d|^2 <= q_cut / lambda_min(Q), and the 2 %
cover FP32 rounding of q.  Checked here in float32 for random conics (the
view-tied range and strongly anisotropic ones) at pixel offsets around mu."""
import numpy as np

Q_CUT = np.float32(11.0826)


def r2_bound(qa, qb, qc):
    f = np.float32
    h = f(0.5) * (qa - qc)
    lmax = f(0.5) * (qa + qc) + np.sqrt(h * h + qb * qb)
    det = qa * qc - qb * qb
    return np.where(det > 0, f(1.0201) * Q_CUT * lmax / det, f(3e38)).astype(f)


def test_every_pixel_within_the_cutoff_lies_in_the_cull_circle():
    rng = np.random.default_rng(0)
    f = np.float32
    n = 20000
    # covariance r^2 J J^T + 0.3 I style conics and anisotropic ones
    s1 = rng.uniform(0.3, 40.0, n)
    s2 = s1 * rng.uniform(0.05, 1.0, n)
    th = rng.uniform(0, np.pi, n)
    c, s = np.cos(th), np.sin(th)
    sxx = c * c * s1 + s * s * s2
    syy = s * s * s1 + c * c * s2
    sxy = c * s * (s1 - s2)
    det = sxx * syy - sxy * sxy
    qa, qb, qc = (syy / det).astype(f), (-sxy / det).astype(f), (sxx / det).astype(f)
    mx = rng.uniform(0, 1, n).astype(f) + f(100)
    my = rng.uniform(0, 1, n).astype(f) + f(200)
    r2 = r2_bound(qa, qb, qc)
    worst = 0.0
    for ox in range(-22, 23):
        for oy in range(-22, 23):
            dx = (np.floor(mx) + f(ox) - mx).astype(f)
            dy = (np.floor(my) + f(oy) - my).astype(f)
            q = (qa * dx) * dx
            q = ((f(2) * qb) * dx * dy + q).astype(f)
            q = ((qc * dy) * dy + q).astype(f)
            inq = q <= Q_CUT
            d2 = (dx * dx + dy * dy).astype(np.float64)
            assert not np.any(inq & (d2 > r2)), (ox, oy)
            if inq.any():
                worst = max(worst, float((d2[inq] / r2[inq]).max()))
    # the bound is tight up to the 2 % margin (the ellipse reaches it)
    assert 0.9 < worst <= 1.0
