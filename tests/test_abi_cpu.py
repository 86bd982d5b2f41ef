"""Host-side checks of the C ABI: the library loads, exports every entry
point ``include/vtgs.h`` declares, and validates arguments before touching
a GPU (plan creation is host-only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "vtgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vtgs_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2506_02741_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2506_02741_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(L):
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    from paper_2506_02741_amd import _lib
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_version_and_defaults(L):
    from paper_2506_02741_amd import _lib
    assert L.vtgs_abi_version() == _lib.VTGS_ABI_VERSION == 2
    p = _lib.default_params()
    assert p.tile == 16 and p.batch == 256
    assert abs(p.alpha_min - 1 / 255) < 1e-9 and abs(p.alpha_max - 0.99) < 1e-7
    assert abs(p.q_cut - 11.0826) < 1e-5 and abs(p.lowpass - 0.3) < 1e-7


def _kf(n=10, W=8, H=4, learnable=0):
    from paper_2506_02741_amd import _lib
    cam = _lib.vtgs_camera(10.0, 10.0, 4.0, 2.0, W, H)
    fake = 0x1000  # never dereferenced: plan creation is host-only
    return _lib.vtgs_keyframe(n, fake, fake, fake, fake, fake, fake, cam, learnable, None, None,
                              None, None)


def _view(W=8, H=4, first=0, count=1):
    from paper_2506_02741_amd import _lib
    return _lib.vtgs_view(_lib.vtgs_camera(10.0, 10.0, 4.0, 2.0, W, H), 0x1000, first, count,
                          None, None, None, None)


def _create(L, kfs, views, **prm):
    from paper_2506_02741_amd import _lib
    ka = (_lib.vtgs_keyframe * max(len(kfs), 1))(*kfs)
    va = (_lib.vtgs_view * max(len(views), 1))(*views)
    h = C.c_void_p()
    p = _lib.default_params(**prm)
    rc = L.vtgs_plan_create(ka, len(kfs), va, len(views), C.byref(p), 0, C.byref(h))
    return rc, h


def test_plan_sizes(L):
    rc, h = _create(L, [_kf(10), _kf(7)], [_view(first=0, count=2), _view(W=20, H=17, first=1)])
    assert rc == 0
    try:
        assert L.vtgs_plan_records(h) == 17 + 7
        assert L.vtgs_plan_pixels(h) == 32 + 340
        assert L.vtgs_plan_view_offset(h, 1) == 32
        assert L.vtgs_plan_view_offset(h, 2) == -1
        assert L.vtgs_plan_tiles(h) == 1 + 2 * 2
        assert L.vtgs_plan_pair_capacity(h) == int(np.ceil(1.5 * (1 + 10 / 16) ** 2 * 24)) + 65536
        assert L.vtgs_plan_workspace_bytes(h) % 256 == 0
    finally:
        L.vtgs_plan_destroy(h)


@pytest.mark.parametrize("bad", [dict(tile=12), dict(batch=100), dict(alpha_max=1.0),
                                 dict(alpha_min=0.5, alpha_max=0.4), dict(q_cut=-1.0)])
def test_plan_rejects_bad_params(L, bad):
    from paper_2506_02741_amd import _lib
    rc, h = _create(L, [_kf()], [_view()], **bad)
    assert rc == _lib.VTGS_E_ARG and not h.value
    assert len(_lib.last_error()) > 0


def test_plan_rejects_bad_views(L):
    from paper_2506_02741_amd import _lib
    rc, _ = _create(L, [_kf()], [_view(first=0, count=2)])
    assert rc == _lib.VTGS_E_ARG and "slice" in _lib.last_error()
    rc, _ = _create(L, [_kf()], [_view(W=0)])
    assert rc == _lib.VTGS_E_ARG
    bad = _kf()
    bad.pix = None
    rc, _ = _create(L, [bad], [_view()])
    assert rc == _lib.VTGS_E_ARG and "NULL" in _lib.last_error()
    rc, _ = _create(L, [], [])
    assert rc == _lib.VTGS_E_ARG


def test_unbound_plan_and_null_args(L):
    from paper_2506_02741_amd import _lib
    rc, h = _create(L, [_kf()], [_view()])
    try:
        assert L.vtgs_render_fwd(h, None, None, None, None) == _lib.VTGS_E_WORKSPACE
        assert L.vtgs_plan_bind(h, None, 0, None) == _lib.VTGS_E_WORKSPACE
        assert L.vtgs_plan_bind(h, 0x1001, 1 << 40, None) == _lib.VTGS_E_WORKSPACE  # misaligned
        assert L.vtgs_plan_bind(h, 0x1000, 16, None) == _lib.VTGS_E_WORKSPACE      # too small
    finally:
        L.vtgs_plan_destroy(h)
    assert L.vtgs_render_fwd(None, None, None, None, None) == _lib.VTGS_E_ARG
    assert L.vtgs_ingest_count(None, None, 4, 4, 1, None, 0, None, None) == _lib.VTGS_E_ARG
    assert L.vtgs_ingest_scratch_bytes(480, 640, 1) > 0
    assert L.vtgs_ingest_scratch_bytes(0, 640, 1) == 0


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_bench_traffic_summary_tracks_kernel_sources(tmp_path, monkeypatch):
    """The committed counter summary is used only while the kernel sources
    still hash to the value it records."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source")
    import hashlib
    good = hashlib.sha256(b"kernel source").hexdigest()
    f = tmp_path / "traffic.txt"
    f.write_text("hbm_bytes_per_launch: 1234\nsources_sha256: %s\n" % good)
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(b, "TRAFFIC_SOURCES", [str(src)])
    assert b.measured_traffic("composite_bwd") == 1234.0
    src.write_bytes(b"kernel source, changed")
    assert b.measured_traffic("composite_bwd") is None


def test_pair_capacity_limit(L):
    """Tile lists are indexed with 32-bit signed positions: an explicit
    capacity above 2^31 - 1 is an argument error, and the default room is
    clamped to it."""
    from paper_2506_02741_amd import _lib
    import ctypes as C
    kfs, views = [_kf()], [_view()]
    ka = (_lib.vtgs_keyframe * 1)(*kfs)
    va = (_lib.vtgs_view * 1)(*views)
    p = _lib.default_params()
    h = C.c_void_p()
    assert L.vtgs_plan_create(ka, 1, va, 1, C.byref(p), (1 << 31), C.byref(h)) == _lib.VTGS_E_ARG
    assert "2^31" in _lib.last_error() and not h.value
    assert L.vtgs_plan_create(ka, 1, va, 1, C.byref(p), (1 << 31) - 1, C.byref(h)) == _lib.VTGS_OK
    try:
        assert L.vtgs_plan_pair_capacity(h) == (1 << 31) - 1
    finally:
        L.vtgs_plan_destroy(h)


def test_debug_entries_need_a_bound_plan(L):
    from paper_2506_02741_amd import _lib
    rc, h = _create(L, [_kf(learnable=1)], [_view()])
    try:
        assert L.vtgs_debug_images(h, None, None, None) == _lib.VTGS_E_WORKSPACE
        assert L.vtgs_debug_gather(h, None) == _lib.VTGS_E_WORKSPACE
    finally:
        L.vtgs_plan_destroy(h)
    assert L.vtgs_debug_gather(None, None) == _lib.VTGS_E_ARG
