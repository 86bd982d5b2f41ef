"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) runs every entry point on a small room scene without a
report: no out-of-bounds access, use after free, leak or undefined
arithmetic in the checker the parity tests rely on."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    from scenes import room_frames
    cam, frames, vpose = room_frames(5, 48, 36)
    fr = frames[0]
    d = tmp_path
    np.array([cam.height, cam.width], np.int32).tofile(d / "dims.bin")
    fr.depth.astype(np.float32).tofile(d / "depth.bin")
    fr.rgb.astype(np.float32).tofile(d / "rgb.bin")
    np.asarray(fr.pose, np.float32).tofile(d / "kpose.bin")
    np.asarray(vpose, np.float32).tofile(d / "vpose.bin")
    np.array([cam.fx, cam.fy, cam.cx, cam.cy], np.float32).tofile(d / "intr.bin")
    exe = d / "oracle_sanitize"
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-std=c11", "-o", str(exe), os.path.join(HERE, "oracle_sanitize_main.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    # (verify_asan_link_order=0: the environment may preload a library of its
    # own ahead of the sanitizer runtime)
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([str(exe), str(d)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.startswith("ok "), r.stdout
