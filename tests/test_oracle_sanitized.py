"""The C half of the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer: a sanitized build of the same source runs the
mirror's steps (skinning, back-face flags, the visibility raster in both
modes and its filters, the shadow-mapping variant, splat projection,
binning, tiled and brute-force compositing, nearest neighbours,
densification) on small scenes in a child process, which must finish
without a sanitizer report."""

import os
import subprocess
import sys

import pytest

from oracle import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
from oracle import cpu
from paper_2407_10707_amd import synth
for seed, n, h, w in ((3, 120, 37, 53), (4, 40, 16, 16)):
    s = synth.micro_scene(seed, n, h, w)
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    front = cpu.front_f32(xo, no, s["cam"].centre.astype(np.float32))
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    raw, cnt = cpu.mesh_visibility(vx, s["faces"], s["view_dirs"], s["vis_res"], s["knn_v"])
    cpu.mesh_visibility_shadow(vx, s["faces"], s["view_dirs"], s["vis_res"], s["knn_v"], 1.5)
    cpu.raster_view(vx, s["faces"], s["view_dirs"][0], s["vis_res"], brute=True)
    pre = cpu.splat_preprocess(s["cam"], xo, Ao, s["quat"], s["log_s"], s["opac"], front)
    keys, vals, ranges = cpu.splat_bin(s["cam"], pre)
    col = np.random.default_rng(seed).random((3, n)).astype(np.float32)
    cpu.composite_tiles(s["cam"], ranges, vals, pre, s["opac"], col, with_applied=True)
    cpu.composite_brute(s["cam"], pre, s["opac"], col)
    cpu.knn(s["pos"], s["verts"], 3)
    r = cpu.densify(s["vidx"], s["verts"], s["faces"], d0=4.0, p0=2.0, seed=seed, cap=64)
    assert int(r["ng"].sum()) == r["n_added"]
print("sanitized oracle ok")
"""


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan is not available")
    lib = build.build_sanitized(str(tmp_path / "librga_oracle_san.so"))
    env = dict(os.environ, RGA_ORACLE_LIBRARY=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "sanitized oracle ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
