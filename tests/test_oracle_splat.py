"""Pins of the splatting oracle (the 3DGS rasterizer of Sec. 3.1): closed
forms for one and two Gaussians, invariants, brute force, and agreement of the
FP32 mirror (C) with the independent FP64 implementation (PyTorch)."""

import math

import numpy as np
import pytest
import torch

from oracle import cpu, ref64
from paper_2407_10707_amd import synth
from tests import helpers
from tests.conftest import scene


def _gauss_set(xyz, sigma, opac, colors, W=64, H=64, quat=None):
    n = len(xyz)
    cam = synth.default_camera(W, H)
    x = np.asarray(xyz, np.float32).T.copy()
    A = np.tile(np.eye(3, dtype=np.float32).reshape(9, 1), (1, n))
    q = np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)) if quat is None else quat
    ls = np.log(np.asarray(sigma, np.float64)).astype(np.float32)
    if ls.ndim == 1:
        ls = np.tile(ls[None, :], (3, 1))
    o = np.asarray(opac, np.float32)
    col = np.asarray(colors, np.float32).T.copy()
    front = np.ones(n, np.uint8)
    return cam, x, A, q, ls, o, col, front


def _render_f32(cam, x, A, q, ls, o, col, front):
    pre = cpu.splat_preprocess(cam, x, A, q, ls, o, front)
    keys, vals, ranges = cpu.splat_bin(cam, pre)
    img, T, margin = cpu.composite_tiles(cam, ranges, vals, pre, o, col)
    return pre, keys, vals, ranges, img, T, margin


def test_exp_and_ln_bound_helpers():
    xs = np.linspace(-12, 6, 4001)
    got = np.array([cpu.exp_f32(float(np.float32(v))) for v in xs], np.float64)
    ref = np.exp(xs.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(got - ref) / ref) < 3e-7
    ys = np.concatenate([np.linspace(1, 255, 3001), 2.0 ** np.arange(0, 8)])
    lb = np.array([cpu.ln_upper_f32(float(np.float32(y))) for y in ys], np.float64)
    ly = np.log(ys.astype(np.float32).astype(np.float64))
    assert np.all(lb >= ly - 1e-6)
    assert np.all(lb - ly < 0.02)


def test_lone_isotropic_gaussian_closed_form():
    """alpha(p) = o exp(-|p - c|^2 / (2 (s^2 + 0.3))), s = f sigma / Z."""
    sigma, o, c = 0.05, 0.6, np.array([0.2, 0.5, 0.9])
    cam, x, A, q, ls, op, col, front = _gauss_set([[0, 0, 0]], [sigma], [o], [c])
    pre, keys, vals, ranges, img, T, margin = _render_f32(cam, x, A, q, ls, op, col, front)
    s = cam.fx * float(np.float32(math.exp(float(ls[0, 0])))) / 3.0
    ii, jj = np.meshgrid(np.arange(cam.width) + 0.5, np.arange(cam.height) + 0.5)
    r2 = (ii - cam.cx) ** 2 + (jj - cam.cy) ** 2
    alpha = np.minimum(0.99, o * np.exp(-0.5 * r2 / (s * s + 0.3)))
    alpha[alpha < 1 / 255] = 0
    ok = np.abs(alpha * 255 - 1) > 1e-3           # away from the cut-off
    for ch in range(3):
        assert np.allclose(img[ch][ok], c[ch] * alpha[ok], rtol=2e-6, atol=1e-7)
    # summed opacity = integral of the truncated Gaussian = 2 pi s2 (o - 1/255)
    mass = 2 * math.pi * (s * s + 0.3) * (o - 1 / 255)
    assert abs((1 - T).sum() / mass - 1) < 3e-3


def test_two_gaussians_over_operator():
    c1, c2 = np.array([1.0, 0.2, 0.1]), np.array([0.1, 0.3, 1.0])
    cam, x, A, q, ls, op, col, front = _gauss_set([[0, 0, 0.4], [0, 0, -0.3]], [0.04, 0.06],
                                                  [0.7, 0.8], [c1, c2])
    pre, keys, vals, ranges, img, T, _ = _render_f32(cam, x, A, q, ls, op, col, front)
    # the pixel nearest the axis
    i, j = int(cam.cx), int(cam.cy)
    px, py = i + 0.5, j + 0.5
    al = []
    for g, Z in ((0, 3 - 0.4), (1, 3 + 0.3)):
        s = cam.fx * float(np.float32(math.exp(float(ls[0, g])))) / Z
        r2 = (px - cam.cx) ** 2 + (py - cam.cy) ** 2
        al.append(min(0.99, float(op[g]) * math.exp(-0.5 * r2 / (s * s + 0.3))))
    want = c1 * al[0] + c2 * al[1] * (1 - al[0])
    assert np.allclose(img[:, j, i], want, rtol=1e-5)
    assert abs(T[j, i] - (1 - al[0]) * (1 - al[1])) < 1e-6


def test_white_splats_satisfy_one_minus_transmittance(scene1):
    """All colours 1: C = sum alpha_i T_i = 1 - T_final at every pixel."""
    s = scene1
    f = helpers.oracle_frame_f32(s, np.ones((3, s["n"]), np.float32))
    for ch in range(3):
        assert np.allclose(f["img"][ch], 1 - f["T"], atol=2e-6)
    assert f["T"].min() >= 0 and f["T"].max() <= 1


@pytest.mark.parametrize("case", ["cfg1", "micro_odd", "micro_ragged"])
def test_tiled_equals_brute_force(case):
    if case == "cfg1":
        s = scene(1)
    elif case == "micro_odd":
        s = synth.micro_scene(1, 300, 37, 53)
    else:
        s = synth.micro_scene(2, 800, 96, 161, log_scale_mean=-3.0)
    col = np.random.default_rng(0).random((3, s["n"])).astype(np.float32)
    f = helpers.oracle_frame_f32(s, col)
    img_b, T_b = cpu.composite_brute(s["cam"], f["pre"], s["opac"], col)
    assert np.array_equal(f["img"], img_b)
    assert np.array_equal(f["T"], T_b)


def test_sort_keys_and_lists(scene1):
    s = scene1
    f = helpers.oracle_frame_f32(s, np.ones((3, s["n"]), np.float32))
    keys, vals, pre = f["keys"], f["vals"], f["pre"]
    assert len(keys) == pre["touched"].sum()
    order = np.lexsort((vals, keys))
    assert np.array_equal(order, np.arange(len(keys)))          # sorted by (key, index)
    tx, ty = cpu.tiles_of(s["cam"])
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    zb = pre["depth"].view(np.uint32)
    assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.uint32), zb[vals])
    for g in np.nonzero(pre["touched"])[0][:200]:
        x0, y0, x1, y1 = pre["rect"][:, g]
        want = {ty_ * tx + tx_ for ty_ in range(y0, y1 + 1) for tx_ in range(x0, x1 + 1)}
        assert set(tiles[vals == g].tolist()) == want


def test_tile_rectangles_cover_every_visible_pixel():
    """Every pixel where the FP64 alpha reaches 1/255 lies in a tile of the
    splat's rectangle (so tiles never change the image)."""
    s = synth.micro_scene(3, 400, 64, 80, log_scale_mean=-3.2)
    front = helpers.front_flags(s)
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    pre = cpu.splat_preprocess(s["cam"], xo, Ao, s["quat"], s["log_s"], s["opac"], front)
    proj = ref64.project(s["cam"], ref64.t64(xo), ref64.t64(Ao), ref64.t64(s["quat"]),
                         ref64.t64(s["log_s"]), ref64.t64(s["opac"]), front)
    H, W = s["height"], s["width"]
    ii, jj = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    checked = 0
    for g in np.nonzero(proj["valid"].numpy())[0]:
        m = proj["mean2d"][:, g].numpy()
        con = proj["conic"][:, g].numpy()
        dx, dy = m[0] - ii, m[1] - jj
        a = s["opac"][g] * np.exp(-0.5 * (con[0] * dx * dx + 2 * con[1] * dx * dy + con[2] * dy * dy))
        hit = np.minimum(a, 0.99) >= (1 / 255) * (1 + 1e-5)
        if not hit.any():
            continue
        checked += 1
        assert pre["touched"][g] > 0
        x0, y0, x1, y1 = pre["rect"][:, g]
        tjj, tii = np.nonzero(hit)
        assert (tii // 16 >= x0).all() and (tii // 16 <= x1).all()
        assert (tjj // 16 >= y0).all() and (tjj // 16 <= y1).all()
    assert checked > 50


def test_fp32_mirror_matches_fp64_composite(scene1):
    s = scene1
    rng = np.random.default_rng(4)
    col = rng.random((3, s["n"])).astype(np.float32)
    f = helpers.oracle_frame_f32(s, col)
    proj = ref64.project(s["cam"], ref64.t64(f["xo"]), ref64.t64(f["Ao"]), ref64.t64(s["quat"]),
                         ref64.t64(s["log_s"]), ref64.t64(s["opac"]), f["front"])
    img64, T64 = ref64.composite(s["cam"], proj, ref64.t64(s["opac"]), ref64.t64(col))
    img64 = img64.numpy().reshape(f["img"].shape)
    ok = f["margin"] > 1e-4
    assert ok.mean() > 0.99
    err = np.abs(img64 - f["img"])[:, ok]
    assert err.max() < 1e-5


def test_needle_splat_takes_the_fp64_path():
    """A long thin splat seen edge-on: the FP32 determinant cancels; the FP64
    path reproduces the FP64 conic to FP32 rounding."""
    ang = math.pi / 4
    q = np.array([[math.cos(ang / 2)], [0.0], [0.0], [math.sin(ang / 2)]], np.float32)
    cam, x, A, _, ls, op, col, front = _gauss_set([[0.0, 0.0, 0.0]], [[3.0, 2e-4, 2e-4]], [0.5],
                                                  [[1, 1, 1]], W=256, H=256, quat=q)
    ls = np.log(np.array([[3.0], [2e-4], [2e-4]])).astype(np.float32)
    pre = cpu.splat_preprocess(cam, x, A, q, ls, op, front)
    assert pre["fp64"][0] == 1
    proj = ref64.project(cam, ref64.t64(x), ref64.t64(A), ref64.t64(q), ref64.t64(ls),
                         ref64.t64(op), front)
    want = proj["conic"][:, 0].numpy()
    got = pre["conic"][:, 0].astype(np.float64)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() / scale < 1e-5


def test_needle_scene_takes_the_fp64_path():
    """The mixed needle scene of the GPU needle tests: every needle, and no
    ordinary splat, takes the FP64 path; the FP64 path's conic agrees with
    the FP64 oracle's to FP32 rounding, where the conic taken in FP32 from
    the same covariance is off by far more (the determinant cancels)."""
    sc = synth.needle_splats(1)
    cam = sc["cam"]
    pre = cpu.splat_preprocess(cam, sc["x"], sc["A"], sc["quat"], sc["log_s"], sc["opac"],
                               sc["front"])
    flagged = np.nonzero(pre["fp64"])[0]
    assert np.array_equal(flagged, np.sort(sc["needle"]))
    proj = ref64.project(cam, ref64.t64(sc["x"]), ref64.t64(sc["A"]), ref64.t64(sc["quat"]),
                         ref64.t64(sc["log_s"]), ref64.t64(sc["opac"]), sc["front"])
    c64 = proj["conic"][:, flagged].numpy()
    scale = np.abs(c64).max(0)
    assert np.max(np.abs(pre["conic"][:, flagged] - c64) / scale) < 1e-6
    sig = proj["sigma"][:, flagged].numpy().astype(np.float32)
    det = sig[0] * sig[2] - sig[1] * sig[1]
    naive = np.stack([sig[2] / det, -sig[1] / det, sig[0] / det])
    assert np.max(np.abs(naive - c64) / scale) > 1e-4
