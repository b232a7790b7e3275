"""The work counts behind bench.py's roofline entries, on the CPU: the
(pixel, splat) pairs the compositing walks and applies (blend_pairs, plain
PyTorch) against a per-pixel walk written out here and the FP32 mirror's
per-pixel applied counts, on two small scenes (Sec. 3.1, last paragraph:
3DGS compositing with alpha >= 1/255, stop before T < 1e-4)."""

import numpy as np
import pytest
import torch

import bench
from oracle import cpu
from paper_2407_10707_amd import synth
from tests.conftest import scene


def _walk_counts(cam, ranges, vals, pre, opac):
    W, H = cam.width, cam.height
    tx = (W + 15) // 16
    m, c = pre["mean2d"].astype(np.float64), pre["conic"].astype(np.float64)
    o = np.asarray(opac, np.float64)
    walked = applied = 0
    for t in range(ranges.shape[0]):
        a, b = ranges[t]
        for yy in range(16):
            for xx in range(16):
                px, py = (t % tx) * 16 + xx, (t // tx) * 16 + yy
                if px >= W or py >= H:
                    continue
                T = 1.0
                for e in range(a, b):
                    g = vals[e]
                    walked += 1
                    dx, dy = m[0, g] - (px + 0.5), m[1, g] - (py + 0.5)
                    pw = -0.5 * (c[0, g] * dx * dx + c[2, g] * dy * dy) - c[1, g] * dx * dy
                    al = min(0.99, o[g] * np.exp(pw))
                    if pw > 0 or al < 1 / 255:
                        continue
                    if T * (1 - al) < 1e-4:
                        break
                    T *= 1 - al
                    applied += 1
    return walked, applied


@pytest.mark.parametrize("name", ["cfg1", "micro"])
def test_blend_pair_counts(name):
    s = scene(1) if name == "cfg1" else synth.micro_scene(5, 333, 70, 45)
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    cam = s["cam"]
    front = cpu.front_f32(xo, no, cam.centre.astype(np.float32))
    pre = cpu.splat_preprocess(cam, xo, Ao, s["quat"], s["log_s"], s["opac"], front)
    _, vals, ranges = cpu.splat_bin(cam, pre)
    got = bench.blend_pairs(torch.tensor(pre["mean2d"]), torch.tensor(pre["conic"]),
                            torch.tensor(np.asarray(s["opac"], np.float32)), torch.tensor(vals),
                            torch.tensor(ranges), cam.width, cam.height)
    walked, applied = _walk_counts(cam, ranges, vals, pre, s["opac"])
    mirror = cpu.composite_tiles(cam, ranges, vals, pre, s["opac"],
                                 np.ones((3, s["n"]), np.float32), with_applied=True)[-1]
    assert got["walked"] == walked
    assert got["applied"] == applied == int(mirror.sum())
    assert bench.blend_bwd_flops(walked, applied) == 15.0 * walked + 59.0 * applied
