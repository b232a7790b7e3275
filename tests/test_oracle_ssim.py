"""Pins of the image loss of the FP64 oracle (Sec. 3.3, image-loss
equation; SSIM as Wang et al.): windowed sums against loops, the closed form
for constant images, identity and symmetry, finite differences of the
gradient."""

import math

import numpy as np
import torch

from oracle import ref64


def test_window_is_a_normalised_gaussian():
    g = ref64.ssim_window().numpy()
    assert g.shape == (11,) and abs(g.sum() - 1) < 1e-15
    assert np.allclose(g, g[::-1])
    assert abs(g[6] / g[5] - math.exp(-1 / (2 * 1.5 ** 2))) < 1e-14


def test_windowed_sums_match_loops_with_zero_padding():
    rng = np.random.default_rng(1)
    x = rng.random((1, 7, 9))
    y = rng.random((1, 7, 9))
    g = ref64.ssim_window().numpy()
    S = ref64.ssim_map(x, y).numpy()
    for (r, c) in [(0, 0), (3, 4), (6, 8), (2, 7)]:
        m = {k: 0.0 for k in ("x", "y", "xx", "yy", "xy")}
        for i in range(11):
            for j in range(11):
                rr, cc = r + i - 5, c + j - 5
                if 0 <= rr < 7 and 0 <= cc < 9:
                    w = g[i] * g[j]
                    a, b = x[0, rr, cc], y[0, rr, cc]
                    m["x"] += w * a
                    m["y"] += w * b
                    m["xx"] += w * a * a
                    m["yy"] += w * b * b
                    m["xy"] += w * a * b
        sx = m["xx"] - m["x"] ** 2
        sy = m["yy"] - m["y"] ** 2
        sxy = m["xy"] - m["x"] * m["y"]
        c1, c2 = 0.01 ** 2, 0.03 ** 2
        want = ((2 * m["x"] * m["y"] + c1) * (2 * sxy + c2)) / \
            ((m["x"] ** 2 + m["y"] ** 2 + c1) * (sx + sy + c2))
        assert abs(S[0, r, c] - want) < 1e-12


def test_constant_images_closed_form_and_identity():
    a, b = 0.3, 0.7
    x = np.full((2, 20, 24), a)
    y = np.full((2, 20, 24), b)
    S = ref64.ssim_map(x, y).numpy()
    c1 = 0.01 ** 2
    inner = S[:, 5:-5, 5:-5]
    assert np.allclose(inner, (2 * a * b + c1) / (a * a + b * b + c1), atol=1e-12)
    z = np.random.default_rng(2).random((3, 16, 16))
    assert np.allclose(ref64.ssim_map(z, z).numpy(), 1.0, atol=1e-12)
    assert abs(float(ref64.image_loss(z, z))) < 1e-12
    w = np.random.default_rng(3).random((3, 16, 16))
    assert np.allclose(ref64.ssim_map(z, w).numpy(), ref64.ssim_map(w, z).numpy(), atol=1e-14)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    x = torch.tensor(rng.random((2, 9, 13)), requires_grad=True)
    y = torch.tensor(rng.random((2, 9, 13)))
    (g,) = torch.autograd.grad(ref64.image_loss(x, y), (x,))
    x = x.detach()
    eps = 1e-6
    for idx in [(0, 0, 0), (1, 4, 6), (0, 8, 12), (1, 2, 11), (0, 5, 1)]:
        e = torch.zeros_like(x)
        e[idx] = eps
        fd = (ref64.image_loss(x + e, y) - ref64.image_loss(x - e, y)) / (2 * eps)
        assert abs(float(fd) - float(g[idx])) <= 1e-7 + 1e-6 * abs(float(fd))


def test_l1_term_against_loops_and_closed_forms():
    """The L1 term of the image loss: the mean over every channel and pixel
    of |x - y| (checked against a loop), |c| for a constant offset c, and its
    gradient sign(x - y) / count with sign(0) = 0 at exact ties."""
    rng = np.random.default_rng(4)
    x = rng.random((3, 5, 7))
    y = rng.random((3, 5, 7))
    y[0, 1, 2] = x[0, 1, 2]                 # exact ties
    y[2, 4, 6] = x[2, 4, 6]
    tot = 0.0
    for c in range(3):
        for r in range(5):
            for k in range(7):
                tot += abs(x[c, r, k] - y[c, r, k])
    assert abs(ref64.l1_loss(torch.tensor(x), y).item() - tot / x.size) < 1e-15
    assert abs(ref64.l1_loss(torch.tensor(x), x + 0.25).item() - 0.25) < 1e-15
    xt = torch.tensor(x, requires_grad=True)
    ref64.l1_loss(xt, y).backward()
    want = np.sign(x - y) / x.size
    assert np.array_equal(xt.grad.numpy(), want)
    assert xt.grad[0, 1, 2].item() == 0.0 and xt.grad[2, 4, 6].item() == 0.0
