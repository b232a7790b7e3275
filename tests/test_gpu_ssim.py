"""Image loss of the training section ((1 - lambda) L1 + lambda D-SSIM,
Sec. 3.3) on the GPU through the C ABI against the FP64 oracle.

Tolerances, from the arithmetic: the GPU forms sigma^2 = E[x^2] - mu^2 and
sigma_xy in FP32, so an absolute error of a few 2^-24 in the windowed sums
(values in [0, 1]) is divided by sigma_x^2 + sigma_y^2 + C2 >= C2 = 9e-4:
up to ~1e-4 relative in flat regions, ~1e-6 in textured ones.  The loss
(a mean over all pixels) is compared to 2e-6 absolute; the gradient per
pixel to 2e-4 of the largest gradient magnitude (flat, smooth images) and
2e-5 (noise images).
"""

import numpy as np
import pytest
import torch

from oracle import ref64
from paper_2407_10707_amd import rga

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    rga.lib()
    yield
    torch.cuda.synchronize()


def _smooth(rng, shape):
    """Low-frequency images in [0, 1] (sums of a few random sinusoids)."""
    C, H, W = shape
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    out = np.zeros(shape)
    for c in range(C):
        for _ in range(4):
            fy, fx, ph = rng.uniform(0, 0.08), rng.uniform(0, 0.08), rng.uniform(0, 6.3)
            out[c] += np.sin(fy * yy + fx * xx + ph)
    return (out - out.min()) / (out.max() - out.min())


def _check(x, y, lam, gtol):
    C, H, W = x.shape
    print(f"[ssim] C={C} H={H} W={W} lambda={lam}", flush=True)
    loss, d = rga.image_loss(torch.tensor(x, dtype=torch.float32).cuda(),
                             torch.tensor(y, dtype=torch.float32).cuda(), lam)
    torch.cuda.synchronize()
    xt = torch.tensor(x.astype(np.float32).astype(np.float64), requires_grad=True)
    yt = torch.tensor(y.astype(np.float32).astype(np.float64))
    ref = ref64.image_loss(xt, yt, lam)
    (g,) = torch.autograd.grad(ref, (xt,))
    dl = abs(float(loss.cpu()) - float(ref.detach()))
    err = np.abs(d.cpu().numpy() - g.numpy()).max() / np.abs(g.numpy()).max()
    print(f"[ssim]   loss err {dl:.3e}  grad err / max {err:.3e}", flush=True)
    assert dl <= 2e-6
    assert err <= gtol


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 37, 53), (3, 64, 64)])
def test_noise_images(shape):
    rng = np.random.default_rng(sum(shape))
    _check(rng.random(shape), rng.random(shape), 0.2, 2e-5)


def test_smooth_images_full_size():
    rng = np.random.default_rng(5)
    x = _smooth(rng, (3, 512, 512))
    y = np.clip(x + 0.05 * rng.standard_normal(x.shape), 0, 1)
    _check(x, y, 0.2, 2e-4)


def test_lambda_limits_and_identical_images():
    rng = np.random.default_rng(6)
    x, y = rng.random((2, 40, 33)), rng.random((2, 40, 33))
    _check(x, y, 0.0, 2e-5)
    _check(x, y, 1.0, 2e-5)
    loss, d = rga.image_loss(torch.tensor(x, dtype=torch.float32).cuda(),
                             torch.tensor(x, dtype=torch.float32).cuda(), 0.2)
    assert abs(float(loss.cpu())) < 1e-6
    assert float(d.abs().max().cpu()) < 1e-6
    loss2, none = rga.image_loss(torch.tensor(x, dtype=torch.float32).cuda(),
                                 torch.tensor(y, dtype=torch.float32).cuda(), 0.2, want_grad=False)
    assert none is None
