"""The L1 term of the image loss (Sec. 3.3, image-loss equation) on the GPU,
through the C ABI, against the FP64 oracle: the loss (a fixed-order FP32
reduction: within 4e-6 relative) and dL/dimage element by element, bit for
bit (sign(image - target) / count rounded to FP32, sign(0) = 0)."""

import numpy as np
import pytest
import torch

from oracle import ref64
from paper_2407_10707_amd import rga

pytestmark = pytest.mark.gpu


def _case(shape, seed, ties=0):
    rng = np.random.default_rng([31, seed])
    x = rng.random(shape).astype(np.float32)
    y = rng.random(shape).astype(np.float32)
    if ties:
        flat = rng.choice(x.size, ties, replace=False)
        y.reshape(-1)[flat] = x.reshape(-1)[flat]
    return x, y


@pytest.mark.parametrize("shape,ties", [((3, 512, 512), 0), ((3, 37, 53), 400), ((1, 1, 1), 0),
                                        ((3, 1024, 1024), 5000), ((1, 1, 7), 7)])
def test_l1_loss_matches_fp64(shape, ties):
    print(f"[l1] shape {shape} ties {ties}", flush=True)
    x, y = _case(shape, sum(shape), ties)
    loss, dimg = rga.l1_loss(torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda())
    torch.cuda.synchronize()
    xt = torch.tensor(x.astype(np.float64), requires_grad=True)
    ref = ref64.l1_loss(xt, y)
    ref.backward()
    got = float(loss.cpu()[0])
    rel = abs(got - ref.item()) / max(ref.item(), 1e-300)
    print(f"  loss rel err {rel:.2e}", flush=True)
    assert rel <= 4e-6 or (ref.item() == 0.0 and got == 0.0)
    want = xt.grad.numpy().astype(np.float32)
    assert np.array_equal(dimg.cpu().numpy(), want)
    if ties:
        tie = (x == y)
        assert tie.sum() >= ties and np.all(dimg.cpu().numpy()[tie] == 0.0)


def test_l1_loss_without_gradient_and_errors():
    x, y = _case((3, 40, 24), 3)
    loss, dimg = rga.l1_loss(torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda(),
                             want_grad=False)
    assert dimg is None
    ref = float(np.abs(x.astype(np.float64) - y).mean())
    assert abs(float(loss.cpu()[0]) - ref) <= 4e-6 * ref
    L = rga.lib()
    assert L.l1_loss(None, 0, None, None, None, None, None, 0) == -1
    xd = torch.as_tensor(x).cuda()
    loss = torch.empty(1, device="cuda")
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    rc = L.l1_loss(None, xd.numel(), rga._p(xd), rga._p(xd), rga._p(loss), None, rga._p(small), 8)
    assert rc == -2 and "workspace" in rga.last_error()
