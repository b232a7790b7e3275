"""The Adam step on the GPU through the C ABI against the oracle's FP64
step: parameters within 1e-6 of their magnitude plus 1e-5 of the learning
rate, moments within 2e-6 relative (FP32 products and square root)."""

import numpy as np
import pytest
import torch

from oracle import ref64
from paper_2407_10707_amd import rga

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("count", [1, 1000003])
def test_adam_steps(count):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print(f"[adam] count={count}", flush=True)
    rng = np.random.default_rng(count)
    p = rng.normal(size=count).astype(np.float32)
    m = np.zeros(count, np.float32)
    v = np.zeros(count, np.float32)
    P, M, V = (torch.tensor(a).cuda() for a in (p, m, v))
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 6):
        g = rng.normal(size=count).astype(np.float32)
        rga.adam_step(P, torch.tensor(g).cuda(), M, V, 1e-2, t)
        # the oracle takes the same hyper-parameters the kernel receives (FP32)
        f = lambda a: float(np.float32(a))
        pr, mr, vr = ref64.adam_step(pr, g.astype(np.float64), mr, vr, f(1e-2), f(0.9), f(0.999),
                                     f(1e-8), t)
    torch.cuda.synchronize()
    gp, gm, gv = (a.cpu().numpy().astype(np.float64) for a in (P, M, V))
    assert np.all(np.abs(gp - pr) <= 1e-6 * np.abs(pr) + 1e-5 * 1e-2)
    assert np.all(np.abs(gm - mr) <= 2e-6 * np.abs(mr) + 1e-7)
    assert np.all(np.abs(gv - vr) <= 2e-6 * np.abs(vr) + 1e-9)
