"""A whole train step (visibility, forward, L1 loss, adjoint) captured in a
HIP graph replays to the eager result, with eager work and synchronisations
between the replays.  The frame bins its splats after the shading on the
captured stream, or on a second stream forked from and joined to it; the
visibility is given to the frame or computed in it.  The forward is
deterministic (images compared bit for bit); the adjoint sums with
floating-point atomics, so gradients are compared to 1e-5 relative."""

import numpy as np
import pytest
import torch

from paper_2407_10707_amd import render, synth
from tests.conftest import scene

pytestmark = pytest.mark.gpu


def _step(R, p, target, own_vis):
    if own_vis:         # the frame computes it, binning on its second stream
        image, _, ctx = R.forward(p)
    else:
        image, _, ctx = R.forward(p, R.visibility())
    loss, dimage = R.loss(image, target)
    grads = R.backward(p, ctx, dimage)
    return image, loss, grads


@pytest.mark.parametrize("own_vis,overlap", [(False, False), (True, True)])
def test_graph_replays_match_eager(own_vis, overlap):
    s = scene(1)
    d = render.upload(s)
    R = render.Renderer(s, d, overlap=overlap)
    p = {k: d[k] for k in render.TRAINABLE}
    target = d["target"]
    img_e, loss_e, g_e = _step(R, p, target, own_vis)
    torch.cuda.synchronize()
    ref_img = img_e.cpu().numpy()
    ref_loss = loss_e.cpu().numpy()
    ref_g = {k: v.cpu().numpy() for k, v in g_e.items()}

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            _step(R, p, target, own_vis)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        img_g, loss_g, g_g = _step(R, p, target, own_vis)
    torch.cuda.synchronize()
    for rep in range(4):
        # eager work between replays, then a replay checked against eager
        _step(R, p, target, own_vis)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(img_g.cpu().numpy(), ref_img), f"replay {rep}: image"
        assert np.allclose(loss_g.cpu().numpy(), ref_loss, rtol=1e-6), f"replay {rep}: loss"
        for k, ref in ref_g.items():
            got = g_g[k].cpu().numpy()
            scale = np.abs(ref).max() + 1e-30
            assert np.abs(got - ref).max() <= 1e-5 * scale, f"replay {rep}: {k}"
