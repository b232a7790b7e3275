"""Pin of the oracle's reference gradients: autograd of the FP64 forward
against central finite differences of the same forward, for every trainable
input of the path (position, normal, rotation, log-scale, opacity, albedo,
roughness, tint and every environment texel)."""

import numpy as np
import pytest
import torch

from paper_2407_10707_amd import synth
from tests import helpers


def _setup(seed=5):
    s = synth.micro_scene(seed, 40, 40, 48, he=4, we=8, hv=4, wv=8, log_scale_mean=-3.0)
    _, _, cnt = helpers.oracle_visibility(s)
    front = helpers.front_flags(s)
    w = torch.tensor(np.random.default_rng(seed).random((3, s["height"] * s["width"])))
    return s, cnt, front, w


def _loss(s, p, cnt, front, w):
    img, _ = helpers.render64(s, p, cnt, front)
    return (img * w).sum()


def test_autograd_matches_central_differences():
    s, cnt, front, w = _setup()
    p = helpers.params64(s, requires_grad=True)
    L = _loss(s, p, cnt, front, w)
    L.backward()
    rng = np.random.default_rng(0)
    steps = dict(pos=1e-5, nrm=1e-5, quat=1e-5, log_s=1e-5, opac=1e-6, albedo=1e-6, rough=1e-6,
                 tint=1e-6, env=1e-6)
    live = np.nonzero(front)[0]
    checked = excluded = 0
    for name in helpers.PARAM_NAMES:
        g = p[name].grad.detach().numpy()
        scale = np.sqrt(np.mean(g ** 2)) + 1e-30
        flat = g.reshape(-1)
        if name == "env":
            cand = np.arange(flat.size)
        else:
            # entries of Gaussians that are drawn
            n = s["n"]
            cols = np.arange(flat.size) % n
            cand = np.nonzero(np.isin(cols, live))[0]
        for idx in rng.choice(cand, size=min(8, len(cand)), replace=False):
            h = steps[name]
            fd = []
            for hh in (h, h / 2):
                vals = []
                for sign in (1, -1):
                    q = {k: v.detach().clone() for k, v in p.items()}
                    q[name].view(-1)[idx] += sign * hh
                    with torch.no_grad():
                        vals.append(_loss(s, q, cnt, front, w).item())
                fd.append((vals[0] - vals[1]) / (2 * hh))
            if abs(fd[0] - fd[1]) > 1e-4 * (abs(fd[0]) + 1e-3 * scale):
                excluded += 1          # a discrete decision flipped inside the stencil
                continue
            checked += 1
            assert abs(flat[idx] - fd[1]) <= 1e-5 * max(abs(fd[1]), scale), (name, idx, flat[idx], fd)
    assert checked >= 60 and excluded <= 8, (checked, excluded)


def test_local_differences_equal_whole_frame_differences():
    """The finite differences of the FP64 chain evaluated locally (only the
    perturbed Gaussian's state and the pixels of its compositing box
    recomputed) equal those of whole-frame renders, on the first 500
    Gaussians of the 1024^2 training workload."""
    from tests.conftest import scene
    s = helpers.subscene(scene(3), np.arange(500))
    _, _, cnt = helpers.oracle_visibility(s)
    front = helpers.front_flags(s)
    w = np.random.default_rng(3).uniform(0.5, 1.5, (3, s["height"], s["width"]))
    F = helpers.LocalFD(s, cnt, front, w)
    wt = torch.as_tensor(w.reshape(3, -1))
    valid = np.nonzero(F.base["proj"]["valid"].numpy())[0]
    g = int(valid[7])
    n = s["n"]
    for name, idx, h in (("pos", 0 * n + g, 1e-4), ("log_s", 2 * n + g, 1e-4),
                         ("albedo", 1 * n + g, 1e-3), ("opac", g, 1e-4)):
        local = F.fd(name, idx, h)
        vals = []
        with torch.no_grad():
            for sgn in (1.0, -1.0):
                q = dict(F.p)
                q[name] = F.p[name].clone()
                q[name].view(-1)[idx] += sgn * h
                img, _ = helpers.render64(s, q, cnt, front)
                vals.append(float((img * wt).sum()))
        full = (vals[0] - vals[1]) / (2 * h)
        assert abs(local - full) <= 1e-9 * max(1.0, abs(full)), (name, local, full)
        assert abs(full) > 1e-6, (name, full)
