"""Pins of the displacement network of the FP64 oracle (Sec. 3.1 attributes,
Sec. 3.5 implementation details): brute force on tiny layers, finite
differences of its gradients, identities of the Fourier features and of a
pose that enters as a bias."""

import math

import numpy as np
import torch

from oracle import ref64
from paper_2407_10707_amd import synth


def _tiny(seed):
    rng = np.random.default_rng(seed)
    shapes = [(5, 2 * 2 + 3), (4, 5), (3, 4)]
    layers = [(torch.tensor(rng.normal(size=(o, i))), torch.tensor(rng.normal(size=o)))
              for o, i in shapes]
    x = rng.normal(size=(3, 6))
    freqs = rng.normal(size=(2, 3))
    theta = rng.normal(size=3)
    return x, freqs, theta, layers


def test_tiny_network_matches_neuron_by_neuron_loops():
    x, freqs, theta, layers = _tiny(1)
    _, out = ref64.mlp_layers(x, freqs, theta, layers)
    for v in range(x.shape[1]):
        feats = []
        for j in range(freqs.shape[0]):
            a = sum(freqs[j][c] * x[c][v] for c in range(3))
            feats.append(math.sin(2 * math.pi * a))
        for j in range(freqs.shape[0]):
            a = sum(freqs[j][c] * x[c][v] for c in range(3))
            feats.append(math.cos(2 * math.pi * a))
        h = feats + list(theta)
        for li, (W, b) in enumerate(layers):
            nxt = []
            for o in range(W.shape[0]):
                s = float(b[o])
                for i in range(W.shape[1]):
                    s += float(W[o][i]) * h[i]
                nxt.append(max(s, 0.0) if li + 1 < len(layers) else s)
            h = nxt
        assert np.allclose(out[:, v].numpy(), h, rtol=1e-12, atol=1e-12)


def test_gradients_match_central_differences():
    inp = synth.mlp_inputs(3, freqs=4, pose=5, width=8)
    shapes = [(8, 2 * 4 + 5), (8, 8), (8, 8), (8, 8), (3, 8)]
    rng = np.random.default_rng(4)
    x = torch.tensor(rng.normal(size=(3, 7)))
    c = torch.tensor(rng.normal(size=(3, 7)))
    p = torch.tensor(inp["params"].astype(np.float64), requires_grad=True)
    th = torch.tensor(inp["thetas"][0].astype(np.float64), requires_grad=True)

    def loss(pp, tt):
        return (ref64.mlp_layers(x, inp["freqs"], tt, ref64.mlp_unpack(pp, shapes))[1] * c).sum()

    gp, gt = torch.autograd.grad(loss(p, th), (p, th))
    p, th = p.detach(), th.detach()
    eps = 1e-6
    for i in rng.choice(p.numel(), 40, replace=False):
        e = torch.zeros_like(p)
        e[i] = eps
        fd = (loss(p + e, th) - loss(p - e, th)) / (2 * eps)
        assert abs(float(fd) - float(gp[i])) <= 1e-6 * max(1.0, abs(float(fd)))
    for i in range(th.numel()):
        e = torch.zeros_like(th)
        e[i] = eps
        fd = (loss(p, th + e) - loss(p, th - e)) / (2 * eps)
        assert abs(float(fd) - float(gt[i])) <= 1e-6 * max(1.0, abs(float(fd)))


def test_fourier_features_identities():
    rng = np.random.default_rng(5)
    B = rng.normal(size=(16, 3))
    x = rng.normal(size=(3, 9))
    g = ref64.rff(x, B).numpy()
    assert np.allclose(g[:16] ** 2 + g[16:] ** 2, 1.0, atol=1e-14)
    g0 = ref64.rff(np.zeros((3, 1)), B).numpy()[:, 0]
    assert np.array_equal(g0, np.concatenate([np.zeros(16), np.ones(16)]))
    # integer frequencies: a shift by a unit vector changes no feature
    Bi = rng.integers(-3, 4, size=(16, 3)).astype(np.float64)
    xs = x + np.array([[1.0], [0.0], [0.0]])
    assert np.allclose(ref64.rff(x, Bi).numpy(), ref64.rff(xs, Bi).numpy(), atol=1e-12)


def test_pose_enters_as_a_shared_bias():
    inp = synth.mlp_inputs(6)
    layers = ref64.mlp_unpack(inp["params"].astype(np.float64))
    x = np.random.default_rng(7).normal(size=(3, 5))
    M = layers[0][0][:, 128:]                       # the pose columns of W_1 [256, 72]
    # remove one direction from their row space; a pose change along it then
    # changes nothing
    _, _, vh = torch.linalg.svd(M)
    null = vh[-1]
    Mc = M - (M @ null)[:, None] * null[None, :]
    layers_c = [(torch.cat([layers[0][0][:, :128], Mc], dim=1), layers[0][1])] + layers[1:]
    th = torch.tensor(inp["thetas"][0].astype(np.float64))
    a = ref64.mlp_layers(x, inp["freqs"], th, layers_c)[1]
    b = ref64.mlp_layers(x, inp["freqs"], th + 0.7 * null, layers_c)[1]
    assert torch.allclose(a, b, atol=1e-12)
    # and the pose's effect is the same for every vertex: z_1(theta) - z_1(0)
    z1 = ref64.mlp_layers(x, inp["freqs"], th, layers)[0][0]
    z0 = ref64.mlp_layers(x, inp["freqs"], torch.zeros(72, dtype=torch.float64), layers)[0][0]
    d = z1 - z0
    assert torch.allclose(d, d[:, :1].expand_as(d), atol=1e-12)


def test_mean_displacement_over_poses():
    inp = synth.mlp_inputs(8, n_pose=3)
    x = np.random.default_rng(9).normal(size=(3, 4))
    m = ref64.mean_displacement(x, inp["freqs"], inp["thetas"], inp["params"])
    each = [ref64.displacement(x, inp["freqs"], t, inp["params"]) for t in inp["thetas"]]
    assert torch.allclose(m, (each[0] + each[1] + each[2]) / 3, atol=1e-14)
    assert ref64.mlp_param_count() == inp["params"].size
