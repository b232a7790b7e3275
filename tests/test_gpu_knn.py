"""K nearest canonical vertices and the interpolation equation of Sec. 3.1
on the GPU (through the C ABI) against the oracle.

Bit-exact: neighbour indices and their order ((FP32 squared distance,
index), the oracle's brute force).  Tolerances: weights vs the FP64 weights
of the same squared distances 2e-6 relative (FP32 square root, reciprocal
and normalisation, a few ulp); interpolated attributes vs the FP64 average
1e-6 |ref| + 1e-7; the adjoint's vertex sums vs the FP64 scatter 1e-5
|ref| + 1e-6 (float atomics change the summation order).
"""

import numpy as np
import pytest
import torch

from oracle import cpu, ref64
from paper_2407_10707_amd import rga, synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    rga.lib()
    yield
    torch.cuda.synchronize()


def _check(q, r, k):
    print(f"[knn] n={q.shape[1]} nr={r.shape[1]} k={k}", flush=True)
    index = rga.KnnIndex(dev(r))
    idx, w = rga.knn(index, dev(q), k)
    gi, gw = host(idx), host(w)
    oi, od = cpu.knn(q, r, k)
    assert np.array_equal(gi, oi)
    ow = ref64.knn_weights(od).numpy()
    assert np.allclose(gw, ow, rtol=2e-6, atol=1e-7)
    return gi, gw


@pytest.mark.parametrize("k", [1, 3, 19, 32])
def test_random_points(k):
    rng = np.random.default_rng(100 + k)
    r = rng.random((3, 700)).astype(np.float32)
    q = (rng.random((3, 3000)) * 1.2 - 0.1).astype(np.float32)   # some outside the box
    _check(q, r, k)


def test_lattice_ties_and_queries_on_vertices():
    g = np.arange(9, dtype=np.float32) * 0.25
    r = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).copy()
    rng = np.random.default_rng(7)
    q = (np.round(rng.random((3, 2000)) * 16) / 8).astype(np.float32)  # on and between lattice points
    q[:, :50] = r[:, rng.integers(0, r.shape[1], 50)]
    gi, gw = _check(q, r, 19)
    assert np.all(gw[0, :50] == 1.0) and np.all(gw[1:, :50] == 0.0)


def test_far_queries_and_degenerate_sets():
    rng = np.random.default_rng(9)
    r = rng.random((3, 300)).astype(np.float32)
    q = (rng.normal(size=(3, 500)) * 50).astype(np.float32)          # far outside
    _check(q, r, 5)
    # every reference point the same: one cell, ties broken by index
    r1 = np.ones((3, 40), np.float32)
    _check(rng.random((3, 100)).astype(np.float32), r1, 7)
    # a single reference point; k = nr
    _check(rng.random((3, 64)).astype(np.float32), rng.random((3, 1)).astype(np.float32), 1)
    _check(rng.random((3, 64)).astype(np.float32), r[:, :20].copy(), 20)


def test_avatar_gaussians_and_vertex_neighbourhood():
    s = synth.make_scene(2)
    verts, pos = s["verts"], s["pos"]
    index = rga.KnnIndex(dev(verts))
    # K_g = 3 for all 100k Gaussians; the oracle on a seeded sample
    idx, w = rga.knn(index, dev(pos), 3)
    gi, gw = host(idx), host(w)
    sel = np.random.default_rng(1).choice(pos.shape[1], 4000, replace=False)
    oi, od = cpu.knn(pos[:, sel].copy(), verts, 3)
    assert np.array_equal(gi[:, sel], oi)
    assert np.allclose(gw[:, sel], ref64.knn_weights(od).numpy(), rtol=2e-6, atol=1e-7)
    # K_v = 19 vertex neighbourhood, all vertices
    vi, vw = rga.knn(index, dev(verts), 19)
    oi, _ = cpu.knn(verts, verts, 19)
    assert np.array_equal(host(vi), oi)
    # each vertex is at distance 0 from its nearest (itself, or a coincident
    # seam vertex of lower index) and so takes that vertex alone
    assert np.all(host(vw)[0] == 1.0)


def test_interpolation_and_adjoint():
    rng = np.random.default_rng(21)
    r = rng.random((3, 900)).astype(np.float32)
    q = rng.random((3, 5000)).astype(np.float32)
    attr = rng.normal(size=(24, 900)).astype(np.float32)
    index = rga.KnnIndex(dev(r))
    for k in (3, 19):
        idx, w = rga.knn(index, dev(q), k)
        out = host(rga.knn_interpolate(idx, w, dev(attr)))
        ref = ref64.interpolate(host(idx), host(w).astype(np.float64), attr).numpy()
        assert np.allclose(out, ref, rtol=1e-6, atol=1e-7)
        dout = rng.normal(size=(24, 5000)).astype(np.float32)
        da = host(rga.knn_interpolate_backward(idx, w, dev(dout), 900))
        gi, gw = host(idx), host(w).astype(np.float64)
        exp = np.zeros((24, 900))
        for t in range(k):
            for c in range(24):
                np.add.at(exp[c], gi[t], gw[t] * dout[c])
        assert np.allclose(da, exp, rtol=1e-5, atol=1e-6)
