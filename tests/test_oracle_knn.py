"""Pins of the K-nearest-vertex oracle and the interpolation equation of
Sec. 3.1 (CPU): the FP32 brute force against a k-d tree in FP64, exact tie
order on lattice points against plain Python, and the limits of the
inverse-distance average."""

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import cpu, ref64


def _pts(rng, n):
    return rng.random((3, n)).astype(np.float32)


@pytest.mark.parametrize("k", [1, 3, 19])
def test_knn_matches_kdtree(k):
    rng = np.random.default_rng(11)
    q, r = _pts(rng, 400), _pts(rng, 300)
    idx, d2 = cpu.knn(q, r, k)
    dt, it = cKDTree(r.T.astype(np.float64)).query(q.T.astype(np.float64), k=k)
    dt = dt.reshape(len(q.T), k).T
    it = it.reshape(len(q.T), k).T
    assert np.allclose(np.sqrt(d2.astype(np.float64)), dt, rtol=2e-6, atol=1e-7)
    # indices agree wherever the k-d tree's distances are well separated
    gap = np.full(dt.shape, np.inf)
    gap[1:] = np.minimum(gap[1:], dt[1:] - dt[:-1])
    gap[:-1] = np.minimum(gap[:-1], dt[1:] - dt[:-1])
    sep = gap > 1e-5
    assert sep.mean() > 0.95
    assert np.array_equal(idx[sep], it[sep])
    assert np.all(np.diff(d2, axis=0) >= 0)


def test_knn_ties_follow_index_order():
    # integer lattice: squared distances are exact, many are equal
    g = np.arange(4, dtype=np.float32)
    r = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    q = np.array([[1.5, 0.0, 2.0, 3.0], [1.5, 0.0, 1.0, 3.5], [1.5, 0.0, 0.5, 3.0]], np.float32)
    k = 12
    idx, d2 = cpu.knn(q, r, k)
    for i in range(q.shape[1]):
        ref = sorted(((float(((r[:, j] - q[:, i]).astype(np.float64) ** 2).sum()), j)
                      for j in range(r.shape[1])))[:k]
        assert [j for _, j in ref] == idx[:, i].tolist()
        assert np.array_equal(d2[:, i].astype(np.float64), [d for d, _ in ref])


def test_knn_all_points_is_a_sorted_permutation():
    rng = np.random.default_rng(3)
    q, r = _pts(rng, 20), _pts(rng, 17)
    idx, d2 = cpu.knn(q, r, 17)
    for i in range(20):
        assert sorted(idx[:, i].tolist()) == list(range(17))
        keys = list(zip(d2[:, i].tolist(), idx[:, i].tolist()))
        assert keys == sorted(keys)


def test_weights_and_interpolation_limits():
    rng = np.random.default_rng(5)
    r = _pts(rng, 50)
    q = _pts(rng, 30)
    q[:, 7] = r[:, 13]                       # a query on a vertex
    idx, d2 = cpu.knn(q, r, 3)
    w = ref64.knn_weights(d2).numpy()
    assert np.allclose(w.sum(axis=0), 1.0, atol=1e-15)
    assert idx[0, 7] == 13 and d2[0, 7] == 0.0 and w[0, 7] == 1.0 and np.all(w[1:, 7] == 0)
    # weights decrease with distance (u = 1/d)
    assert np.all(np.diff(w[:, np.arange(30) != 7], axis=0) <= 0)
    # a constant attribute interpolates to itself; the vertex query to its vertex
    attr = np.vstack([np.full(50, 0.7), rng.random(50)])
    out = ref64.interpolate(idx, w, attr).numpy()
    assert np.allclose(out[0], 0.7, rtol=1e-15)
    assert out[1, 7] == attr[1, 13]
    # closed form for one query: the inverse-distance average written out
    d = np.sqrt(d2[:, 3].astype(np.float64))
    assert np.isclose(out[1, 3], (attr[1, idx[:, 3]] / d).sum() / (1.0 / d).sum(), rtol=1e-14)
