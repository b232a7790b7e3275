"""Pins of the training regularisers of the FP64 oracle (Sec. 3.3): loops
over tiny inputs, closed forms (constant materials, Gaussians on their
vertices, scales below the threshold) and finite differences."""

import math

import numpy as np
import torch

from oracle import ref64


def _tiny(seed, nv=6, n=5, kv=3, kg=2):
    rng = np.random.default_rng(seed)
    return dict(mat=rng.random((5, nv)), knn_v=rng.integers(0, nv, (nv, kv)),
                xg=rng.normal(size=(3, n)), verts=rng.normal(size=(3, nv)),
                vidx=rng.integers(0, nv, (kg, n)), disp=rng.normal(size=(3, nv)) * 0.01,
                log_s=rng.normal(-5.3, 0.5, (3, n)))


def test_terms_match_loops():
    t = _tiny(1)
    sm, md, dl, sc, tot = (float(v) for v in ref64.regularisers(**t))
    nv, n = t["mat"].shape[1], t["xg"].shape[1]
    want_sm = sum(abs(t["mat"][a, i] - t["mat"][a, k]) for i in range(nv) for k in t["knn_v"][i]
                  for a in range(5))
    want_md = sum(math.dist(t["xg"][:, g], t["verts"][:, k]) for g in range(n)
                  for k in t["vidx"][:, g])
    want_dl = sum(math.hypot(*t["disp"][:, i]) for i in range(nv))
    want_sc = sum(max(0.0, math.exp(v) - 0.005) for v in t["log_s"].ravel())
    assert abs(sm - want_sm) < 1e-12 and abs(md - want_md) < 1e-12
    assert abs(dl - want_dl) < 1e-14 and abs(sc - want_sc) < 1e-14
    assert abs(tot - (0.002 * want_sm + 0.1 * want_md + 0.02 * want_dl + 10 * want_sc)) < 1e-12


def test_closed_forms():
    t = _tiny(2)
    t["mat"] = np.ones_like(t["mat"]) * 0.4
    t["xg"] = t["verts"][:, t["vidx"][0]]
    t["vidx"] = t["vidx"][:1]
    t["log_s"] = np.full_like(t["log_s"], math.log(0.004))
    t["disp"] = np.zeros_like(t["disp"])
    sm, md, dl, sc, tot = (float(v) for v in ref64.regularisers(**t))
    assert sm == 0 and md == 0 and dl == 0 and sc == 0 and tot == 0


def test_gradients_match_central_differences():
    t = _tiny(3)
    names = ["mat", "xg", "disp", "log_s"]
    ts = {k: torch.tensor(t[k], requires_grad=(k in names)) if k in names else t[k] for k in t}
    tot = ref64.regularisers(**ts)[4]
    grads = torch.autograd.grad(tot, [ts[k] for k in names])
    rng = np.random.default_rng(4)
    eps = 1e-7
    for name, g in zip(names, grads):
        base = t[name]
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in base.shape)
            hi, lo = dict(t), dict(t)
            hi[name] = base.copy()
            lo[name] = base.copy()
            hi[name][idx] += eps
            lo[name][idx] -= eps
            fd = (float(ref64.regularisers(**hi)[4]) - float(ref64.regularisers(**lo)[4])) / (2 * eps)
            assert abs(fd - float(g[idx])) <= 1e-6 * max(1.0, abs(fd)), (name, idx)
