"""Storage order of the Gaussians (they are a set; Sec. 3.1 has each one read
the visibility counts of its nearest mesh vertices): vertex_order is a
stable sort by nearest vertex, bit-exact against numpy's stable argsort, on
one and several radix passes, ragged and empty inputs; gather_columns is
bit-exact against numpy indexing; and shading with its adjoint gives the
oracle's results in the grouped layout on launches whose walk is split over
the eight XCDs (even and ragged eighths) and on one that is not."""

import numpy as np
import pytest
import torch

from oracle import cpu, ref64
from paper_2407_10707_amd import render, rga, synth
from tests import helpers
from tests.conftest import scene

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _want(vidx0, nv):
    return np.argsort(np.clip(vidx0, 0, nv - 1), kind="stable").astype(np.int32)


def test_vertex_order_avatar_workload():
    s = scene(2)
    print(f"[layout] avatar n={s['n']} nv={s['verts'].shape[1]}", flush=True)
    got = host(rga.vertex_order(dev(s["vidx"]), s["verts"].shape[1]))
    assert np.array_equal(got, _want(s["vidx"][0], s["verts"].shape[1]))


# (n, nv): one pass (nv <= 2048), two (nv <= 2^22) and three; ragged blocks;
# every Gaussian on one vertex; ids out of range (clamped)
@pytest.mark.parametrize("n,nv,kind", [(1, 1, "random"), (511, 7, "random"),
                                       (513, 2048, "random"), (4099, 2049, "random"),
                                       (70001, 100000, "random"), (3000, 5_000_000, "random"),
                                       (5000, 10, "one"), (2000, 50, "outside")])
def test_vertex_order_is_the_stable_sort(n, nv, kind):
    print(f"[layout] vertex_order n={n} nv={nv} {kind}", flush=True)
    rng = np.random.default_rng(n + nv)
    v = rng.integers(0, nv, (3, n)).astype(np.int32)
    if kind == "one":
        v[0] = 3
    elif kind == "outside":
        v[0] = rng.integers(-20, nv + 20, n)
    got = host(rga.vertex_order(dev(v), nv))
    assert np.array_equal(got, _want(v[0], nv))


def test_vertex_order_empty_and_errors():
    assert rga.vertex_order(dev(np.zeros((3, 0), np.int32)), 5).numel() == 0
    L = rga.lib()
    assert L.vertex_order(None, 10, None, 0, None, None, 0) != 0
    assert "nv >= 1" in rga.last_error()
    assert L.gather_columns(None, -1, 4, None, None, None) != 0


@pytest.mark.parametrize("shape", [(5,), (3, 1000), (4, 777)])
def test_gather_columns_bit_exact(shape):
    rng = np.random.default_rng(len(shape) * 100 + shape[-1])
    n = shape[-1]
    order = rng.permutation(n).astype(np.int32)
    a = rng.standard_normal(shape).astype(np.float32)
    b = rng.integers(-1000, 1000, shape).astype(np.int32)
    assert np.array_equal(host(rga.gather_columns(dev(a), dev(order))).view(np.uint32),
                          a[..., order].view(np.uint32))
    assert np.array_equal(host(rga.gather_columns(dev(b), dev(order))), b[..., order])


def test_layout_by_vertex_matches_host_permutation():
    s = synth.micro_scene(9, 900, 32, 32)
    d, order = render.layout_by_vertex(render.upload(s))
    o = host(order)
    assert np.array_equal(o, _want(s["vidx"][0], s["verts"].shape[1]))
    sp = render.scene_in_order(s, order)
    for k in render.PER_GAUSSIAN:
        assert np.array_equal(host(d[k]), np.asarray(sp[k], dtype=host(d[k]).dtype)), k
    assert np.all(np.diff(host(d["vidx"])[0]) >= 0)


# n = 300: 38 workgroups (the plain walk); 703 and 704: 88 workgroups, the
# walk split in eighths, ragged and even
@pytest.mark.parametrize("n", [300, 703, 704])
def test_shading_in_grouped_layout(n):
    print(f"[layout shading] n={n}", flush=True)
    s0 = synth.micro_scene(41, n, 40, 48, he=16, we=32, hv=16, wv=16)
    d, order = render.layout_by_vertex(render.upload(s0))
    s = render.scene_in_order(s0, order)
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    _, _, cnt = helpers.oracle_visibility(s)
    campos = s["cam"].centre.astype(np.float32)
    c64 = campos.astype(np.float64)
    front = cpu.front_f32(xo, no, campos)
    args = (dev(xo), dev(no), d["albedo"], d["rough"], d["tint"], d["vidx"], d["vw"], dev(cnt),
            s["kv"], s["he"], s["we"], s["hv"], s["wv"], d["env"])
    col, fr = rga.shade_gaussians(*args, campos)
    assert np.array_equal(host(fr), front)
    ecol, _ = ref64.shade(ref64.t64(xo), ref64.t64(no), s["albedo"], s["rough"], s["tint"],
                          s["vidx"], s["vw"], cnt, s["kv"], s["he"], s["we"], s["hv"], s["wv"],
                          s["env"], c64, front)
    ecol = ecol.numpy()
    err = np.abs(host(col) - ecol)
    assert np.all(err <= 1e-5 * np.abs(ecol) + 1e-7)
    w = np.random.default_rng(3).uniform(-1.0, 1.0, (3, n)).astype(np.float32)
    w[np.abs(ecol - 0.04045) <= 2e-5 * 0.04045] = 0.0   # the transfer curve's breakpoint
    g = rga.shade_gaussians_backward(*args, campos, col, fr, dev(w))
    leaves = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True)
              for k, v in (("x", xo), ("n", no), ("albedo", s["albedo"]), ("rough", s["rough"]),
                           ("tint", s["tint"]), ("env", s["env"]))}
    e2, _ = ref64.shade(leaves["x"], leaves["n"], leaves["albedo"], leaves["rough"],
                        leaves["tint"], s["vidx"], s["vw"], cnt, s["kv"], s["he"], s["we"],
                        s["hv"], s["wv"], leaves["env"], c64, front)
    (e2 * torch.tensor(w.astype(np.float64))).sum().backward()
    for gk, lk in (("dx", "x"), ("dn", "n"), ("dalbedo", "albedo"), ("drough", "rough"),
                   ("dtint", "tint"), ("denv", "env")):
        helpers.check_grad(lk, host(g[gk]), leaves[lk].grad.numpy())
