"""Pins of the oracle's skinning and visibility (Sec. 3.1 deformation,
Sec. 3.2 visibility) against closed forms, special cases, invariants and brute
force -- nothing here compares the oracle with itself."""

import math

import numpy as np
import torch
import pytest

from oracle import cpu, ref64
from paper_2407_10707_amd import synth
from tests.conftest import scene


# ---------------------------------------------------------------- LBS (Sec. 3.1)
def _rand_skin(rng, J=24):
    S = np.zeros((J, 3, 4))
    for j in range(J):
        S[j, :, :3] = synth.axis_angle(rng.normal(size=3), rng.uniform(0, math.pi))
        S[j, :, 3] = rng.normal(0, 0.3, size=3)
    return S


def test_lbs_identity_pose_is_bit_exact():
    s = scene(1, identity_pose=True)
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    assert np.array_equal(xo, s["pos"])
    assert np.array_equal(no, s["nrm"])
    eye = np.eye(3, dtype=np.float32).reshape(9, 1)
    assert np.array_equal(Ao, np.broadcast_to(eye, Ao.shape))


def test_lbs_single_joint_is_rigid_motion():
    rng = np.random.default_rng(0)
    S = _rand_skin(rng)
    n = 500
    x = rng.normal(size=(3, n))
    nrm = rng.normal(size=(3, n))
    jidx = np.zeros((4, n), np.int32)
    jidx[0] = rng.integers(0, 24, n)
    jidx[1:] = rng.integers(0, 24, (3, n))
    jw = np.zeros((4, n))
    jw[0] = 1.0
    xo, no, Ao = cpu.lbs_f32(S.reshape(24, 12), jidx, jw, x, nrm)
    R = S[jidx[0], :, :3]                      # [n,3,3]
    t = S[jidx[0], :, 3]
    x32 = x.astype(np.float32).astype(np.float64)
    want = np.einsum("nab,bn->an", R.astype(np.float32).astype(np.float64), x32) + t.astype(np.float32).T
    assert np.allclose(xo, want, rtol=0, atol=2e-6)
    assert np.allclose(Ao.T.reshape(n, 3, 3), R, atol=1e-6)
    wantn = np.einsum("nab,bn->an", R, nrm.astype(np.float32))
    assert np.allclose(no, wantn, atol=2e-6)
    # the FP64 oracle (standard-form LBS) agrees with the closed form too
    xp64, np64, _ = ref64.lbs(S.reshape(24, 12), jidx, jw, x32, ref64.t64(nrm.astype(np.float32)))
    assert np.allclose(xp64.numpy(), np.einsum("nab,bn->an", R, x32) + t.T, atol=1e-12)


def test_lbs_translation_only_pose():
    rng = np.random.default_rng(1)
    S = np.zeros((24, 3, 4), np.float32)
    S[:, :, :3] = np.eye(3)
    S[:, :, 3] = rng.normal(size=(24, 3))
    n = 300
    x = rng.normal(size=(3, n)).astype(np.float32)
    jidx = rng.integers(0, 24, (4, n)).astype(np.int32)
    jw = np.zeros((4, n), np.float32)
    jw[0] = 1.0
    xo, _, _ = cpu.lbs_f32(S.reshape(24, 12), jidx, jw, x)
    assert np.array_equal(xo, x + S[jidx[0], :, 3].T)


def test_lbs_fp32_mirror_matches_fp64_standard_form(scene1):
    s = scene1
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    x64, n64, A64 = ref64.lbs(s["skin"], s["jidx"], s["jw"], s["pos"], ref64.t64(s["nrm"]))
    assert np.allclose(xo, x64.numpy(), rtol=0, atol=3e-7)
    assert np.allclose(no, n64.numpy(), rtol=0, atol=3e-7)
    assert np.allclose(Ao, A64.numpy(), rtol=0, atol=3e-7)


# ---------------------------------------------------------------- raster (Sec. 3.2)
def test_raster_bbox_equals_brute_force(scene1):
    s = scene1
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    for k in (0, 7, 21, 40, 63):
        d = s["view_dirs"][k]
        a = cpu.raster_view(vx, s["faces"], d, s["vis_res"], brute=False)
        b = cpu.raster_view(vx, s["faces"], d, s["vis_res"], brute=True)
        assert np.array_equal(a, b)
        assert (a != np.uint64(2 ** 64 - 1)).any()


def test_raster_shared_edges_are_watertight():
    """A fan and a grid whose edges pass exactly through sample points: every
    covered sample is claimed by exactly one triangle (tie rule)."""
    res = 16
    rng = np.random.default_rng(2)
    # grid of 4x4 quads, vertices exactly on sample centres (256 i + 128)
    pts = [[256 * i + 128 + (0 if (i % 2) else 0), 256 * j + 128] for j in range(0, 17, 4)
           for i in range(0, 17, 4)]
    tris = []
    for j in range(4):
        for i in range(4):
            a, b = j * 5 + i, j * 5 + i + 1
            c, d = (j + 1) * 5 + i, (j + 1) * 5 + i + 1
            if rng.random() < 0.5:
                tris += [(a, b, d), (a, d, c)]
            else:
                tris += [(a, b, c), (b, d, c)]
    pts = np.array(pts)
    xy = np.stack([pts[list(t)] for t in tris]).astype(np.int32)
    z = rng.random((len(tris), 3)).astype(np.float32) + 1
    # random orientation flips (two-sided raster)
    flip = rng.random(len(tris)) < 0.5
    xy[flip] = xy[flip][:, ::-1]
    z[flip] = z[flip][:, ::-1]
    _, claims = cpu.raster_fixed(xy, z, res, brute=True, claims=True)
    # samples strictly inside the grid's square must be claimed exactly once
    inner = claims[0:16, 0:16]
    lo, hi = 0, 16  # grid spans sample indices 0..16 (right/top boundary belongs to one side)
    assert inner.max() == 1
    # everything in [0, 16) x [0, 16) is inside the closed square [128, 16*256+128]
    assert (inner == 1).sum() >= (hi - lo - 1) ** 2
    # a fan around a centre vertex that is itself a sample point
    cx, cy = 256 * 8 + 128, 256 * 8 + 128
    ring = [(cx + int(1024 * math.cos(a)), cy + int(1024 * math.sin(a)))
            for a in np.linspace(0, 2 * math.pi, 9)[:-1]]
    fan = np.array([[(cx, cy), ring[i], ring[(i + 1) % 8]] for i in range(8)], np.int32)
    _, cl = cpu.raster_fixed(fan, np.ones((8, 3), np.float32), res, brute=True, claims=True)
    assert cl.max() == 1
    assert cl[8, 8] == 1          # the shared centre vertex is claimed once


def test_raster_nearest_triangle_wins_parallel_quads():
    """Two parallel quads facing the light: the far one is hidden."""
    near = np.array([[-0.5, -0.5, 0.2], [0.5, -0.5, 0.2], [0.5, 0.5, 0.2], [-0.5, 0.5, 0.2]])
    far = near.copy()
    far[:, 2] = -0.2
    far[:, :2] *= 0.5      # smaller: entirely behind the near quad
    verts = np.concatenate([near, far]).T.astype(np.float32)
    faces = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7]], np.int32)
    d = np.array([0, 0, 1.0], np.float32)      # light along +z: near quad (z=0.2) is closer
    zb = cpu.raster_view(verts, faces, d, 32)
    won = set((zb[zb != np.uint64(2 ** 64 - 1)] & np.uint64(0xFFFFFFFF)).astype(int).tolist())
    assert won == {0, 1}
    zb2 = cpu.raster_view(verts, faces, -d, 32)   # from the other side the far quad wins
    won2 = set((zb2[zb2 != np.uint64(2 ** 64 - 1)] & np.uint64(0xFFFFFFFF)).astype(int).tolist())
    assert {2, 3} <= won2


def _icosphere(level=3):
    t = (1 + 5 ** 0.5) / 2
    v = [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t],
         [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]]
    f = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
         [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8],
         [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    v = [list(np.array(p) / np.linalg.norm(p)) for p in v]
    for _ in range(level):
        mid = {}
        nf = []

        def m(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                p = np.array(v[a]) + np.array(v[b])
                v.append(list(p / np.linalg.norm(p)))
                mid[key] = len(v) - 1
            return mid[key]
        for a, b, c in f:
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = nf
    return np.array(v), np.array(f, np.int32)


def test_raster_convex_sphere_visibility_is_the_lit_hemisphere():
    """Convex body: a vertex is seen from direction d iff n.d > 0, away from
    grazing angles where triangles shrink below a sample."""
    v, f = _icosphere()
    dirs = synth.latlong_centres(4, 8)
    verts = v.T.astype(np.float32)
    nv = len(v)
    for d in dirs:
        zb = cpu.raster_view(verts, f, d.astype(np.float32), 128)
        vis = np.zeros(nv, bool)
        tri = (zb[zb != np.uint64(2 ** 64 - 1)] & np.uint64(0xFFFFFFFF)).astype(int)
        vis[f[tri].reshape(-1)] = True
        ndotd = v @ d
        assert vis[ndotd > 0.25].all()          # lit side visible
        assert not vis[ndotd < -0.1].any()      # far side hidden


def test_filters_match_sort_median_brute_force():
    rng = np.random.default_rng(3)
    for nv, kv, p in ((200, 19, 0.5), (97, 5, 0.3), (64, 1, 0.7)):
        pts = rng.normal(size=(nv, 3))
        _, knn = synth.nearest(pts, pts, kv)
        raw = (rng.random(nv) < p).astype(np.uint8)
        m1, m2, cnt = cpu.vis_filter(raw, knn)
        e1 = np.median(raw[knn], axis=1).astype(np.uint8)
        e2 = np.median(e1[knn], axis=1).astype(np.uint8)
        ec = e2[knn].sum(axis=1)
        assert np.array_equal(m1, e1) and np.array_equal(m2, e2) and np.array_equal(cnt, ec)


def test_mesh_visibility_counts_are_filtered_raw_bits(scene1):
    s = scene1
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    raw, cnt = cpu.mesh_visibility(vx, s["faces"], s["view_dirs"], s["vis_res"], s["knn_v"])
    V = s["view_dirs"].shape[0]
    bits = np.unpackbits(raw.view(np.uint8), axis=1, bitorder="little")[:, :V]
    for k in (0, 13, 63):
        zb = cpu.raster_view(vx, s["faces"], s["view_dirs"][k], s["vis_res"])
        tri = (zb[zb != np.uint64(2 ** 64 - 1)] & np.uint64(0xFFFFFFFF)).astype(int)
        vis = np.zeros(s["nv"], np.uint8)
        vis[s["faces"][tri].reshape(-1)] = 1
        assert np.array_equal(bits[:, k], vis)
        knn = s["knn_v"]
        e2 = np.median(np.median(vis[knn], axis=1).astype(np.uint8)[knn], axis=1).astype(np.uint8)
        assert np.array_equal(cnt[:, k], e2[knn].sum(axis=1))
    assert cnt.max() <= s["kv"]


def test_shadow_map_variant_sees_the_lit_hemisphere_and_hides_occluded_vertices():
    """The shadow-mapping depth test (the alternative discussed in Sec. 3.2):
    on a convex body the vertices facing the light pass and those facing
    away fail; behind a nearer quad, the covered vertices of a farther quad
    fail and the uncovered ones pass."""
    v, f = _icosphere()
    dirs = synth.latlong_centres(4, 8).astype(np.float32)
    _, knn = synth.nearest(v, v, 1)
    raw, _ = cpu.mesh_visibility_shadow(v.T.astype(np.float32), f, dirs, 128, knn, 2.0)
    for k, d in enumerate(dirs):
        vis = ((raw[:, k >> 5] >> (k & 31)) & 1).astype(bool)
        ndotd = v @ d
        assert vis[ndotd > 0.5].all()
        # (near the silhouette a vertex's pixel sample may miss the body and
        # pass: the grazing band is left out)
        assert not vis[ndotd < -0.3].any()
    # a far 4x4 grid (z = 0) under a near 2x2 quad (z = 1), light along +z
    g = np.linspace(-2.0, 2.0, 5)
    far = np.array([[x, y, 0.0] for y in g for x in g])
    near = np.array([[-1.2, -1.2, 1.0], [1.2, -1.2, 1.0], [1.2, 1.2, 1.0], [-1.2, 1.2, 1.0]])
    pts = np.concatenate([far, near])
    tris = []
    for r in range(4):
        for c in range(4):
            a = r * 5 + c
            tris += [[a, a + 1, a + 6], [a, a + 6, a + 5]]
    tris += [[25, 26, 27], [25, 27, 28]]
    _, knn = synth.nearest(pts, pts, 1)
    raw, _ = cpu.mesh_visibility_shadow(pts.T.astype(np.float32), np.array(tris),
                                        np.array([[0.0, 0.0, 1.0]], np.float32), 64, knn, 1.0)
    vis = (raw[:, 0] & 1).astype(bool)
    covered = (np.abs(far[:, 0]) < 1.2) & (np.abs(far[:, 1]) < 1.2)
    assert vis[25:].all()
    assert not vis[:25][covered].any() and vis[:25][~covered].all()


def test_skinning_matrix_gradient_single_joint_closed_form_and_fd():
    """dL/dS_j of forward LBS (the pose gradient of Sec. 3.3's pose
    optimisation): for one joint with weight 1 it is sum_i dx'_i [x_i, 1]^T +
    dn'_i [n_i, 0]^T; with four blended joints it matches finite
    differences of the FP64 oracle."""
    rng = np.random.default_rng(8)
    n = 7
    x = rng.normal(size=(3, n))
    nrm = rng.normal(size=(3, n))
    gx, gn = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    xt, nt = torch.tensor(x), torch.tensor(nrm)
    S = torch.tensor(rng.normal(size=(2, 12)), requires_grad=True)
    jidx = np.zeros((4, n), np.int32)
    jw = np.zeros((4, n))
    jw[0] = 1.0
    xp, npr, _ = ref64.lbs(S, jidx, jw, xt, nt)
    loss = (xp * torch.tensor(gx)).sum() + (npr * torch.tensor(gn)).sum()
    (g,) = torch.autograd.grad(loss, (S,))
    want = np.zeros((3, 4))
    want[:, :3] = gx @ x.T + gn @ nrm.T
    want[:, 3] = gx.sum(axis=1)
    assert np.allclose(g[0].numpy().reshape(3, 4), want, atol=1e-12)
    assert np.all(g[1].numpy() == 0)
    # blended joints: finite differences
    jidx = rng.integers(0, 2, (4, n)).astype(np.int32)
    jw = rng.dirichlet(np.ones(4), n).T
    S0 = rng.normal(size=(2, 12))

    def L(Sv):
        xp, npr, _ = ref64.lbs(torch.tensor(Sv), jidx, jw, xt, nt)
        return float((xp * torch.tensor(gx)).sum() + (npr * torch.tensor(gn)).sum())

    St = torch.tensor(S0, requires_grad=True)
    xp, npr, _ = ref64.lbs(St, jidx, jw, xt, nt)
    (g,) = torch.autograd.grad((xp * torch.tensor(gx)).sum() + (npr * torch.tensor(gn)).sum(),
                               (St,))
    for j, c in [(0, 0), (1, 5), (0, 11), (1, 3)]:
        e = np.zeros_like(S0)
        e[j, c] = 1e-6
        fd = (L(S0 + e) - L(S0 - e)) / 2e-6
        assert abs(fd - float(g[j, c])) < 1e-6 * max(1.0, abs(fd))
