"""Parity of the HIP path (through the C ABI) with the oracle.

Bit-exact: posed positions/normals/A, raw visibility bits and filtered counts,
back-face flags, per-splat tile rectangles and depth keys, D, tile ranges and
per-tile lists.  Tolerances: shaded colours vs the FP64 oracle
|d| <= 1e-5 |ref| + 1e-7; pixels vs the FP32 mirror |d| <= 1e-5 |ref| + 1e-6
(pixels whose compositing decisions sit within 1e-4 of a threshold are
exempt and counted); gradients vs the FP64 oracle's autograd, per element
(|g - g64| <= rtol |g64| + 1e-3 RMS(g64)) and per tensor (relative L2 <= 1e-4).
"""

import numpy as np
import pytest
import torch

from oracle import cpu, ref64
from paper_2407_10707_amd import render, rga, synth
from tests import helpers
from tests.conftest import scene

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    rga.lib()
    yield
    torch.cuda.synchronize()


def _scenes():
    return {
        "cfg1": lambda: scene(1),
        "cfg1_identity": lambda: scene(1, identity_pose=True),
        "micro_odd": lambda: synth.micro_scene(11, 333, 37, 53),
        "micro_ragged": lambda: synth.micro_scene(12, 900, 100, 161, log_scale_mean=-3.0),
    }


# ------------------------------------------------------------------ LBS
@pytest.mark.parametrize("name", list(_scenes()))
def test_lbs_bit_exact(name):
    print(f"[lbs] {name}", flush=True)
    s = _scenes()[name]()
    xo, no, Ao = rga.lbs_skin(dev(s["skin"]), dev(s["jidx"]), dev(s["jw"]), dev(s["pos"]),
                              dev(s["nrm"]))
    ex, en, eA = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    assert np.array_equal(host(xo), ex)
    assert np.array_equal(host(no), en)
    assert np.array_equal(host(Ao), eA)


def test_lbs_backward_is_A_transpose():
    s = scene(1)
    rng = np.random.default_rng(0)
    gx = rng.normal(size=(3, s["n"])).astype(np.float32)
    gn = rng.normal(size=(3, s["n"])).astype(np.float32)
    dx, dn = rga.lbs_skin_backward(dev(s["skin"]), dev(s["jidx"]), dev(s["jw"]), dev(gx), dev(gn))
    _, _, A64 = ref64.lbs(s["skin"], s["jidx"], s["jw"], s["pos"])
    A = A64.numpy().T.reshape(-1, 3, 3)
    assert np.allclose(host(dx), np.einsum("nba,bn->an", A, gx), atol=2e-6)
    assert np.allclose(host(dn), np.einsum("nba,bn->an", A, gn), atol=2e-6)


@pytest.mark.parametrize("which", ["cfg1", "avatar"])
def test_lbs_pose_gradient(which):
    """dL/d skinning matrices against the FP64 oracle's autograd; the bound
    is 1e-5 of the sum of the absolute terms of each entry (FP32 products
    and per-chunk sums of up to 100k terms)."""
    print(f"[lbs-pose] {which}", flush=True)
    s = scene(1) if which == "cfg1" else scene(2)
    n, J = s["n"], s["n_joints"]
    rng = np.random.default_rng(4)
    gx = rng.normal(size=(3, n)).astype(np.float32)
    gn = rng.normal(size=(3, n)).astype(np.float32)
    g = host(rga.lbs_skin_pose_grad(J, dev(s["jidx"]), dev(s["jw"]), dev(s["pos"]), dev(gx),
                                    dev(s["nrm"]), dev(gn)))
    S = torch.tensor(s["skin"].astype(np.float64), requires_grad=True)
    x64 = torch.tensor(s["pos"].astype(np.float64))
    n64 = torch.tensor(s["nrm"].astype(np.float64))
    xp, npr, _ = ref64.lbs(S, s["jidx"], s["jw"], x64, n64)
    (ref,) = torch.autograd.grad((xp * torch.tensor(gx.astype(np.float64))).sum() +
                                 (npr * torch.tensor(gn.astype(np.float64))).sum(), (S,))
    Sa = torch.tensor(np.abs(s["skin"]).astype(np.float64), requires_grad=True)
    xa, na, _ = ref64.lbs(Sa, s["jidx"], s["jw"], x64.abs(), n64.abs())
    (bound,) = torch.autograd.grad((xa * torch.tensor(np.abs(gx).astype(np.float64))).sum() +
                                   (na * torch.tensor(np.abs(gn).astype(np.float64))).sum(), (Sa,))
    err = np.abs(g - ref.numpy())
    print(f"[lbs-pose]   max err / bound {(err / (bound.numpy() + 1e-30)).max():.3e}", flush=True)
    assert np.all(err <= 1e-5 * bound.numpy() + 1e-7)


def test_pose_to_skin_and_its_adjoint():
    """Skinning matrices of random poses (one joint at the rest pose, one
    with a tiny rotation) against the FP64 oracle: matrices to 2e-6, the
    pose gradient to 2e-5 of its largest magnitude (FP32 chain of 24
    joints)."""
    print("[pose] forward kinematics", flush=True)
    rng = np.random.default_rng(9)
    J = len(synth.PARENTS)
    th = rng.normal(0.0, 0.4, (J, 3))
    th[1] = 0.0
    th[2] = [1e-4, -2e-4, 0.0]
    th = th.astype(np.float32)
    joints = synth.JOINTS_REST.astype(np.float32)
    parents = synth.PARENTS.astype(np.int32)
    S = host(rga.pose_to_skin(dev(th), dev(joints), dev(parents)))
    tt = torch.tensor(th.astype(np.float64).reshape(-1), requires_grad=True)
    ref = ref64.pose_to_skin(tt, joints.astype(np.float64), parents)
    assert np.abs(S - ref.detach().numpy()).max() <= 2e-6
    C = rng.normal(size=(J, 12)).astype(np.float32)
    (g,) = torch.autograd.grad((ref * torch.tensor(C.astype(np.float64))).sum(), (tt,))
    dth = host(rga.pose_to_skin_backward(dev(th), dev(joints), dev(parents), dev(C)))
    err = np.abs(dth.reshape(-1) - g.numpy()).max() / np.abs(g.numpy()).max()
    print(f"[pose]   dtheta err / max {err:.3e}", flush=True)
    assert err <= 2e-5


def test_lbs_empty_and_errors():
    s = scene(1)
    x = torch.empty((3, 0), device="cuda")
    out = rga.lbs_skin(dev(s["skin"]), torch.empty((4, 0), dtype=torch.int32, device="cuda"),
                       torch.empty((4, 0), device="cuda"), x, None)
    assert out[0].shape == (3, 0)
    L = rga.lib()
    assert L.lbs_skin(None, 10, 0, None, None, None, None, None, None, None, None, None) == -1
    assert "n_joints" in rga.last_error()


# ------------------------------------------------------------------ visibility
@pytest.mark.parametrize("name", ["cfg1", "micro_odd"])
def test_visibility_bit_exact(name):
    print(f"[vis] {name}", flush=True)
    s = _scenes()[name]()
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    count, raw = rga.mesh_visibility(dev(vx), dev(s["faces"]), dev(s["view_dirs"]), s["vis_res"],
                                     dev(s["knn_v"]), want_raw=True)
    eraw, ecnt = cpu.mesh_visibility(vx, s["faces"], s["view_dirs"], s["vis_res"], s["knn_v"])
    assert np.array_equal(host(raw).view(np.uint32), eraw)
    assert np.array_equal(host(count), ecnt)


def test_visibility_bit_exact_avatar_scale():
    """7k-vertex / 14k-triangle mesh, 512 views at 128^2 (the avatar workload)."""
    print("[vis] avatar scale", flush=True)
    s = scene(2, n_gauss=1000)
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    count, raw = rga.mesh_visibility(dev(vx), dev(s["faces"]), dev(s["view_dirs"]), s["vis_res"],
                                     dev(s["knn_v"]), want_raw=True)
    eraw, ecnt = cpu.mesh_visibility(vx, s["faces"], s["view_dirs"], s["vis_res"], s["knn_v"])
    assert np.array_equal(host(raw).view(np.uint32), eraw)
    assert np.array_equal(host(count), ecnt)


@pytest.mark.parametrize("case", [("cfg1", 0.0), ("cfg1", 1.5), ("avatar", 2.0)])
def test_shadow_map_visibility_bit_exact(case):
    """The shadow-mapping variant: raw depth-test bits and filtered counts."""
    name, bias = case
    print(f"[vis-shadow] {name} bias={bias}", flush=True)
    s = scene(2, n_gauss=1000) if name == "avatar" else _scenes()[name]()
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    count, raw = rga.mesh_visibility(dev(vx), dev(s["faces"]), dev(s["view_dirs"]), s["vis_res"],
                                     dev(s["knn_v"]), want_raw=True, shadow_bias_px=bias)
    eraw, ecnt = cpu.mesh_visibility_shadow(vx, s["faces"], s["view_dirs"], s["vis_res"],
                                            s["knn_v"], bias)
    assert np.array_equal(host(raw).view(np.uint32), eraw)
    assert np.array_equal(host(count), ecnt)


# ------------------------------------------------------------------ shading
@pytest.mark.parametrize("name", ["cfg1", "micro_odd"])
def test_shading_matches_fp64(name):
    print(f"[shade] {name}", flush=True)
    s = _scenes()[name]()
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    _, _, cnt = helpers.oracle_visibility(s)
    campos = s["cam"].centre.astype(np.float32)
    col, front = rga.shade_gaussians(dev(xo), dev(no), dev(s["albedo"]), dev(s["rough"]),
                                     dev(s["tint"]), dev(s["vidx"]), dev(s["vw"]), dev(cnt),
                                     s["kv"], s["he"], s["we"], s["hv"], s["wv"], dev(s["env"]),
                                     campos)
    efront = cpu.front_f32(xo, no, campos)
    assert np.array_equal(host(front), efront)
    ecol, _ = ref64.shade(ref64.t64(xo), ref64.t64(no), s["albedo"], s["rough"], s["tint"],
                          s["vidx"], s["vw"], cnt, s["kv"], s["he"], s["we"], s["hv"], s["wv"],
                          s["env"], campos.astype(np.float64), efront)
    ecol = ecol.numpy()
    got = host(col)
    err = np.abs(got - ecol)
    assert np.all(err <= 1e-5 * np.abs(ecol) + 1e-7), err.max()


@pytest.mark.parametrize("name", ["cfg1", "micro_odd"])
def test_shading_bf16x3_matches_fp64(name):
    """BF16 operands (hi + lo split) on MFMA with FP32 accumulation: colours
    within 1e-4 relative of the FP64 oracle; back-face flags bit-exact."""
    print(f"[shade bf16x3] {name}", flush=True)
    s = _scenes()[name]()
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    _, _, cnt = helpers.oracle_visibility(s)
    campos = s["cam"].centre.astype(np.float32)
    col, front = rga.shade_gaussians(dev(xo), dev(no), dev(s["albedo"]), dev(s["rough"]),
                                     dev(s["tint"]), dev(s["vidx"]), dev(s["vw"]), dev(cnt),
                                     s["kv"], s["he"], s["we"], s["hv"], s["wv"], dev(s["env"]),
                                     campos, precision="bf16x3")
    efront = cpu.front_f32(xo, no, campos)
    assert np.array_equal(host(front), efront)
    ecol, _ = ref64.shade(ref64.t64(xo), ref64.t64(no), s["albedo"], s["rough"], s["tint"],
                          s["vidx"], s["vw"], cnt, s["kv"], s["he"], s["we"], s["hv"], s["wv"],
                          s["env"], campos.astype(np.float64), efront)
    ecol = ecol.numpy()
    got = host(col)
    rel = np.abs(got - ecol) / (np.abs(ecol) + 1e-30)
    print(f"  max rel {rel[ecol > 1e-3].max():.2e}", flush=True)
    assert np.all(np.abs(got - ecol) <= 1e-4 * np.abs(ecol) + 1e-6)


# ------------------------------------------------------------------ splatting
def _splat_case(s, color):
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    front = cpu.front_f32(xo, no, s["cam"].centre.astype(np.float32))
    return xo, Ao, front


def _tile_scenes():
    """Image sizes at the tile sort's pass boundaries: 2048 tiles (one pass of
    11-bit digits), 2080 and 4096 (one pass of 12-bit digits), 4160 (two
    passes, then the tile-range and work-item launches)."""
    return {f"tiles_{h // 16 * ((w + 15) // 16)}": (lambda h=h, w=w: synth.micro_scene(
        21, 3000, h, w, log_scale_mean=-3.0)) for h, w in ((512, 1024), (512, 1040),
                                                           (1024, 1024), (1024, 1040))}


@pytest.mark.parametrize("name", list(_scenes()) + list(_tile_scenes()))
def test_splat_forward_parity(name):
    print(f"[splat] {name}", flush=True)
    s = {**_scenes(), **_tile_scenes()}[name]()
    rng = np.random.default_rng(1)
    col = rng.random((3, s["n"])).astype(np.float32)
    xo, Ao, front = _splat_case(s, col)
    cam = s["cam"]
    # room for every (tile, splat) pair: the 1024^2 scenes reach about 107 per Gaussian
    ws = rga.SplatWorkspace(s["n"], cam.width, cam.height, 160 * s["n"] + 1024, "cuda")
    img, T = rga.splat_forward(cam, dev(xo), dev(Ao), dev(s["quat"]), dev(s["log_s"]),
                               dev(s["opac"]), dev(col), dev(front), ws)
    pre = cpu.splat_preprocess(cam, xo, Ao, s["quat"], s["log_s"], s["opac"], front)
    keys, vals, ranges = cpu.splat_bin(cam, pre)
    eimg, eT, margin = cpu.composite_tiles(cam, ranges, vals, pre, s["opac"], col)
    D = ws.count()
    assert D == len(keys)
    assert D <= ws.capacity, "workspace too small for this scene's lists"
    st = ws.state()
    n = s["n"]

    tdt = {np.int32: torch.int32, np.float32: torch.float32, np.uint8: torch.uint8}

    def grab(ptr, shape, dtype):
        return host(ws.view(ptr, shape, tdt[dtype]))

    touched = grab(st.touched, (n,), np.int32)
    assert np.array_equal(touched, pre["touched"])
    rect = grab(st.rect, (4, n), np.int32)
    live = touched > 0
    assert np.array_equal(rect[:, live], pre["rect"][:, live])
    depth = grab(st.depth, (n,), np.float32)
    assert np.array_equal(depth.view(np.uint32)[live], pre["depth"].view(np.uint32)[live])
    gm = grab(st.mean2d, (2, n), np.float32)
    assert np.array_equal(gm[:, live], pre["mean2d"][:, live])
    gfp = grab(st.fp64, (n,), np.uint8)
    assert np.array_equal(gfp[live], pre["fp64"][live])
    tiles = st.tiles_x * st.tiles_y
    granges = grab(st.ranges, (tiles, 2), np.int32)
    nonempty = ranges[:, 1] > ranges[:, 0]
    assert np.array_equal(granges[nonempty], ranges[nonempty])
    assert np.all(granges[~nonempty, 1] == granges[~nonempty, 0])
    if D:
        gvals = grab(st.sorted, (D,), np.int32)
        assert np.array_equal(gvals, vals)
        # keys rebuilt from the GPU's own tile ranges and depths
        tile_of = np.repeat(np.arange(tiles), granges[:, 1] - granges[:, 0])
        gkeys = (tile_of.astype(np.uint64) << np.uint64(32)) | depth.view(np.uint32)[gvals].astype(np.uint64)
        assert np.array_equal(gkeys, keys)
    gi, gT = host(img), host(T)
    ok = margin > 1e-4
    tol = 1e-5 * np.abs(eimg) + 1e-6
    bad = (np.abs(gi - eimg) > tol) & ok[None]
    assert not bad.any(), (f"{int(bad.sum())} pixel values off; max err "
                           f"{np.abs(gi - eimg)[:, ok].max():.3e}; worst rel "
                           f"{(np.abs(gi - eimg) / (np.abs(eimg) + 1e-30))[bad].max():.3e}")
    assert np.all(np.abs(gT - eT)[ok] <= 1e-5 * eT[ok] + 1e-6)
    print(f"  D={D} exempt={int((~ok).sum())}/{ok.size}", flush=True)


@pytest.mark.parametrize("mode", ["albedo", "normal"])
def test_editing_maps(mode):
    """Albedo and normal maps (Sec. 3.4): the splatting of the albedo or of
    the skinned normal, against the FP32 mirror with the same colours."""
    print(f"[map] {mode}", flush=True)
    from paper_2407_10707_amd import render
    s = _scenes()["cfg1"]()
    R = render.Renderer(s, render.upload(s), capacity=64 * s["n"] + 1024)
    p = {k: R.d[k] for k in ("pos", "nrm", "quat", "log_s", "opac", "albedo", "rough", "tint",
                             "env")}
    count = R.visibility()
    img = host(R.render_map(p, count, mode))
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    col = s["albedo"] if mode == "albedo" else no
    ref = helpers.oracle_frame_f32(s, np.ascontiguousarray(col, dtype=np.float32))
    ok = ref["margin"] > 1e-4
    tol = 1e-5 * np.abs(ref["img"]) + 1e-6
    assert not ((np.abs(img - ref["img"]) > tol) & ok[None]).any()


def test_splat_deep_tiles_parity():
    """Thousands of faint splats over a few tiles: lists span many 256-entry
    chunks and most pixels stop in a later chunk with an incoming
    transmittance near the 1e-4 stop, where the chunk combine and the
    restart must carry T exactly.  Image and T_final against the FP32
    mirror, with the tolerance and the decision exemption scaled by the
    number of splats composited per pixel (chunked vs sequential rounding)."""
    print("[splat] deep tiles", flush=True)
    rng = np.random.default_rng(5)
    cam = synth.default_camera(48, 32)
    n = 4000
    x = np.stack([rng.uniform(-1.7, 0.6, n), rng.uniform(-0.3, 1.2, n),
                  rng.uniform(-0.2, 0.2, n)]).astype(np.float32)
    A = np.tile(np.eye(3, dtype=np.float32).reshape(9, 1), (1, n))
    q = rng.normal(size=(4, n)).astype(np.float32)
    log_s = rng.normal(-1.0, 0.2, (3, n)).astype(np.float32)
    opac = rng.uniform(0.005, 0.03, n).astype(np.float32)
    col = rng.random((3, n)).astype(np.float32)
    front = np.ones(n, np.uint8)
    ws = rga.SplatWorkspace(n, cam.width, cam.height, 8 * n, "cuda")
    img, T = rga.splat_forward(cam, dev(x), dev(A), dev(q), dev(log_s), dev(opac), dev(col),
                               dev(front), ws)
    pre = cpu.splat_preprocess(cam, x, A, q, log_s, opac, front)
    keys, vals, ranges = cpu.splat_bin(cam, pre)
    eimg, eT, margin, napp = cpu.composite_tiles(cam, ranges, vals, pre, opac, col,
                                                 with_applied=True)
    assert ws.count() == len(keys)
    st = ws.state()
    assert np.array_equal(host(ws.view(st.sorted, (len(keys),), torch.int32)), vals)
    lens = ranges[:, 1] - ranges[:, 0]
    deep = int((napp > 300).sum())
    print(f"  D={len(keys)} longest list {lens.max()} pixels past 300 splats {deep}", flush=True)
    assert lens.max() > 4 * 256 and deep > 100
    u = 2.0 ** -24
    rel = 1e-5 + 8.0 * (napp + 2) * u
    ok = margin > np.maximum(1e-4, rel)
    gi, gT = host(img), host(T)
    bad = (np.abs(gi - eimg) > rel[None] * np.abs(eimg) + 1e-6) & ok[None]
    assert not bad.any(), int(bad.sum())
    # T_final >= 1e-4 everywhere a walk stopped: compare relatively
    badT = (np.abs(gT - eT) > rel * eT) & ok
    assert not badT.any(), (int(badT.sum()), float(np.max(np.abs(gT - eT)[ok] / eT[ok])))


@pytest.mark.parametrize("n", [20000, 40000])
def test_splat_long_lists_bit_exact(n):
    """Tile lists longer than a workgroup sorts in LDS (8192 entries): large
    splats over a 3 x 2-tile image, each tile holding all of them (3 and 5
    sorted runs, merged in 2 and 3 passes, the last run unpaired in the
    first), drawn from 1,000 positions, so that many depths tie exactly
    (ties go to the lower index).  D, the ranges and every list against the
    oracle's (depth bits, index) order."""
    print(f"[splat] long lists n={n}", flush=True)
    rng = np.random.default_rng(9)
    cam = synth.default_camera(48, 32)
    pts = np.stack([rng.uniform(-0.3, 0.3, 1000), rng.uniform(-0.2, 0.2, 1000),
                    rng.uniform(-0.5, 0.5, 1000)]).astype(np.float32)
    x = np.ascontiguousarray(pts[:, rng.integers(0, 1000, n)])
    A = np.tile(np.eye(3, dtype=np.float32).reshape(9, 1), (1, n))
    q = rng.normal(size=(4, n)).astype(np.float32)
    log_s = rng.normal(-0.5, 0.1, (3, n)).astype(np.float32)
    opac = rng.uniform(0.3, 0.9, n).astype(np.float32)
    col = rng.random((3, n)).astype(np.float32)
    front = np.ones(n, np.uint8)
    ws = rga.SplatWorkspace(n, cam.width, cam.height, 8 * n, "cuda")
    rga.splat_forward(cam, dev(x), dev(A), dev(q), dev(log_s), dev(opac), dev(col), dev(front), ws)
    pre = cpu.splat_preprocess(cam, x, A, q, log_s, opac, front)
    keys, vals, ranges = cpu.splat_bin(cam, pre)
    lens = ranges[:, 1] - ranges[:, 0]
    print(f"  D={len(keys)} list lengths {lens.tolist()}", flush=True)
    assert lens.max() > 2 * 8192
    assert ws.count() == len(keys)
    st = ws.state()
    assert np.array_equal(host(ws.view(st.ranges, (len(lens), 2), torch.int32)), ranges)
    assert np.array_equal(host(ws.view(st.sorted, (len(keys),), torch.int32)), vals)


def test_splat_empty_and_all_culled():
    cam = synth.default_camera(40, 24)
    ws = rga.SplatWorkspace(0, 40, 24, 16, "cuda")
    z = lambda *sh: torch.zeros(sh, device="cuda")
    img, T = rga.splat_forward(cam, z(3, 0), z(9, 0), z(4, 0), z(3, 0), z(0), z(3, 0),
                               torch.zeros(0, dtype=torch.uint8, device="cuda"), ws)
    assert torch.all(img == 0) and torch.all(T == 1)
    # all Gaussians behind the camera
    n = 50
    x = torch.zeros(3, n, device="cuda")
    x[2] = 10.0
    A = torch.eye(3, device="cuda").reshape(9, 1).repeat(1, n).contiguous()
    q = torch.zeros(4, n, device="cuda")
    q[0] = 1
    ws = rga.SplatWorkspace(n, 40, 24, 1024, "cuda")
    img, T = rga.splat_forward(cam, x, A, q, z(3, n) - 3, z(n) + 0.5, z(3, n) + 1,
                               torch.ones(n, dtype=torch.uint8, device="cuda"), ws)
    assert torch.all(img == 0) and torch.all(T == 1)
    assert ws.count() == 0


def test_splat_capacity_overflow_is_reported():
    """More duplicates than the workspace holds: D is reported, the image
    and T_final are poisoned (NaN) and so are the adjoint's gradients."""
    s = scene(1)
    col = np.ones((3, s["n"]), np.float32)
    xo, Ao, front = _splat_case(s, col)
    cam = s["cam"]
    ws = rga.SplatWorkspace(s["n"], cam.width, cam.height, 16, "cuda")
    args = (dev(xo), dev(Ao), dev(s["quat"]), dev(s["log_s"]), dev(s["opac"]), dev(col),
            dev(front))
    img, T = rga.splat_forward(cam, *args, ws)
    assert ws.count() > 16
    assert torch.isnan(img).all() and torch.isnan(T).all()
    g = rga.splat_backward(cam, *args, ws, img, torch.ones_like(img), want_dA=True)
    for k in ("dx", "dquat", "dlog_s", "dopac", "dcolor", "dA"):
        assert torch.isnan(g[k]).all(), k
    # a large enough workspace on the same inputs is clean again
    ws2 = rga.SplatWorkspace(s["n"], cam.width, cam.height, 64 * s["n"], "cuda")
    img2, _ = rga.splat_forward(cam, *args, ws2)
    assert torch.isfinite(img2).all()


@pytest.mark.parametrize("overlap", [False, True])
def test_renderer_refuses_stale_backward_and_overflow(overlap):
    """A backward whose forward's splat state has been overwritten by a later
    render on the same Renderer is refused; the autograd path raises on an
    overflowed frame, and train_step re-renders it in a larger workspace --
    with the splats binned after the shading or on the second stream."""
    s = scene(1)
    d = render.upload(s)
    R = render.Renderer(s, d, capacity=64 * s["n"], overlap=overlap)
    p = {k: d[k] for k in render.TRAINABLE}
    count = R.visibility()
    _, _, ctx1 = R.forward(p, count)
    R.render_map(p, count, "albedo")
    with pytest.raises(rga.RgaError, match="overwritten"):
        R.backward(p, ctx1, torch.zeros(3, s["height"], s["width"], device="cuda"))
    R2 = render.Renderer(s, d, capacity=16, overlap=overlap)
    q = {k: v.clone().requires_grad_(True) for k, v in p.items()}
    img, _ = render.render(R2, count, q)
    with pytest.raises(rga.RgaError, match="overflowed"):
        img.sum().backward()
    R3 = render.Renderer(s, d, capacity=16, overlap=overlap)
    loss, g = R3.train_step(p, count, d["target"])
    assert R3.ws.capacity > 16 and torch.isfinite(loss).all()
    assert all(torch.isfinite(t).all() for t in g.values())
    # the frame computing its own visibility overflows and recovers the same way
    R4 = render.Renderer(s, d, capacity=16, overlap=overlap)
    loss4, g4 = R4.train_step(p, None, d["target"])
    assert R4.ws.capacity > 16 and torch.equal(loss4, loss)
    for k in g:
        a4, a3 = g4[k].cpu().numpy(), g[k].cpu().numpy()
        assert np.abs(a4 - a3).max() <= 1e-5 * (np.abs(a3).max() + 1e-30), k


# ------------------------------------------------------------------ gradients
def _grad_case(seed=5):
    s = synth.micro_scene(seed, 60, 48, 64, he=4, we=8, hv=4, wv=8, log_scale_mean=-3.0)
    _, _, cnt = helpers.oracle_visibility(s)
    front = helpers.front_flags(s)
    w = np.random.default_rng(seed).random((3, s["height"], s["width"]))
    return s, cnt, front, w


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_gradients_match_fp64_oracle(precision):
    print(f"[grad] micro {precision}", flush=True)
    s, cnt, front, w = _grad_case()
    p = helpers.params64(s, requires_grad=True)
    img, _ = helpers.render64(s, p, cnt, front)
    (img * torch.tensor(w.reshape(3, -1))).sum().backward()
    d = render.upload(s)
    R = render.Renderer(s, d, precision=precision)
    pd = {k: d[k] for k in render.TRAINABLE}
    image, T, ctx = R.forward(pd, dev(cnt))
    g = R.backward(pd, ctx, dev(w.astype(np.float32)))
    # forward image against the FP64 oracle as a sanity check of the chain
    # per element |g - g64| <= rtol |g64| + 1e-3 RMS(g64), per tensor relL2 <= 1e-4;
    # the split bf16 product's colours carry up to 1e-4 relative error, so
    # its per-element rtol is 1e-3
    tol_img, rtol = (2e-5, 1e-4) if precision == "fp32" else (2e-4, 1e-3)
    assert np.abs(host(image).reshape(3, -1) - img.detach().numpy()).max() < tol_img
    for k in render.TRAINABLE:
        helpers.check_grad(k, host(g[k]), p[k].grad.numpy(), rtol=rtol)


def test_pose_to_skin_edge_cases():
    """One joint, and a skeleton whose parents are all out of range (every
    joint a root), against the oracle."""
    print("[pose] edge cases", flush=True)
    rng = np.random.default_rng(10)
    for J, parents in ((1, np.array([-1], np.int32)), (5, np.array([-1, 7, 3, -2, 4], np.int32))):
        th = rng.normal(0.0, 0.5, (J, 3)).astype(np.float32)
        joints = rng.normal(size=(J, 3)).astype(np.float32)
        S = host(rga.pose_to_skin(dev(th), dev(joints), dev(parents)))
        eff = np.array([p if 0 <= p < j else -1 for j, p in enumerate(parents)])
        ref = ref64.pose_to_skin(th.astype(np.float64).reshape(-1), joints.astype(np.float64), eff)
        assert np.abs(S - ref.numpy()).max() <= 2e-6
