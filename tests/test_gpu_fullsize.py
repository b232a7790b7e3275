"""Parity at the workloads' full sizes, in the launch configuration and the
storage layout bench.py uses (Gaussians grouped by nearest vertex; Renderer:
skin mesh -> visibility -> skin -> shade -> splat, and the adjoint), on
outputs the oracle can compute:

* bit-exact: skinned positions/normals/A (all), visibility counts (all
  views), back-face flags (all), D, tile ranges and lists (all);
* shaded colours of a seeded sample of 1500 Gaussians vs the FP64 oracle;
* the whole image vs the FP32 mirror's tiled compositing of the GPU colours;
* gradients of a loss on 32 sampled pixels of one tile vs the FP64 oracle's autograd,
  restricted to the Gaussians those pixels can see.
"""

import numpy as np
import pytest
import torch

from oracle import cpu, ref64
from paper_2407_10707_amd import render, rga, synth
from tests import helpers

pytestmark = pytest.mark.gpu

_CASES = {
    # config id, overrides (pose / env index), precision
    "avatar_512": (2, {}, "fp32"),
    "train_1024": (3, {}, "fp32"),
    "precision_200k_bf16x3": (4, {}, "bf16x3"),
    "anim_300k_1080_pose7_env2": (5, {"pose_index": 7, "env_index": 2}, "bf16x3"),
}


def _image_tol(ref, napp):
    """Tolerance of a composited pixel against the FP32 mirror.  The GPU sums
    each pixel in 256-splat chunks and combines them (C = C_before + T_in C_chunk,
    T_in a product of chunk transmittances) where the mirror multiplies and
    adds one splat at a time; with n splats composited, the transmittance
    products and the sum of non-negative terms each carry a relative
    rounding error of about 3 n u on either side (u = 2^-24), and the two
    sides' expf may differ by an ulp per splat: 8 (n + 2) u |ref| bounds the
    difference, on top of the 1e-5 relative and 1e-6 absolute floor."""
    u = 2.0 ** -24
    return (1e-5 + 8.0 * (napp[None] + 2) * u) * np.abs(ref) + 1e-6


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module", params=list(_CASES))
def case(request):
    cfg, kw, precision = _CASES[request.param]
    print(f"[fullsize] {request.param}: building scene", flush=True)
    s = synth.make_scene(cfg, **kw)
    # the layout bench.py times: Gaussians grouped by nearest vertex
    d, order = render.layout_by_vertex(render.upload(s))
    s = render.scene_in_order(s, order)
    R = render.Renderer(s, d, precision=precision)
    p = {k: d[k] for k in render.TRAINABLE}
    # the frame computes its own visibility, binning beside it (as bench.py)
    image, T, ctx = R.forward(p)
    if R.ensure_capacity():
        image, T, ctx = R.forward(p, ctx["count"])
    count = ctx["count"]
    torch.cuda.synchronize()
    return dict(name=request.param, s=s, d=d, R=R, p=p, count=count, image=image, T=T, ctx=ctx,
                precision=precision)


def test_skinning_visibility_and_flags_bit_exact(case):
    s = case["s"]
    print(f"[fullsize] {case['name']}: skinning/visibility", flush=True)
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    assert np.array_equal(_host(case["ctx"]["xo"]), xo)
    assert np.array_equal(_host(case["ctx"]["no"]), no)
    assert np.array_equal(_host(case["ctx"]["A"]), Ao)
    _, _, cnt = helpers.oracle_visibility(s)
    assert np.array_equal(_host(case["count"]), cnt)
    front = cpu.front_f32(xo, no, s["cam"].centre.astype(np.float32))
    assert np.array_equal(_host(case["ctx"]["front"]), front)
    assert np.array_equal(_host(case["R"].front_bin), front)     # the binning's own flags


def test_sampled_colours_match_fp64(case):
    s = case["s"]
    print(f"[fullsize] {case['name']}: sampled shading", flush=True)
    col = _host(case["ctx"]["color"])
    xo = _host(case["ctx"]["xo"])
    no = _host(case["ctx"]["no"])
    front = _host(case["ctx"]["front"])
    cnt = _host(case["count"])
    idx = np.sort(np.random.default_rng(7).choice(s["n"], 1500, replace=False))
    ecol, _ = ref64.shade(ref64.t64(xo[:, idx]), ref64.t64(no[:, idx]), s["albedo"][:, idx],
                          s["rough"][idx], s["tint"][idx], s["vidx"][:, idx], s["vw"][:, idx], cnt,
                          s["kv"], s["he"], s["we"], s["hv"], s["wv"], s["env"],
                          s["cam"].centre.astype(np.float32).astype(np.float64), front[idx])
    ecol = ecol.numpy()
    rtol = 1e-5 if case["precision"] == "fp32" else 1e-4
    err = np.abs(col[:, idx] - ecol)
    print(f"  max rel {np.max(err / (np.abs(ecol) + 1e-30)):.2e}", flush=True)
    assert np.all(err <= rtol * np.abs(ecol) + (1e-7 if case["precision"] == "fp32" else 1e-6))


def test_lists_and_image_match_fp32_mirror(case):
    s, R = case["s"], case["R"]
    print(f"[fullsize] {case['name']}: lists and image", flush=True)
    cam = s["cam"]
    col = _host(case["ctx"]["color"])
    xo = _host(case["ctx"]["xo"])
    Ao = _host(case["ctx"]["A"])
    front = _host(case["ctx"]["front"])
    pre = cpu.splat_preprocess(cam, xo, Ao, s["quat"], s["log_s"], s["opac"], front)
    keys, vals, ranges = cpu.splat_bin(cam, pre)
    D = R.ws.count()
    assert D == len(keys) and D <= R.ws.capacity
    st = R.ws.state()
    tiles = st.tiles_x * st.tiles_y
    gr = _host(R.ws.view(st.ranges, (tiles, 2), torch.int32))
    ne = ranges[:, 1] > ranges[:, 0]
    assert np.array_equal(gr[ne], ranges[ne])
    assert np.array_equal(_host(R.ws.view(st.sorted, (D,), torch.int32)), vals)
    eimg, eT, margin, napp = cpu.composite_tiles(cam, ranges, vals, pre, s["opac"], col,
                                                 with_applied=True)
    gi = _host(case["image"])
    # a decision (skip, clamp, stop) within the arithmetic's error of its
    # threshold may go either way on the two sides: such pixels are exempt
    ok = margin > np.maximum(1e-4, 8.0 * (napp + 2) * 2.0 ** -24)
    tol = _image_tol(eimg, napp)
    err = np.abs(gi - eimg)
    bad = (err > tol) & ok[None]
    u = 2.0 ** -24
    ratio = (err / ((napp[None] + 2) * u * np.abs(eimg) + 1e-30))[:, ok]
    print(f"  D={D} exempt={int((~ok).sum())}/{ok.size} max err {err[:, ok].max():.2e} "
          f"max rel {np.max(err[:, ok] / (np.abs(eimg[:, ok]) + 1e-6)):.2e} "
          f"max err/((n+2) u |ref|) {ratio.max():.2f} n max {napp.max()}", flush=True)
    assert not bad.any(), int(bad.sum())


def test_sampled_pixel_gradients_match_fp64(case):
    """L = sum over 32 sampled pixels of w . image; the GPU adjoint (dimage = w
    on those pixels, 0 elsewhere) against autograd of the FP64 oracle for
    the Gaussians whose tile lists cover the sampled pixels."""
    s, R, p = case["s"], case["R"], case["p"]
    print(f"[fullsize] {case['name']}: sampled gradients", flush=True)
    H, W = s["height"], s["width"]
    rng = np.random.default_rng(11)
    img = _host(case["image"])
    lit = np.nonzero(img.sum(0).reshape(-1) > 0.05)[0]
    # 32 lit pixels of one tile (keeps the FP64 oracle's share small)
    t0 = rng.choice(lit)
    ty, tx = (t0 // W) // 16, (t0 % W) // 16
    in_tile = lit[((lit // W) // 16 == ty) & ((lit % W) // 16 == tx)]
    pix = np.sort(rng.choice(in_tile, min(32, len(in_tile)), replace=False))
    w = np.zeros((3, H * W), np.float32)
    w[:, pix] = rng.uniform(0.5, 1.5, size=(3, len(pix)))
    g = R.backward(p, case["ctx"], torch.as_tensor(w.reshape(3, H, W)).cuda())
    # Gaussians that can reach the sampled pixels: their tiles' lists
    st = R.ws.state()
    D = R.ws.count()
    ranges = _host(R.ws.view(st.ranges, (st.tiles_x * st.tiles_y, 2), torch.int32))
    vals = _host(R.ws.view(st.sorted, (D,), torch.int32))
    tiles = np.unique((pix // W) // 16 * st.tiles_x + (pix % W) // 16)
    sub = np.unique(np.concatenate([vals[ranges[t, 0]:ranges[t, 1]] for t in tiles]))
    print(f"  {len(sub)} Gaussians reach the {len(pix)} pixels", flush=True)
    sub_s = dict(s)
    for k in ("pos", "nrm", "quat", "log_s", "albedo", "jidx", "jw", "vidx", "vw"):
        sub_s[k] = np.ascontiguousarray(s[k][:, sub])
    for k in ("opac", "rough", "tint"):
        sub_s[k] = np.ascontiguousarray(s[k][sub])
    sub_s["n"] = len(sub)
    cnt = _host(case["count"])
    front = _host(case["ctx"]["front"])[sub]
    p64 = helpers.params64(sub_s, requires_grad=True)
    img64, _ = helpers.render64(sub_s, p64, cnt, front, pixels=pix)
    (img64 * torch.tensor(w[:, pix].astype(np.float64))).sum().backward()
    rtol = 1e-4 if case["precision"] == "fp32" else 1e-3
    for k in render.TRAINABLE:
        got = _host(g[k])
        got = got if k == "env" else got[..., sub]
        helpers.check_grad(k, got, p64[k].grad.numpy(), rtol=rtol)


def _subscene(s, sub):
    sub_s = dict(s)
    for k in ("pos", "nrm", "quat", "log_s", "albedo", "jidx", "jw", "vidx", "vw"):
        sub_s[k] = np.ascontiguousarray(s[k][:, sub])
    for k in ("opac", "rough", "tint"):
        sub_s[k] = np.ascontiguousarray(s[k][sub])
    sub_s["n"] = len(sub)
    return sub_s


def test_image_error_vs_fp64_on_sampled_tiles(case):
    """Image error of the whole GPU path against the FP64 oracle's whole chain
    (skinning, shading, projection, compositing) on every pixel of 8 sampled
    lit tiles, as PSNR (peak 1), relative L2 and max abs.  For the workloads
    that use the BF16X3 shading the plain FP32 form is measured beside it."""
    s, R, d, p = case["s"], case["R"], case["d"], case["p"]
    H, W = s["height"], s["width"]
    st = R.ws.state()
    TX, TY = st.tiles_x, st.tiles_y
    img = _host(case["image"])
    tmean = np.zeros(TX * TY)
    for t in range(TX * TY):
        ty, tx = divmod(t, TX)
        tmean[t] = img[:, ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16].mean()
    rng = np.random.default_rng(13)
    tiles = np.sort(rng.choice(np.nonzero(tmean > 0.05)[0], 8, replace=False))
    pix = []
    for t in tiles:
        ty, tx = divmod(int(t), TX)
        yy, xx = np.meshgrid(np.arange(ty * 16, min(H, ty * 16 + 16)),
                             np.arange(tx * 16, min(W, tx * 16 + 16)), indexing="ij")
        pix.append((yy * W + xx).reshape(-1))
    pix = np.sort(np.concatenate(pix))
    D = R.ws.count()
    ranges = _host(R.ws.view(st.ranges, (TX * TY, 2), torch.int32))
    vals = _host(R.ws.view(st.sorted, (D,), torch.int32))
    sub = np.unique(np.concatenate([vals[ranges[t, 0]:ranges[t, 1]] for t in tiles]))
    print(f"[fullsize] {case['name']}: image error, {len(pix)} pixels, {len(sub)} Gaussians",
          flush=True)
    cnt = _host(case["count"])
    front = _host(case["ctx"]["front"])[sub]
    sub_s = _subscene(s, sub)
    with torch.no_grad():
        ref, _ = helpers.render64(sub_s, helpers.params64(sub_s), cnt, front, pixels=pix)
    ref = ref.numpy()
    forms = [case["precision"]] + (["fp32"] if case["precision"] == "bf16x3" else [])
    for form in forms:
        if form == case["precision"]:
            got = img.reshape(3, -1)[:, pix]
        else:
            R2 = render.Renderer(s, d, capacity=R.ws.capacity, precision=form)
            got = _host(R2.forward(p, case["count"])[0]).reshape(3, -1)[:, pix]
            del R2
        err = got - ref
        mse = float(np.mean(err ** 2))
        psnr = 10 * np.log10(1.0 / max(mse, 1e-300))
        rel = float(np.linalg.norm(err) / np.linalg.norm(ref))
        print(f"[report] {case['name']} {form}: PSNR {psnr:.1f} dB, relL2 {rel:.2e}, "
              f"max abs {np.abs(err).max():.2e}", flush=True)
        assert psnr > 110.0 and rel < 1e-5, (form, psnr, rel)
