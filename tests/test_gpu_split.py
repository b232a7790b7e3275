"""The forward split that lets the binning overlap the shading (Sec. 3.1,
last paragraph, and the back-face rule of the rendering-equation
paragraph): back_face gives the shading's back-face flags bit for bit;
splat_bin then splat_blend give splat_forward's image, T_final, duplicate
count and tile lists bit for bit, also when the colours change between two
blends of one binning; the renderer's frame that computes the visibility
itself, binning on a second stream, equals the frame given the visibility
(image bit for bit, gradients to 1e-5 relative: the adjoint sums with float
atomics)."""

import ctypes as C

import numpy as np
import pytest
import torch

from oracle import cpu
from paper_2407_10707_amd import render, rga, synth
from tests.conftest import scene

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _scenes():
    return {"cfg1": lambda: scene(1),
            "micro_ragged": lambda: synth.micro_scene(5, 333, 70, 45)}


@pytest.mark.parametrize("name", list(_scenes()))
def test_back_face_matches_shading_and_mirror(name):
    print(f"[split] back_face {name}", flush=True)
    s = _scenes()[name]()
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    cam = s["cam"].centre.astype(np.float32)
    fb = host(rga.back_face(dev(xo), dev(no), cam))
    assert np.array_equal(fb, cpu.front_f32(xo, no, cam))
    count = torch.zeros((int(s["verts"].shape[1]), s["hv"] * s["wv"]), dtype=torch.uint8,
                        device="cuda")
    _, fs = rga.shade_gaussians(dev(xo), dev(no), dev(s["albedo"]), dev(s["rough"]),
                                dev(s["tint"]), dev(s["vidx"]), dev(s["vw"]), count, s["kv"],
                                s["he"], s["we"], s["hv"], s["wv"], dev(s["env"]), cam)
    assert np.array_equal(fb, host(fs))
    # a normal exactly perpendicular to the view ray is back-facing (n.w = 0)
    x = dev(np.zeros((3, 2), np.float32))
    nrm = dev(np.array([[1.0, 0.0], [0.0, 0.0], [0.0, 1.0]], np.float32))
    assert host(rga.back_face(x, nrm, [0.0, 0.0, 2.0])).tolist() == [0, 1]


@pytest.mark.parametrize("name", list(_scenes()))
def test_bin_then_blend_equals_forward(name):
    print(f"[split] bin + blend {name}", flush=True)
    s = _scenes()[name]()
    n, cam = s["n"], s["cam"]
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    front = dev(cpu.front_f32(xo, no, cam.centre.astype(np.float32)))
    rng = np.random.default_rng(3)
    cols = [dev(rng.random((3, n)).astype(np.float32)) for _ in range(2)]
    geo = (dev(xo), dev(Ao), dev(s["quat"]), dev(s["log_s"]), dev(s["opac"]))
    cap = 64 * n + 1024
    ref = []
    for col in cols:
        ws = rga.SplatWorkspace(n, cam.width, cam.height, cap, "cuda")
        img, T = rga.splat_forward(cam, *geo, col, front, ws)
        st = ws.state()
        D = ws.count()
        lists = host(ws.view(st.sorted, (D,), torch.int32))
        ref.append((host(img), host(T), D, lists))
    ws = rga.SplatWorkspace(n, cam.width, cam.height, cap, "cuda")
    rga.splat_bin(cam, *geo, front, ws)
    for (eimg, eT, eD, elists), col in zip(ref, cols):
        img, T = rga.splat_blend(cam, col, ws)
        assert np.array_equal(host(img), eimg)
        assert np.array_equal(host(T), eT)
        assert ws.count() == eD
        st = ws.state()
        assert np.array_equal(host(ws.view(st.sorted, (eD,), torch.int32)), elists)
    # the adjoint of the last blend equals the adjoint after splat_forward
    dimg = dev(rng.random((3, cam.height, cam.width)).astype(np.float32))
    g1 = rga.splat_backward(cam, *geo, cols[1], front, ws, img, dimg)
    ws2 = rga.SplatWorkspace(n, cam.width, cam.height, cap, "cuda")
    img2, _ = rga.splat_forward(cam, *geo, cols[1], front, ws2)
    g2 = rga.splat_backward(cam, *geo, cols[1], front, ws2, img2, dimg)
    for k in ("dx", "dquat", "dlog_s", "dopac", "dcolor"):
        a, b = host(g1[k]), host(g2[k])
        assert np.abs(a - b).max() <= 1e-5 * (np.abs(b).max() + 1e-30), k


def test_split_entry_points_refuse_bad_arguments():
    s = scene(1)
    n, cam = s["n"], s["cam"]
    ws = rga.SplatWorkspace(n, cam.width, cam.height, 1024, "cuda")
    L = rga.lib()
    c = rga.camera(cam)
    assert L.splat_bin(None, n, C.byref(c), None, None, None, None, None, None,
                       rga._p(ws.buf), ws.bytes, ws.capacity) == -1
    assert L.splat_blend(None, n, C.byref(c), None, rga._p(ws.buf), ws.bytes, ws.capacity,
                         None, None) == -1
    assert L.splat_blend(None, n, C.byref(c), None, rga._p(ws.buf), 16, ws.capacity,
                         None, None) != 0
    assert L.back_face(None, -1, None, None, None, None) == -1
    assert L.back_face(None, 4, None, None, None, None) == -1
    assert L.back_face(None, 0, None, None, None, None) == 0
    # the binding refuses a blend on a workspace no binning has filled
    with pytest.raises(rga.RgaError, match="splat_bin first"):
        rga.splat_blend(cam, torch.zeros((3, n), dtype=torch.float32, device="cuda"), ws)


@pytest.mark.parametrize("cfg", [1, 2])
def test_renderer_frame_with_its_own_visibility(cfg):
    """R.forward(p) (visibility inside the frame, binning on the second
    stream) against R.forward(p, R.visibility()) and against a renderer
    that bins after the shading on one stream, and their adjoints."""
    print(f"[split] renderer cfg {cfg}", flush=True)
    s = scene(cfg)
    d, order = render.layout_by_vertex(render.upload(s))
    so = render.scene_in_order(s, order)
    R1 = render.Renderer(so, d, overlap=False)
    assert render.Renderer(so, d).overlap == (s["n"] >= render.Renderer.OVERLAP_MIN_GAUSSIANS)
    p = {k: d[k] for k in render.TRAINABLE}
    w = dev(np.random.default_rng(cfg).random((3, s["cam"].height, s["cam"].width))
            .astype(np.float32))
    count = R1.visibility()
    img1, T1, c1 = R1.forward(p, count)
    if R1.ensure_capacity():
        img1, T1, c1 = R1.forward(p, count)
    g1 = R1.backward(p, c1, w)
    R = render.Renderer(so, d, capacity=R1.ws.capacity, overlap=True)
    for given in (False, True):
        img2, T2, c2 = R.forward(p, count if given else None)
        assert torch.equal(c2["count"], count)
        assert torch.equal(img1, img2) and torch.equal(T1, T2)
        assert torch.equal(R.front_bin, c2["front"])
        g2 = R.backward(p, c2, w)
        for k in render.TRAINABLE:
            a, b = host(g1[k]), host(g2[k])
            err = np.abs(a - b).max() / (np.abs(b).max() + 1e-30)
            print(f"  {k:8s} {err:.1e}", flush=True)
            assert err <= 1e-5, (k, err)
