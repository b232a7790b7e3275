"""The paper's vertex parametrisation composed from the library's entry
points (Sec. 3.1: materials and the displacement network's output on the
canonical vertices, interpolated to each Gaussian over its K_g = 3 nearest
vertices; skinning matrices from the pose theta), with the total loss of
Sec. 3.3 (an image term plus the four weighted regularisers, their
gradients merged inside the library), against the same composition of the
FP64 oracle, differentiated by autograd.

The neighbour indices come from the oracle's FP32 brute force (bit-exact
with the GPU search); the visibility counts and back-face flags, FP32
decisions, come from the oracle's FP32 mirror of the posed scene.  Gradients
per element as the render-path gradient test: |g - g64| <= 1e-4 |g64| +
1e-3 RMS(g64), and relative L2 <= 1e-4 per tensor."""

import numpy as np
import pytest
import torch

from oracle import cpu, ref64
from paper_2407_10707_amd import render, rga, synth
from tests import helpers

pytestmark = pytest.mark.gpu


def test_vertex_model_gradients_match_fp64_oracle():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print("[vertex-model] micro scene", flush=True)
    s = synth.micro_scene(5, 60, 48, 64, he=4, we=8, hv=4, wv=8, log_scale_mean=-3.0)
    nv, n = int(s["nv"]), int(s["n"])
    rng = np.random.default_rng(12)
    inp = synth.mlp_inputs(12)
    params = inp["params"].copy()
    params[-(3 * 256 + 3):] *= 0.01          # displacements of a few millimetres
    theta = (0.3 * rng.standard_normal((24, 3))).astype(np.float32)
    v_alb = rng.random((3, nv)).astype(np.float32)
    v_rough = rng.uniform(0.2, 0.9, nv).astype(np.float32)
    v_tint = rng.uniform(0.0, 1.0, nv).astype(np.float32)
    joints = synth.JOINTS_REST.astype(np.float32)
    parents = synth.PARENTS.astype(np.int32)

    # ---- oracle: FP64 composition, FP32 decisions from the mirror
    idx, d2 = cpu.knn(s["pos"], s["verts"], 3)
    wk = ref64.knn_weights(d2)
    t64 = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), requires_grad=True)
    th64, mlp64, alb64, ro64, ti64 = t64(theta), t64(params), t64(v_alb), t64(v_rough), t64(v_tint)
    pos64 = t64(s["pos"])
    dxv = ref64.displacement(s["verts"].astype(np.float64), inp["freqs"].astype(np.float64),
                             th64.reshape(-1), mlp64)
    attrs = torch.cat([alb64, ro64[None], ti64[None], dxv])
    ag = ref64.interpolate(idx, wk, attrs)
    skin64 = ref64.pose_to_skin(th64.reshape(-1), joints.astype(np.float64), parents)
    skin32 = skin64.detach().numpy().astype(np.float32)
    s2 = dict(s, skin=skin32)
    pos_d32 = (pos64 + ag[5:8]).detach().numpy().astype(np.float32)
    s3 = dict(s2, pos=pos_d32)
    _, _, cnt = helpers.oracle_visibility(s2)
    front = helpers.front_flags(s3)
    p = helpers.params64(s)
    ls64 = p["log_s"].detach().clone().requires_grad_(True)
    p.update(pos=pos64 + ag[5:8], albedo=ag[0:3], rough=ag[3], tint=ag[4], log_s=ls64)
    img, _ = helpers.render64(dict(s, skin=skin64), p, cnt, front)
    wimg = np.random.default_rng(13).random(img.shape)
    # the total loss of Sec. 3.3: an image term (here sum w . image) plus the
    # weighted regularisers of the vertex materials, the Gaussians' mesh
    # distance, the vertex displacements and the scales
    reg = ref64.regularisers(attrs[0:5], s["knn_v"], pos64, s["verts"].astype(np.float64), idx,
                             dxv, ls64)
    total = (img * torch.tensor(wimg)).sum() + reg[4]
    total.backward()

    # ---- GPU: the same composition through the C ABI
    d = render.upload(s)
    R = render.Renderer(s, d)
    M = render.VertexModel(R, torch.tensor(inp["freqs"]).cuda(), torch.tensor(joints).cuda(),
                           torch.tensor(parents).cuda())
    dev = lambda a: torch.tensor(np.ascontiguousarray(a)).cuda()
    v = dict(theta=dev(theta), mlp=dev(params), v_albedo=dev(v_alb), v_rough=dev(v_rough),
             v_tint=dev(v_tint), pos=d["pos"], nrm=d["nrm"], quat=d["quat"], log_s=d["log_s"],
             opac=d["opac"], env=d["env"])
    image, _, ctx = M.forward(v, dev(cnt))
    assert np.abs(image.cpu().numpy().reshape(3, -1) - img.detach().numpy()).max() < 2e-5
    loss = torch.full((1,), 0.25, device="cuda")
    g = M.backward(v, ctx, dev(wimg.reshape(image.shape).astype(np.float32)), loss=loss)
    torch.cuda.synchronize()
    terms = ctx["reg_terms"].cpu().numpy()
    want = np.array([float(t) for t in reg])
    print(f"[vertex-model]   regulariser terms {terms} vs {want}", flush=True)
    assert np.all(np.abs(terms - want) <= 2e-6 * np.abs(want) + 1e-7)
    assert abs(float(loss.cpu()[0]) - (0.25 + want[4])) <= 2e-6 * (0.25 + abs(want[4]))
    for name, ref in (("theta", th64), ("mlp", mlp64), ("v_albedo", alb64), ("v_rough", ro64),
                      ("v_tint", ti64), ("pos", pos64), ("log_s", ls64)):
        r = ref.grad.numpy()
        got = g[name].cpu().numpy().astype(np.float64).reshape(r.shape)
        helpers.check_grad(name, got, r, rtol=1e-4, tag="[vertex-model] ")
