"""The live-pair tape of the shading (Sec. 3.1 rendering equation, App.
A BRDF): shade_gaussians records, per Gaussian, the live (direction,
visibility) pairs it summed (the FP32 walk; the BF16X3 form's MFMA forward
too, tested last), and shade_gaussians_backward replays them
instead of testing every direction again.  The adjoint with the tape
matches the adjoint without it (per-Gaussian gradients to 1e-6 relative,
the environment gradient, summed with LDS atomics in either case, to 1e-5)
on small scenes over several view grids (the walk split over the XCDs or
not, Gaussians with more than K/2 live pairs), at the avatar workload, and
against the FP64 oracle; the colours are unchanged by recording; the tape's
counts are the numbers of directions with n.w > 0 and visibility > 0;
misuse is refused."""

import numpy as np
import pytest
import torch

from oracle import cpu, ref64
from paper_2407_10707_amd import render, rga, synth
from tests import helpers

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _close(a, b, rtol):
    a, b = host(a).astype(np.float64), host(b).astype(np.float64)
    scale = np.abs(b).max() + 1e-30
    err = np.abs(a - b).max() / scale
    return err <= rtol, err


def _compare(args, campos, n, he, we, seed):
    tape = rga.shade_tape(n, he, we, "cuda")
    c0, f0 = rga.shade_gaussians(*args, campos)
    c1, f1 = rga.shade_gaussians(*args, campos, tape=tape)
    assert torch.equal(c0, c1) and torch.equal(f0, f1)
    w = dev(np.random.default_rng(seed).uniform(-1, 1, (3, n)).astype(np.float32))
    g0 = rga.shade_gaussians_backward(*args, campos, c0, f0, w)
    g1 = rga.shade_gaussians_backward(*args, campos, c0, f0, w, tape=tape)
    for k in ("dx", "dn", "dalbedo", "drough", "dtint"):
        ok, err = _close(g1[k], g0[k], 1e-6)
        print(f"  {k:8s} max err / max |g| {err:.1e}", flush=True)
        assert ok, (k, err)
    ok, err = _close(g1["denv"], g0["denv"], 1e-5)
    assert ok, ("denv", err)
    return tape, c1, f1, g1


@pytest.mark.parametrize("n,grid", [(300, (16, 32, 16, 16)), (704, (16, 32, 16, 32)),
                                    (703, (8, 16, 4, 8)), (1, (4, 8, 4, 8)),
                                    (257, (32, 64, 32, 32))])
def test_tape_replay_matches_the_walk(n, grid):
    he, we, hv, wv = grid
    print(f"[tape] n={n} grid={grid}", flush=True)
    s = synth.micro_scene(43, n, 40, 48, he=he, we=we, hv=hv, wv=wv)
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    _, _, cnt = helpers.oracle_visibility(s)
    campos = s["cam"].centre.astype(np.float32)
    args = (dev(xo), dev(no), dev(s["albedo"]), dev(s["rough"]), dev(s["tint"]), dev(s["vidx"]),
            dev(s["vw"]), dev(cnt), s["kv"], he, we, hv, wv, dev(s["env"]))
    tape, col, fr, g = _compare(args, campos, n, he, we, n)
    # the counts: directions with n.w > 0 and interpolated visibility > 0,
    # for the front-facing Gaussians (FP64 decisions; a direction within
    # rounding of the horizon may go either way)
    counts = host(tape[:4 * n].view(torch.int32))
    dirs, _ = ref64.env_geometry(he, we)
    vk = ref64.texel_view(he, we, hv, wv).numpy()
    nn = no.astype(np.float64) / np.linalg.norm(no, axis=0)
    ci = dirs.numpy() @ nn                                          # [K, n]
    vis = sum(s["vw"][j][None, :] * cnt[s["vidx"][j]][:, vk].T for j in range(3))
    live = (ci > 0) & (vis > 0)
    front = host(fr).astype(bool)
    near = (np.abs(ci) < 1e-5).sum(0)
    want = np.where(front, live.sum(0), 0)
    assert np.all(np.abs(counts - want) <= near), np.abs(counts - want).max()
    if he * we >= 512:                 # several groups of 64 pairs per Gaussian
        assert counts.max() > 64
    # and the taped adjoint against the FP64 oracle
    c64 = campos.astype(np.float64)
    w = np.random.default_rng(n).uniform(-1, 1, (3, n)).astype(np.float32)
    ecol, _ = ref64.shade(ref64.t64(xo), ref64.t64(no), s["albedo"], s["rough"], s["tint"],
                          s["vidx"], s["vw"], cnt, s["kv"], he, we, hv, wv, s["env"], c64,
                          front.astype(np.uint8))
    w[np.abs(ecol.numpy() - 0.04045) <= 2e-5 * 0.04045] = 0.0
    g = rga.shade_gaussians_backward(*args, campos, col, fr, dev(w), tape=tape)
    leaves = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True)
              for k, v in (("x", xo), ("n", no), ("albedo", s["albedo"]), ("rough", s["rough"]),
                           ("tint", s["tint"]), ("env", s["env"]))}
    e2, _ = ref64.shade(leaves["x"], leaves["n"], leaves["albedo"], leaves["rough"],
                        leaves["tint"], s["vidx"], s["vw"], cnt, s["kv"], he, we, hv, wv,
                        leaves["env"], c64, front.astype(np.uint8))
    (e2 * torch.tensor(w.astype(np.float64))).sum().backward()
    for gk, lk in (("dx", "x"), ("dn", "n"), ("dalbedo", "albedo"), ("drough", "rough"),
                   ("dtint", "tint"), ("denv", "env")):
        helpers.check_grad(lk, host(g[gk]), leaves[lk].grad.numpy())


def test_tape_at_the_avatar_workload():
    s = synth.make_scene(2)
    print(f"[tape] avatar n={s['n']}", flush=True)
    d, _ = render.layout_by_vertex(render.upload(s))
    R = render.Renderer(s, d)
    p = {k: d[k] for k in render.TRAINABLE}
    count = R.visibility()
    xo, no, _ = rga.lbs_skin(d["skin"], d["jidx"], d["jw"], p["pos"], p["nrm"])
    args = (xo, no, p["albedo"], p["rough"], p["tint"], d["vidx"], d["vw"], count, s["kv"],
            s["he"], s["we"], s["hv"], s["wv"], p["env"])
    tape, _, fr, _ = _compare(args, R.cam_pos, s["n"], s["he"], s["we"], 11)
    counts = host(tape[:4 * s["n"]].view(torch.int32))
    assert np.all(counts[host(fr) == 0] == 0)
    print(f"  live pairs {counts.sum()} of {int(host(fr).sum()) * s['he'] * s['we']} tested",
          flush=True)


def test_tape_refused_when_misused():
    s = synth.micro_scene(3, 50, 32, 32)
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    _, _, cnt = helpers.oracle_visibility(s)
    campos = s["cam"].centre.astype(np.float32)
    args = (dev(xo), dev(no), dev(s["albedo"]), dev(s["rough"]), dev(s["tint"]), dev(s["vidx"]),
            dev(s["vw"]), dev(cnt), s["kv"], s["he"], s["we"], s["hv"], s["wv"], dev(s["env"]))
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(rga.RgaError, match="tape"):
        rga.shade_gaussians(*args, campos, tape=small)
    tape = rga.shade_tape(50, s["he"], s["we"], "cuda")
    with pytest.raises(rga.RgaError, match="aligned"):
        rga.shade_gaussians(*args, campos, tape=tape[1:])


def test_renderer_frames_with_and_without_tape():
    """A training frame records the tape and its adjoint replays it; a
    display frame records none and its adjoint tests every direction: the
    gradients agree."""
    s = synth.micro_scene(17, 400, 64, 64, he=16, we=32, hv=16, wv=32)
    d, _ = render.layout_by_vertex(render.upload(s))
    R = render.Renderer(s, d)
    p = {k: d[k] for k in render.TRAINABLE}
    _, _, cnt = helpers.oracle_visibility(s)
    count = dev(cnt)
    w = dev(np.random.default_rng(2).random((3, s["height"], s["width"])).astype(np.float32))
    img1, _, ctx1 = R.forward(p, count)
    assert ctx1["tape"] is not None
    g1 = R.backward(p, ctx1, w)
    img2, _, ctx2 = R.forward(p, count, for_backward=False)
    assert ctx2["tape"] is None
    g2 = R.backward(p, ctx2, w)
    assert torch.equal(img1, img2)
    for k in render.TRAINABLE:
        ok, err = _close(g1[k], g2[k], 1e-5)
        print(f"  {k:8s} {err:.1e}", flush=True)
        assert ok, (k, err)


@pytest.mark.parametrize("grid", [(16, 32, 16, 16), (16, 32, 16, 32), (6, 16, 6, 16)])
def test_bf16x3_forward_tape(grid):
    """The BF16X3 form's MFMA forward writes the same tape (its pairs in step
    order; texel patches or not): its colours are unchanged by recording,
    its counts are those of the FP32 walk up to directions within rounding
    of the horizon, and the replay of its tape (the adjoint given one)
    matches the FP32 form's replay and the FP64 oracle."""
    he, we, hv, wv = grid
    n = 500
    print(f"[tape] bf16x3 grid={grid}", flush=True)
    s = synth.micro_scene(47, n, 40, 48, he=he, we=we, hv=hv, wv=wv)
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    _, _, cnt = helpers.oracle_visibility(s)
    campos = s["cam"].centre.astype(np.float32)
    args = (dev(xo), dev(no), dev(s["albedo"]), dev(s["rough"]), dev(s["tint"]), dev(s["vidx"]),
            dev(s["vw"]), dev(cnt), s["kv"], he, we, hv, wv, dev(s["env"]))
    tb = rga.shade_tape(n, he, we, "cuda")
    tf = rga.shade_tape(n, he, we, "cuda")
    c0, f0 = rga.shade_gaussians(*args, campos, precision="bf16x3")
    cb, fb = rga.shade_gaussians(*args, campos, precision="bf16x3", tape=tb)
    assert torch.equal(c0, cb) and torch.equal(f0, fb)
    cf, ff = rga.shade_gaussians(*args, campos, tape=tf)
    assert torch.equal(ff, fb)
    nb = host(tb[:4 * n].view(torch.int32))
    nf = host(tf[:4 * n].view(torch.int32))
    dirs, _ = ref64.env_geometry(he, we)
    nn = no.astype(np.float64) / np.linalg.norm(no, axis=0)
    near = (np.abs(dirs.numpy() @ nn) < 1e-5).sum(0)
    assert np.all(np.abs(nb - nf) <= near), np.abs(nb - nf).max()
    # the pairs themselves: the same (direction, visibility) sets per Gaussian
    K = he * we
    pairs_b = host(tb[256 * ((4 * n + 255) // 256):].view(torch.int32)).reshape(n, K, 2)
    pairs_f = host(tf[256 * ((4 * n + 255) // 256):].view(torch.int32)).reshape(n, K, 2)
    for g in np.nonzero((nb == nf) & (nb > 0))[0][:50]:
        a = sorted(map(tuple, pairs_b[g, :nb[g]]))
        b = sorted(map(tuple, pairs_f[g, :nf[g]]))
        assert a == b, g
    w = np.random.default_rng(5).uniform(-1, 1, (3, n)).astype(np.float32)
    gb = rga.shade_gaussians_backward(*args, campos, cb, fb, dev(w), precision="bf16x3", tape=tb)
    gf = rga.shade_gaussians_backward(*args, campos, cf, ff, dev(w), tape=tf)
    for k in ("dx", "dn", "dalbedo", "drough", "dtint", "denv"):
        ok, err = _close(gb[k], gf[k], 1e-4)
        print(f"  {k:8s} replay of the BF16X3 tape vs the FP32 tape {err:.1e}", flush=True)
        assert ok, (k, err)
    c64 = campos.astype(np.float64)
    ecol, _ = ref64.shade(ref64.t64(xo), ref64.t64(no), s["albedo"], s["rough"], s["tint"],
                          s["vidx"], s["vw"], cnt, s["kv"], he, we, hv, wv, s["env"], c64,
                          host(fb).astype(np.uint8))
    w[np.abs(ecol.numpy() - 0.04045) <= 2e-5 * 0.04045] = 0.0
    gb = rga.shade_gaussians_backward(*args, campos, cb, fb, dev(w), precision="bf16x3", tape=tb)
    leaves = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True)
              for k, v in (("x", xo), ("n", no), ("albedo", s["albedo"]), ("rough", s["rough"]),
                           ("tint", s["tint"]), ("env", s["env"]))}
    e2, _ = ref64.shade(leaves["x"], leaves["n"], leaves["albedo"], leaves["rough"],
                        leaves["tint"], s["vidx"], s["vw"], cnt, s["kv"], he, we, hv, wv,
                        leaves["env"], c64, host(fb).astype(np.uint8))
    (e2 * torch.tensor(w.astype(np.float64))).sum().backward()
    for gk, lk in (("dx", "x"), ("dn", "n"), ("dalbedo", "albedo"), ("drough", "rough"),
                   ("dtint", "tint"), ("denv", "env")):
        helpers.check_grad(lk, host(gb[gk]), leaves[lk].grad.numpy())
