"""Shared test helpers: the FP64 reference forward of the whole path, built
only from the oracle (``oracle.ref64`` for values, ``oracle.cpu`` for the FP32
decisions that must match bit for bit)."""

from __future__ import annotations

import math

import numpy as np
import torch

from oracle import cpu, ref64

PARAM_NAMES = ("pos", "nrm", "quat", "log_s", "opac", "albedo", "rough", "tint", "env")


def oracle_visibility(s):
    """Posed mesh (FP32 mirror LBS) -> raw bits, counts."""
    vx, _, _ = cpu.lbs_f32(s["skin"], s["mesh_jidx"], s["mesh_jw"], s["verts"])
    raw, cnt = cpu.mesh_visibility(vx, s["faces"], s["view_dirs"], s["vis_res"], s["knn_v"])
    return vx, raw, cnt


def front_flags(s):
    xo, no, _ = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    return cpu.front_f32(xo, no, s["cam"].centre.astype(np.float32))


def params64(s, requires_grad=False):
    p = {k: torch.tensor(np.asarray(s[k], dtype=np.float64), requires_grad=requires_grad)
         for k in PARAM_NAMES}
    return p


def render64(s, p, count, front, pixels=None, return_parts=False):
    """FP64 forward of the full path: LBS -> shading -> projection ->
    compositing.  ``front`` (FP32 decision) is held fixed."""
    xp, npr, A = ref64.lbs(s["skin"], s["jidx"], s["jw"], p["pos"], p["nrm"])
    col, Lo = ref64.shade(xp, npr, p["albedo"], p["rough"], p["tint"], s["vidx"], s["vw"], count,
                          s["kv"], s["he"], s["we"], s["hv"], s["wv"], p["env"],
                          s["cam"].centre, front)
    proj = ref64.project(s["cam"], xp, A, p["quat"], p["log_s"], p["opac"], front)
    img, T = ref64.composite(s["cam"], proj, p["opac"], col, pixels=pixels)
    if return_parts:
        return img, T, dict(xp=xp, npr=npr, A=A, col=col, Lo=Lo, proj=proj)
    return img, T


def oracle_frame_f32(s, color):
    """FP32-mirror projection, binning and tiled compositing of a frame whose
    shaded colours are given."""
    xo, no, Ao = cpu.lbs_f32(s["skin"], s["jidx"], s["jw"], s["pos"], s["nrm"])
    front = cpu.front_f32(xo, no, s["cam"].centre.astype(np.float32))
    pre = cpu.splat_preprocess(s["cam"], xo, Ao, s["quat"], s["log_s"], s["opac"], front)
    keys, vals, ranges = cpu.splat_bin(s["cam"], pre)
    img, T, margin = cpu.composite_tiles(s["cam"], ranges, vals, pre, s["opac"], color)
    return dict(xo=xo, no=no, Ao=Ao, front=front, pre=pre, keys=keys, vals=vals, ranges=ranges,
                img=img, T=T, margin=margin)


def check_grad(name, got, ref, rtol=1e-4, floor=1e-3, rel_l2=1e-4, tag=""):
    """Per-element and per-tensor check of a GPU gradient against the FP64
    oracle's: |g - g64| <= rtol |g64| + floor RMS(g64) for every element and
    ||g - g64|| <= rel_l2 ||g64||.  Prints the worst ratios."""
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    rms = float(np.sqrt(np.mean(ref * ref))) if ref.size else 0.0
    err = np.abs(got - ref)
    lim = rtol * np.abs(ref) + floor * rms + 1e-300
    rl2 = float(np.linalg.norm(got - ref) / (np.linalg.norm(ref) + 1e-300))
    worst = float((err / lim).max()) if ref.size else 0.0
    print(f"  {tag}{name:8s} relL2={rl2:.2e} worst err/limit={worst:.3f}", flush=True)
    assert worst <= 1.0, (name, worst, int((err > lim).sum()))
    assert rl2 <= rel_l2, (name, rl2)


def subscene(s, sub):
    """The scene restricted to the Gaussians `sub` (mesh, camera and
    environment unchanged)."""
    out = dict(s)
    for k in ("pos", "nrm", "quat", "log_s", "albedo", "jidx", "jw", "vidx", "vw"):
        out[k] = np.ascontiguousarray(s[k][:, sub])
    for k in ("opac", "rough", "tint"):
        out[k] = np.ascontiguousarray(s[k][sub])
    out["n"] = len(sub)
    return out


GAUSS_PARAMS = ("pos", "nrm", "quat", "log_s", "opac", "albedo", "rough", "tint")


class LocalFD:
    """Central finite differences of L = sum(w * image) through the FP64
    oracle's whole chain (render64), evaluated cheaply but exactly:

    * a parameter of Gaussian g changes only g's skinned state, colour and
      projection (each computed per Gaussian) and the pixels inside g's
      compositing box (alpha < 1/255 outside it, so they never see g); the
      difference L(p + h e) - L(p - h e) is therefore the difference of the
      loss over those pixels, composited with every Gaussian;
    * an environment texel changes every colour: the whole frame is
      re-shaded and re-composited.
    `fd(name, flat_index, h)` returns (L(+h) - L(-h)) / 2h."""

    def __init__(self, s, count, front, w):
        self.s, self.count, self.front = s, count, np.asarray(front)
        self.w = torch.as_tensor(np.asarray(w, dtype=np.float64).reshape(3, -1))
        self.p = params64(s)
        with torch.no_grad():
            _, _, parts = render64(s, self.p, count, front, return_parts=True)
        self.base = parts

    def _gauss_state(self, q, g):
        s = self.s
        sl = slice(g, g + 1)
        xp, npr, A = ref64.lbs(s["skin"], s["jidx"][:, sl], s["jw"][:, sl], q["pos"][:, sl],
                               q["nrm"][:, sl])
        col, _ = ref64.shade(xp, npr, q["albedo"][:, sl], q["rough"][sl], q["tint"][sl],
                             s["vidx"][:, sl], s["vw"][:, sl], self.count, s["kv"], s["he"],
                             s["we"], s["hv"], s["wv"], q["env"], s["cam"].centre,
                             self.front[sl])
        proj = ref64.project(s["cam"], xp, A, q["quat"][:, sl], q["log_s"][:, sl],
                             q["opac"][sl], self.front[sl])
        return col, proj

    def _box(self, g):
        cam = self.s["cam"]
        pr = self.base["proj"]
        if not bool(pr["valid"][g]):
            return np.zeros(0, np.int64)
        m, sig = pr["mean2d"][:, g], pr["sigma"][:, g]
        r2 = 2.0 * math.log(255.0 * float(self.p["opac"][g]))
        hx = math.sqrt(r2 * float(sig[0])) + 3.0
        hy = math.sqrt(r2 * float(sig[2])) + 3.0
        x0, x1 = max(0, math.floor(float(m[0]) - hx)), min(cam.width - 1, math.ceil(float(m[0]) + hx))
        y0, y1 = max(0, math.floor(float(m[1]) - hy)), min(cam.height - 1, math.ceil(float(m[1]) + hy))
        if x0 > x1 or y0 > y1:
            return np.zeros(0, np.int64)
        yy, xx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
        return (yy * cam.width + xx).reshape(-1)

    def _loss_gauss(self, q, g, pix):
        col_g, proj_g = self._gauss_state(q, g)
        col = self.base["col"].clone()
        col[:, g] = col_g[:, 0]
        proj = {k: v.clone() for k, v in self.base["proj"].items()}
        for k in proj:
            proj[k][..., g] = proj_g[k][..., 0]
        img, _ = ref64.composite(self.s["cam"], proj, q["opac"], col, pixels=pix)
        return float((img * self.w[:, pix]).sum())

    def _loss_frame(self, q):
        img, _ = render64(self.s, q, self.count, self.front)
        return float((img * self.w).sum())

    def fd(self, name, idx, h):
        vals = []
        with torch.no_grad():
            if name == "env":
                for sgn in (1.0, -1.0):
                    q = dict(self.p)
                    q["env"] = self.p["env"].clone()
                    q["env"].view(-1)[idx] += sgn * h
                    vals.append(self._loss_frame(q))
            else:
                g = idx % self.s["n"]
                pix = self._box(g)
                if len(pix) == 0:
                    return 0.0
                for sgn in (1.0, -1.0):
                    q = dict(self.p)
                    q[name] = self.p[name].clone()
                    q[name].view(-1)[idx] += sgn * h
                    vals.append(self._loss_gauss(q, g, pix))
        return (vals[0] - vals[1]) / (2.0 * h)
