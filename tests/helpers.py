"""Shared test helpers: the FP64 reference forward of the whole path, built
only from the oracle (``oracle.ref64`` for values, ``oracle.cpu`` for the FP32
decisions that must match bit for bit)."""

from __future__ import annotations

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
