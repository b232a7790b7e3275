"""FP64 oracle of the render path -- TEST INFRASTRUCTURE ONLY.

Plain PyTorch CPU operations in float64, written from the paper's equations
with no blocking or fusion.  Gradients of this forward (through
``torch.autograd``) are the reference gradients; finite differences of the
same forward pin them.  Only ``tests/``, the smoke check and the CPU baseline
of the benchmark use this module.

Integer decisions whose FP32 result is compared bit for bit (the back-face
flag, tile lists) come from the FP32 mirror in ``rga_oracle.c``; this module
takes the back-face flag as an input so that both oracles agree on which
Gaussians exist.
"""

from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

f64 = torch.float64


def t64(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(f64)
    return torch.as_tensor(np.asarray(a), dtype=f64)


# ---------------------------------------------------------------------------
# Sec. 3.1, deformation: forward linear blend skinning.
# x' = sum_j w_j (R_j x + t_j); the linear part A = sum_j w_j R_j carries the
# normal (n' = A n) and the covariance factor (A R S).
# ---------------------------------------------------------------------------
def lbs(skin, jidx, jw, x, nrm=None):
    """skin [J,12] (rows [R|t]); jidx, jw [4,n]; x, nrm [3,n] -> x', n', A [9,n]."""
    S = t64(skin).reshape(-1, 3, 4)
    jidx = torch.as_tensor(np.asarray(jidx), dtype=torch.long)
    jw = t64(jw)
    x = t64(x) if not isinstance(x, torch.Tensor) else x
    Rsel = S[jidx][..., :3]                      # [4,n,3,3]
    tsel = S[jidx][..., 3]                       # [4,n,3]
    A = torch.einsum("jn,jnab->nab", jw, Rsel)   # [n,3,3]
    t = torch.einsum("jn,jna->na", jw, tsel)     # [n,3]
    xp = torch.einsum("nab,bn->an", A, x) + t.T
    npr = None
    if nrm is not None:
        npr = torch.einsum("nab,bn->an", A, nrm)
    return xp, npr, A.reshape(-1, 9).T


# ---------------------------------------------------------------------------
# The pose theta (72 = 24 joints x axis-angle, Sec. 3.1 attributes) and the
# skinning matrices it gives (the quantity pose optimisation of Sec. 3.3
# differentiates).  Reading: SMPL-style forward kinematics on a skeleton of
# rest joint positions J and parents (parent index below the child's):
# R_j = exp([theta_j]x) (Rodrigues), G_j = G_parent R_j,
# P_j = P_parent + G_parent (J_j - J_parent) (G_root = R_root, P_root = J_root),
# skin_j = [G_j | P_j - G_j J_j].
# ---------------------------------------------------------------------------
def rodrigues(theta):
    """theta [J, 3] axis-angle -> R [J, 3, 3]."""
    th = t64(theta)
    t2 = (th * th).sum(dim=1)
    small = t2 < 1e-12                  # the series (no square root near 0)
    ts = torch.sqrt(torch.where(small, torch.ones_like(t2), t2))
    a = torch.where(small, 1.0 - t2 / 6.0, torch.sin(ts) / ts)
    b = torch.where(small, 0.5 - t2 / 24.0, (1.0 - torch.cos(ts)) / (ts * ts))
    z = torch.zeros_like(t2)
    K = torch.stack([torch.stack([z, -th[:, 2], th[:, 1]], -1),
                     torch.stack([th[:, 2], z, -th[:, 0]], -1),
                     torch.stack([-th[:, 1], th[:, 0], z], -1)], 1)
    eye = torch.eye(3, dtype=f64).expand(th.shape[0], 3, 3)
    return eye + a[:, None, None] * K + b[:, None, None] * (K @ K)


def pose_to_skin(theta, joints, parents):
    """theta [J*3], joints [J, 3] rest positions, parents [J] -> skin [J, 12]."""
    J = len(parents)
    R = rodrigues(t64(theta).reshape(J, 3))
    Jt = t64(joints)
    G, P = [None] * J, [None] * J
    for j in range(J):
        p = int(parents[j])
        if p < 0:
            G[j], P[j] = R[j], Jt[j]
        else:
            G[j] = G[p] @ R[j]
            P[j] = P[p] + G[p] @ (Jt[j] - Jt[p])
    rows = [torch.cat([G[j], (P[j] - G[j] @ Jt[j])[:, None]], dim=1).reshape(12) for j in range(J)]
    return torch.stack(rows)


# ---------------------------------------------------------------------------
# Sec. 3.1: the environment map is a lat-long grid of He x We area lights.
# Texel (r, c): polar angle (r + 1/2) pi / He from +Y, azimuth (c + 1/2) 2 pi / We;
# its area A is the exact solid angle of the texel.
# ---------------------------------------------------------------------------
def env_geometry(he: int, we: int):
    r = torch.arange(he, dtype=f64)
    c = torch.arange(we, dtype=f64)
    th = (r + 0.5) * math.pi / he
    ph = (c + 0.5) * 2.0 * math.pi / we
    TH, PH = torch.meshgrid(th, ph, indexing="ij")
    dirs = torch.stack([torch.sin(TH) * torch.sin(PH), torch.cos(TH),
                        torch.sin(TH) * torch.cos(PH)], dim=-1).reshape(-1, 3)
    band = (2.0 * math.pi / we) * (torch.cos(r * math.pi / he) - torch.cos((r + 1) * math.pi / he))
    solid = band[:, None].expand(he, we).reshape(-1)
    return dirs, solid


def texel_view(he: int, we: int, hv: int, wv: int) -> torch.Tensor:
    """View used for texel (r, c) when the visibility views form a coarser
    Hv x Wv lat-long grid that divides the He x We map."""
    r = torch.arange(he)[:, None].expand(he, we)
    c = torch.arange(we)[None, :].expand(he, we)
    return ((r * hv) // he * wv + (c * wv) // we).reshape(-1)


# ---------------------------------------------------------------------------
# App. A: simplified Disney BRDF (Karis' real-time forms).
# ---------------------------------------------------------------------------
F0 = 0.04


def ggx_d(nh, alpha):
    a2 = alpha * alpha
    return a2 / (math.pi * (nh * nh * (a2 - 1.0) + 1.0) ** 2)


def fresnel(oh):
    return F0 + (1.0 - F0) * torch.pow(torch.as_tensor(2.0, dtype=f64),
                                       (-5.55473 * oh - 6.98316) * oh)


def smith_g1(x, k):
    return x / (x * (1.0 - k) + k)


def brdf(wi, wo, n, albedo, gamma, tint):
    """R(w_i, w_o, n) of App. A for unit vectors [...,3]; albedo [...,3]."""
    h = wi + wo
    h = h / torch.linalg.norm(h, dim=-1, keepdim=True)
    ci = (n * wi).sum(-1)
    co = (n * wo).sum(-1)
    nh = (n * h).sum(-1)
    oh = (wo * h).sum(-1)
    alpha = gamma * gamma
    k = (gamma + 1.0) ** 2 / 8.0
    spec = ggx_d(nh, alpha) * fresnel(oh) * smith_g1(ci, k) * smith_g1(co, k) / (4.0 * ci * co)
    return albedo / math.pi + (tint * spec)[..., None]


def srgb_oetf(x):
    """Gamma correction of the output radiance: the sRGB transfer curve."""
    lo = 12.92 * x
    hi = 1.055 * torch.pow(torch.clamp(x, min=0.0031308), 1.0 / 2.4) - 0.055
    return torch.where(x <= 0.0031308, lo, hi)


# ---------------------------------------------------------------------------
# Sec. 3.1, rendering equation: L_o = sum_k L^k A^k R v_g[k] max(0, w_i^k . n).
# Sec. 3.2 / Eq. interpolate: v_g[k] = sum_j u_j count[vertex_j][view(k)] / K_v.
# ---------------------------------------------------------------------------
def bf16_round(x):
    """Round to bfloat16 (8 significant bits, round to nearest even) by way
    of FP32, as a GPU rounds an FP32 operand: returned in float64."""
    return t64(x).to(torch.float32).to(torch.bfloat16).to(f64)


def contract(W, E, operands: str = "exact"):
    """The shading contraction sum_k W[g, k] E[k, c] of the rendering
    equation.  ``operands`` emulates the operand precision of a matrix-core
    form, with exact products and an FP64 sum: "exact" (FP64 operands),
    "bf16" (both operands rounded to bfloat16), "bf16x3" (each operand
    split into a bfloat16 high part and the bfloat16 of the FP32 remainder,
    W E ~ W_hi E_hi + W_hi E_lo + W_lo E_hi; Henry, Tang and Heinecke,
    ARITH 2019)."""
    if operands == "exact":
        return W @ E
    W32, E32 = t64(W).to(torch.float32), t64(E).to(torch.float32)
    Wh, Eh = bf16_round(W32), bf16_round(E32)
    if operands == "bf16":
        return Wh @ Eh
    if operands == "bf16x3":
        Wl = bf16_round(W32.to(f64) - Wh)
        El = bf16_round(E32.to(f64) - Eh)
        return Wh @ Eh + Wh @ El + Wl @ Eh
    raise ValueError(operands)


def shade(xp, npr, albedo, rough, tint, vidx, vw, count, kv, he, we, hv, wv, env, cam_pos,
          front, chunk: int = 4096, operands: str = "exact"):
    """Returns (colour [3,n], L_o [3,n]) in float64.  ``front`` [n] (0/1) is the
    FP32 back-face decision; non-front Gaussians get colour 0.  ``operands``
    selects the emulated operand precision of the contraction (`contract`)."""
    xp, npr, albedo, rough, tint = (t64(v) for v in (xp, npr, albedo, rough, tint))
    n = xp.shape[1]
    dirs, solid = env_geometry(he, we)
    vk = texel_view(he, we, hv, wv)
    env = t64(env)
    E = env * solid[:, None]                                      # [K,3]
    count = torch.as_tensor(np.asarray(count), dtype=f64)         # [nv,V]
    vidx = torch.as_tensor(np.asarray(vidx), dtype=torch.long)
    vw = t64(vw)
    cam = t64(cam_pos)
    front = torch.as_tensor(np.asarray(front)).to(torch.bool)
    outs = []
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        nn = npr[:, s:e].T
        nn = nn / torch.linalg.norm(nn, dim=1, keepdim=True)       # [m,3]
        wo = cam[None, :] - xp[:, s:e].T
        wo = wo / torch.linalg.norm(wo, dim=1, keepdim=True)
        vis = sum(vw[j, s:e, None] * count[vidx[j, s:e]][:, vk] for j in range(3)) / kv
        ci = nn @ dirs.T                                           # [m,K]
        live = (ci > 0) & (vis > 0)
        ci_s = torch.where(live, ci, torch.ones_like(ci))
        co = (nn * wo).sum(1).clamp(min=1e-300)[:, None]
        h = dirs[None, :, :] + wo[:, None, :]
        h = h / torch.linalg.norm(h, dim=-1, keepdim=True)
        nh = (h * nn[:, None, :]).sum(-1)
        oh = (h * wo[:, None, :]).sum(-1)
        g = rough[s:e, None]
        alpha = g * g
        k = (g + 1.0) ** 2 / 8.0
        spec = ggx_d(nh, alpha) * fresnel(oh) * smith_g1(ci_s, k) * smith_g1(co, k) / (4.0 * ci_s * co)
        wgt = torch.where(live, vis * ci_s, torch.zeros_like(ci))  # v * max(0, w.n)
        diff_sum = contract(wgt, E, operands)                      # [m,3]
        spec_sum = contract(wgt * spec, E, operands)
        Lo = albedo[:, s:e].T / math.pi * diff_sum + tint[s:e, None] * spec_sum
        Lo = torch.where(front[s:e, None], Lo, torch.zeros_like(Lo))
        outs.append(Lo)
    Lo = torch.cat(outs, 0).T
    col = torch.where(front[None, :], srgb_oetf(Lo), torch.zeros_like(Lo))
    return col, Lo


# ---------------------------------------------------------------------------
# Splatting (the 3DGS method): EWA projection, front-to-back compositing.
# ---------------------------------------------------------------------------
def quat_to_rot(q):
    """q [4,n] (w, x, y, z), normalised here -> [n,3,3]."""
    q = q / torch.linalg.norm(q, dim=0, keepdim=True)
    w, x, y, z = q
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def project(cam, xp, A, quat, log_s, opac, front):
    """Camera-space projection of every Gaussian.  Returns a dict with mean2d
    [2,n], conic [3,n] (A, B, C of the inverse covariance), sigma [3,n] (the
    2D covariance a, b, c), depth [n] and valid [n] (bool)."""
    R = t64(cam.R)
    tc = t64(cam.t)
    Xc = R @ xp + tc[:, None]
    X, Y, Z = Xc
    front = torch.as_tensor(np.asarray(front)).to(torch.bool)
    valid = (Z > 0.2) & front & (opac >= 1.0 / 255.0)
    Zs = torch.where(valid, Z, torch.ones_like(Z))
    s = torch.exp(log_s)                                          # [3,n]
    Rq = quat_to_rot(quat)                                        # [n,3,3]
    Am = A.T.reshape(-1, 3, 3)
    M = Am @ Rq * s.T[:, None, :]                                 # A R diag(s)
    V = R[None] @ M
    zero = torch.zeros_like(Zs)
    J = torch.stack([torch.stack([cam.fx / Zs, zero, -cam.fx * X / Zs ** 2], -1),
                     torch.stack([zero, cam.fy / Zs, -cam.fy * Y / Zs ** 2], -1)], -2)
    T = J @ V                                                     # [n,2,3]
    Sig = T @ T.transpose(1, 2)
    a = Sig[:, 0, 0] + 0.3
    b = Sig[:, 0, 1]
    c = Sig[:, 1, 1] + 0.3
    det = a * c - b * b
    valid = valid & (det > 0)
    dets = torch.where(valid, det, torch.ones_like(det))
    conic = torch.stack([c / dets, -b / dets, a / dets])
    mean2d = torch.stack([cam.fx * X / Zs + cam.cx, cam.fy * Y / Zs + cam.cy])
    return dict(mean2d=mean2d, conic=conic, sigma=torch.stack([a, b, c]), depth=Z, valid=valid)


def composite(cam, proj, opac, color, pixels: Optional[np.ndarray] = None):
    """Front-to-back alpha compositing over Gaussians in (depth, index) order.

    Per pixel centre p: alpha = min(0.99, o exp(-d^T Conic d / 2)), d = mean - p;
    skip if the exponent is positive or alpha < 1/255; stop before the entry
    that takes the transmittance below 1e-4; C = sum c alpha T, T_final = T.
    Black background.  Only pixels inside a Gaussian's alpha >= 1/255 ellipse
    box can receive it, so (pixel, Gaussian) pairs are enumerated from those
    boxes; ``pixels`` optionally restricts to a subset of flat pixel indices.
    Returns (image [3, P], T_final [P]) where P = H*W or len(pixels).
    """
    H, W = cam.height, cam.width
    valid = proj["valid"]
    gid = torch.nonzero(valid).flatten()
    if pixels is None:
        pix_list = None
        P = H * W
    else:
        pix_list = torch.as_tensor(np.asarray(pixels), dtype=torch.long)
        P = len(pix_list)
    if len(gid) == 0:
        return torch.zeros(3, P, dtype=f64), torch.ones(P, dtype=f64)
    depth = proj["depth"].detach()[gid]
    order = torch.argsort(depth, stable=True)          # ties keep index order
    rank = torch.empty_like(order)
    rank[order] = torch.arange(len(order))
    m = proj["mean2d"].detach()[:, gid]
    sig = proj["sigma"].detach()[:, gid]
    o = opac.detach()[gid]
    r2 = 2.0 * torch.log(255.0 * o)
    hx = torch.sqrt(r2 * sig[0]) + 1.0
    hy = torch.sqrt(r2 * sig[2]) + 1.0
    x0 = torch.clamp(torch.floor(m[0] - hx - 0.5), 0, W - 1).long()
    x1 = torch.clamp(torch.ceil(m[0] + hx - 0.5), 0, W - 1).long()
    y0 = torch.clamp(torch.floor(m[1] - hy - 0.5), 0, H - 1).long()
    y1 = torch.clamp(torch.ceil(m[1] + hy - 0.5), 0, H - 1).long()
    onscreen = (m[0] + hx > 0) & (m[0] - hx < W) & (m[1] + hy > 0) & (m[1] - hy < H)
    nx = torch.where(onscreen, x1 - x0 + 1, torch.zeros_like(x0))
    ny = torch.where(onscreen, y1 - y0 + 1, torch.zeros_like(y0))
    if pix_list is None:
        cnt = nx * ny
        gi = torch.repeat_interleave(torch.arange(len(gid)), cnt)
        start = torch.cumsum(cnt, 0) - cnt
        local = torch.arange(int(cnt.sum())) - start[gi]
        px = x0[gi] + local % nx[gi]
        py = y0[gi] + local // nx[gi]
        slot = py * W + px
    else:
        # only the requested pixels: test every box against each pixel
        qx, qy = pix_list % W, pix_list // W
        parts = []
        for a in range(0, P, 256):
            b = min(P, a + 256)
            inside = ((qx[a:b, None] >= x0[None]) & (qx[a:b, None] <= x0[None] + nx[None] - 1) &
                      (qy[a:b, None] >= y0[None]) & (qy[a:b, None] <= y0[None] + ny[None] - 1))
            sl, g = torch.nonzero(inside, as_tuple=True)
            parts.append((g, sl + a))
        gi = torch.cat([t[0] for t in parts])
        slot = torch.cat([t[1] for t in parts])
        px, py = qx[slot], qy[slot]
    if len(slot) == 0:
        return torch.zeros(3, P, dtype=f64), torch.ones(P, dtype=f64)
    key = slot * len(gid) + rank[gi]
    srt = torch.argsort(key)
    gi, px, py, slot = gi[srt], px[srt], py[srt], slot[srt]
    g = gid[gi]
    mean = proj["mean2d"][:, g]
    con = proj["conic"][:, g]
    dx = mean[0] - (px.to(f64) + 0.5)
    dy = mean[1] - (py.to(f64) + 0.5)
    q = con[0] * dx * dx + 2.0 * con[1] * dx * dy + con[2] * dy * dy
    power = -0.5 * q
    araw = opac[g] * torch.exp(power)
    alpha = torch.minimum(araw, torch.full_like(araw, 0.99))
    keep = (power <= 0) & (alpha >= 1.0 / 255.0)
    a_eff = torch.where(keep, alpha, torch.zeros_like(alpha))
    l1m = torch.log1p(-a_eff)
    # per-pixel running sums of log(1 - alpha), one padded row per pixel
    seg_start = torch.ones_like(slot, dtype=torch.bool)
    seg_start[1:] = slot[1:] != slot[:-1]
    first = torch.nonzero(seg_start).flatten()
    seg_id = torch.cumsum(seg_start.long(), 0) - 1
    pos = torch.arange(len(slot)) - first[seg_id]
    incl_parts = []
    nseg = len(first)
    lmax_all = int(pos.max()) + 1
    block = max(1, 4_000_000 // lmax_all)
    for b0 in range(0, nseg, block):
        b1 = min(nseg, b0 + block)
        lo = int(first[b0])
        hi = int(first[b1]) if b1 < nseg else len(slot)
        sid = seg_id[lo:hi] - b0
        ps = pos[lo:hi]
        pad = torch.zeros(b1 - b0, lmax_all, dtype=f64)
        pad = pad.index_put((sid, ps), l1m[lo:hi])
        incl_parts.append(torch.cumsum(pad, 1)[sid, ps])
    incl = torch.cat(incl_parts)
    excl = incl - l1m
    T_incl = torch.exp(incl)
    T_excl = torch.exp(excl)
    active = keep & (T_incl >= 1e-4)
    w = torch.where(active, a_eff * T_excl, torch.zeros_like(a_eff))
    img = torch.zeros(3, P, dtype=f64)
    img = img.index_add(1, slot, color[:, g] * w[None, :])
    logT = torch.zeros(P, dtype=f64).index_add(0, slot, torch.where(active, l1m, torch.zeros_like(l1m)))
    return img, torch.exp(logT)


def l1_loss(image, target):
    """Mean absolute error over all 3HW values (the L1 term of the image loss)."""
    return (image - t64(target)).abs().mean()


# ---------------------------------------------------------------------------
# Image loss (Sec. 3.3, image-loss equation): L_img = (1 - lambda) L_1 +
# lambda L_D-SSIM with lambda = 0.2.  Readings (the paper names D-SSIM only):
# SSIM of Wang et al. with an 11 x 11 Gaussian window of std 1.5, C1 = 0.01^2,
# C2 = 0.03^2 (values in [0, 1]), each channel filtered separately with zero
# padding (the window is cut at the border and not renormalised), D-SSIM =
# 1 - the mean of the SSIM map over all channels and pixels.
# ---------------------------------------------------------------------------
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window(size: int = 11, sigma: float = 1.5) -> torch.Tensor:
    t = torch.arange(size, dtype=f64) - (size - 1) / 2.0
    g = torch.exp(-t * t / (2.0 * sigma * sigma))
    return g / g.sum()


def ssim_map(x, y):
    """x, y [C, H, W] -> the SSIM of every channel and pixel [C, H, W]."""
    x, y = t64(x), t64(y)
    C = x.shape[0]
    g = ssim_window()
    w = torch.outer(g, g)[None, None].expand(C, 1, -1, -1)
    pad = (g.numel() - 1) // 2

    def filt(a):
        return torch.nn.functional.conv2d(a[None], w, padding=pad, groups=C)[0]

    mx, my = filt(x), filt(y)
    sxx = filt(x * x) - mx * mx
    syy = filt(y * y) - my * my
    sxy = filt(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / \
        ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def image_loss(x, y, lam: float = 0.2):
    """(1 - lam) mean |x - y| + lam (1 - mean SSIM(x, y))."""
    x, y = t64(x), t64(y)
    return (1.0 - lam) * (x - y).abs().mean() + lam * (1.0 - ssim_map(x, y).mean())


# ---------------------------------------------------------------------------
# Regularisers of the training loss (Sec. 3.3): smoothness of the vertex
# materials over the K_v nearest vertices (L1 of the differences of a, gamma,
# p), distance of each Gaussian to its K_g nearest vertices (Euclidean),
# length of each vertex displacement, and the scale hinge
# sum max(0, s - s_0) with s_0 = 0.005 over every scale component (s =
# exp(log-scale)); the total weights them by lambda_smooth = 0.002,
# lambda_mdist = 0.1, lambda_disp = 0.02, lambda_scale = 10.
# ---------------------------------------------------------------------------
REG_LAMBDAS = (0.002, 0.1, 0.02, 10.0)
REG_S0 = 0.005


def regularisers(mat, knn_v, xg, verts, vidx, disp, log_s, s0=REG_S0, lams=REG_LAMBDAS):
    """mat [5, nv] (albedo rgb, roughness, tint), knn_v [nv, kv], xg [3, n],
    verts [3, nv], vidx [kg, n], disp [3, nv], log_s [3, n] ->
    (smooth, mdist, disp, scale, weighted total)."""
    mat, xg, verts, disp, log_s = t64(mat), t64(xg), t64(verts), t64(disp), t64(log_s)
    kn = torch.as_tensor(np.asarray(knn_v), dtype=torch.long)
    vi = torch.as_tensor(np.asarray(vidx), dtype=torch.long)
    smooth = (mat[:, :, None] - mat[:, kn]).abs().sum()
    dv = xg[:, None, :] - verts[:, vi]                     # [3, kg, n]
    mdist = torch.sqrt((dv * dv).sum(dim=0)).sum()
    dlen = torch.sqrt((disp * disp).sum(dim=0)).sum()
    scale = torch.clamp(torch.exp(log_s) - s0, min=0.0).sum()
    total = lams[0] * smooth + lams[1] * mdist + lams[2] * dlen + lams[3] * scale
    return smooth, mdist, dlen, scale, total


# ---------------------------------------------------------------------------
# Sec. 3.1, interpolation equation: a Gaussian's attribute is the average of
# its K_g nearest canonical vertices' attributes weighted by
# u_j = 1 / ||x_g - x_j||.  The neighbour set comes from the FP32 mirror
# (`cpu.knn`, an integer decision); the weights and the average are taken
# here in FP64 from the same squared distances.  A query that coincides with
# a vertex (distance 0) takes that vertex's attribute (the limit of the
# weights); among several such vertices, the first in (distance, index) order.
# ---------------------------------------------------------------------------
def knn_weights(d2):
    """d2 [k,n] squared distances in (distance, index) order -> w [k,n]."""
    d2 = t64(d2)
    k = d2.shape[0]
    zero = d2[0] == 0
    u = 1.0 / torch.sqrt(torch.where(zero[None].expand(k, -1), torch.ones_like(d2), d2))
    w = u / u.sum(dim=0, keepdim=True)
    first = torch.zeros_like(d2)
    first[0] = 1.0
    return torch.where(zero[None].expand(k, -1), first, w)


def interpolate(idx, w, attr):
    """idx [k,n] vertex indices, w [k,n], attr [C,nv] -> [C,n]: sum_t w_t attr[:, idx_t]."""
    idx = torch.as_tensor(np.asarray(idx), dtype=torch.long)
    w = t64(w)
    attr = t64(attr)
    out = torch.zeros(attr.shape[0], idx.shape[1], dtype=f64)
    for t in range(idx.shape[0]):
        out = out + w[t][None] * attr[:, idx[t]]
    return out


# ---------------------------------------------------------------------------
# Sec. 3.1 (attributes) and Sec. 3.5 (implementation details): the pose-
# dependent vertex displacement dx = d(x, theta), an MLP of four hidden
# layers of width 256 with ReLU, whose coordinate input goes through random
# Fourier features.  Readings (the paper gives neither the encoding's size
# nor how the pose enters): gamma(x) = [sin(2 pi B x), cos(2 pi B x)] with a
# fixed B [64, 3]; the network input is [gamma(x), theta] (128 + 72 = 200);
# layers h_l = relu(W_l h_{l-1} + b_l), l = 1..4, and a linear output
# dx = W_5 h_4 + b_5 (3).  Parameters are one flat vector in the order
# W_1 [256, 200], b_1, W_2 [256, 256], b_2, W_3, b_3, W_4, b_4, W_5 [3, 256], b_5.
# ---------------------------------------------------------------------------
MLP_FREQS = 64
MLP_POSE = 72
MLP_WIDTH = 256
MLP_SHAPES = [(MLP_WIDTH, 2 * MLP_FREQS + MLP_POSE), (MLP_WIDTH, MLP_WIDTH),
              (MLP_WIDTH, MLP_WIDTH), (MLP_WIDTH, MLP_WIDTH), (3, MLP_WIDTH)]


def mlp_param_count(shapes=MLP_SHAPES) -> int:
    return sum(o * i + o for o, i in shapes)


def mlp_unpack(params, shapes=MLP_SHAPES):
    """Flat parameter vector -> [(W_l, b_l)] in layer order."""
    p = t64(params)
    out, o = [], 0
    for n_out, n_in in shapes:
        W = p[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = p[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == p.numel()
    return out


def rff(x, freqs):
    """x [3, n], freqs B [m, 3] -> gamma [2m, n] = [sin(2 pi B x); cos(2 pi B x)]."""
    f = 2.0 * math.pi * (t64(freqs) @ t64(x))
    return torch.cat([torch.sin(f), torch.cos(f)], dim=0)


def mlp_layers(x, freqs, theta, layers):
    """Pre-activations z_l [out_l, n] of every layer and the output dx [3, n].

    The pose is the same for every vertex: it is appended to each column of
    the encoded coordinates."""
    g = rff(x, freqs)
    th = t64(theta).reshape(-1, 1).expand(-1, g.shape[1])
    h = torch.cat([g, th], dim=0)
    zs = []
    for li, (W, b) in enumerate(layers):
        z = W @ h + b[:, None]
        zs.append(z)
        h = torch.relu(z) if li + 1 < len(layers) else z
    return zs, h


def displacement(x, freqs, theta, params):
    """d(x, theta) for every column of x: [3, n]."""
    return mlp_layers(x, freqs, theta, mlp_unpack(params))[1]


def mean_displacement(x, freqs, thetas, params):
    """Average displacement over a set of poses (used for novel poses)."""
    return torch.stack([displacement(x, freqs, th, params) for th in thetas]).mean(dim=0)


# ---------------------------------------------------------------------------
# The optimiser of the training loop.  Reading: the paper trains as 3DGS
# does, with Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v +
# (1 - b2) g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
# ---------------------------------------------------------------------------
def adam_step(p, g, m, v, lr, b1, b2, eps, t):
    """One Adam step at step number t (1-based) -> (p, m, v)."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
