"""Render-and-train path on top of the C ABI (marshalling only).

Per frame (Sec. 3.1-3.2 of the paper):
  lbs_skin(mesh) -> mesh_visibility          (once per pose, no gradient)
  lbs_skin(Gaussians) -> shade_gaussians -> splat_forward -> image
and the adjoint
  splat_backward -> shade_gaussians_backward (accumulates into dx') ->
  lbs_skin_backward.
Every arithmetic step runs in librga.so; this module only owns buffers.
"""

from __future__ import annotations

from typing import Dict, Optional

import numpy as np
import torch

from . import rga

TRAINABLE = ("pos", "nrm", "quat", "log_s", "opac", "albedo", "rough", "tint", "env")
STATIC_F32 = ("verts", "mesh_jw", "skin", "jw", "vw", "view_dirs", "target")
STATIC_I32 = ("faces", "mesh_jidx", "knn_v", "jidx", "vidx")


def upload(scene: dict, device="cuda") -> Dict[str, torch.Tensor]:
    """Copy a synthetic scene's arrays to the device (float32 / int32)."""
    out = {}
    for k in TRAINABLE + STATIC_F32:
        out[k] = torch.as_tensor(np.ascontiguousarray(scene[k], dtype=np.float32)).to(device)
    for k in STATIC_I32:
        out[k] = torch.as_tensor(np.ascontiguousarray(scene[k], dtype=np.int32)).to(device)
    return out


# the arrays with one column per Gaussian
PER_GAUSSIAN = ("pos", "nrm", "quat", "log_s", "opac", "albedo", "rough", "tint", "jidx", "jw",
                "vidx", "vw")


def layout_by_vertex(d: Dict[str, torch.Tensor]):
    """The device scene with its Gaussians stored grouped by nearest mesh
    vertex: vertex_order (a stable sort by vidx row 0) applied to every
    per-Gaussian array with gather_columns.  Returns (new dict, order) with
    new[k][..., j] = d[k][..., order[j]]; the other arrays are shared.  The
    Gaussians are a set, so this changes no result, only where each one
    lives: the shading kernels then gather count rows that their neighbours
    have just brought into the cache."""
    order = rga.vertex_order(d["vidx"], int(d["verts"].shape[1]))
    out = dict(d)
    for k in PER_GAUSSIAN:
        out[k] = rga.gather_columns(d[k], order)
    return out, order


def scene_in_order(scene: dict, order) -> dict:
    """The host scene with its Gaussians in `order` (as layout_by_vertex
    returns it), so that host-side checks see the device layout."""
    o = np.asarray(order.cpu() if isinstance(order, torch.Tensor) else order, dtype=np.int64)
    out = dict(scene)
    for k in PER_GAUSSIAN:
        out[k] = np.ascontiguousarray(np.asarray(scene[k])[..., o])
    return out


class Renderer:
    """Holds the static inputs and workspaces of one scene/camera."""

    # below this many Gaussians a frame is bound by the host's launches, and
    # the second stream's events cost more than the overlap saves
    OVERLAP_MIN_GAUSSIANS = 16384

    def __init__(self, scene: dict, dev: Dict[str, torch.Tensor], capacity: Optional[int] = None,
                 precision: str = "fp32", overlap: Optional[bool] = None):
        self.s = scene
        self.d = dev
        self.cam = scene["cam"]
        self.cam_pos = [float(v) for v in np.asarray(self.cam.centre, dtype=np.float32)]
        self.n = int(scene["n"])
        self.precision = precision
        cap = capacity if capacity is not None else max(1 << 16, 24 * self.n)
        self.ws = rga.SplatWorkspace(self.n, self.cam.width, self.cam.height, cap,
                                     dev["pos"].device)
        self.vis_ws = None
        self.shade_ws = None
        self.l1_ws = None
        self.img_ws = None
        self.image_loss = False
        # the FP32 shading records its live (Gaussian, direction) pairs on a
        # tape that the adjoint replays instead of testing every direction
        self.tape = None
        # the stream that bins the splats while the shading runs, and the
        # back-face flags it computes for them
        self.side = None
        self.front_bin = None
        self.overlap = (int(scene["n"]) >= self.OVERLAP_MIN_GAUSSIANS) if overlap is None \
            else bool(overlap)
        # every splat_forward on self.ws overwrites the lists and blend state
        # that the adjoint reads: a forward's context records the generation
        # it was rendered in, and a backward of an older forward is refused
        self.generation = 0

    # ------------------------------------------------------------------ per pose
    def visibility(self):
        d, s = self.d, self.s
        vx, _, _ = rga.lbs_skin(d["skin"], d["mesh_jidx"], d["mesh_jw"], d["verts"], None,
                                want_A=False)
        count, _ = rga.mesh_visibility(vx, d["faces"], d["view_dirs"], s["vis_res"], d["knn_v"],
                                       ws=self.vis_ws)
        return count

    def ensure_capacity(self):
        """Synchronises; grows the splat workspace if the last frame overflowed.
        Returns True if the frame must be re-rendered."""
        D = self.ws.count()
        if D > self.ws.capacity:
            self.ws = rga.SplatWorkspace(self.n, self.cam.width, self.cam.height,
                                         int(D * 1.25) + 1024, self.d["pos"].device)
            self.generation += 1
            return True
        return False

    def _splat(self, *args):
        self.generation += 1
        return rga.splat_forward(self.cam, *args, self.ws)

    # ------------------------------------------------------------------ forward
    def forward(self, p: Dict[str, torch.Tensor], count: Optional[torch.Tensor] = None,
                for_backward: bool = True):
        """One frame.  count: the visibility of the current pose
        (mesh_visibility), or None to compute it in this frame.  With
        for_backward (the default) the shading (either form) also records
        the tape its adjoint replays; a frame only for display skips it (a backward of
        such a frame still works: it tests every direction again).

        With overlap (the default from OVERLAP_MIN_GAUSSIANS Gaussians on),
        the splats are binned (back-face flags, projection, sorts, tile
        lists: nothing the colours enter) on a second stream while this
        stream computes the visibility and the shading; the blend waits for
        both.  Every buffer the second stream touches is allocated before
        the fork and this stream joins it before anything else runs.
        Without, splat_forward runs after the shading on this stream."""
        d, s = self.d, self.s
        xo, no, A = rga.lbs_skin(d["skin"], d["jidx"], d["jw"], p["pos"], p["nrm"],
                                 disp=p.get("disp"))
        main = torch.cuda.current_stream(xo.device)
        self.generation += 1
        if self.overlap:
            if self.side is None:
                self.side = torch.cuda.Stream(device=xo.device)
                self.forked, self.binned = torch.cuda.Event(), torch.cuda.Event()
            if self.front_bin is None:
                self.front_bin = torch.empty((self.n,), dtype=torch.uint8, device=xo.device)
            self.forked.record(main)
        # the visibility's launches are queued first: the host then queues
        # the binning's short kernels while the raster runs
        if count is None:
            count = self.visibility()
        if self.overlap:
            self.side.wait_event(self.forked)
            with torch.cuda.stream(self.side):
                rga.back_face(xo, no, self.cam_pos, out=self.front_bin)
                rga.splat_bin(self.cam, xo, A, p["quat"], p["log_s"], p["opac"], self.front_bin,
                              self.ws)
                self.binned.record(self.side)
        tape = None
        if for_backward:
            if self.tape is None:
                self.tape = rga.shade_tape(self.n, s["he"], s["we"], xo.device)
            tape = self.tape
        color, front = rga.shade_gaussians(xo, no, p["albedo"], p["rough"], p["tint"], d["vidx"],
                                           d["vw"], count, s["kv"], s["he"], s["we"], s["hv"],
                                           s["wv"], p["env"], self.cam_pos, self.precision,
                                           tape=tape)
        if self.overlap:
            main.wait_event(self.binned)
            image, T = rga.splat_blend(self.cam, color, self.ws)
        else:
            image, T = rga.splat_forward(self.cam, xo, A, p["quat"], p["log_s"], p["opac"],
                                         color, front, self.ws)
        # the tape, like the splat workspace, holds this forward's state until
        # the next forward (the generation check below covers both)
        ctx = dict(xo=xo, no=no, A=A, color=color, front=front, image=image, count=count,
                   generation=self.generation, ws=self.ws, tape=tape)
        return image, T, ctx

    # ------------------------------------------------------------------ editing maps
    def render_map(self, p: Dict[str, torch.Tensor], count: torch.Tensor, mode: str = "albedo"):
        """The albedo or normal map of the appearance-editing paradigm
        (Sec. 3.4): the same splatting with each Gaussian's colour set to
        its albedo, or to its posed normal (the skinned normal's components,
        as LBS returns them).  The back-face rule of the shading decides
        which Gaussians exist, as in the shaded frame."""
        if mode not in ("albedo", "normal"):
            raise ValueError("mode must be 'albedo' or 'normal'")
        d, s = self.d, self.s
        xo, no, A = rga.lbs_skin(d["skin"], d["jidx"], d["jw"], p["pos"], p["nrm"],
                                 disp=p.get("disp"))
        _, front = rga.shade_gaussians(xo, no, p["albedo"], p["rough"], p["tint"], d["vidx"],
                                       d["vw"], count, s["kv"], s["he"], s["we"], s["hv"],
                                       s["wv"], p["env"], self.cam_pos, self.precision)
        color = p["albedo"] if mode == "albedo" else no
        image, _ = self._splat(xo, A, p["quat"], p["log_s"], p["opac"], color, front)
        return image

    # ------------------------------------------------------------------ backward
    def backward(self, p: Dict[str, torch.Tensor], ctx, dimage: torch.Tensor,
                 want_dA: bool = False):
        d, s = self.d, self.s
        if ctx.get("generation") != self.generation or ctx.get("ws") is not self.ws:
            raise rga.RgaError("splat workspace overwritten since this forward (another "
                               "render on the same Renderer): run backward before the next "
                               "forward, or render again")
        g = rga.splat_backward(self.cam, ctx["xo"], ctx["A"], p["quat"], p["log_s"], p["opac"],
                               ctx["color"], ctx["front"], self.ws, ctx["image"], dimage,
                               want_dA=want_dA)
        sh = rga.shade_gaussians_backward(
            ctx["xo"], ctx["no"], p["albedo"], p["rough"], p["tint"], d["vidx"], d["vw"],
            ctx["count"], s["kv"], s["he"], s["we"], s["hv"], s["wv"], p["env"], self.cam_pos,
            ctx["color"], ctx["front"], g["dcolor"], dx_accum=g["dx"], precision=self.precision,
            ws=self.shade_ws, tape=ctx.get("tape"))
        dpos, dnrm = rga.lbs_skin_backward(d["skin"], d["jidx"], d["jw"], sh["dx"], sh["dn"])
        out = dict(pos=dpos, nrm=dnrm, quat=g["dquat"], log_s=g["dlog_s"], opac=g["dopac"],
                   albedo=sh["dalbedo"], rough=sh["drough"], tint=sh["dtint"], env=sh["denv"],
                   color=g["dcolor"], posed_x=sh["dx"], posed_n=sh["dn"])
        if want_dA:
            out["posed_A"] = g["dA"]
        return out

    def loss(self, image: torch.Tensor, target: torch.Tensor):
        """L1 (the hot path's loss), or with image_loss set the image loss
        of the training section, (1 - 0.2) L1 + 0.2 D-SSIM."""
        if getattr(self, "image_loss", False):
            if self.img_ws is None:
                n = int(rga.lib().image_loss_workspace(*(int(v) for v in image.shape)))
                self.img_ws = torch.empty(n, dtype=torch.uint8, device=image.device)
            return rga.image_loss(image, target, 0.2, ws=self.img_ws)
        if self.l1_ws is None:              # allocated once, kept across steps
            n = int(rga.lib().l1_loss_workspace(image.numel()))
            self.l1_ws = torch.empty(n, dtype=torch.uint8, device=image.device)
        return rga.l1_loss(image, target, ws=self.l1_ws)

    def train_step(self, p, count, target, check: bool = True):
        """fwd + loss + bwd; returns (loss [1] on device, grads).  With check
        (the default) the duplicate count is read back after the forward
        (one host synchronisation) and the frame re-rendered in a larger
        workspace if it overflowed; without it nothing synchronises and an
        overflowed frame yields NaN loss and gradients (the kernels poison
        them), so a caller that skips the check still sees the failure."""
        image, _, ctx = self.forward(p, count)
        if check and self.ensure_capacity():
            image, _, ctx = self.forward(p, ctx["count"])
        loss, dimage = self.loss(image, target)
        grads = self.backward(p, ctx, dimage)
        return loss, grads


class RenderFunction(torch.autograd.Function):
    """image = render(pos, nrm, quat, log_s, opac, albedo, rough, tint, env)
    with the hand-written adjoint of librga.so as its backward."""

    @staticmethod
    def forward(ctx, renderer: Renderer, count, pos, nrm, quat, log_s, opac, albedo, rough, tint,
                env):
        p = dict(pos=pos, nrm=nrm, quat=quat, log_s=log_s, opac=opac, albedo=albedo,
                 rough=rough, tint=tint, env=env)
        image, T, c = renderer.forward(p, count)
        ctx.renderer = renderer
        ctx.p = p
        ctx.c = c
        ctx.mark_non_differentiable(T)
        return image, T

    @staticmethod
    def backward(ctx, dimage, dT):
        R = ctx.renderer
        D = R.ws.count()          # synchronises
        if D > R.ws.capacity:
            raise rga.RgaError(f"splat workspace overflowed ({D} duplicates, capacity "
                               f"{R.ws.capacity}): the forward image is invalid; call "
                               "Renderer.ensure_capacity() and render again")
        g = R.backward(ctx.p, ctx.c, dimage.contiguous())
        return (None, None, g["pos"], g["nrm"], g["quat"], g["log_s"], g["opac"], g["albedo"],
                g["rough"], g["tint"], g["env"])


def render(renderer: Renderer, count, p: Dict[str, torch.Tensor]):
    return RenderFunction.apply(renderer, count, *[p[k] for k in TRAINABLE])


class VertexModel:
    """The paper's parametrisation (Sec. 3.1): materials and the pose-
    dependent displacement live on the canonical mesh vertices and reach a
    Gaussian through the interpolation equation over its K_g = 3 nearest
    vertices; the skinning matrices come from the pose theta (forward
    kinematics).  Quaternion, scale, opacity and normal stay per Gaussian
    here.  forward / backward compose the library's entry points:
    knn -> displacement network -> interpolation -> pose_to_skin -> the
    render path (the interpolated displacement is added to each Gaussian by
    the skinning call), and back through the same adjoints: the two routes
    of theta (through the network and through the skinning) meet in
    pose_to_skin_backward, which adds its share to the network's; with
    `regularise` the regularisers of Sec. 3.3 add their gradients to the
    image loss's inside the library (the total loss of Sec. 3.3)."""

    LAMBDAS = (0.002, 0.1, 0.02, 10.0)     # smooth, mesh distance, displacement, scale
    S0 = 0.005

    def __init__(self, R: Renderer, freqs, joints, parents, regularise: bool = True):
        self.R = R
        self.index = rga.KnnIndex(R.d["verts"])
        self.net = rga.Displacement(R.d["verts"], freqs)
        self.joints = joints
        self.parents = parents
        self.regularise = regularise

    def forward(self, v: Dict[str, torch.Tensor], count: Optional[torch.Tensor]):
        """v: theta [24, 3], mlp [params], v_albedo [3, nv], v_rough [nv],
        v_tint [nv], pos, nrm, quat, log_s, opac, env (per Gaussian).
        count: the visibility of v's pose, or None to compute it."""
        R = self.R
        idx, w = rga.knn(self.index, v["pos"], 3)
        dxv = self.net.forward(v["theta"].reshape(-1), v["mlp"])
        # vertex attributes [8][nv]: albedo (3), roughness, tint, displacement (3)
        attrs = torch.cat([v["v_albedo"], v["v_rough"][None], v["v_tint"][None], dxv])
        ag = rga.knn_interpolate(idx, w, attrs)
        p = dict(pos=v["pos"], disp=ag[5:8], nrm=v["nrm"], quat=v["quat"], log_s=v["log_s"],
                 opac=v["opac"], albedo=ag[0:3], rough=ag[3], tint=ag[4], env=v["env"])
        R.d["skin"] = rga.pose_to_skin(v["theta"], self.joints, self.parents)
        image, T, ctx = R.forward(p, count)
        ctx.update(idx=idx, w=w, p=p, attrs=attrs)
        return image, T, ctx

    def backward(self, v: Dict[str, torch.Tensor], ctx, dimage: torch.Tensor,
                 loss: Optional[torch.Tensor] = None):
        """Gradients of the image loss whose gradient is `dimage` plus, with
        `regularise`, the weighted regularisers; `loss` (device float [1],
        the image loss) then receives their weighted total, and ctx gets
        the four unweighted terms and the total under "reg_terms"."""
        R = self.R
        p = ctx["p"]
        g = R.backward(p, ctx, dimage, want_dA=True)
        nv = int(R.d["verts"].shape[1])
        dg = torch.cat([g["albedo"], g["rough"][None], g["tint"][None], g["pos"]])
        dv = rga.knn_interpolate_backward(ctx["idx"], ctx["w"], dg, nv)
        if self.regularise:
            attrs = ctx["attrs"]
            ctx["reg_terms"] = rga.regularisers(
                attrs[0:5], R.d["knn_v"], v["pos"], R.d["verts"], ctx["idx"], attrs[5:8],
                v["log_s"], s0=self.S0, lams=self.LAMBDAS,
                accum=(dv[0:5], g["pos"], dv[5:8], g["log_s"]), loss_accum=loss)[0]
        dmlp, dth = self.net.backward(dv[5:8])
        dskin = rga.lbs_skin_pose_grad(int(self.parents.numel()), R.d["jidx"], R.d["jw"], p["pos"],
                                       g["posed_x"], p["nrm"], g["posed_n"], g["posed_A"],
                                       disp=p["disp"])
        rga.pose_to_skin_backward(v["theta"], self.joints, self.parents, dskin, dtheta_accum=dth)
        return dict(theta=dth.reshape(-1, 3), mlp=dmlp, v_albedo=dv[0:3], v_rough=dv[3],
                    v_tint=dv[4], pos=g["pos"], nrm=g["nrm"], quat=g["quat"], log_s=g["log_s"],
                    opac=g["opac"], env=g["env"])
