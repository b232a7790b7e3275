"""ctypes binding of librga.so: argument marshalling only.

Every function here checks tensor placement/shape/dtype, allocates outputs
with torch (device memory and streams are PyTorch's), and calls the C entry
point of the same name on the current HIP stream.  There is no fallback: if
the library is not built, ``lib()`` raises.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# RGA_LIBRARY may name another build of the same library (same ABI)
LIB_PATH = os.environ.get("RGA_LIBRARY") or os.path.join(_HERE, "librga.so")
_lib = None

RGA_FP32 = 0
RGA_BF16X3 = 1
PRECISIONS = {"fp32": RGA_FP32, "bf16x3": RGA_BF16X3}

_VP = C.c_void_p
_I = C.c_int
_I64 = C.c_int64
_SZ = C.c_size_t

_SIGS = {
    "rga_last_error": (C.c_char_p, []),
    "rga_abi_version": (_I, []),
    "lbs_skin": (_I, [_VP, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "lbs_skin_backward": (_I, [_VP, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "pose_to_skin": (_I, [_VP, _I, _VP, _VP, _VP, _VP]),
    "pose_to_skin_backward": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _I]),
    "lbs_skin_pose_grad_workspace": (_SZ, [_I, _I]),
    "lbs_skin_pose_grad": (_I, [_VP, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                _SZ]),
    "mesh_visibility_workspace": (_SZ, [_I, _I]),
    "mesh_visibility": (_I, [_VP, _I, _I, _VP, _VP, _I, _VP, _I, _VP, _I, _VP, _VP, _VP, _SZ]),
    "mesh_visibility_shadowmap": (_I, [_VP, _I, _I, _VP, _VP, _I, _VP, _I, _VP, _I, C.c_float,
                                       _VP, _VP, _VP, _SZ]),
    "mesh_visibility_noalloc_limit": (_SZ, []),
    "mesh_visibility_noalloc": (_I, [_VP, _I, _I, _VP, _VP, _I, _VP, _I, _VP, _I, _VP, _VP]),
    "shade_gaussians": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _I, _I, _I, _I, _I,
                             _I, _VP, _VP, _I, _VP, _VP, _VP, _SZ]),
    "shade_tape_bytes": (_SZ, [_I, _I, _I]),
    "back_face": (_I, [_VP, _I, _VP, _VP, _VP, _VP]),
    "shade_gaussians_workspace": (_SZ, [_I, _I, _I]),
    "shade_gaussians_backward": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _I, _I, _I,
                                      _I, _I, _I, _VP, _VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                      _VP, _VP, _VP, _SZ, _VP, _SZ]),
    "splat_workspace_size": (_SZ, [_I, _I, _I, _I64]),
    "splat_forward": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _I64, _VP,
                           _VP]),
    "splat_bin": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _I64]),
    "splat_blend": (_I, [_VP, _I, _VP, _VP, _VP, _SZ, _I64, _VP, _VP]),
    "splat_read_count": (_I, [_VP, _VP, _I, _I, _I, _I64, _VP]),
    "splat_state": (_I, [_VP, _I, _I, _I, _I64, _VP]),
    "splat_backward": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _I64, _VP,
                            _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "l1_loss_workspace": (_SZ, [_I64]),
    "l1_loss": (_I, [_VP, _I64, _VP, _VP, _VP, _VP, _VP, _SZ]),
    "knn_workspace": (_SZ, [_I]),
    "knn_build": (_I, [_VP, _I, _VP, _VP, _SZ]),
    "knn_query_workspace": (_SZ, [_I]),
    "knn_query": (_I, [_VP, _I, _VP, _I, _I, _VP, _VP, _VP, _SZ, _VP, _SZ]),
    "knn_interpolate": (_I, [_VP, _I, _I, _VP, _VP, _I, _I, _VP, _VP]),
    "knn_interpolate_backward": (_I, [_VP, _I, _I, _VP, _VP, _I, _I, _VP, _VP]),
    "regularisers_workspace": (_SZ, [_I, _I]),
    "regularisers": (_I, [_VP, _I, _I, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP] +
                     [C.c_float] * 5 + [_VP] * 5 + [_I, _VP, _VP, _SZ]),
    "adam_step": (_I, [_VP, C.c_int64, _VP, _VP, _VP, _VP] + [C.c_float] * 4 + [_I]),
    "image_loss_workspace": (_SZ, [_I, _I, _I]),
    "image_loss": (_I, [_VP, _I, _I, _I, _VP, _VP, C.c_float, _VP, _VP, _VP, _SZ]),
    "mlp_workspace": (_SZ, [_I]),
    "mlp_forward": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "mlp_backward": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP, _VP]),
    "densify_workspace": (_SZ, [_I]),
    "densify": (_I, [_VP, _I, _I, _VP, _I, _VP, _I, _VP, C.c_double, C.c_double, C.c_uint64,
                     _I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ]),
    "vertex_order_workspace": (_SZ, [_I]),
    "vertex_order": (_I, [_VP, _I, _VP, _I, _VP, _VP, _SZ]),
    "gather_columns": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "rga_timing_enable": (_I, [_I]),
    "rga_timing_reset": (_I, []),
    "rga_timing_filter": (_I, [C.c_char_p]),
    "rga_timing_read": (_I, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
}


class RgaError(RuntimeError):
    pass


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class SplatState(C.Structure):
    _fields_ = [("mean2d", _VP), ("conic", _VP), ("depth", _VP), ("rect", _VP),
                ("touched", _VP), ("fp64", _VP), ("sorted", _VP), ("ranges", _VP),
                ("count", _VP), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32)]


def lib():
    """Load librga.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().rga_last_error().decode()


def _check(rc: int, name: str):
    if rc != 0:
        raise RgaError(f"{name} failed ({rc}): {last_error()}")


def _p(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise RgaError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise RgaError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise RgaError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise RgaError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def camera(cam) -> Camera:
    c = Camera()
    R = [float(v) for v in torch.as_tensor(cam.R).reshape(-1).tolist()]
    c.R[:] = R
    c.t[:] = [float(v) for v in torch.as_tensor(cam.t).reshape(-1).tolist()]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _f32(t, name, shape=None):
    return _dev(t, torch.float32, name, shape)


def _i32(t, name, shape=None):
    return _dev(t, torch.int32, name, shape)


def _u8(t, name, shape=None):
    return _dev(t, torch.uint8, name, shape)


# ----------------------------------------------------------------------------- LBS
def lbs_skin(skin, jidx, jw, x, nrm=None, want_A: bool = True, disp=None):
    """Skinned positions (of x + disp when disp [3, n] is given), normals, A."""
    n = x.shape[1]
    J = skin.shape[0]
    _f32(skin, "skin", (J, 12))
    _i32(jidx, "jidx", (4, n))
    _f32(jw, "jw", (4, n))
    _f32(x, "x", (3, n))
    if nrm is not None:
        _f32(nrm, "nrm", (3, n))
    if disp is not None:
        _f32(disp, "disp", (3, n))
    xo = torch.empty_like(x)
    no = torch.empty_like(nrm) if nrm is not None else None
    Ao = torch.empty((9, n), dtype=torch.float32, device=x.device) if want_A else None
    _check(lib().lbs_skin(_stream(), n, J, _p(skin), _p(jidx), _p(jw), _p(x), _p(disp), _p(nrm),
                          _p(xo), _p(no), _p(Ao)), "lbs_skin")
    return xo, no, Ao


def pose_to_skin(theta, joints, parents):
    """theta [J, 3] axis-angle, joints [J, 3], parents [J] int32 -> skin [J, 12]."""
    theta, joints, parents = _f32(theta, "theta"), _f32(joints, "joints"), _i32(parents, "parents")
    J = int(parents.numel())
    skin = torch.empty((J, 12), dtype=torch.float32, device=theta.device)
    _check(lib().pose_to_skin(_stream(), J, _p(theta), _p(joints), _p(parents), _p(skin)),
           "pose_to_skin")
    return skin


def pose_to_skin_backward(theta, joints, parents, dskin, dtheta_accum=None):
    """dskin [J, 12] -> dtheta [J, 3]; with dtheta_accum (J * 3 floats) the
    gradient is added into it in place and it is returned."""
    theta, joints, parents = _f32(theta, "theta"), _f32(joints, "joints"), _i32(parents, "parents")
    dskin = _f32(dskin, "dskin")
    J = int(parents.numel())
    if dtheta_accum is None:
        dtheta = torch.empty((J, 3), dtype=torch.float32, device=theta.device)
    else:
        dtheta = _f32(dtheta_accum, "dtheta_accum")
        if dtheta.numel() != 3 * J:
            raise RgaError("dtheta_accum must hold 3 floats per joint")
    _check(lib().pose_to_skin_backward(_stream(), J, _p(theta), _p(joints), _p(parents),
                                       _p(dskin), _p(dtheta), int(dtheta_accum is not None)),
           "pose_to_skin_backward")
    return dtheta


def lbs_skin_pose_grad(n_joints: int, jidx, jw, x, dx_out, nrm=None, dn_out=None, dA=None,
                       disp=None):
    """dskin [n_joints, 12]: the gradient w.r.t. the skinning matrices (of
    the points x + disp when disp is given)."""
    n = int(x.shape[1])
    _f32(x, "x", (3, n))
    _f32(dx_out, "dx_out", (3, n))
    if disp is not None:
        _f32(disp, "disp", (3, n))
    dskin = torch.empty((n_joints, 12), dtype=torch.float32, device=x.device)
    nb = int(lib().lbs_skin_pose_grad_workspace(n, n_joints))
    ws = torch.empty(nb, dtype=torch.uint8, device=x.device)
    _check(lib().lbs_skin_pose_grad(_stream(), n, n_joints, _p(jidx), _p(jw), _p(x), _p(disp),
                                    _p(nrm), _p(dx_out), _p(dn_out), _p(dA), _p(dskin), _p(ws),
                                    nb), "lbs_skin_pose_grad")
    return dskin


def lbs_skin_backward(skin, jidx, jw, dx_out, dn_out=None):
    n = dx_out.shape[1]
    J = skin.shape[0]
    _f32(dx_out, "dx_out", (3, n))
    dx = torch.empty_like(dx_out)
    dn = torch.empty_like(dn_out) if dn_out is not None else None
    _check(lib().lbs_skin_backward(_stream(), n, J, _p(skin), _p(jidx), _p(jw), _p(dx_out),
                                   _p(dn_out), _p(dx), _p(dn)), "lbs_skin_backward")
    return dx, dn


# ----------------------------------------------------------------------------- visibility
def mesh_visibility(verts, faces, view_dirs, res: int, knn, want_raw: bool = False, ws=None,
                    shadow_bias_px: Optional[float] = None):
    """(count [nv, V] uint8, raw bits or None).  With shadow_bias_px set, the
    raw maps come from the shadow-mapping depth test with that bias."""
    nv = verts.shape[1]
    nf = faces.shape[0]
    V = view_dirs.shape[0]
    kv = knn.shape[1]
    _f32(verts, "verts", (3, nv))
    _i32(faces, "faces", (nf, 3))
    _f32(view_dirs, "view_dirs", (V, 3))
    _i32(knn, "knn", (nv, kv))
    need = int(lib().mesh_visibility_workspace(nv, V))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=verts.device)
    count = torch.empty((nv, V), dtype=torch.uint8, device=verts.device)
    raw = torch.empty((nv, (V + 31) // 32), dtype=torch.int32, device=verts.device) if want_raw else None
    if shadow_bias_px is None:
        _check(lib().mesh_visibility(_stream(), nv, nf, _p(verts), _p(faces), V, _p(view_dirs),
                                     res, _p(knn), kv, _p(raw), _p(count), _p(ws), ws.numel()),
               "mesh_visibility")
    else:
        _check(lib().mesh_visibility_shadowmap(_stream(), nv, nf, _p(verts), _p(faces), V,
                                               _p(view_dirs), res, _p(knn), kv,
                                               float(shadow_bias_px), _p(raw), _p(count), _p(ws),
                                               ws.numel()), "mesh_visibility_shadowmap")
    return count, raw


def mesh_visibility_noalloc(verts, faces, view_dirs, res: int, knn, want_raw: bool = False,
                            count=None, raw=None):
    """mesh_visibility through the entry point that allocates nothing on the
    device (its workspace is the library's fixed array).  The outputs may be
    passed in, so that the call itself allocates nothing either."""
    nv = verts.shape[1]
    nf = faces.shape[0]
    V = view_dirs.shape[0]
    kv = knn.shape[1]
    _f32(verts, "verts", (3, nv))
    _i32(faces, "faces", (nf, 3))
    _f32(view_dirs, "view_dirs", (V, 3))
    _i32(knn, "knn", (nv, kv))
    if count is None:
        count = torch.empty((nv, V), dtype=torch.uint8, device=verts.device)
    _u8(count, "count", (nv, V))
    if raw is None and want_raw:
        raw = torch.empty((nv, (V + 31) // 32), dtype=torch.int32, device=verts.device)
    if raw is not None:
        _i32(raw, "raw", (nv, (V + 31) // 32))
    _check(lib().mesh_visibility_noalloc(_stream(), nv, nf, _p(verts), _p(faces), V,
                                         _p(view_dirs), res, _p(knn), kv, _p(raw), _p(count)),
           "mesh_visibility_noalloc")
    return count, raw


# ----------------------------------------------------------------------------- shading
def shade_tape(n: int, he: int, we: int, device):
    """A live-pair tape for shade_gaussians / shade_gaussians_backward."""
    return torch.empty(max(16, int(lib().shade_tape_bytes(n, he, we))), dtype=torch.uint8,
                       device=device)


def _tape(tape):
    if tape is None:
        return None, 0
    _u8(tape, "tape")
    return _p(tape), tape.numel()


def shade_gaussians(x, nrm, albedo, rough, tint, vidx, vw, count, kv, he, we, hv, wv, env,
                    cam_pos, precision: str = "fp32", tape=None):
    """tape: None, or a buffer from shade_tape that receives the live pairs
    (either form) for a shade_gaussians_backward of the same inputs."""
    n = x.shape[1]
    nv = count.shape[0]
    _f32(x, "x", (3, n))
    _f32(nrm, "nrm", (3, n))
    _f32(albedo, "albedo", (3, n))
    _f32(rough, "rough", (n,))
    _f32(tint, "tint", (n,))
    _i32(vidx, "vidx", (3, n))
    _f32(vw, "vw", (3, n))
    _u8(count, "count", (nv, hv * wv))
    _f32(env, "env", (he * we, 3))
    color = torch.empty((3, n), dtype=torch.float32, device=x.device)
    front = torch.empty((n,), dtype=torch.uint8, device=x.device)
    cp = (C.c_float * 3)(*[float(v) for v in cam_pos])
    _check(lib().shade_gaussians(_stream(), n, _p(x), _p(nrm), _p(albedo), _p(rough), _p(tint),
                                 _p(vidx), _p(vw), _p(count), nv, kv, he, we, hv, wv, _p(env),
                                 C.cast(cp, C.c_void_p), PRECISIONS[precision], _p(color),
                                 _p(front), *_tape(tape)), "shade_gaussians")
    return color, front


def back_face(x, nrm, cam_pos, out=None):
    """The back-face flags of shade_gaussians on their own (uint8 [n])."""
    n = x.shape[1]
    _f32(x, "x", (3, n))
    _f32(nrm, "nrm", (3, n))
    front = torch.empty((n,), dtype=torch.uint8, device=x.device) if out is None else out
    _u8(front, "front", (n,))
    cp = (C.c_float * 3)(*[float(v) for v in cam_pos])
    _check(lib().back_face(_stream(), n, _p(x), _p(nrm), C.cast(cp, C.c_void_p), _p(front)),
           "back_face")
    return front


def shade_gaussians_backward(x, nrm, albedo, rough, tint, vidx, vw, count, kv, he, we, hv, wv,
                             env, cam_pos, color, front, dcolor, dx_accum=None,
                             precision: str = "fp32", ws=None, tape=None):
    """tape: None, or the tape shade_gaussians filled for these inputs."""
    n = x.shape[1]
    nv = count.shape[0]
    _f32(dcolor, "dcolor", (3, n))
    dx = torch.zeros((3, n), dtype=torch.float32, device=x.device) if dx_accum is None else dx_accum
    dn = torch.empty((3, n), dtype=torch.float32, device=x.device)
    dalb = torch.empty((3, n), dtype=torch.float32, device=x.device)
    drough = torch.empty((n,), dtype=torch.float32, device=x.device)
    dtint = torch.empty((n,), dtype=torch.float32, device=x.device)
    denv = torch.empty((he * we, 3), dtype=torch.float32, device=x.device)
    need = int(lib().shade_gaussians_workspace(n, he, we))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    cp = (C.c_float * 3)(*[float(v) for v in cam_pos])
    _check(lib().shade_gaussians_backward(
        _stream(), n, _p(x), _p(nrm), _p(albedo), _p(rough), _p(tint), _p(vidx), _p(vw),
        _p(count), nv, kv, he, we, hv, wv, _p(env), C.cast(cp, C.c_void_p), PRECISIONS[precision],
        _p(color), _p(front), _p(dcolor), _p(dx), _p(dn), _p(dalb), _p(drough), _p(dtint),
        _p(denv), _p(ws), ws.numel(), *_tape(tape)), "shade_gaussians_backward")
    return dict(dx=dx, dn=dn, dalbedo=dalb, drough=drough, dtint=dtint, denv=denv)


# ----------------------------------------------------------------------------- splatting
class SplatWorkspace:
    """Device workspace of splat_forward/splat_backward for one (n, image,
    capacity); grows when a frame needs more duplicates than it holds."""

    def __init__(self, n: int, width: int, height: int, capacity: int, device):
        self.n, self.width, self.height, self.capacity = n, width, height, int(capacity)
        self.bytes = int(lib().splat_workspace_size(n, width, height, self.capacity))
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        self.binned = False       # holds the lists of a splat_bin / splat_forward

    def count(self) -> int:
        D = C.c_int64()
        _check(lib().splat_read_count(_stream(), _p(self.buf), self.n, self.width, self.height,
                                      self.capacity, C.byref(D)), "splat_read_count")
        return int(D.value)

    def view(self, ptr: int, shape, dtype: torch.dtype) -> torch.Tensor:
        """Tensor view of a region of the workspace (for inspection)."""
        off = int(ptr) - self.buf.data_ptr()
        nbytes = int(np.prod(shape)) * torch.empty((), dtype=dtype).element_size()
        if off < 0 or off + nbytes > self.bytes:
            raise RgaError("pointer outside the splat workspace")
        return self.buf[off:off + nbytes].view(dtype).reshape(shape)

    def state(self) -> SplatState:
        st = SplatState()
        _check(lib().splat_state(_p(self.buf), self.n, self.width, self.height, self.capacity,
                                 C.byref(st)), "splat_state")
        return st


def splat_forward(cam, x, A, quat, log_s, opac, color, front, ws: SplatWorkspace):
    n = x.shape[1]
    _f32(x, "x", (3, n))
    _f32(A, "A", (9, n))
    _f32(quat, "quat", (4, n))
    _f32(log_s, "log_s", (3, n))
    _f32(opac, "opac", (n,))
    _f32(color, "color", (3, n))
    _u8(front, "front", (n,))
    H, W = int(cam.height), int(cam.width)
    if (ws.n, ws.width, ws.height) != (n, W, H):
        raise RgaError("splat workspace was sized for another problem")
    image = torch.empty((3, H, W), dtype=torch.float32, device=x.device)
    T = torch.empty((H, W), dtype=torch.float32, device=x.device)
    c = camera(cam)
    _check(lib().splat_forward(_stream(), n, C.byref(c), _p(x), _p(A), _p(quat), _p(log_s),
                               _p(opac), _p(color), _p(front), _p(ws.buf), ws.bytes, ws.capacity,
                               _p(image), _p(T)), "splat_forward")
    ws.binned = True
    return image, T


def splat_bin(cam, x, A, quat, log_s, opac, front, ws: SplatWorkspace):
    """The colour-free part of splat_forward (projection, sorts, tile lists)."""
    n = x.shape[1]
    _f32(x, "x", (3, n))
    _f32(A, "A", (9, n))
    _f32(quat, "quat", (4, n))
    _f32(log_s, "log_s", (3, n))
    _f32(opac, "opac", (n,))
    _u8(front, "front", (n,))
    if (ws.n, ws.width, ws.height) != (n, int(cam.width), int(cam.height)):
        raise RgaError("splat workspace was sized for another problem")
    c = camera(cam)
    _check(lib().splat_bin(_stream(), n, C.byref(c), _p(x), _p(A), _p(quat), _p(log_s), _p(opac),
                           _p(front), _p(ws.buf), ws.bytes, ws.capacity), "splat_bin")
    ws.binned = True


def splat_blend(cam, color, ws: SplatWorkspace):
    """The rest of splat_forward on the lists of the last splat_bin on ws."""
    n = color.shape[1]
    _f32(color, "color", (3, n))
    H, W = int(cam.height), int(cam.width)
    if (ws.n, ws.width, ws.height) != (n, W, H):
        raise RgaError("splat workspace was sized for another problem")
    if not ws.binned:
        raise RgaError("splat_blend: the workspace holds no lists (run splat_bin first)")
    image = torch.empty((3, H, W), dtype=torch.float32, device=color.device)
    T = torch.empty((H, W), dtype=torch.float32, device=color.device)
    c = camera(cam)
    _check(lib().splat_blend(_stream(), n, C.byref(c), _p(color), _p(ws.buf), ws.bytes,
                             ws.capacity, _p(image), _p(T)), "splat_blend")
    return image, T


def splat_backward(cam, x, A, quat, log_s, opac, color, front, ws: SplatWorkspace, image,
                   dimage, want_dA: bool = False):
    n = x.shape[1]
    _f32(dimage, "dimage", tuple(image.shape))
    dx = torch.empty((3, n), dtype=torch.float32, device=x.device)
    dq = torch.empty((4, n), dtype=torch.float32, device=x.device)
    ds = torch.empty((3, n), dtype=torch.float32, device=x.device)
    do = torch.empty((n,), dtype=torch.float32, device=x.device)
    dc = torch.empty((3, n), dtype=torch.float32, device=x.device)
    dA = torch.empty((9, n), dtype=torch.float32, device=x.device) if want_dA else None
    c = camera(cam)
    _check(lib().splat_backward(_stream(), n, C.byref(c), _p(x), _p(A), _p(quat), _p(log_s),
                                _p(opac), _p(color), _p(front), _p(ws.buf), ws.bytes,
                                ws.capacity, _p(image), _p(dimage), _p(dx), _p(dq), _p(ds),
                                _p(do), _p(dc), _p(dA)), "splat_backward")
    return dict(dx=dx, dquat=dq, dlog_s=ds, dopac=do, dcolor=dc, dA=dA)


# ----------------------------------------------------------------------------- loss
def l1_loss(image, target, want_grad: bool = True, ws=None):
    _f32(image, "image")
    _f32(target, "target", tuple(image.shape))
    cnt = image.numel()
    loss = torch.empty((1,), dtype=torch.float32, device=image.device)
    dimage = torch.empty_like(image) if want_grad else None
    need = int(lib().l1_loss_workspace(cnt))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=image.device)
    _check(lib().l1_loss(_stream(), cnt, _p(image), _p(target), _p(loss), _p(dimage), _p(ws),
                         ws.numel()), "l1_loss")
    return loss, dimage


# ----------------------------------------------------------------------------- timing
class KnnIndex:
    """Uniform grid over a reference point set (e.g. the canonical mesh
    vertices), built on the device; query it with `knn`."""

    def __init__(self, ref):
        ref = _f32(ref, "ref")
        if ref.dim() != 2 or ref.shape[0] != 3:
            raise RgaError("ref must be [3, nr]")
        self.ref = ref
        self.nr = int(ref.shape[1])
        self.bytes = int(lib().knn_workspace(self.nr))
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=ref.device)
        _check(lib().knn_build(_stream(), self.nr, _p(ref), _p(self.buf), self.bytes), "knn_build")


def knn(index: KnnIndex, q, k: int):
    """(idx [k,n] int32, w [k,n]) of the k nearest reference points of q [3,n]."""
    q = _f32(q, "q")
    n = int(q.shape[1])
    idx = torch.empty((k, n), dtype=torch.int32, device=q.device)
    w = torch.empty((k, n), dtype=torch.float32, device=q.device)
    sb = int(lib().knn_query_workspace(n))
    scratch = torch.empty(sb, dtype=torch.uint8, device=q.device)
    _check(lib().knn_query(_stream(), n, _p(q), index.nr, int(k), _p(idx), _p(w), _p(index.buf),
                           index.bytes, _p(scratch), sb), "knn_query")
    return idx, w


def knn_interpolate(idx, w, attr):
    """attr [C, nr] -> [C, n] with the weights of `knn`."""
    idx = _i32(idx, "idx")
    w = _f32(w, "w")
    attr = _f32(attr, "attr")
    k, n = int(idx.shape[0]), int(idx.shape[1])
    C_, nr = int(attr.shape[0]), int(attr.shape[1])
    out = torch.empty((C_, n), dtype=torch.float32, device=attr.device)
    _check(lib().knn_interpolate(_stream(), n, k, _p(idx), _p(w), C_, nr, _p(attr), _p(out)),
           "knn_interpolate")
    return out


def knn_interpolate_backward(idx, w, dout, nr: int):
    """dout [C, n] -> dattr [C, nr]."""
    idx = _i32(idx, "idx")
    w = _f32(w, "w")
    dout = _f32(dout, "dout")
    k, n = int(idx.shape[0]), int(idx.shape[1])
    C_ = int(dout.shape[0])
    dattr = torch.empty((C_, nr), dtype=torch.float32, device=dout.device)
    _check(lib().knn_interpolate_backward(_stream(), n, k, _p(idx), _p(w), C_, int(nr), _p(dout),
                                          _p(dattr)), "knn_interpolate_backward")
    return dattr


def image_loss(image, target, lam: float = 0.2, want_grad: bool = True, ws=None):
    """(loss [1], dimage [C, H, W] or None) of (1 - lam) L1 + lam D-SSIM."""
    image = _f32(image, "image")
    target = _f32(target, "target")
    if image.dim() != 3 or tuple(target.shape) != tuple(image.shape):
        raise RgaError("image and target must be [C, H, W] of one shape")
    C_, H, W = (int(v) for v in image.shape)
    nb = int(lib().image_loss_workspace(C_, H, W))
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=image.device)
    nb = ws.numel()
    loss = torch.empty(1, dtype=torch.float32, device=image.device)
    dimage = torch.empty_like(image) if want_grad else None
    _check(lib().image_loss(_stream(), C_, H, W, _p(image), _p(target), float(lam), _p(loss),
                            _p(dimage) if want_grad else None, _p(ws), nb), "image_loss")
    return loss, dimage


def regularisers(mat, knn_v, xg, verts, vidx, disp, log_s, s0: float = 0.005,
                 lams=(0.002, 0.1, 0.02, 10.0), accum=None, loss_accum=None):
    """(terms [5]: smooth, mdist, disp, scale, weighted total; gradients of
    the total w.r.t. mat [5, nv], xg [3, n], disp [3, nv], log_s [3, n]).
    With accum = (dmat, dxg, ddisp, dlogs) the gradients are added into those
    tensors in place (and they are returned); with loss_accum (a device
    float [1]) the weighted total is added to it."""
    mat, xg, verts = _f32(mat, "mat"), _f32(xg, "xg"), _f32(verts, "verts")
    disp, log_s = _f32(disp, "disp"), _f32(log_s, "log_s")
    knn_v, vidx = _i32(knn_v, "knn_v"), _i32(vidx, "vidx")
    nv, n = int(mat.shape[1]), int(xg.shape[1])
    kv, kg = int(knn_v.shape[1]), int(vidx.shape[0])
    nb = int(lib().regularisers_workspace(nv, n))
    ws = torch.empty(nb, dtype=torch.uint8, device=mat.device)
    terms = torch.empty(5, dtype=torch.float32, device=mat.device)
    if accum is None:
        dmat, ddisp = torch.empty_like(mat), torch.empty_like(disp)
        dxg, dlogs = torch.empty_like(xg), torch.empty_like(log_s)
    else:
        dmat, dxg, ddisp, dlogs = accum
        for t, nm, like in ((dmat, "dmat", mat), (dxg, "dxg", xg), (ddisp, "ddisp", disp),
                            (dlogs, "dlogs", log_s)):
            _f32(t, nm, tuple(like.shape))
    if loss_accum is not None:
        _f32(loss_accum, "loss_accum", (1,))
    _check(lib().regularisers(_stream(), nv, n, kv, kg, _p(mat), _p(knn_v), _p(xg), _p(verts),
                              _p(vidx), _p(disp), _p(log_s), float(s0), *(float(v) for v in lams),
                              _p(terms), _p(dmat), _p(dxg), _p(ddisp), _p(dlogs),
                              int(accum is not None), _p(loss_accum), _p(ws), nb),
           "regularisers")
    return terms, dmat, dxg, ddisp, dlogs


def adam_step(param, grad, m, v, lr: float, step: int, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step in place on param, m, v (same shape as grad)."""
    for t, nm in ((param, "param"), (grad, "grad"), (m, "m"), (v, "v")):
        _f32(t, nm, tuple(param.shape))
    _check(lib().adam_step(_stream(), param.numel(), _p(param), _p(grad), _p(m), _p(v),
                           float(lr), float(beta1), float(beta2), float(eps), int(step)),
           "adam_step")


def densify(sg, verts, faces, d0: float = 1.0, p0: float = 0.02, seed: int = 0,
            cap: Optional[int] = None, sync: bool = True):
    """Density-based densification (App. B, Alg. 1) on the device.
    sg [kg, n] int32, verts [3, nv], faces [nf, 3] int32.  Returns a dict of
    device tensors Dv [nv], df [nf], ng [nf], x [3, cap], face [cap],
    summary int64 [2] = (sum(Q), N'); with sync, also n_added = N' (a host
    read) and x / face cut to the draws that were written."""
    kg, n = (int(sg.shape[0]), int(sg.shape[1])) if sg.dim() == 2 else (0, 0)
    _i32(sg, "sg", (kg, n))
    nv = int(verts.shape[1])
    _f32(verts, "verts", (3, nv))
    nf = int(faces.shape[0])
    _i32(faces, "faces", (nf, 3))
    if cap is None:
        cap = max(1, nf)
    devc = verts.device
    Dv = torch.empty(nv, dtype=torch.int32, device=devc)
    df = torch.empty(nf, dtype=torch.float32, device=devc)
    ng = torch.empty(nf, dtype=torch.int32, device=devc)
    x = torch.zeros((3, cap), dtype=torch.float32, device=devc)
    fo = torch.zeros(cap, dtype=torch.int32, device=devc)
    summary = torch.empty(2, dtype=torch.int64, device=devc)
    need = int(lib().densify_workspace(nf))
    ws = torch.empty(max(need, 16), dtype=torch.uint8, device=devc)
    _check(lib().densify(_stream(), n, kg, _p(sg), nv, _p(verts), nf, _p(faces), float(d0),
                         float(p0), C.c_uint64(int(seed) & (2**64 - 1)), int(cap), _p(Dv), _p(df),
                         _p(ng), _p(x) if cap > 0 else None, _p(fo) if cap > 0 else None,
                         _p(summary), _p(ws), ws.numel()), "densify")
    out = dict(Dv=Dv, df=df, ng=ng, x=x, face=fo, summary=summary)
    if sync:
        N = int(summary[1].item())
        m = min(N, cap)
        out.update(n_added=N, x=x[:, :m], face=fo[:m])
    return out


def vertex_order(vidx, nv: int):
    """The Gaussians' indices sorted stably by nearest mesh vertex (vidx
    [3, n] int32, row 0), on the device: an int32 permutation [n]."""
    n = int(vidx.shape[1])
    _i32(vidx, "vidx", (3, n))
    order = torch.empty((n,), dtype=torch.int32, device=vidx.device)
    ws = torch.empty(max(16, int(lib().vertex_order_workspace(n))), dtype=torch.uint8,
                     device=vidx.device)
    _check(lib().vertex_order(_stream(), n, _p(vidx), int(nv), _p(order), _p(ws), ws.numel()),
           "vertex_order")
    return order


def gather_columns(src, order):
    """dst[..., j] = src[..., order[j]] for a contiguous float32 or int32
    tensor whose last dimension is the Gaussians (n); a new tensor."""
    if src.dtype not in (torch.float32, torch.int32):
        raise RgaError("gather_columns: float32 or int32 tensor expected")
    _dev(src, src.dtype, "src")
    n = int(src.shape[-1])
    _i32(order, "order", (n,))
    rows = src.numel() // n if n > 0 else 0
    dst = torch.empty_like(src)
    _check(lib().gather_columns(_stream(), rows, n, _p(src), _p(order), _p(dst)),
           "gather_columns")
    return dst


MLP_PARAMS = 249603


class Displacement:
    """The displacement network d(x, theta) over a fixed set of vertices:
    holds the workspace that `forward` fills and `backward` reads."""

    def __init__(self, x, freqs):
        self.x = _f32(x, "x")
        if self.x.dim() != 2 or self.x.shape[0] != 3:
            raise RgaError("x must be [3, nv]")
        self.freqs = _f32(freqs, "freqs")
        if tuple(self.freqs.shape) != (64, 3):
            raise RgaError("freqs must be [64, 3]")
        self.nv = int(self.x.shape[1])
        self.bytes = int(lib().mlp_workspace(self.nv))
        self.ws = torch.empty(self.bytes, dtype=torch.uint8, device=self.x.device)

    def forward(self, theta, params):
        """dx [3, nv] for pose theta [72] and the flat parameters."""
        self.theta = _f32(theta, "theta").reshape(-1)
        self.params = _f32(params, "params").reshape(-1)
        if self.theta.numel() != 72 or self.params.numel() != MLP_PARAMS:
            raise RgaError("theta must hold 72 and params %d floats" % MLP_PARAMS)
        dx = torch.empty((3, self.nv), dtype=torch.float32, device=self.x.device)
        _check(lib().mlp_forward(_stream(), self.nv, _p(self.x), _p(self.freqs), _p(self.theta),
                                 _p(self.params), _p(self.ws), self.bytes, _p(dx)), "mlp_forward")
        return dx

    def backward(self, ddx):
        """(dparams, dtheta) of the last forward for ddx [3, nv]."""
        ddx = _f32(ddx, "ddx")
        if tuple(ddx.shape) != (3, self.nv):
            raise RgaError("ddx must be [3, nv]")
        dp = torch.empty(MLP_PARAMS, dtype=torch.float32, device=ddx.device)
        dt = torch.empty(72, dtype=torch.float32, device=ddx.device)
        _check(lib().mlp_backward(_stream(), self.nv, _p(self.x), _p(self.freqs), _p(self.theta),
                                  _p(self.params), _p(ddx), _p(self.ws), self.bytes, _p(dp),
                                  _p(dt)), "mlp_backward")
        return dp, dt


def timing_enable(on: bool = True):
    _check(lib().rga_timing_enable(int(on)), "rga_timing_enable")


def timing_filter(kernel: Optional[str]):
    _check(lib().rga_timing_filter(kernel.encode() if kernel else None), "rga_timing_filter")


def timing_reset():
    _check(lib().rga_timing_reset(), "rga_timing_reset")


def timing_read(kernel: str) -> Tuple[float, int]:
    ms = C.c_double()
    cnt = C.c_int64()
    _check(lib().rga_timing_read(kernel.encode(), C.byref(ms), C.byref(cnt)), "rga_timing_read")
    return float(ms.value), int(cnt.value)
