"""ctypes binding of the FP32-mirror oracle ``rga_oracle.c`` -- TEST INFRASTRUCTURE ONLY.

Arrays are numpy, C-contiguous; per-Gaussian arrays are SoA planes [C][n].
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RGA_ORACLE_LIBRARY may name another build of the same source (the
# sanitizer build of the CPU tests)
_LIB_PATH = os.environ.get("RGA_ORACLE_LIBRARY") or os.path.join(_HERE, "librga_oracle.so")
_lib = None


class OracleCamera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        _lib.oracle_splat_bin.restype = C.c_int64
        _lib.oracle_exp_f32.restype = C.c_float
        _lib.oracle_exp_f32.argtypes = [C.c_float]
        _lib.oracle_ln_upper_f32.restype = C.c_float
        _lib.oracle_ln_upper_f32.argtypes = [C.c_float]
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(C.c_void_p)


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def camera(cam) -> OracleCamera:
    c = OracleCamera()
    c.R[:] = [float(v) for v in np.asarray(cam.R, dtype=np.float32).reshape(-1)]
    c.t[:] = [float(v) for v in np.asarray(cam.t, dtype=np.float32).reshape(-1)]
    c.fx, c.fy, c.cx, c.cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def lbs_f32(skin, jidx, jw, x, nrm=None):
    x = _f(x)
    n = x.shape[1]
    xo = np.empty((3, n), np.float32)
    no = np.empty((3, n), np.float32) if nrm is not None else None
    Ao = np.empty((9, n), np.float32)
    skin = _f(skin)
    lib().oracle_lbs_f32(C.c_int(n), C.c_int(skin.shape[0]), _p(skin), _p(_i(jidx)), _p(_f(jw)),
                         _p(x), _p(_f(nrm)) if nrm is not None else None, _p(xo), _p(no), _p(Ao))
    return xo, no, Ao


def front_f32(x, nrm, cam_pos):
    x = _f(x)
    n = x.shape[1]
    out = np.empty(n, np.uint8)
    lib().oracle_front_f32(C.c_int(n), _p(x), _p(_f(nrm)), _p(_f(cam_pos)), _p(out))
    return out


def vis_frame(verts):
    v = _f(verts)
    c = np.empty(3, np.float32)
    rho = C.c_float()
    lib().oracle_vis_frame(C.c_int(v.shape[1]), _p(v), _p(c), C.byref(rho))
    return c, np.float32(rho.value)


def raster_view(verts, faces, d, res, brute=False):
    v = _f(verts)
    f = _i(faces)
    z = np.empty(res * res, np.uint64)
    lib().oracle_raster_view(C.c_int(v.shape[1]), C.c_int(f.shape[0]), _p(v), _p(f), _p(_f(d)),
                             C.c_int(res), C.c_int(int(brute)), _p(z))
    return z.reshape(res, res)


def vis_filter(raw, knn):
    raw = np.ascontiguousarray(raw, dtype=np.uint8)
    knn = _i(knn)
    nv, kv = knn.shape
    m1, m2, cnt = (np.empty(nv, np.uint8) for _ in range(3))
    lib().oracle_vis_filter(C.c_int(nv), _p(raw), _p(knn), C.c_int(kv), _p(m1), _p(m2), _p(cnt))
    return m1, m2, cnt


def mesh_visibility(verts, faces, view_dirs, res, knn):
    v = _f(verts)
    f = _i(faces)
    dirs = _f(view_dirs)
    knn = _i(knn)
    nv, kv = knn.shape
    V = dirs.shape[0]
    nw = (V + 31) // 32
    raw = np.zeros((nv, nw), np.uint32)
    cnt = np.zeros((nv, V), np.uint8)
    lib().oracle_mesh_visibility(C.c_int(nv), C.c_int(f.shape[0]), _p(v), _p(f), C.c_int(V),
                                 _p(dirs), C.c_int(res), _p(knn), C.c_int(kv), _p(raw), _p(cnt))
    return raw, cnt


def mesh_visibility_shadow(verts, faces, view_dirs, res, knn, bias_px):
    """The shadow-mapping depth test instead of triangle ids (same filters)."""
    v = _f(verts)
    f = _i(faces)
    dirs = _f(view_dirs)
    knn = _i(knn)
    nv, kv = knn.shape
    V = dirs.shape[0]
    nw = (V + 31) // 32
    raw = np.zeros((nv, nw), np.uint32)
    cnt = np.zeros((nv, V), np.uint8)
    lib().oracle_mesh_visibility_shadow(C.c_int(nv), C.c_int(f.shape[0]), _p(v), _p(f), C.c_int(V),
                                        _p(dirs), C.c_int(res), _p(knn), C.c_int(kv),
                                        C.c_float(bias_px), _p(raw), _p(cnt))
    return raw, cnt


def exp_f32(x: float) -> np.float32:
    return np.float32(lib().oracle_exp_f32(C.c_float(x)))


def ln_upper_f32(y: float) -> np.float32:
    return np.float32(lib().oracle_ln_upper_f32(C.c_float(y)))


def splat_preprocess(cam, xp, A, quat, log_s, opac, front):
    xp = _f(xp)
    n = xp.shape[1]
    out = dict(valid=np.empty(n, np.uint8), mean2d=np.empty((2, n), np.float32),
               conic=np.empty((3, n), np.float32), depth=np.empty(n, np.float32),
               rect=np.empty((4, n), np.int32), touched=np.empty(n, np.int32),
               fp64=np.empty(n, np.uint8))
    c = camera(cam)
    lib().oracle_splat_preprocess_f32(
        C.c_int(n), C.byref(c), _p(xp), _p(_f(A)), _p(_f(quat)), _p(_f(log_s)), _p(_f(opac)),
        _p(np.ascontiguousarray(front, dtype=np.uint8)), _p(out["valid"]), _p(out["mean2d"]),
        _p(out["conic"]), _p(out["depth"]), _p(out["rect"]), _p(out["touched"]), _p(out["fp64"]))
    return out


def tiles_of(cam):
    return (cam.width + 15) // 16, (cam.height + 15) // 16


def splat_bin(cam, pre):
    tx, ty = tiles_of(cam)
    n = pre["touched"].shape[0]
    D = int(lib().oracle_splat_bin(C.c_int(n), C.c_int(tx), C.c_int(ty), _p(pre["rect"]),
                                   _p(pre["touched"]), _p(pre["depth"]), None, None, None))
    keys = np.empty(max(D, 1), np.uint64)
    vals = np.empty(max(D, 1), np.int32)
    ranges = np.zeros((tx * ty, 2), np.int32)
    lib().oracle_splat_bin(C.c_int(n), C.c_int(tx), C.c_int(ty), _p(pre["rect"]),
                           _p(pre["touched"]), _p(pre["depth"]), _p(keys), _p(vals), _p(ranges))
    return keys[:D], vals[:D], ranges


def composite_tiles(cam, ranges, values, pre, opac, color, with_applied=False):
    """Tiled FP32-mirror compositing: image [3][H][W], T_final, the smallest
    relative decision margin per pixel and, if asked, the number of splats
    composited into each pixel."""
    H, W = cam.height, cam.width
    tx, _ = tiles_of(cam)
    n = pre["mean2d"].shape[1]
    img = np.empty((3, H, W), np.float32)
    T = np.empty((H, W), np.float32)
    margin = np.empty((H, W), np.float32)
    applied = np.empty((H, W), np.int32)
    vals = _i(values) if len(values) else np.zeros(1, np.int32)
    lib().oracle_composite_tiles_f32(C.c_int(H), C.c_int(W), C.c_int(tx), _p(_i(ranges)),
                                     _p(vals), C.c_int(n), _p(pre["mean2d"]), _p(pre["conic"]),
                                     _p(_f(opac)), _p(_f(color)), _p(img), _p(T), _p(margin),
                                     _p(applied))
    if with_applied:
        return img, T, margin, applied
    return img, T, margin


def composite_brute(cam, pre, opac, color):
    H, W = cam.height, cam.width
    n = pre["mean2d"].shape[1]
    img = np.empty((3, H, W), np.float32)
    T = np.empty((H, W), np.float32)
    lib().oracle_composite_brute_f32(C.c_int(H), C.c_int(W), C.c_int(n), _p(pre["valid"]),
                                     _p(pre["depth"]), _p(pre["mean2d"]), _p(pre["conic"]),
                                     _p(_f(opac)), _p(_f(color)), _p(img), _p(T))
    return img, T


def raster_fixed(xy, z, res, brute=False, claims=False):
    """xy [nt,3,2] int32 fixed-point (1/256 px) vertices, z [nt,3]."""
    xy = _i(xy)
    z = _f(z)
    nt = xy.shape[0]
    zb = np.empty(res * res, np.uint64)
    cl = np.empty(res * res, np.int32) if claims else None
    lib().oracle_raster_fixed(C.c_int(nt), _p(xy), _p(z), C.c_int(res), C.c_int(int(brute)),
                              _p(zb), _p(cl))
    return zb.reshape(res, res), (cl.reshape(res, res) if claims else None)


def project_view(verts, d, res):
    v = _f(verts)
    nv = v.shape[1]
    U = np.empty(nv, np.int32)
    V = np.empty(nv, np.int32)
    z = np.empty(nv, np.float32)
    lib().oracle_project_view(C.c_int(nv), _p(v), _p(_f(d)), C.c_int(res), _p(U), _p(V), _p(z))
    return U, V, z


def knn(q, ref, k):
    """k nearest rows of ref [3,nr] for every query [3,n], ordered by (distance^2,
    index), distance^2 in FP32 (rga_oracle.c) -> idx [k,n] int32, d2 [k,n] f32."""
    q = _f(q)
    ref = _f(ref)
    n, nr = q.shape[1], ref.shape[1]
    idx = np.empty((k, n), np.int32)
    d2 = np.empty((k, n), np.float32)
    lib().oracle_knn(C.c_int(n), _p(q), C.c_int(nr), _p(ref), C.c_int(k), _p(idx), _p(d2))
    return idx, d2


def splitmix64(seed: int, k: int) -> int:
    """The k-th output (k >= 1) of SplitMix64 from state `seed`."""
    L = lib()
    L.oracle_splitmix64.restype = C.c_uint64
    L.oracle_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    return int(L.oracle_splitmix64(C.c_uint64(seed), C.c_uint64(k)))


def densify(sg, verts, faces, d0=1.0, p0=0.02, seed=0, cap=None):
    """App. B, Alg. 1 (rga_oracle.c): sg [kg,n] K_g nearest vertices of each
    Gaussian, verts [3,nv], faces [nf,3] -> dict(Dv [nv], df [nf], ng [nf],
    n_added, x [3,min(n_added, cap)], face [min(n_added, cap)])."""
    sg = _i(sg)
    verts = _f(verts)
    faces = _i(faces)
    kg, n = sg.shape
    nv, nf = verts.shape[1], faces.shape[0]
    if cap is None:
        cap = max(1, nf)
    Dv = np.empty(nv, np.int32)
    df = np.empty(nf, np.float32)
    ng = np.empty(nf, np.int32)
    x = np.zeros((3, cap), np.float32)
    fo = np.zeros(cap, np.int32)
    L = lib()
    L.oracle_densify.restype = C.c_int64
    L.oracle_densify.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                 C.c_void_p, C.c_double, C.c_double, C.c_uint64, C.c_int64] + \
        [C.c_void_p] * 5
    N = int(L.oracle_densify(n, kg, _p(sg), nv, _p(verts), nf, _p(faces), float(d0), float(p0),
                             C.c_uint64(seed), cap, _p(Dv), _p(df), _p(ng), _p(x), _p(fo)))
    m = min(N, cap)
    return dict(Dv=Dv, df=df, ng=ng, n_added=N, x=x[:, :m].copy(), face=fo[:m].copy())
