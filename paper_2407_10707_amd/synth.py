"""Seeded synthetic avatar scenes (inputs only).

This module produces the *inputs* of the render-and-train path: a procedural
capsule body mesh on a 24-joint skeleton, skinning matrices from a random pose,
canonical Gaussians sampled on the mesh, nearest-vertex tables, an environment
map, visibility view directions and a camera.  It holds none of the method's
arithmetic (no skinning, no shading, no splatting); both the HIP path and the
CPU oracle consume what it returns.

The shapes follow the paper's workloads (Sec. 3.5 "Implementation Details": about
100K Gaussians, K_g = 3, K_v = 19; Sec. 3.1: a 16x32 light-probe map of 512
area lights; the proxy mesh of Sec. 3.1).  Captured avatars are not available,
so every array is synthetic and a pure function of (config id, stream seed).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np
from scipy.spatial import cKDTree

# --------------------------------------------------------------------------
# Skeleton: SMPL-like 24-joint tree, canonical A-pose, body 1.7 units tall,
# centred on the origin with +Y up.
# --------------------------------------------------------------------------
PARENTS = np.array([-1, 0, 0, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 9, 9, 12, 13, 14,
                    16, 17, 18, 19, 20, 21], dtype=np.int64)

JOINTS_REST = np.array([
    [0.00, 0.00, 0.00],    # 0 pelvis
    [0.09, -0.08, 0.00],   # 1 left hip
    [-0.09, -0.08, 0.00],  # 2 right hip
    [0.00, 0.10, 0.00],    # 3 spine 1
    [0.10, -0.45, 0.00],   # 4 left knee
    [-0.10, -0.45, 0.00],  # 5 right knee
    [0.00, 0.23, 0.00],    # 6 spine 2
    [0.10, -0.78, 0.00],   # 7 left ankle
    [-0.10, -0.78, 0.00],  # 8 right ankle
    [0.00, 0.28, 0.00],    # 9 spine 3
    [0.11, -0.81, 0.12],   # 10 left foot
    [-0.11, -0.81, 0.12],  # 11 right foot
    [0.00, 0.48, 0.00],    # 12 neck
    [0.07, 0.40, 0.00],    # 13 left collar
    [-0.07, 0.40, 0.00],   # 14 right collar
    [0.00, 0.58, 0.00],    # 15 head
    [0.17, 0.42, 0.00],    # 16 left shoulder
    [-0.17, 0.42, 0.00],   # 17 right shoulder
    [0.36, 0.24, 0.00],    # 18 left elbow
    [-0.36, 0.24, 0.00],   # 19 right elbow
    [0.54, 0.06, 0.00],    # 20 left wrist
    [-0.54, 0.06, 0.00],   # 21 right wrist
    [0.61, -0.01, 0.00],   # 22 left hand
    [-0.61, -0.01, 0.00],  # 23 right hand
], dtype=np.float64)

# (joint a, joint b or None for an explicit end point, radius)
_HEAD_TOP = np.array([0.0, 0.72, 0.0])
CAPSULES = [
    (0, 6, 0.14), (6, 12, 0.15), (12, 15, 0.05), (15, None, 0.11),
    (1, 4, 0.08), (4, 7, 0.055), (2, 5, 0.08), (5, 8, 0.055),
    (7, 10, 0.045), (8, 11, 0.045),
    (13, 16, 0.055), (14, 17, 0.055),
    (16, 18, 0.05), (18, 20, 0.04), (17, 19, 0.05), (19, 21, 0.04),
    (20, 22, 0.035), (21, 23, 0.035),
]


@dataclasses.dataclass(frozen=True)
class SceneConfig:
    """Sizes of one synthetic workload."""
    name: str
    n_gauss: int
    seg: int            # capsule segments around the axis
    rings: int          # capsule rings along the profile
    he: int             # environment rows (He x We texels = K directions)
    we: int
    hv: int             # visibility view grid rows (Hv x Wv = V views)
    wv: int
    vis_res: int        # visibility raster resolution
    height: int         # camera image
    width: int
    n_env: int = 1
    n_pose: int = 1
    kv: int = 19
    kg: int = 3
    log_scale_mean: float = -4.0
    log_scale_std: float = 0.3


CONFIGS: Dict[int, SceneConfig] = {
    1: SceneConfig("tiny-2k-128px", 2000, 7, 4, 8, 16, 8, 8, 64, 128, 128),
    2: SceneConfig("avatar-100k-512px", 100_000, 18, 21, 16, 32, 16, 32, 128, 512, 512),
    3: SceneConfig("train-100k-1024px", 100_000, 18, 21, 16, 32, 16, 32, 128, 1024, 1024),
    4: SceneConfig("precision-200k-2048dir-1024px", 200_000, 18, 21, 32, 64, 32, 32, 128,
                   1024, 1024),
    5: SceneConfig("anim-relight-300k-1080px", 300_000, 18, 21, 32, 64, 32, 32, 128, 1080,
                   1080, n_env=4, n_pose=16),
    # paper-shaped supplementary workload: ~40K-vertex mesh, 500^2, small scales
    6: SceneConfig("paper-shape-100k-500px", 100_000, 48, 46, 16, 32, 16, 32, 128, 500, 500,
                   log_scale_mean=math.log(0.005)),
}


def rng_for(cfg_id: int, stream: int, salt: int = 0) -> np.random.Generator:
    """Streams: 0 mesh, 1 pose, 2 sampling, 3 attributes, 4 env, 5 target, 6 FD subset."""
    return np.random.default_rng([cfg_id, stream, salt])


# --------------------------------------------------------------------------
# Mesh
# --------------------------------------------------------------------------
def _frame(axis: np.ndarray):
    axis = axis / np.linalg.norm(axis)
    helper = np.array([1.0, 0.0, 0.0]) if abs(axis[0]) < 0.9 else np.array([0.0, 0.0, 1.0])
    u = np.cross(axis, helper)
    u /= np.linalg.norm(u)
    v = np.cross(axis, u)
    return axis, u, v


def capsule(a: np.ndarray, b: np.ndarray, radius: float, seg: int, rings: int):
    """UV capsule with seg*rings+2 vertices and 2*seg*rings outward-facing triangles."""
    axis, u, v = _frame(b - a)
    length = float(np.linalg.norm(b - a))
    cap = 0.5 * math.pi * radius
    total = 2 * cap + length
    verts = [a - axis * radius]
    for i in range(rings):
        s = total * (i + 1) / (rings + 1)
        if s < cap:
            ang = s / radius                      # 0 at the bottom pole
            h, r = -radius * math.cos(ang), radius * math.sin(ang)
        elif s > cap + length:
            ang = (s - cap - length) / radius
            h, r = length + radius * math.sin(ang), radius * math.cos(ang)
        else:
            h, r = s - cap, radius
        for j in range(seg):
            phi = 2.0 * math.pi * j / seg
            verts.append(a + axis * h + r * (math.cos(phi) * u + math.sin(phi) * v))
    verts.append(b + axis * radius)
    verts = np.asarray(verts)
    faces = []
    top = 1 + seg * rings
    for j in range(seg):
        faces.append((0, 1 + (j + 1) % seg, 1 + j))
    for i in range(rings - 1):
        r0, r1 = 1 + i * seg, 1 + (i + 1) * seg
        for j in range(seg):
            j1 = (j + 1) % seg
            faces.append((r0 + j, r0 + j1, r1 + j1))
            faces.append((r0 + j, r1 + j1, r1 + j))
    last = 1 + (rings - 1) * seg
    for j in range(seg):
        faces.append((last + j, last + (j + 1) % seg, top))
    return verts, np.asarray(faces, dtype=np.int64)


def body_mesh(seg: int, rings: int):
    vs, fs, off = [], [], 0
    for ja, jb, rad in CAPSULES:
        a = JOINTS_REST[ja]
        b = JOINTS_REST[jb] if jb is not None else _HEAD_TOP
        v, f = capsule(a, b, rad, seg, rings)
        vs.append(v)
        fs.append(f + off)
        off += len(v)
    return np.concatenate(vs), np.concatenate(fs)


def nearest(points: np.ndarray, ref: np.ndarray, k: int) -> tuple:
    """k nearest rows of ref for every point, ordered by (distance, index)."""
    tree = cKDTree(ref)
    kk = min(len(ref), k + 8)
    d, idx = tree.query(points, k=kk)
    d = np.atleast_2d(d)
    idx = np.atleast_2d(idx)
    # (distance, index) order per row
    out_i = np.empty((len(points), k), dtype=np.int64)
    out_d = np.empty((len(points), k), dtype=np.float64)
    for start in range(0, len(points), 65536):
        dd = d[start:start + 65536]
        ii = idx[start:start + 65536]
        o = np.lexsort((ii, dd))  # sorts along the last axis row-wise
        out_i[start:start + 65536] = np.take_along_axis(ii, o, axis=1)[:, :k]
        out_d[start:start + 65536] = np.take_along_axis(dd, o, axis=1)[:, :k]
    return out_d, out_i


# --------------------------------------------------------------------------
# Pose -> skinning matrices (host forward kinematics in FP64)
# --------------------------------------------------------------------------
def axis_angle(axis: np.ndarray, ang: float) -> np.ndarray:
    axis = axis / np.linalg.norm(axis)
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * k + (1 - math.cos(ang)) * (k @ k)


def random_pose(rng: np.random.Generator, n_joints: int = 24, max_deg: float = 30.0):
    rots = []
    for _ in range(n_joints):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        rots.append(axis_angle(axis, math.radians(rng.uniform(0.0, max_deg))))
    return np.stack(rots)


def skinning_matrices(local_rots: np.ndarray) -> np.ndarray:
    """[J][3][4] rows [R | t] mapping canonical points to the posed space."""
    J = len(PARENTS)
    G = np.zeros((J, 3, 3))
    P = np.zeros((J, 3))
    for j in range(J):
        p = PARENTS[j]
        if p < 0:
            G[j] = local_rots[j]
            P[j] = JOINTS_REST[j]
        else:
            G[j] = G[p] @ local_rots[j]
            P[j] = P[p] + G[p] @ (JOINTS_REST[j] - JOINTS_REST[p])
    S = np.zeros((J, 3, 4))
    S[:, :, :3] = G
    S[:, :, 3] = P - np.einsum("jab,jb->ja", G, JOINTS_REST)
    return S


def identity_skinning(n_joints: int = 24) -> np.ndarray:
    S = np.zeros((n_joints, 3, 4))
    S[:, :, :3] = np.eye(3)
    return S


# --------------------------------------------------------------------------
# Directions of a lat-long grid (view directions for visibility)
# --------------------------------------------------------------------------
def latlong_centres(rows: int, cols: int) -> np.ndarray:
    r = (np.arange(rows) + 0.5) * math.pi / rows
    c = (np.arange(cols) + 0.5) * 2.0 * math.pi / cols
    th, ph = np.meshgrid(r, c, indexing="ij")
    d = np.stack([np.sin(th) * np.sin(ph), np.cos(th), np.sin(th) * np.cos(ph)], axis=-1)
    return d.reshape(-1, 3)


# --------------------------------------------------------------------------
# Camera
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    R: np.ndarray       # world->camera rotation, row-major 3x3
    t: np.ndarray       # world->camera translation
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def centre(self) -> np.ndarray:
        return -(self.R.T @ self.t)


def default_camera(width: int, height: int, fov_y_deg: float = 40.0, dist: float = 3.0) -> Camera:
    f = height / (2.0 * math.tan(math.radians(fov_y_deg) / 2.0))
    R = np.diag([1.0, -1.0, -1.0])
    t = np.array([0.0, 0.0, dist])
    return Camera(R, t, f, f, width / 2.0, height / 2.0, width, height)


# --------------------------------------------------------------------------
# Scene assembly
# --------------------------------------------------------------------------
def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def pose_skin(cfg_id: int, pose_index: int = 0) -> np.ndarray:
    """Skinning matrices [24][3][4] of pose `pose_index` of a configuration."""
    return skinning_matrices(random_pose(rng_for(cfg_id, 1, pose_index)))


def env_map(cfg_id: int, env_index: int = 0) -> np.ndarray:
    """Environment radiance [He*We][3]: log-normal per texel and channel."""
    cfg = CONFIGS[cfg_id]
    re = rng_for(cfg_id, 4, env_index)
    return np.exp(re.normal(-1.0, 1.0, size=(cfg.he * cfg.we, 3)))


def make_scene(cfg_id: int, n_gauss: Optional[int] = None, pose_index: int = 0,
               env_index: int = 0, identity_pose: bool = False,
               height: Optional[int] = None, width: Optional[int] = None) -> dict:
    """Return the inputs of one frame of a configuration.

    Per-Gaussian arrays are SoA planes ``[C][N]`` float32 (int32 for indices).
    """
    cfg = CONFIGS[cfg_id]
    N = cfg.n_gauss if n_gauss is None else n_gauss
    H = cfg.height if height is None else height
    W = cfg.width if width is None else width

    verts, faces = body_mesh(cfg.seg, cfg.rings)
    nv = len(verts)

    # vertex -> vertex neighbours (canonical space, includes the vertex itself)
    _, knn_v = nearest(verts, verts, cfg.kv)

    # mesh skin: 4 nearest joints, Gaussian falloff
    dj = np.linalg.norm(verts[:, None, :] - JOINTS_REST[None], axis=-1)
    jn = np.argsort(dj, axis=1, kind="stable")[:, :4]
    d4 = np.take_along_axis(dj, jn, axis=1)
    w4 = np.exp(-(d4 ** 2 - d4[:, :1] ** 2) / (2 * 0.08 ** 2))
    w4 /= w4.sum(axis=1, keepdims=True)

    # pose
    skin = identity_skinning() if identity_pose else pose_skin(cfg_id, pose_index)

    # Gaussians: area-weighted triangle, uniform barycentric point, face normal
    rs = rng_for(cfg_id, 2)
    tri = verts[faces]
    fn = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    area = 0.5 * np.linalg.norm(fn, axis=1)
    fn = fn / np.maximum(2.0 * area[:, None], 1e-30)
    fsel = rs.choice(len(faces), size=N, p=area / area.sum())
    r1, r2 = rs.random(N), rs.random(N)
    s1 = np.sqrt(r1)
    bary = np.stack([1 - s1, s1 * (1 - r2), s1 * r2], axis=1)
    pos = np.einsum("nk,nkd->nd", bary, tri[fsel])
    nrm = fn[fsel]

    ra = rng_for(cfg_id, 3)
    quat = ra.normal(size=(N, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    log_s = ra.normal(cfg.log_scale_mean, cfg.log_scale_std, size=(N, 3))
    opac = ra.uniform(0.3, 0.95, size=N)
    albedo = ra.uniform(0.0, 1.0, size=(N, 3))
    rough = ra.uniform(0.2, 0.9, size=N)
    tint = ra.uniform(0.0, 1.0, size=N)
    djg = np.linalg.norm(pos[:, None, :] - JOINTS_REST[None], axis=-1)
    gj = np.argsort(djg, axis=1, kind="stable")[:, :4]
    gw = ra.dirichlet(np.ones(4), size=N)

    # Gaussian -> nearest canonical vertices with normalised inverse-distance weights
    gd, gi = nearest(pos, verts, cfg.kg)
    u = 1.0 / np.maximum(gd, 1e-12)
    u /= u.sum(axis=1, keepdims=True)

    env = env_map(cfg_id, env_index)

    cam = default_camera(W, H)
    target = rng_for(cfg_id, 5).random((3, H, W))

    return dict(
        cfg_id=cfg_id, cfg=cfg, n=N, nv=nv, nf=len(faces), height=H, width=W,
        verts=_f32(verts.T), faces=_i32(faces), mesh_jidx=_i32(jn.T), mesh_jw=_f32(w4.T),
        knn_v=_i32(knn_v), kv=cfg.kv,
        skin=_f32(skin.reshape(-1, 12)), n_joints=24,
        pos=_f32(pos.T), nrm=_f32(nrm.T), quat=_f32(quat.T), log_s=_f32(log_s.T),
        opac=_f32(opac), albedo=_f32(albedo.T), rough=_f32(rough), tint=_f32(tint),
        jidx=_i32(gj.T), jw=_f32(gw.T), vidx=_i32(gi.T), vw=_f32(u.T),
        he=cfg.he, we=cfg.we, hv=cfg.hv, wv=cfg.wv, env=_f32(env),
        view_dirs=_f32(latlong_centres(cfg.hv, cfg.wv)), vis_res=cfg.vis_res,
        cam=cam, target=_f32(target),
    )


def micro_scene(seed: int, n: int, height: int, width: int, he: int = 4, we: int = 8,
                hv: int = 4, wv: int = 8, vis_res: int = 32, seg: int = 5, rings: int = 3,
                log_scale_mean: float = -3.5, posed: bool = True) -> dict:
    """Small randomized scene for edge-case tests (odd sizes, ragged tiles)."""
    rng = np.random.default_rng([1000, seed])
    verts, faces = body_mesh(seg, rings)
    nv = len(verts)
    _, knn_v = nearest(verts, verts, 19 if nv >= 19 else nv)
    kv = knn_v.shape[1]
    dj = np.linalg.norm(verts[:, None, :] - JOINTS_REST[None], axis=-1)
    jn = np.argsort(dj, axis=1, kind="stable")[:, :4]
    w4 = rng.dirichlet(np.ones(4), size=nv)
    skin = skinning_matrices(random_pose(rng)) if posed else identity_skinning()
    pos = rng.uniform([-0.5, -0.8, -0.2], [0.5, 0.8, 0.2], size=(n, 3))
    nrm = rng.normal(size=(n, 3))
    nrm[:, 2] = np.abs(nrm[:, 2]) + 0.2          # mostly towards the camera
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    quat = rng.normal(size=(n, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    log_s = rng.normal(log_scale_mean, 0.4, size=(n, 3))
    gj = rng.integers(0, 24, size=(n, 4))
    gw = rng.dirichlet(np.ones(4), size=n)
    gd, gi = nearest(pos, verts, 3)
    u = 1.0 / np.maximum(gd, 1e-12)
    u /= u.sum(axis=1, keepdims=True)
    cam = default_camera(width, height)
    return dict(
        cfg_id=None, cfg=None, n=n, nv=nv, nf=len(faces), height=height, width=width,
        verts=_f32(verts.T), faces=_i32(faces), mesh_jidx=_i32(jn.T), mesh_jw=_f32(w4.T),
        knn_v=_i32(knn_v), kv=kv, skin=_f32(skin.reshape(-1, 12)), n_joints=24,
        pos=_f32(pos.T), nrm=_f32(nrm.T), quat=_f32(quat.T), log_s=_f32(log_s.T),
        opac=_f32(rng.uniform(0.02, 0.99, size=n)), albedo=_f32(rng.random((3, n))),
        rough=_f32(rng.uniform(0.2, 0.9, size=n)), tint=_f32(rng.random(n)),
        jidx=_i32(gj.T), jw=_f32(gw.T), vidx=_i32(gi.T), vw=_f32(u.T),
        he=he, we=we, hv=hv, wv=wv, env=_f32(np.exp(rng.normal(-1, 1, size=(he * we, 3)))),
        view_dirs=_f32(latlong_centres(hv, wv)), vis_res=vis_res, cam=cam,
        target=_f32(rng.random((3, height, width))),
    )


def mlp_inputs(seed: int, n_pose: int = 1, freqs: int = 64, pose: int = 72, width: int = 256,
               sigma: float = 1.0) -> dict:
    """Inputs of the displacement network: the Fourier matrix B [freqs, 3]
    (normal, std sigma, per unit of length), poses [n_pose, pose] (axis-angle
    components, normal with std 0.2) and a flat parameter vector drawn as a
    freshly initialised network would be (each layer's weights and biases
    uniform in +-1/sqrt(fan_in)), in the order W_1, b_1, ..., W_5, b_5 with
    W_1 [width, 2 freqs + pose], W_2..W_4 [width, width], W_5 [3, width]."""
    rng = np.random.default_rng([7, seed])
    shapes = [(width, 2 * freqs + pose), (width, width), (width, width), (width, width),
              (3, width)]
    parts = []
    for n_out, n_in in shapes:
        bound = 1.0 / math.sqrt(n_in)
        parts.append(rng.uniform(-bound, bound, n_out * n_in))
        parts.append(rng.uniform(-bound, bound, n_out))
    return dict(freqs=_f32(rng.normal(0.0, sigma, (freqs, 3))),
                thetas=_f32(rng.normal(0.0, 0.2, (n_pose, pose))),
                params=_f32(np.concatenate(parts)))


def needle_splats(seed: int, n_plain: int = 300, width: int = 99, height: int = 75,
                  n_needles: int = 8) -> dict:
    """Splat-level inputs (posed positions, linear part A = I, quaternions,
    log-scales, opacities, colours) of ordinary splats mixed with needles:
    one axis 4-8 units long and two of 2e-4, turned about the camera's
    optical axis by angles in 25-65 or 115-155 degrees (off the image axes,
    where the 2D covariance's determinant cancels), so that their projected
    2D covariance is nearly rank one.  The order is shuffled."""
    rng = np.random.default_rng([2000, seed])
    cam = default_camera(width, height)
    n = n_plain + n_needles
    x = np.stack([rng.uniform(-0.7, 0.7, n), rng.uniform(-0.5, 0.5, n),
                  rng.uniform(-0.3, 0.3, n)])
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0)
    ls = rng.normal(-3.3, 0.3, (3, n))
    op = rng.uniform(0.3, 0.95, n)
    angs = (rng.uniform(25.0, 65.0, n_needles) + 90.0 * (np.arange(n_needles) % 2)) * math.pi / 180
    for i, a in enumerate(angs):
        g = n_plain + i
        q[:, g] = [math.cos(a / 2), 0.0, 0.0, math.sin(a / 2)]
        ls[:, g] = [math.log(rng.uniform(4.0, 8.0)), math.log(2e-4), math.log(2e-4)]
        op[g] = rng.uniform(0.5, 0.9)
    perm = rng.permutation(n)
    A = np.tile(np.eye(3).reshape(9, 1), (1, n))
    return dict(cam=cam, n=n, x=_f32(x[:, perm]), A=_f32(A), quat=_f32(q[:, perm]),
                log_s=_f32(ls[:, perm]), opac=_f32(op[perm]), color=_f32(rng.random((3, n))),
                front=np.ones(n, np.uint8), needle=np.argsort(perm)[n_plain:])
