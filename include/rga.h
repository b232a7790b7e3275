/*
 * rga.h -- C ABI of the relightable Gaussian-avatar render-and-train path
 * (Zhan et al., "Interactive Rendering of Relightable and Animatable Gaussian
 * Avatars"), implemented as hand-written HIP kernels for gfx950 (MI355X).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array pointers are DEVICE pointers owned by the caller, except the
 *    camera struct and cam_pos, which live in host memory.  The library never
 *    allocates device memory and keeps no state between calls; scratch space
 *    is a caller-provided workspace whose size the *_workspace functions give
 *    (one exception: mesh_visibility_noalloc uses a fixed array of its own).
 *  - Per-item arrays are structure-of-arrays planes: "[C][n]" means C
 *    contiguous planes of n float32 (or int32) values each.  Device pointers
 *    must be 16-byte aligned.
 *  - Every call is asynchronous on the HIP stream `stream` (hipStream_t passed
 *    as void*; NULL is the default stream).  No entry point synchronises the
 *    device except splat_read_count.
 *  - Return value: RGA_OK (0) or a negative error code; rga_last_error()
 *    returns a thread-local message for the last failure.  Argument checks
 *    happen on the host before any launch; on error nothing is launched.
 *  - Backward entry points OVERWRITE their gradient outputs, except where an
 *    argument is documented as accumulating.
 *  - Index inputs (joint, vertex, neighbour indices) must be in range; they
 *    are clamped on the device for memory safety, which silently changes the
 *    result of out-of-range input rather than faulting.
 */
#ifndef RGA_H
#define RGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RGA_OK 0
#define RGA_EINVAL (-1)        /* null pointer, bad size or misalignment     */
#define RGA_ECAPACITY (-2)     /* workspace too small                        */
#define RGA_EHIP (-3)          /* HIP launch or runtime error                */
#define RGA_EUNSUPPORTED (-4)  /* configuration outside the supported range  */

#define RGA_FP32 0             /* shading contraction in FP32 on VALU        */
#define RGA_BF16X3 1           /* shading contraction on BF16 MFMA, hi+lo split */

/* Pinhole camera, world -> camera x_c = R x + t (row-major R), camera frame
 * x right, y down, z forward; pixel (i, j) has its centre at (i+0.5, j+0.5). */
typedef struct rga_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} rga_camera;

const char* rga_last_error(void);
/* 3: splat_bin / splat_blend / back_face; splat_backward reads `color`;
 * the live-pair tape in both shading forms.                                */
int rga_abi_version(void);

/* ------------------------------------------------------------------------
 * Sec. 3.1 (deformation): forward linear blend skinning of canonical points
 * (Gaussians or mesh vertices) to the posed space, with four joints per point.
 *   x' = x + sum_j w_j ((R_j - I) x + t_j)      (= sum_j w_j (R_j x + t_j))
 *   A  = I + sum_j w_j (R_j - I)                 (blended linear part)
 *   n' = A n                                     (unnormalised normal)
 * skin   [n_joints][3][4]  row-major [R_j | t_j], n_joints in 1..256
 * jidx   [4][n] int32, jw [4][n]: joint indices and weights (sum 1)
 * x      [3][n]  canonical positions;  nrm [3][n] canonical normals or NULL
 * disp   [3][n]  displacement added to x before skinning (the paper's
 *        "Gaussians are first added with position displacements", Sec. 1 /
 *        Sec. 3.1), or NULL for none: the point skinned is the FP32 sum x + disp
 * x_out  [3][n]; n_out [3][n] or NULL (needs nrm); A_out [9][n] or NULL
 * The sums run in joint-slot order with fused multiply-adds, so the result is
 * reproducible bit for bit.  The adjoint with respect to disp equals that
 * with respect to x (lbs_skin_backward).                                    */
int lbs_skin(void* stream, int n, int n_joints, const float* skin, const int32_t* jidx,
             const float* jw, const float* x, const float* disp, const float* nrm, float* x_out,
             float* n_out, float* A_out);

/* Adjoint of lbs_skin with respect to x and nrm (the gradient with respect
 * to the skinning matrices is lbs_skin_pose_grad's):  dx = A^T dx_out,
 * dn = A^T dn_out.
 * dn_out / dn may both be NULL.  Overwrites dx and dn.                      */
int lbs_skin_backward(void* stream, int n, int n_joints, const float* skin,
                      const int32_t* jidx, const float* jw, const float* dx_out,
                      const float* dn_out, float* dx, float* dn);

/* The pose gradient of lbs_skin (the skinning matrices are what pose
 * optimisation, Sec. 3.3, differentiates): dskin [n_joints][3][4] =
 * sum_i w_ij (dx_out_i (x_i, 1)^T + dn_out_i (nrm_i, 0)^T + (dA_i, 0)),
 * summed over the slots of each Gaussian that name joint j (dA [9][n], the
 * gradient with respect to A from splat_backward, may be NULL); x_i is the
 * skinned point x + disp of lbs_skin (disp may be NULL).  nrm and dn_out are
 * both set or both NULL.  ws: lbs_skin_pose_grad_workspace(n, n_joints)
 * bytes of device memory (per-chunk sums, added in a fixed order).
 * Overwrites dskin.
 * Errors: RGA_EINVAL (sizes, null pointers), RGA_ECAPACITY (ws too small). */
/* The skinning matrices of an axis-angle pose (theta in R^72 for 24 joints,
 * Sec. 3.1 attributes; pose optimisation, Sec. 3.3).  Reading: forward
 * kinematics R_j = exp([theta_j]x) (Rodrigues), G_j = G_parent R_j,
 * P_j = P_parent + G_parent (J_j - J_parent), skin_j = [G_j | P_j - G_j J_j];
 * a joint whose parent is not in 0..j-1 is a root (G = R, P = J_j).
 * theta [n_joints][3], joints [n_joints][3] rest positions, parents
 * [n_joints] int32, skin [n_joints][3][4] (the layout of lbs_skin), all
 * device memory; n_joints in 1..256.  pose_to_skin_backward: dskin ->
 * dtheta [n_joints][3], overwritten, or with accumulate != 0 added to what
 * dtheta holds (theta also reaches the loss through the displacement
 * network, whose adjoint writes its share first).  Errors: RGA_EINVAL.    */
int pose_to_skin(void* stream, int n_joints, const float* theta, const float* joints,
                 const int32_t* parents, float* skin);
int pose_to_skin_backward(void* stream, int n_joints, const float* theta, const float* joints,
                          const int32_t* parents, const float* dskin, float* dtheta,
                          int accumulate);
size_t lbs_skin_pose_grad_workspace(int n, int n_joints);
int lbs_skin_pose_grad(void* stream, int n, int n_joints, const int32_t* jidx, const float* jw,
                       const float* x, const float* disp, const float* nrm, const float* dx_out,
                       const float* dn_out, const float* dA, float* dskin, void* ws,
                       size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Sec. 3.2 (visibility computation): orthographic rasterization of the posed
 * mesh along each of V view directions into a res x res triangle-index image;
 * the three vertices of every triangle that wins a sample are visible; then
 * mean(median(median(V))) over the kv nearest vertices (filter equations).
 * verts     [3][nv] posed vertex positions;  faces [nf][3] int32
 * view_dirs [V][3] unit directions (from the body toward the light)
 * res       raster resolution, 1..128
 * knn       [nv][kv] int32 nearest canonical vertices of each vertex (the
 *           vertex itself included), kv odd, 1..31
 * raw_bits  [nv][ceil(V/32)] uint32 raw visibility bits (bit k&31 of word
 *           k>>5 for view k), or NULL
 * count     [nv][V] uint8 filtered visibility in 0..kv (the mean filter's
 *           value is count/kv)
 * ws        device workspace of at least mesh_visibility_workspace(nv, V) bytes
 * Raster rules: the frame is the posed mesh's bounding box centre and 1.01x
 * half its diagonal; projected coordinates snap to 1/256 pixel; samples at
 * pixel centres; triangles are two-sided, zero-area ones skipped; a sample on
 * an edge belongs to the edge's owner by a fixed tie rule; the nearest
 * triangle wins, ties to the lower index.  Outputs are bit-exact.           */
size_t mesh_visibility_workspace(int nv, int V);
int mesh_visibility(void* stream, int nv, int nf, const float* verts, const int32_t* faces,
                    int V, const float* view_dirs, int res, const int32_t* knn, int kv,
                    uint32_t* raw_bits, uint8_t* count, void* ws, size_t ws_bytes);

/* The shadow-mapping alternative discussed in Sec. 3.2 (discussion with
 * shadow mapping): the same raster and filters, but a vertex's raw
 * visibility from a view is a depth test: its depth is at most the depth
 * map's at the raster sample of the pixel it projects into plus bias_px
 * pixel widths (one pixel = 2 rho / res of the view's frame), or that
 * sample holds no triangle.  bias_px in [0, 64] (RGA_EINVAL otherwise);
 * the other arguments are those of mesh_visibility.                       */
int mesh_visibility_shadowmap(void* stream, int nv, int nf, const float* verts,
                              const int32_t* faces, int V, const float* view_dirs, int res,
                              const int32_t* knn, int kv, float bias_px, uint32_t* raw_bits,
                              uint8_t* count, void* ws, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * visibility of mesh_visibility (same arguments without the workspace, same
 * bit-exact outputs), its workspace taken from a fixed device array of the
 * library, mesh_visibility_noalloc_limit() bytes (32 MiB) per GPU, held from
 * the first call on that GPU until the process ends.  Sizes whose workspace
 * (mesh_visibility_workspace(nv, V)) exceeds that limit return RGA_ECAPACITY
 * before any launch.  Calls that overlap on one GPU (concurrent streams or
 * host threads) share the array and race; serialise them.  Allocates
 * nothing and calls no allocating routine.                                  */
size_t mesh_visibility_noalloc_limit(void);
int mesh_visibility_noalloc(void* stream, int nv, int nf, const float* verts,
                            const int32_t* faces, int V, const float* view_dirs, int res,
                            const int32_t* knn, int kv, uint32_t* raw_bits, uint8_t* count);

/* ------------------------------------------------------------------------
 * Sec. 3.1, rendering equation, and App. A (BRDF): per-Gaussian shading
 *   L_o = sum_k L^k A^k R(w_k, w_o, n) v_g[k] max(0, w_k . n),
 *   R = a/pi + p D F G / (4 (n.w_i)(n.w_o)),  GGX D with alpha = gamma^2,
 *   F = F0 + (1-F0) 2^((-5.55473 oh - 6.98316) oh), F0 = 0.04,
 *   G = G1(w_i) G1(w_o), G1(x) = x / (x (1-k) + k), k = (gamma+1)^2 / 8,
 * then colour = sRGB transfer curve of L_o (gamma correction).  Gaussians
 * whose normal faces away from the camera (n'.(cam - x') <= 0 in FP32) get
 * front = 0 and colour 0.
 * x, nrm     [3][n] posed positions and (unnormalised) normals
 * albedo [3][n], rough [n] (gamma > 0), tint [n] (specular tint p)
 * vidx [3][n] int32, vw [3][n]: the K_g = 3 nearest mesh vertices of each
 *            Gaussian and their normalised inverse-distance weights (Eq.
 *            interpolate): v_g[k] = sum_j vw_j count[vidx_j][view(k)] / kv
 * count      [nv][V] uint8 from mesh_visibility, V = hv * wv
 * env        [he*we][3] radiance of the lat-long map; texel (r, c) has polar
 *            angle (r+0.5) pi/he from +Y, azimuth (c+0.5) 2pi/we, direction
 *            (sin th sin ph, cos th, sin th cos ph), area = its solid angle
 * hv, wv     the view grid (a coarser lat-long grid dividing he x we): texel
 *            (r, c) uses view (r*hv/he)*wv + c*wv/we
 * cam_pos    host float[3], camera centre in world space
 * precision  RGA_FP32 or RGA_BF16X3
 * color      [3][n] out;  front [n] uint8 out
 * tape       NULL, or tape_bytes >= shade_tape_bytes(n, he, we) of device
 *            memory (16-byte aligned) that receives the live (Gaussian,
 *            direction) pairs the sum visited: per Gaussian their number
 *            and, in the order visited (the FP32 walk's, or the BF16X3
 *            form's 32-direction steps), each pair's direction and
 *            interpolated visibility.  The adjoint of the same inputs can
 *            read them instead of testing every direction again.
 * Limits (RGA_EUNSUPPORTED otherwise): V % 16 == 0 and V <= 2048; hv | he
 * and wv | we; he*we <= 3584 directions; the LDS tables must fit 160 KB:
 * 32 K + 48 V bytes (forward) and 44 K + 48 V + 1536 bytes (adjoint) for
 * K = he*we directions and V views (e.g. 2048 directions with 1024 views).
 * RGA_BF16X3 also needs K % 32 == 0, one or two texels per view (hv == he,
 * we == wv or we == 2 wv), and at most 3296 directions in the forward and
 * 2272 in the adjoint.                                                      */
int shade_gaussians(void* stream, int n, const float* x, const float* nrm, const float* albedo,
                    const float* rough, const float* tint, const int32_t* vidx, const float* vw,
                    const uint8_t* count, int nv, int kv, int he, int we, int hv, int wv,
                    const float* env, const float* cam_pos, int precision, float* color,
                    uint8_t* front, void* tape, size_t tape_bytes);

/* Bytes of a live-pair tape for n Gaussians and an he x we map: an int32
 * count per Gaussian (rounded up to 256 bytes), then 8 bytes per
 * (Gaussian, direction) slot.                                               */
size_t shade_tape_bytes(int n, int he, int we);

/* Adjoint of shade_gaussians.  Recomputes the BRDF weights; L_o is recovered
 * from `color` (the forward output) by inverting the transfer curve.
 * dcolor [3][n] in.  Outputs: dx [3][n] (ACCUMULATES: dx += d/dx'),
 * dn [3][n], dalbedo [3][n], drough [n], dtint [n] (overwritten),
 * denv [he*we][3] (overwritten).  ws: shade_gaussians_workspace bytes.
 * tape: NULL (every direction is tested again), or the tape that
 * shade_gaussians wrote for these same inputs (x, nrm, rough, vidx, vw,
 * count, env, cam_pos, the grids): the live pairs are read from it, which
 * gives the same sums with less work.  A tape from other inputs gives wrong
 * gradients (it is not checked).  Given a tape the adjoint is the FP32
 * replay in either form (for RGA_BF16X3 the tape of its MFMA forward); the
 * MFMA adjoint runs for RGA_BF16X3 without one.                             */
size_t shade_gaussians_workspace(int n, int he, int we);
int shade_gaussians_backward(void* stream, int n, const float* x, const float* nrm,
                             const float* albedo, const float* rough, const float* tint,
                             const int32_t* vidx, const float* vw, const uint8_t* count, int nv,
                             int kv, int he, int we, int hv, int wv, const float* env,
                             const float* cam_pos, int precision, const float* color,
                             const uint8_t* front, const float* dcolor, float* dx, float* dn,
                             float* dalbedo, float* drough, float* dtint, float* denv, void* ws,
                             size_t ws_bytes, const void* tape, size_t tape_bytes);

/* ------------------------------------------------------------------------
 * Sec. 3.1, last paragraph: splatting with the 3DGS tile rasterizer.
 * Projection: X = R x' + t; culled if Z <= 0.2, front == 0, opacity < 1/255
 * or the 2D covariance is not positive definite.  Covariance factor
 * M = A R(q/|q|) diag(exp(log_s)); Sigma2D = J R M M^T R^T J^T + 0.3 I with
 * the perspective Jacobian J at the centre.  Near-degenerate splats
 * (det <= 2^-12 a c in FP32) take the 2x2 covariance, determinant and
 * inverse in FP64.  Each splat is binned into the 16x16-pixel tiles of the
 * box bounding its alpha >= 1/255 ellipse; per tile, splats are ordered by
 * (float bits of Z, index); pixels composite front to back with
 * alpha = min(0.99, o exp(-d^T Conic d / 2)), skipping alpha < 1/255 and
 * stopping before the transmittance drops below 1e-4; black background.
 * Inputs: x [3][n], A [9][n] (from lbs_skin), quat [4][n] (w,x,y,z),
 * log_s [3][n], opac [n], color [3][n], front [n].
 * capacity   maximum number of (splat, tile) duplicates D the workspace holds
 * ws         splat_workspace_size(n, width, height, capacity) bytes; holds the
 *            per-splat records, sorted lists, tile ranges and, per pixel,
 *            the (colour, transmittance) state at every 64th entry of each
 *            tile list that splat_backward and splat_state read.  Keep it
 *            alive and unmodified until the backward pass.
 * image [3][H][W], T_final [H][W] out.
 * No host synchronisation: if D exceeds capacity the lists are truncated, the
 * image and T_final are poisoned (every value NaN) and splat_read_count
 * reports D > capacity (retry larger); a splat_backward on that workspace
 * writes NaN gradients.                                                    */
size_t splat_workspace_size(int n, int width, int height, int64_t capacity);
int splat_forward(void* stream, int n, const rga_camera* cam, const float* x, const float* A,
                  const float* quat, const float* log_s, const float* opac, const float* color,
                  const uint8_t* front, void* ws, size_t ws_bytes, int64_t capacity,
                  float* image, float* T_final);

/* splat_forward in two calls, so that the part the colours do not enter can
 * run while the shading computes them.  splat_bin: projection, depth sort,
 * duplication, tile sort, tile ranges and work items (arguments as for
 * splat_forward).  splat_blend: the compositing of the colours [3][n];
 * image and T_final as for splat_forward.
 * splat_blend reads what the last splat_bin left in ws (same n, camera and
 * capacity): the caller orders the two (one stream, or an event between
 * two); a workspace no splat_bin (or splat_forward) has filled holds no
 * valid lists, and splat_blend on it is undefined (its indices are read
 * from the workspace).  splat_forward = splat_bin then splat_blend on one
 * stream.  Errors as for splat_forward.                                    */
int splat_bin(void* stream, int n, const rga_camera* cam, const float* x, const float* A,
              const float* quat, const float* log_s, const float* opac, const uint8_t* front,
              void* ws, size_t ws_bytes, int64_t capacity);
int splat_blend(void* stream, int n, const rga_camera* cam, const float* color, void* ws,
                size_t ws_bytes, int64_t capacity, float* image, float* T_final);

/* Sec. 3.1, the back-face rule (a Gaussian whose normal faces away from the
 * camera gets zero opacity) on its own: front[g] = 1 if
 * nrm_g . (cam_pos - x_g) > 0 in FP32 on the unnormalised posed normal,
 * evaluated as fma(n_z, w_z, fma(n_y, w_y, n_x w_x)) with w = cam_pos - x_g,
 * else 0 -- bit for bit the flags shade_gaussians writes, for a caller that
 * bins the splats (splat_bin) before the shading runs.  x, nrm [3][n]
 * device; cam_pos host float[3]; front [n] uint8 device out.
 * Errors: RGA_EINVAL (n < 0, null pointers).                               */
int back_face(void* stream, int n, const float* x, const float* nrm, const float* cam_pos,
              uint8_t* front);

/* Synchronises `stream` and returns the duplicate count D of the last
 * splat_forward (or splat_bin) that used ws (may exceed capacity: then
 * re-run larger).                                                          */
int splat_read_count(void* stream, const void* ws, int n, int width, int height,
                     int64_t capacity, int64_t* D);

/* Device pointers into a splat workspace (valid after splat_forward):
 * mean2d [2][n] f32, conic [3][n] f32 (A, B, C of the inverse covariance),
 * depth [n] f32, rect [4][n] int32 (tx0, ty0, tx1, ty1), touched [n] int32,
 * fp64 [n] uint8, sorted [D] int32 splat indices per tile in tile order,
 * ranges [tiles][2] int32 [start, end), count: device int64 D.             */
typedef struct rga_splat_state {
  float* mean2d;
  float* conic;
  float* depth;
  int32_t* rect;
  int32_t* touched;
  uint8_t* fp64;
  int32_t* sorted;
  int32_t* ranges;
  int64_t* count;
  int32_t tiles_x, tiles_y;
} rga_splat_state;
int splat_state(void* ws, int n, int width, int height, int64_t capacity, rga_splat_state* st);

/* Adjoint of splat_forward given dL/dimage.  Re-walks every tile list front to
 * back recomputing the transmittance (nothing per (pixel, splat) is stored);
 * `image` is the forward output and `color` the colours it composited.  Outputs (overwritten): dx [3][n],
 * dquat [4][n], dlog_s [3][n], dopac [n], dcolor [3][n], and, unless NULL,
 * dA [9][n]: the gradient with respect to the skinning's linear part A
 * through the covariance (A R S), which the pose gradient needs.           */
int splat_backward(void* stream, int n, const rga_camera* cam, const float* x, const float* A,
                   const float* quat, const float* log_s, const float* opac,
                   const float* color, const uint8_t* front, void* ws, size_t ws_bytes,
                   int64_t capacity, const float* image, const float* dimage, float* dx,
                   float* dquat, float* dlog_s, float* dopac, float* dcolor, float* dA);

/* ------------------------------------------------------------------------
 * Sec. 3.3, image loss (its L1 term): loss = mean |image - target| over
 * `count` values; dimage = sign(image - target) / count (sign(0) = 0).
 * loss: device float[1]; dimage may be NULL.  ws: l1_loss_workspace bytes.  */
size_t l1_loss_workspace(int64_t count);
int l1_loss(void* stream, int64_t count, const float* image, const float* target, float* loss,
            float* dimage, void* ws, size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Sec. 3.1, interpolation equation: the K_g (or K_v) nearest canonical mesh
 * vertices of each Gaussian (or vertex), and the attribute average
 *   *_g = sum_{j in S_g} u_j *^j / sum_{j in S_g} u_j,  u_j = 1 / |x_g - x_j|.
 * Neighbours are ordered by (squared distance, vertex index); the squared
 * distance is computed in FP32 as fmaf(dz, dz, fmaf(dy, dy, dx * dx)) with
 * d = x_j - x_g, so the sets and their order are exact (ties: lower index
 * first).  w_t = u_t / sum u (normalised, FP32); a query at distance 0 from
 * its nearest vertex gets w = (1, 0, ...).  No gradient flows through the
 * choice of neighbours or the weights (decisions of the method).
 *
 * knn_build: ref [3][nr] reference points (e.g. the canonical vertices); ws
 *   is knn_workspace(nr) bytes of device memory owned by the caller, filled
 *   with a uniform grid over ref; keep it unmodified while querying.
 * knn_query: q [3][n] query points; k in 1..min(32, nr); idx [k][n] int32 and
 *   w [k][n] out (t-th nearest in row t).  Queries may lie outside ref's box.
 *   scratch: knn_query_workspace(n) bytes of device memory (the queries are
 *   taken in grid-cell order); ws is the built grid, read only.
 * knn_interpolate: attr [C][nr] vertex attributes -> out [C][n] =
 *   sum_t w[t][i] attr[c][idx[t][i]] (t in order, FP32).
 * knn_interpolate_backward: dout [C][n] -> dattr [C][nr] (overwritten) =
 *   sum over (i, t) with idx[t][i] = j of w[t][i] dout[c][i] (partial sums
 *   per workgroup, added with float atomics: the rounding of the sum may
 *   vary between runs).  C <= 65535.
 * Errors: RGA_EINVAL for bad sizes or NULL pointers, RGA_ECAPACITY for a
 * short workspace; all calls are asynchronous on `stream`.                  */
size_t knn_workspace(int nr);
int knn_build(void* stream, int nr, const float* ref, void* ws, size_t ws_bytes);
size_t knn_query_workspace(int n);
int knn_query(void* stream, int n, const float* q, int nr, int k, int32_t* idx, float* w,
              const void* ws, size_t ws_bytes, void* scratch, size_t scratch_bytes);
int knn_interpolate(void* stream, int n, int k, const int32_t* idx, const float* w, int C, int nr,
                    const float* attr, float* out);
int knn_interpolate_backward(void* stream, int n, int k, const int32_t* idx, const float* w,
                             int C, int nr, const float* dout, float* dattr);

/* ------------------------------------------------------------------------
 * Image loss of the training section (Sec. 3.3, image-loss equation):
 * L = (1 - lambda) L_1 + lambda L_D-SSIM (the paper sets lambda = 0.2).
 * Readings: L_1 = mean |image - target| over C H W; L_D-SSIM = 1 - the mean
 * SSIM over C H W, SSIM of Wang et al. with an 11 x 11 Gaussian window of
 * std 1.5, C1 = 0.01^2, C2 = 0.03^2, every channel filtered on its own with
 * zero padding (the window is cut at the border, not renormalised).
 * image, target [C][H][W] device float; loss device float[1]; dimage
 * [C][H][W] = dL/dimage (written; may be NULL to skip the adjoint; the
 * sign of 0 is 0).  ws: image_loss_workspace(C, H, W) bytes of device memory
 * owned by the caller (the adjoint's per-pixel terms and per-tile sums).
 * Errors: RGA_EINVAL (sizes outside 1..65535 channels, 1..2^20 pixels per
 * side, lambda outside [0, 1], null pointer), RGA_ECAPACITY (ws too small);
 * nothing is launched then.                                                */
size_t image_loss_workspace(int C, int H, int W);
int image_loss(void* stream, int C, int H, int W, const float* image, const float* target,
               float lambda, float* loss, float* dimage, void* ws, size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Regularisers of the training loss (Sec. 3.3): L_smooth = sum_i sum_{k in
 * S_v(i)} |m_i - m_k|_1 over the materials (albedo rgb, roughness, tint),
 * L_mdist = sum_g sum_{k in S_g(g)} |x_g - x_k|_2, L_disp = sum_i |dx_i|_2,
 * L_scale = sum_g sum_c max(0, s_gc - s_0) with s = exp(log-scale) (the
 * paper: s_0 = 0.005, lambdas 0.002, 0.1, 0.02, 10).
 * mat [5][nv]; knn_v [nv][kv] int32 (the K_v nearest vertices of each
 * vertex); xg [3][n] canonical Gaussian positions; verts [3][nv]; vidx
 * [kg][n] int32 (the K_g nearest vertices of each Gaussian); disp [3][nv];
 * log_s [3][n]; all device memory, indices clamped to 0..nv-1.
 * terms device float[5]: the four unweighted sums and the weighted total.
 * dmat [5][nv], dxg [3][n], ddisp [3][nv], dlogs [3][n]: gradients of the
 * weighted total (a zero difference or length gives 0), written, or with
 * accumulate != 0 added to what they hold (so that the image loss's
 * gradients and these meet inside the library: the total loss of Sec. 3.3).
 * loss_accum: device float[1] to which the weighted total is added (e.g. the
 * image loss), or NULL.
 * ws: regularisers_workspace(nv, n) bytes of device memory.
 * Errors: RGA_EINVAL (nv < 1, n < 0, kv or kg outside 1..nv, null pointer),
 * RGA_ECAPACITY (ws too small); nothing is launched then.                 */
size_t regularisers_workspace(int nv, int n);
int regularisers(void* stream, int nv, int n, int kv, int kg, const float* mat,
                 const int32_t* knn_v, const float* xg, const float* verts, const int32_t* vidx,
                 const float* disp, const float* log_s, float s0, float lam_smooth,
                 float lam_mdist, float lam_disp, float lam_scale, float* terms, float* dmat,
                 float* dxg, float* ddisp, float* dlogs, int accumulate, float* loss_accum,
                 void* ws, size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Pose-dependent vertex displacement dx = d(x, theta) (Sec. 3.1, attribute
 * paragraph: an MLP of the canonical position and the pose; Sec. 3.5,
 * implementation details: four layers of width 256 with ReLU and random
 * Fourier features of the coordinates).  Readings: gamma(x) =
 * [sin(2 pi B x), cos(2 pi B x)] with B [RGA_MLP_FREQS][3]; the input of
 * the first layer is [gamma(x), theta] (128 + 72); four hidden layers
 * h_l = relu(W_l h_{l-1} + b_l) and a linear output dx = W_5 h_4 + b_5.
 *
 * params: RGA_MLP_PARAMS floats, W_1 [256][200], b_1 [256], W_2 [256][256],
 *   b_2, W_3, b_3, W_4, b_4, W_5 [3][256], b_5 [3] (row-major, out x in).
 * x [3][nv] canonical vertex positions; freqs B [64][3]; theta [72]; all
 *   device memory.  ws: mlp_workspace(nv) bytes of device memory owned by
 *   the caller, 16-byte aligned: the operands packed from params, the
 *   kept activations and the adjoint's partial sums.
 * mlp_forward: dx [3][nv] (written).  The products run on bf16 MFMA with
 *   FP32 accumulation, each operand split into bf16 high and low parts
 *   (hi.hi + lo.hi + hi.lo): about FP32 accuracy.
 * mlp_backward: the adjoint of the last mlp_forward on the same ws (same
 *   nv, x, freqs, theta, params; it reads the packed operands and the kept
 *   activations): ddx [3][nv] -> dparams [RGA_MLP_PARAMS] and dtheta [72]
 *   (overwritten).  Calls on one ws must not overlap.
 * Errors: RGA_EINVAL (nv outside 0..2^26, null pointer, unaligned ws),
 *   RGA_ECAPACITY (ws too small); nothing is launched then.              */
#define RGA_MLP_FREQS 64
#define RGA_MLP_POSE 72
#define RGA_MLP_WIDTH 256
#define RGA_MLP_PARAMS 249603
size_t mlp_workspace(int nv);
int mlp_forward(void* stream, int nv, const float* x, const float* freqs, const float* theta,
                const float* params, void* ws, size_t ws_bytes, float* dx);
int mlp_backward(void* stream, int nv, const float* x, const float* freqs, const float* theta,
                 const float* params, const float* ddx, void* ws, size_t ws_bytes,
                 float* dparams, float* dtheta);

/* ------------------------------------------------------------------------
 * App. B (Gaussian densification algorithm, Alg. 1): density-based
 * densification.  D_v[k] counts the Gaussians whose K_g nearest vertices
 * include vertex k; a triangle's density is the sum of its three vertices'
 * counts over 6 K_g (each vertex taken to touch six triangles); triangles
 * below the threshold d0 get the weight P = max(0, d0 - d_f); sum(P) p0
 * Gaussians (rounded down) are drawn multinomially with probabilities
 * P / sum(P), each at a uniform random point of its triangle.
 * P is held exactly as the integer Q = max(0, round(d0 6 K_g 65536) - 65536 S)
 * (S the vertex sum), so the draws are reproducible: draw j takes outputs
 * 3j+1, 3j+2, 3j+3 of SplitMix64 seeded with `seed` (Steele, Lea and Flood,
 * OOPSLA 2014); the first selects the triangle whose cumulative range of Q
 * holds floor(r sum(Q) / 2^64), the other two (shifted right by 40, times
 * 2^-24) give u1, u2 and the point with barycentric weights (1 - s,
 * s (1 - u2), s u2), s = sqrt(u1), over the triangle's vertices in order.
 * sg     [kg][n] int32 K_g nearest vertices of each Gaussian; kg in 1..64
 * verts  [3][nv] vertex positions (the canonical mesh); faces [nf][3] int32
 * d0, p0 the density threshold and the fraction added per call (the paper
 *        uses 1 and 0.02), each in [0, 1e6]
 * cap    room for new positions: draws j < cap write x_out[:, j] and
 *        f_out[j] (draw order); every draw is counted in ng
 * Outputs (device, overwritten): Dv [nv], df [nf] float, ng [nf],
 * x_out [3][cap], f_out [cap], summary int64[2] = {sum(Q), N'} (N' may
 * exceed cap; read it to size the next call).  ws: densify_workspace(nf)
 * bytes.  Bit-exact against the oracle.  Errors: RGA_EINVAL (sizes, range,
 * null pointers), RGA_ECAPACITY (ws too small); nothing is launched then. */
size_t densify_workspace(int nf);
int densify(void* stream, int n, int kg, const int32_t* sg, int nv, const float* verts, int nf,
            const int32_t* faces, double d0, double p0, uint64_t seed, int64_t cap, int32_t* Dv,
            float* df, int32_t* ng, float* x_out, int32_t* f_out, int64_t* summary, void* ws,
            size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Storage order of the Gaussians (Sec. 3.1: each Gaussian reads the
 * visibility counts of its K_g nearest mesh vertices).  The Gaussians are a
 * set: their order in memory is free, and storing them grouped by nearest
 * vertex lets the shading kernels' nearby waves gather the same count rows
 * (and each XCD's L2 hold its share of the table).
 *
 * vertex_order: order [n] int32 out, the indices 0..n-1 sorted stably by
 * vidx row 0 (vertex ids clamped to 0..nv-1; ties in index order), i.e. a
 * permutation; vidx [3][n] int32 (row 0 read).  ws: vertex_order_workspace(n)
 * bytes, 16-byte aligned.  Errors: RGA_EINVAL (n < 0, nv < 1, null
 * pointers, misaligned ws), RGA_ECAPACITY (ws too small); nothing is
 * launched then.  Bit-exact (a stable sort has one result).
 *
 * gather_columns: dst[r][j] = src[r][order[j]] for `rows` rows of n 4-byte
 * elements (float or int32), to apply an order to every per-Gaussian array
 * (and its optimiser state).  src and dst must not overlap; order entries
 * are clamped to 0..n-1.  Errors: RGA_EINVAL (negative sizes, null
 * pointers, src == dst), RGA_EUNSUPPORTED (rows * n beyond 2^39).           */
size_t vertex_order_workspace(int n);
int vertex_order(void* stream, int n, const int32_t* vidx, int nv, int32_t* order, void* ws,
                 size_t ws_bytes);
int gather_columns(void* stream, int rows, int n, const void* src, const int32_t* order,
                   void* dst);

/* ------------------------------------------------------------------------
 * The optimiser of the training loop (the paper trains as 3DGS does; the
 * reading is Adam): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * param -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * param, m, v [count] updated in place; grad [count]; device memory; step
 * is 1-based.  Errors: RGA_EINVAL (count < 0, step < 1, betas outside
 * [0, 1), eps <= 0, null pointer).                                         */
int adam_step(void* stream, int64_t count, float* param, const float* grad, float* m, float* v,
              float lr, float beta1, float beta2, float eps, int step);

/* ------------------------------------------------------------------------
 * Kernel timing with HIP events, for measurement.  While enabled, every
 * kernel launch is bracketed by events on its stream; rga_timing_read
 * synchronises and returns the summed milliseconds and launch count of the
 * kernels whose name matches `kernel` exactly.                              */
int rga_timing_enable(int on);
/* Restrict timing to kernels named `kernel` (NULL or "" times every kernel). */
int rga_timing_filter(const char* kernel);
int rga_timing_reset(void);
int rga_timing_read(const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* RGA_H */
