/*
 * CPU oracle for the relightable Gaussian-avatar render path -- TEST
 * INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load this library; the product path never does.
 *
 * This file is the FP32 "mirror" half of the oracle: the parts of the method
 * whose floating-point arithmetic decides an integer (which triangle wins a
 * raster sample, which tiles a splat touches, the depth order of splats, the
 * back-face flag) written out plainly in single precision with a fixed,
 * documented operation order and explicit fmaf, so that those integers can be
 * compared bit for bit.  Values with no integer consequence (shaded colours,
 * gradients) are checked against the FP64 oracle in ref64.py instead.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 * (no contraction: every fused multiply-add below is an explicit fmaf).
 *
 * Sections of the paper this follows:
 *   - Sec. 3.1 (deformation): forward linear blend skinning of Gaussians and mesh.
 *   - Sec. 3.2 (visibility): orthographic triangle-index rasterization of the
 *     posed mesh from each light direction, "triangle appears -> its three
 *     vertices visible", then mean(median(median(V))) over the K_v nearest
 *     vertices (the filter equations of Sec. 3.2).
 *   - Sec. 3.1, last paragraph: Gaussians whose normal faces away from the
 *     camera get zero opacity (back-face flag).
 *   - Sec. 3.1, last paragraph: the 3DGS tile rasterizer (projection, tile
 *     binning, depth sort, front-to-back alpha compositing).
 *   - Sec. 3.1, interpolation equation: the K_g (K_v) nearest canonical
 *     vertices of each Gaussian (vertex), brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Threads used by the parallel loops (reported by the CPU baseline).        */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ======================================================================== */
/* Sec. 3.1: forward LBS.  The posed point is x + sum_j w_j ((R_j - I) x + t_j)
 * (equal to sum_j w_j (R_j x + t_j) when the weights sum to one), the blended
 * linear part is A = I + sum_j w_j (R_j - I), and the normal is carried as A n.
 * skin: [J][3][4] rows [R | t]; jidx/jw: [4][n]; x, nrm: [3][n].            */
void oracle_lbs_f32(int n, int J, const float* skin, const int32_t* jidx,
                    const float* jw, const float* x, const float* nrm,
                    float* x_out, float* n_out, float* A_out) {
  (void)J;
  for (int i = 0; i < n; ++i) {
    const float p0 = x[i], p1 = x[n + i], p2 = x[2 * n + i];
    float acc[3] = {0.f, 0.f, 0.f};
    float Aacc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < 4; ++j) {
      const float w = jw[j * n + i];
      const float* S = skin + 12 * jidx[j * n + i];
      for (int a = 0; a < 3; ++a) {
        const float d0 = S[4 * a + 0] - (a == 0 ? 1.f : 0.f);
        const float d1 = S[4 * a + 1] - (a == 1 ? 1.f : 0.f);
        const float d2 = S[4 * a + 2] - (a == 2 ? 1.f : 0.f);
        const float pa = fmaf(d2, p2, fmaf(d1, p1, fmaf(d0, p0, S[4 * a + 3])));
        acc[a] = fmaf(w, pa, acc[a]);
        Aacc[3 * a + 0] = fmaf(w, d0, Aacc[3 * a + 0]);
        Aacc[3 * a + 1] = fmaf(w, d1, Aacc[3 * a + 1]);
        Aacc[3 * a + 2] = fmaf(w, d2, Aacc[3 * a + 2]);
      }
    }
    x_out[i] = p0 + acc[0];
    x_out[n + i] = p1 + acc[1];
    x_out[2 * n + i] = p2 + acc[2];
    float A[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) A[3 * a + b] = (a == b ? 1.f : 0.f) + Aacc[3 * a + b];
    if (A_out)
      for (int k = 0; k < 9; ++k) A_out[k * n + i] = A[k];
    if (nrm && n_out) {
      const float m0 = nrm[i], m1 = nrm[n + i], m2 = nrm[2 * n + i];
      for (int a = 0; a < 3; ++a)
        n_out[a * n + i] = fmaf(A[3 * a + 2], m2, fmaf(A[3 * a + 1], m1, A[3 * a + 0] * m0));
    }
  }
}

/* Sec. 3.1: a Gaussian whose (posed) normal faces away from the camera is
 * dropped.  front = n' . (cam - x') > 0, decided in FP32.                    */
void oracle_front_f32(int n, const float* x, const float* nrm, const float* cam,
                      uint8_t* front) {
  for (int i = 0; i < n; ++i) {
    const float w0 = cam[0] - x[i], w1 = cam[1] - x[n + i], w2 = cam[2] - x[2 * n + i];
    const float d = fmaf(nrm[2 * n + i], w2, fmaf(nrm[n + i], w1, nrm[i] * w0));
    front[i] = d > 0.f ? 1 : 0;
  }
}

/* ======================================================================== */
/* Sec. 3.2: visibility by orthographic rasterization of the posed mesh.     */

/* Bounding frame of the posed mesh: centre c and radius rho (1.01 x half the
 * AABB diagonal) so that every vertex projects inside the raster.           */
void oracle_vis_frame(int nv, const float* v, float* c, float* rho) {
  float lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = v[a * nv];
    hi[a] = v[a * nv];
    for (int i = 1; i < nv; ++i) {
      lo[a] = fminf(lo[a], v[a * nv + i]);
      hi[a] = fmaxf(hi[a], v[a * nv + i]);
    }
  }
  float e[3];
  for (int a = 0; a < 3; ++a) {
    c[a] = (lo[a] + hi[a]) * 0.5f;
    e[a] = hi[a] - lo[a];
  }
  float r = 1.01f * (0.5f * sqrtf(fmaf(e[2], e[2], fmaf(e[1], e[1], e[0] * e[0]))));
  if (!(r > 0.f)) r = 1.f;
  *rho = r;
}

/* Orthonormal basis (t, b) perpendicular to the unit direction d, by the
 * branch-free construction of Duff et al. (JCGT 6(1), 2017).                */
static void basis_f32(const float* d, float* t, float* b) {
  const float sgn = copysignf(1.f, d[2]);
  const float a = -1.f / (sgn + d[2]);
  const float bb = (d[0] * d[1]) * a;
  t[0] = 1.f + ((sgn * d[0]) * d[0]) * a;
  t[1] = sgn * bb;
  t[2] = -(sgn * d[0]);
  b[0] = bb;
  b[1] = sgn + (d[1] * d[1]) * a;
  b[2] = -d[1];
}

/* Project every vertex for one view: 8-bit sub-pixel fixed point (U, V) and
 * depth z = rho - d.(x - c) (smaller is nearer the light).                  */
static void project_view(int nv, const float* v, const float* c, float rho, const float* d,
                         int res, int32_t* U, int32_t* V, float* z) {
  float t[3], b[3];
  basis_f32(d, t, b);
  const float scale = 0.5f * (float)res;
  const float irho = 1.f / rho;   /* u = (t.(x - c) (1/rho) + 1) res / 2 */
  for (int i = 0; i < nv; ++i) {
    const float q0 = v[i] - c[0], q1 = v[nv + i] - c[1], q2 = v[2 * nv + i] - c[2];
    const float pu = fmaf(t[2], q2, fmaf(t[1], q1, t[0] * q0));
    const float pv = fmaf(b[2], q2, fmaf(b[1], q1, b[0] * q0));
    const float pd = fmaf(d[2], q2, fmaf(d[1], q1, d[0] * q0));
    const float u = (pu * irho + 1.f) * scale;
    const float w = (pv * irho + 1.f) * scale;
    U[i] = (int32_t)rintf(u * 256.f);
    V[i] = (int32_t)rintf(w * 256.f);
    z[i] = rho - pd;
  }
}

static int64_t edge_fn(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t sx, int64_t sy) {
  return (bx - ax) * (sy - ay) - (by - ay) * (sx - ax);
}

/* Tie rule for samples exactly on an edge A->B of a positively oriented
 * triangle: the edge owns them if dy > 0, or dy == 0 and dx < 0.  For two
 * triangles sharing an edge exactly one of them owns it.                    */
static int owns(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  const int64_t dx = bx - ax, dy = by - ay;
  return dy > 0 || (dy == 0 && dx < 0);
}

static int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

/* Raster triangles given in 8-bit sub-pixel fixed point (x, y) with depths z
 * into zbuf[res*res] of keys (float bits of depth << 32 | triangle id); the
 * smallest key wins, so the nearest triangle wins and ties go to the lower
 * id.  Samples sit at pixel centres (256 i + 128, 256 j + 128).  brute != 0
 * tests every sample against every triangle instead of the triangle's
 * bounding box (same result by construction).  claims (may be NULL) counts,
 * per sample, how many triangles cover it.                                  */
static void raster_fixed(int nt, const int64_t* X, const int64_t* Y, const float* Zv,
                         const int32_t* ids, int res, int brute, uint64_t* zbuf,
                         int32_t* claims) {
  for (int p = 0; p < res * res; ++p) zbuf[p] = ~(uint64_t)0;
  if (claims) memset(claims, 0, sizeof(int32_t) * res * res);
  for (int f = 0; f < nt; ++f) {
    int64_t x0 = X[3 * f], y0 = Y[3 * f], x1 = X[3 * f + 1], y1 = Y[3 * f + 1];
    int64_t x2 = X[3 * f + 2], y2 = Y[3 * f + 2];
    float z0 = Zv[3 * f], z1 = Zv[3 * f + 1], z2 = Zv[3 * f + 2];
    int64_t area = edge_fn(x0, y0, x1, y1, x2, y2);
    if (area == 0) continue;
    if (area < 0) {               /* two-sided: make it positively oriented */
      int64_t tx = x1, ty = y1;
      x1 = x2; y1 = y2; x2 = tx; y2 = ty;
      float tz = z1; z1 = z2; z2 = tz;
      area = -area;
    }
    const float ia = 1.f / (float)area;
    int64_t i_lo = 0, i_hi = res - 1, j_lo = 0, j_hi = res - 1;
    if (!brute) {
      int64_t mnx = x0, mxx = x0, mny = y0, mxy = y0;
      if (x1 < mnx) mnx = x1; if (x2 < mnx) mnx = x2;
      if (x1 > mxx) mxx = x1; if (x2 > mxx) mxx = x2;
      if (y1 < mny) mny = y1; if (y2 < mny) mny = y2;
      if (y1 > mxy) mxy = y1; if (y2 > mxy) mxy = y2;
      i_lo = -floor_div(-(mnx - 128), 256);   /* ceil((mnx-128)/256) */
      i_hi = floor_div(mxx - 128, 256);
      j_lo = -floor_div(-(mny - 128), 256);
      j_hi = floor_div(mxy - 128, 256);
      if (i_lo < 0) i_lo = 0;
      if (j_lo < 0) j_lo = 0;
      if (i_hi > res - 1) i_hi = res - 1;
      if (j_hi > res - 1) j_hi = res - 1;
    }
    const int o12 = owns(x1, y1, x2, y2), o20 = owns(x2, y2, x0, y0), o01 = owns(x0, y0, x1, y1);
    for (int64_t j = j_lo; j <= j_hi; ++j) {
      const int64_t sy = 256 * j + 128;
      for (int64_t i = i_lo; i <= i_hi; ++i) {
        const int64_t sx = 256 * i + 128;
        const int64_t w0 = edge_fn(x1, y1, x2, y2, sx, sy);
        const int64_t w1 = edge_fn(x2, y2, x0, y0, sx, sy);
        const int64_t w2 = edge_fn(x0, y0, x1, y1, sx, sy);
        const int in0 = w0 > 0 || (w0 == 0 && o12);
        const int in1 = w1 > 0 || (w1 == 0 && o20);
        const int in2 = w2 > 0 || (w2 == 0 && o01);
        if (!(in0 && in1 && in2)) continue;
        /* depth: barycentric weights w_e / area through the reciprocal */
        const float bz = fmaf((float)w2, z2, fmaf((float)w1, z1, (float)w0 * z0)) * ia;
        uint32_t zb;
        memcpy(&zb, &bz, 4);
        const uint64_t key = ((uint64_t)zb << 32) | (uint32_t)ids[f];
        uint64_t* slot = &zbuf[j * res + i];
        if (key < *slot) *slot = key;
        if (claims) ++claims[j * res + i];
      }
    }
  }
}

/* Raster triangles already in fixed point: xy [nt][3][2] int32, z [nt][3];
 * triangle ids are their indices.                                           */
void oracle_raster_fixed(int nt, const int32_t* xy, const float* z, int res, int brute,
                         uint64_t* zbuf, int32_t* claims) {
  int64_t* X = (int64_t*)malloc(sizeof(int64_t) * 3 * (nt > 0 ? nt : 1));
  int64_t* Y = (int64_t*)malloc(sizeof(int64_t) * 3 * (nt > 0 ? nt : 1));
  int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (nt > 0 ? nt : 1));
  for (int f = 0; f < nt; ++f) {
    ids[f] = f;
    for (int c = 0; c < 3; ++c) {
      X[3 * f + c] = xy[6 * f + 2 * c];
      Y[3 * f + c] = xy[6 * f + 2 * c + 1];
    }
  }
  raster_fixed(nt, X, Y, z, ids, res, brute, zbuf, claims);
  free(X);
  free(Y);
  free(ids);
}

/* Raster one view of the posed mesh along direction d.                      */
void oracle_raster_view(int nv, int nf, const float* v, const int32_t* faces, const float* d,
                        int res, int brute, uint64_t* zbuf) {
  float c[3], rho;
  oracle_vis_frame(nv, v, c, &rho);
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * nv);
  int32_t* V = (int32_t*)malloc(sizeof(int32_t) * nv);
  float* z = (float*)malloc(sizeof(float) * nv);
  project_view(nv, v, c, rho, d, res, U, V, z);
  int64_t* X = (int64_t*)malloc(sizeof(int64_t) * 3 * (nf > 0 ? nf : 1));
  int64_t* Y = (int64_t*)malloc(sizeof(int64_t) * 3 * (nf > 0 ? nf : 1));
  float* Z = (float*)malloc(sizeof(float) * 3 * (nf > 0 ? nf : 1));
  int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (nf > 0 ? nf : 1));
  for (int f = 0; f < nf; ++f) {
    ids[f] = f;
    for (int k = 0; k < 3; ++k) {
      const int vi = faces[3 * f + k];
      X[3 * f + k] = U[vi];
      Y[3 * f + k] = V[vi];
      Z[3 * f + k] = z[vi];
    }
  }
  raster_fixed(nf, X, Y, Z, ids, res, brute, zbuf, NULL);
  free(X);
  free(Y);
  free(Z);
  free(ids);
  free(U);
  free(V);
  free(z);
}

/* Projected fixed-point coordinates and depths of every vertex for one view
 * (exposed for tests): U, V [nv] int32, z [nv].                             */
void oracle_project_view(int nv, const float* v, const float* d, int res, int32_t* U,
                         int32_t* V, float* z) {
  float c[3], rho;
  oracle_vis_frame(nv, v, c, &rho);
  project_view(nv, v, c, rho, d, res, U, V, z);
}

/* Filters of Sec. 3.2 on one view's 0/1 vertex map (kv odd):
 *   median over the kv nearest vertices of a 0/1 map = [count >= (kv+1)/2];
 *   m1 = median(raw), m2 = median(m1), cnt = sum of m2 over the neighbours
 *   (the mean filter is cnt / kv).                                          */
void oracle_vis_filter(int nv, const uint8_t* raw, const int32_t* knn, int kv,
                       uint8_t* m1, uint8_t* m2, uint8_t* cnt) {
  const int half = (kv + 1) / 2;
  for (int i = 0; i < nv; ++i) {
    int s = 0;
    for (int j = 0; j < kv; ++j) s += raw[knn[i * kv + j]];
    m1[i] = s >= half;
  }
  for (int i = 0; i < nv; ++i) {
    int s = 0;
    for (int j = 0; j < kv; ++j) s += m1[knn[i * kv + j]];
    m2[i] = s >= half;
  }
  for (int i = 0; i < nv; ++i) {
    int s = 0;
    for (int j = 0; j < kv; ++j) s += m2[knn[i * kv + j]];
    cnt[i] = (uint8_t)s;
  }
}

/* The shadow-mapping alternative the paper discusses (Sec. 3.2, discussion
 * with shadow mapping): a vertex is seen from a view when its own depth is
 * at most the depth map's at the raster sample of the pixel it projects
 * into, plus a bias of bias_px pixel widths (2 rho / res per pixel), or
 * when that sample holds no triangle.  raw[nv] gets the 0/1 map.           */
static void shadow_view(int nv, int nf, const float* v, const int32_t* faces, const float* d,
                        int res, float bias_px, uint64_t* zbuf, uint8_t* raw) {
  float c[3], rho;
  oracle_vis_frame(nv, v, c, &rho);
  oracle_raster_view(nv, nf, v, faces, d, res, 0, zbuf);
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * nv);
  int32_t* W = (int32_t*)malloc(sizeof(int32_t) * nv);
  float* z = (float*)malloc(sizeof(float) * nv);
  project_view(nv, v, c, rho, d, res, U, W, z);
  const float bias = bias_px * (2.f * rho) / (float)res;
  for (int i = 0; i < nv; ++i) {
    int px = U[i] >> 8, py = W[i] >> 8;   /* the pixel holding the point */
    px = px < 0 ? 0 : (px > res - 1 ? res - 1 : px);
    py = py < 0 ? 0 : (py > res - 1 ? res - 1 : py);
    const uint64_t key = zbuf[(size_t)py * res + px];
    if (key == ~(uint64_t)0) {
      raw[i] = 1;
    } else {
      const uint32_t hi = (uint32_t)(key >> 32);
      float zd;
      memcpy(&zd, &hi, 4);
      raw[i] = z[i] <= zd + bias;
    }
  }
  free(U);
  free(W);
  free(z);
}

static void mesh_visibility_impl(int nv, int nf, const float* v, const int32_t* faces, int V,
                                 const float* dirs, int res, const int32_t* knn, int kv,
                                 uint32_t* raw_bits, uint8_t* count, int shadow, float bias_px);

/* Full visibility of Sec. 3.2 for V view directions.
 * raw_bits: [nv][ceil(V/32)] words, bit (k & 31) of word k >> 5 is the raw
 *           (unfiltered) visibility of vertex i from view k; may be NULL.
 * count:    [nv][V] filtered counts in 0..kv.                                */
void oracle_mesh_visibility(int nv, int nf, const float* v, const int32_t* faces, int V,
                            const float* dirs, int res, const int32_t* knn, int kv,
                            uint32_t* raw_bits, uint8_t* count) {
  mesh_visibility_impl(nv, nf, v, faces, V, dirs, res, knn, kv, raw_bits, count, 0, 0.f);
}

/* The same with the raw maps of the shadow-mapping depth test.              */
void oracle_mesh_visibility_shadow(int nv, int nf, const float* v, const int32_t* faces, int V,
                                   const float* dirs, int res, const int32_t* knn, int kv,
                                   float bias_px, uint32_t* raw_bits, uint8_t* count) {
  mesh_visibility_impl(nv, nf, v, faces, V, dirs, res, knn, kv, raw_bits, count, 1, bias_px);
}

static void mesh_visibility_impl(int nv, int nf, const float* v, const int32_t* faces, int V,
                                 const float* dirs, int res, const int32_t* knn, int kv,
                                 uint32_t* raw_bits, uint8_t* count, int shadow, float bias_px) {
  const int nw = (V + 31) / 32;
  if (raw_bits) memset(raw_bits, 0, sizeof(uint32_t) * (size_t)nv * nw);
#pragma omp parallel
  {
    uint64_t* zbuf = (uint64_t*)malloc(sizeof(uint64_t) * res * res);
    uint8_t* raw = (uint8_t*)malloc(nv);
    uint8_t* m1 = (uint8_t*)malloc(nv);
    uint8_t* m2 = (uint8_t*)malloc(nv);
    uint8_t* cnt = (uint8_t*)malloc(nv);
#pragma omp for schedule(dynamic, 1)
    for (int k = 0; k < V; ++k) {
      if (shadow) {
        shadow_view(nv, nf, v, faces, dirs + 3 * k, res, bias_px, zbuf, raw);
      } else {
        oracle_raster_view(nv, nf, v, faces, dirs + 3 * k, res, 0, zbuf);
        memset(raw, 0, nv);
        for (int p = 0; p < res * res; ++p) {
          if (zbuf[p] == ~(uint64_t)0) continue;
          const int f = (int)(uint32_t)(zbuf[p] & 0xffffffffu);
          raw[faces[3 * f]] = 1;
          raw[faces[3 * f + 1]] = 1;
          raw[faces[3 * f + 2]] = 1;
        }
      }
      if (raw_bits) {
        for (int i = 0; i < nv; ++i)
          if (raw[i]) {
#pragma omp atomic
            raw_bits[(size_t)i * nw + (k >> 5)] |= 1u << (k & 31);
          }
      }
      oracle_vis_filter(nv, raw, knn, kv, m1, m2, cnt);
      for (int i = 0; i < nv; ++i) count[(size_t)i * V + k] = cnt[i];
    }
    free(zbuf);
    free(raw);
    free(m1);
    free(m2);
    free(cnt);
  }
}

/* ======================================================================== */
/* Splatting (the 3DGS rasterizer the paper renders with, Sec. 3.1).         */

typedef struct {
  float R[9];   /* world -> camera rotation, row-major */
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} oracle_camera;

/* exp for the scale s = exp(log s): Cody-Waite reduction by ln 2 and a
 * degree-7 Taylor polynomial, all in FP32 with a fixed order, so that the
 * scales (which decide tile coverage) are reproducible bit for bit.         */
float oracle_exp_f32(float x) {
  x = fminf(fmaxf(x, -87.f), 88.f);
  const float k = rintf(x * 1.44269502f);
  float r = fmaf(-k, 0.693145752f, x);
  r = fmaf(-k, 1.42860677e-6f, r);
  float p = 1.f / 5040.f;
  p = fmaf(p, r, 1.f / 720.f);
  p = fmaf(p, r, 1.f / 120.f);
  p = fmaf(p, r, 1.f / 24.f);
  p = fmaf(p, r, 1.f / 6.f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.f);
  p = fmaf(p, r, 1.f);
  return ldexpf(p, (int)k);
}

/* Upper bound of ln y for y >= 1 from exact operations only:
 * y = m 2^e with m in [1, 2); ln y <= e ln2 + (m - 1)/sqrt(m).              */
float oracle_ln_upper_f32(float y) {
  int e;
  const float m = frexpf(y, &e) * 2.f;
  return (float)(e - 1) * 0.693147182f + (m - 1.f) / sqrtf(m);
}

/* Per-Gaussian projection.  Outputs (all [.][n]):
 *   valid   1 if the Gaussian survives near-plane, back-face, opacity and
 *           determinant culls (screen extent not considered);
 *   mean2d  pixel coordinates; conic (A, B, C) of the inverse 2D covariance;
 *   depth   camera z; rect (tx0, ty0, tx1, ty1) inclusive tile range;
 *   touched number of tiles (0 if invalid or off screen);
 *   fp64    1 if the 2x2 covariance determinant and inverse were taken in FP64.
 * Conventions: camera frame x right, y down, z forward; pixel (i, j) has its
 * centre at (i + 0.5, j + 0.5); 16x16-pixel tiles.                          */
void oracle_splat_preprocess_f32(int n, const oracle_camera* cam, const float* x,
                                 const float* A, const float* q, const float* log_s,
                                 const float* opac, const uint8_t* front, uint8_t* valid,
                                 float* mean2d, float* conic, float* depth, int32_t* rect,
                                 int32_t* touched, uint8_t* fp64) {
  const int TX = (cam->width + 15) / 16, TY = (cam->height + 15) / 16;
  const float* Rc = cam->R;
  for (int g = 0; g < n; ++g) {
    valid[g] = 0;
    touched[g] = 0;
    fp64[g] = 0;
    mean2d[g] = mean2d[n + g] = 0.f;
    conic[g] = conic[n + g] = conic[2 * n + g] = 0.f;
    depth[g] = 0.f;
    rect[g] = rect[n + g] = 0;
    rect[2 * n + g] = rect[3 * n + g] = -1;
    const float x0 = x[g], x1 = x[n + g], x2 = x[2 * n + g];
    const float X = fmaf(Rc[2], x2, fmaf(Rc[1], x1, fmaf(Rc[0], x0, cam->t[0])));
    const float Y = fmaf(Rc[5], x2, fmaf(Rc[4], x1, fmaf(Rc[3], x0, cam->t[1])));
    const float Z = fmaf(Rc[8], x2, fmaf(Rc[7], x1, fmaf(Rc[6], x0, cam->t[2])));
    depth[g] = Z;
    if (!(Z > 0.2f)) continue;
    if (!front[g]) continue;
    const float o = opac[g];
    if (!(o >= 1.f / 255.f)) continue;
    float s[3];
    for (int j = 0; j < 3; ++j) s[j] = oracle_exp_f32(log_s[j * n + g]);
    const float q0 = q[g], q1 = q[n + g], q2 = q[2 * n + g], q3 = q[3 * n + g];
    const float qq = fmaf(q3, q3, fmaf(q2, q2, fmaf(q1, q1, q0 * q0)));
    if (!(qq > 0.f)) continue;
    const float inv = 1.f / sqrtf(qq);
    const float qw = q0 * inv, qx = q1 * inv, qy = q2 * inv, qz = q3 * inv;
    const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
    const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
    const float Rq[9] = {1.f - 2.f * (yy + zz), 2.f * (xy - wz), 2.f * (xz + wy),
                         2.f * (xy + wz), 1.f - 2.f * (xx + zz), 2.f * (yz - wx),
                         2.f * (xz - wy), 2.f * (yz + wx), 1.f - 2.f * (xx + yy)};
    float Ag[9];
    for (int k = 0; k < 9; ++k) Ag[k] = A[k * n + g];
    /* M = A Rq diag(s): the posed Gaussian's covariance factor */
    float M[9], V[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        M[3 * i + j] = fmaf(Ag[3 * i + 2], Rq[6 + j], fmaf(Ag[3 * i + 1], Rq[3 + j],
                                                              Ag[3 * i] * Rq[j])) * s[j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        V[3 * i + j] = fmaf(Rc[3 * i + 2], M[6 + j], fmaf(Rc[3 * i + 1], M[3 + j],
                                                          Rc[3 * i] * M[j]));
    const float xzr = X / Z, yzr = Y / Z;
    const float J00 = cam->fx / Z, J11 = cam->fy / Z;
    const float J02 = -(J00 * xzr), J12 = -(J11 * yzr);
    float T[6];
    for (int j = 0; j < 3; ++j) {
      T[j] = fmaf(J02, V[6 + j], J00 * V[j]);
      T[3 + j] = fmaf(J12, V[6 + j], J11 * V[3 + j]);
    }
    const float a = fmaf(T[2], T[2], fmaf(T[1], T[1], T[0] * T[0])) + 0.3f;
    const float b = fmaf(T[2], T[5], fmaf(T[1], T[4], T[0] * T[3]));
    const float c = fmaf(T[5], T[5], fmaf(T[4], T[4], T[3] * T[3])) + 0.3f;
    const float det = fmaf(a, c, -(b * b));
    float ca, cb, cc;
    if (det <= (a * c) * 0x1p-12f) {
      /* near-degenerate 2x2 covariance: determinant and inverse in FP64,
       * from the same FP32 inputs (scales, rotation, A, camera, X/Z, Y/Z) */
      double Md[9], Vd[9], Td[6];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          Md[3 * i + j] = fma((double)Ag[3 * i + 2], (double)Rq[6 + j],
                              fma((double)Ag[3 * i + 1], (double)Rq[3 + j],
                                  (double)Ag[3 * i] * (double)Rq[j])) * (double)s[j];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          Vd[3 * i + j] = fma((double)Rc[3 * i + 2], Md[6 + j],
                              fma((double)Rc[3 * i + 1], Md[3 + j], (double)Rc[3 * i] * Md[j]));
      const double Zd = (double)Z;
      const double j00 = (double)cam->fx / Zd, j11 = (double)cam->fy / Zd;
      const double j02 = -(j00 * ((double)X / Zd)), j12 = -(j11 * ((double)Y / Zd));
      for (int j = 0; j < 3; ++j) {
        Td[j] = fma(j02, Vd[6 + j], j00 * Vd[j]);
        Td[3 + j] = fma(j12, Vd[6 + j], j11 * Vd[3 + j]);
      }
      const double ad = fma(Td[2], Td[2], fma(Td[1], Td[1], Td[0] * Td[0])) + 0.3;
      const double bd = fma(Td[2], Td[5], fma(Td[1], Td[4], Td[0] * Td[3]));
      const double cd = fma(Td[5], Td[5], fma(Td[4], Td[4], Td[3] * Td[3])) + 0.3;
      const double dd = fma(ad, cd, -(bd * bd));
      if (!(dd > 0.0)) continue;
      ca = (float)(cd / dd);
      cb = (float)(-bd / dd);
      cc = (float)(ad / dd);
      fp64[g] = 1;
    } else {
      ca = c / det;
      cb = -b / det;
      cc = a / det;
    }
    const float u = fmaf(cam->fx, xzr, cam->cx);
    const float v = fmaf(cam->fy, yzr, cam->cy);
    valid[g] = 1;
    mean2d[g] = u;
    mean2d[n + g] = v;
    conic[g] = ca;
    conic[n + g] = cb;
    conic[2 * n + g] = cc;
    /* Axis-aligned box of the ellipse where o exp(-q/2) >= 1/255, i.e.
     * q <= 2 ln(255 o); half-widths sqrt(r2 * Sigma_xx), sqrt(r2 * Sigma_yy),
     * with a conservative ln and a small inflation.                          */
    const float r2 = 2.f * oracle_ln_upper_f32(255.f * o);
    const float hx = sqrtf(r2 * a) * 1.001f + 1e-3f;
    const float hy = sqrtf(r2 * c) * 1.001f + 1e-3f;
    float fx0 = floorf((u - hx) * 0.0625f), fx1 = floorf((u + hx) * 0.0625f);
    float fy0 = floorf((v - hy) * 0.0625f), fy1 = floorf((v + hy) * 0.0625f);
    if (!(fx0 == fx0) || !(fx1 == fx1) || !(fy0 == fy0) || !(fy1 == fy1)) continue;
    fx0 = fmaxf(fx0, 0.f);
    fy0 = fmaxf(fy0, 0.f);
    fx1 = fminf(fx1, (float)(TX - 1));
    fy1 = fminf(fy1, (float)(TY - 1));
    if (fx0 > fx1 || fy0 > fy1) continue;
    rect[g] = (int32_t)fx0;
    rect[n + g] = (int32_t)fy0;
    rect[2 * n + g] = (int32_t)fx1;
    rect[3 * n + g] = (int32_t)fy1;
    touched[g] = (rect[2 * n + g] - rect[g] + 1) * (rect[3 * n + g] - rect[n + g] + 1);
  }
}

typedef struct {
  uint64_t key;
  int32_t g;
} kv_pair;

static int cmp_pair(const void* pa, const void* pb) {
  const kv_pair* a = (const kv_pair*)pa;
  const kv_pair* b = (const kv_pair*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return a->g < b->g ? -1 : (a->g > b->g ? 1 : 0);
}

/* Tile binning: one entry per (Gaussian, touched tile) with key
 * (tile id << 32 | float bits of depth), sorted by (key, Gaussian index).
 * Returns D.  keys/values may be NULL to query D.  ranges: [tiles][2] of
 * [start, end) into the sorted entries.                                     */
int64_t oracle_splat_bin(int n, int tiles_x, int tiles_y, const int32_t* rect,
                         const int32_t* touched, const float* depth, uint64_t* keys,
                         int32_t* values, int32_t* ranges) {
  int64_t D = 0;
  for (int g = 0; g < n; ++g) D += touched[g];
  if (!keys || !values) return D;
  kv_pair* pairs = (kv_pair*)malloc(sizeof(kv_pair) * (D > 0 ? D : 1));
  int64_t k = 0;
  for (int g = 0; g < n; ++g) {
    if (touched[g] <= 0) continue;
    uint32_t zb;
    memcpy(&zb, &depth[g], 4);
    for (int ty = rect[n + g]; ty <= rect[3 * n + g]; ++ty)
      for (int tx = rect[g]; tx <= rect[2 * n + g]; ++tx) {
        pairs[k].key = ((uint64_t)(uint32_t)(ty * tiles_x + tx) << 32) | zb;
        pairs[k].g = g;
        ++k;
      }
  }
  qsort(pairs, (size_t)D, sizeof(kv_pair), cmp_pair);
  for (int t = 0; t < tiles_x * tiles_y; ++t) ranges[2 * t] = ranges[2 * t + 1] = 0;
  for (int64_t i = 0; i < D; ++i) {
    keys[i] = pairs[i].key;
    values[i] = pairs[i].g;
    const int t = (int)(pairs[i].key >> 32);
    if (i == 0 || (int)(pairs[i - 1].key >> 32) != t) ranges[2 * t] = (int32_t)i;
    ranges[2 * t + 1] = (int32_t)(i + 1);
  }
  free(pairs);
  return D;
}

/* Front-to-back compositing of one pixel over an ordered list of Gaussians:
 * alpha = min(0.99, o exp(-q/2)) with q = d^T Conic d, d = mean - pixel
 * centre; entries with q < 0 or alpha < 1/255 are skipped; the walk stops
 * before the entry that would take the transmittance below 1e-4.
 * margin is the smallest relative distance of any such decision from its
 * threshold (used to exempt knife-edge pixels from tolerance checks).      */
static void composite_pixel(float px, float py, const int32_t* list, int64_t len,
                            const float* mean2d, const float* conic, const float* opac,
                            const float* color, int n, float* out_c, float* out_T,
                            float* out_margin, int32_t* out_applied) {
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, margin = INFINITY;
  int32_t applied = 0;
  for (int64_t e = 0; e < len; ++e) {
    const int g = list[e];
    const float dx = mean2d[g] - px, dy = mean2d[n + g] - py;
    const float ca = conic[g], cb = conic[n + g], cc = conic[2 * n + g];
    const float qf = fmaf(ca * dx, dx, fmaf(cc * dy, dy, 2.f * ((cb * dx) * dy)));
    const float power = -0.5f * qf;
    if (power > 0.f) continue;
    /* exp(power) evaluated as 2^(power log2 e), the product in FP32: the
     * GPU takes the same skip / clamp / stop decisions from the same value */
    const float araw = opac[g] * exp2f(power * 1.44269504f);
    const float alpha = fminf(0.99f, araw);
    {
      const float m1 = fabsf(araw - 1.f / 255.f) * 255.f;
      const float m2 = fabsf(araw - 0.99f) / 0.99f;
      if (m1 < margin) margin = m1;
      if (m2 < margin) margin = m2;
    }
    if (alpha < 1.f / 255.f) continue;
    const float Tn = T * (1.f - alpha);
    {
      const float m3 = fabsf(Tn - 1e-4f) / 1e-4f;
      if (m3 < margin) margin = m3;
    }
    if (Tn < 1e-4f) break;
    const float w = alpha * T;
    C0 = fmaf(color[g], w, C0);
    C1 = fmaf(color[n + g], w, C1);
    C2 = fmaf(color[2 * n + g], w, C2);
    ++applied;
    T = Tn;
  }
  out_c[0] = C0;
  out_c[1] = C1;
  out_c[2] = C2;
  *out_T = T;
  if (out_margin) *out_margin = margin;
  if (out_applied) *out_applied = applied;
}

/* Tiled compositing: each pixel walks the sorted list of its 16x16 tile.
 * image [3][H][W], T_final [H][W], margin [H][W] and applied [H][W] (the
 * number of splats composited into the pixel) may be NULL.                */
void oracle_composite_tiles_f32(int H, int W, int tiles_x, const int32_t* ranges,
                                const int32_t* values, int n, const float* mean2d,
                                const float* conic, const float* opac, const float* color,
                                float* image, float* T_final, float* margin, int32_t* applied) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int t = (y / 16) * tiles_x + (x / 16);
      float c[3], T, m;
      int32_t na;
      composite_pixel((float)x + 0.5f, (float)y + 0.5f, values + ranges[2 * t],
                      (int64_t)ranges[2 * t + 1] - ranges[2 * t], mean2d, conic, opac, color, n,
                      c, &T, &m, &na);
      for (int ch = 0; ch < 3; ++ch) image[(size_t)ch * H * W + (size_t)y * W + x] = c[ch];
      T_final[(size_t)y * W + x] = T;
      if (margin) margin[(size_t)y * W + x] = m;
      if (applied) applied[(size_t)y * W + x] = na;
    }
}

typedef struct {
  uint32_t zb;
  int32_t g;
} depth_item;

static int cmp_depth(const void* pa, const void* pb) {
  const depth_item* a = (const depth_item*)pa;
  const depth_item* b = (const depth_item*)pb;
  if (a->zb != b->zb) return a->zb < b->zb ? -1 : 1;
  return a->g < b->g ? -1 : (a->g > b->g ? 1 : 0);
}

/* Brute force: every pixel walks every valid Gaussian in (depth bits, index)
 * order, with no tiles at all.  Equal to the tiled result by construction.  */
void oracle_composite_brute_f32(int H, int W, int n, const uint8_t* valid, const float* depth,
                                const float* mean2d, const float* conic, const float* opac,
                                const float* color, float* image, float* T_final) {
  depth_item* items = (depth_item*)malloc(sizeof(depth_item) * (n > 0 ? n : 1));
  int m = 0;
  for (int g = 0; g < n; ++g)
    if (valid[g]) {
      memcpy(&items[m].zb, &depth[g], 4);
      items[m].g = g;
      ++m;
    }
  qsort(items, (size_t)m, sizeof(depth_item), cmp_depth);
  int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (m > 0 ? m : 1));
  for (int i = 0; i < m; ++i) list[i] = items[i].g;
#pragma omp parallel for schedule(dynamic, 4)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      float c[3], T;
      composite_pixel((float)x + 0.5f, (float)y + 0.5f, list, m, mean2d, conic, opac, color, n,
                      c, &T, NULL, NULL);
      for (int ch = 0; ch < 3; ++ch) image[(size_t)ch * H * W + (size_t)y * W + x] = c[ch];
      T_final[(size_t)y * W + x] = T;
    }
  free(list);
  free(items);
}

/* ---- Sec. 3.1, interpolation equation: the K nearest canonical vertices ----
 * For every query point (a Gaussian's canonical position) the k reference
 * points (canonical mesh vertices) with the smallest squared distance,
 * ordered by (distance^2, index).  distance^2 in FP32 with d = ref - query,
 * evaluated as fmaf(dz, dz, fmaf(dy, dy, dx * dx)); the order on equal
 * distances is the lower index first.  Plain brute force over all pairs,
 * keeping the k best in a sorted array.  k <= nr.                        */
void oracle_knn(int n, const float* q, int nr, const float* ref, int k, int32_t* idx, float* d2) {
#pragma omp parallel
  {
    float* bd = (float*)malloc(sizeof(float) * (size_t)(k > 0 ? k : 1));
    int32_t* bi = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      const float qx = q[i], qy = q[n + i], qz = q[2 * n + i];
      int m = 0;
      for (int j = 0; j < nr; ++j) {
        const float dx = ref[j] - qx, dy = ref[nr + j] - qy, dz = ref[2 * nr + j] - qz;
        const float dd = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        /* j is larger than every index already kept, so on equal distance it
         * goes after them */
        if (m == k && !(dd < bd[k - 1])) continue;
        int p = m < k ? m : k - 1;
        while (p > 0 && dd < bd[p - 1]) {
          bd[p] = bd[p - 1];
          bi[p] = bi[p - 1];
          --p;
        }
        bd[p] = dd;
        bi[p] = j;
        if (m < k) ++m;
      }
      for (int t = 0; t < k; ++t) {
        idx[(size_t)t * n + i] = bi[t];
        d2[(size_t)t * n + i] = bd[t];
      }
    }
    free(bd);
    free(bi);
  }
}

/* ======================================================================== */
/* App. B (Gaussian densification algorithm, Alg. 1): density-based
 * densification.
 *
 * Random numbers: the k-th output (k >= 1) of SplitMix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) from
 * the state `seed`: the state advances by the golden-ratio increment and each
 * output is the state passed through the mixing function.                   */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Alg. 1, step by step:
 *   D_v[k]  = number of Gaussians whose K_g nearest vertices S_g include k;
 *   d_f[i]  = sum over the three vertices of triangle i of D_v, / (6 K_g)
 *             (each vertex is taken to touch six triangles);
 *   P[i]    = max(0, d0 - d_f[i]);  N' = sum(P) p0;
 *   n_g     = multinomial counts of N' draws with probabilities P / sum(P);
 *   every draw adds one Gaussian at a uniformly random point of its triangle.
 * Readings: P is held exactly as an integer in units of 1 / (6 K_g 65536):
 * Q[i] = max(0, round(d0 6 K_g 65536) - 65536 S[i]) with S[i] the vertex sum
 * (exact for the paper's d0 = 1); N' = floor(sum(Q) p0 / (6 K_g 65536)) in
 * double precision (the count is an integer); draw j (from 0) takes
 * r = SplitMix64 output 3j + 1 and picks the triangle whose cumulative range
 * of Q holds u = floor(r sum(Q) / 2^64); its point takes outputs 3j + 2 and
 * 3j + 3 as u1, u2 = (output >> 40) 2^-24 and lands at barycentric
 * (1 - s, s (1 - u2), s u2) with s = sqrt(u1) (the uniform-triangle map of
 * Osada et al., 2002), x = fmaf(b2, v2, fmaf(b1, v1, b0 v0)) per coordinate
 * in FP32.  New Gaussians are listed in draw order; only the first `cap`
 * positions are written, the counts always cover every draw.
 * sg [kg][n] int32, verts [3][nv], faces [nf][3]; outputs Dv [nv], df [nf],
 * ng [nf], x_out [3][cap], f_out [cap]; returns N'.                        */
int64_t oracle_densify(int n, int kg, const int32_t* sg, int nv, const float* verts, int nf,
                       const int32_t* faces, double d0, double p0, uint64_t seed, int64_t cap,
                       int32_t* Dv, float* df, int32_t* ng, float* x_out, int32_t* f_out) {
  for (int v = 0; v < nv; ++v) Dv[v] = 0;
  for (int i = 0; i < n; ++i)
    for (int t = 0; t < kg; ++t) Dv[sg[(size_t)t * n + i]] += 1;
  const int64_t unit = 6LL * kg * 65536LL;
  const int64_t T = llround(d0 * (double)unit);
  int64_t* C = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nf > 0 ? nf : 1));
  int64_t total = 0;
  for (int f = 0; f < nf; ++f) {
    int64_t S = 0;
    for (int c = 0; c < 3; ++c) S += Dv[faces[3 * f + c]];
    df[f] = (float)((double)S / (double)(6 * kg));
    int64_t q = T - 65536LL * S;
    if (q < 0) q = 0;
    total += q;
    C[f] = total;              /* inclusive cumulative sum */
    ng[f] = 0;
  }
  const int64_t N = total > 0 ? (int64_t)floor((double)total * p0 / (double)unit) : 0;
  for (int64_t j = 0; j < N; ++j) {
    const uint64_t r = oracle_splitmix64(seed, 3 * (uint64_t)j + 1);
    const uint64_t u = (uint64_t)(((unsigned __int128)r * (uint64_t)total) >> 64);
    /* first triangle whose inclusive cumulative sum exceeds u */
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      if (C[mid] > (int64_t)u) hi = mid; else lo = mid + 1;
    }
    const int f = lo;
    ng[f] += 1;
    if (j < cap) {
      const float u1 = (float)(oracle_splitmix64(seed, 3 * (uint64_t)j + 2) >> 40) * 0x1p-24f;
      const float u2 = (float)(oracle_splitmix64(seed, 3 * (uint64_t)j + 3) >> 40) * 0x1p-24f;
      const float s = sqrtf(u1);
      const float b0 = 1.f - s, b1 = s * (1.f - u2), b2 = s * u2;
      const int a = faces[3 * f], b = faces[3 * f + 1], c = faces[3 * f + 2];
      for (int k = 0; k < 3; ++k)
        x_out[(size_t)k * cap + j] = fmaf(b2, verts[(size_t)k * nv + c],
                                          fmaf(b1, verts[(size_t)k * nv + b],
                                               b0 * verts[(size_t)k * nv + a]));
      f_out[j] = f;
    }
  }
  free(C);
  return N;
}
