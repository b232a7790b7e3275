// Per-vertex visibility from orthographic rasterization of the posed mesh
// (Sec. 3.2 of the paper), bit-exact.
//
//   raster     one workgroup per view: the res x res z-buffer of 64-bit keys
//              (float bits of depth << 32 | triangle id) lives in LDS
//              (128 KB at 128^2, within gfx950's 160 KB), filled with LDS
//              64-bit atomic-min; winning triangles mark their three
//              vertices in an LDS bitmask that is written out view-major
//   transpose  32x32 bit-matrix transposes by wave ballots -> vertex-major words
//              raw[v][w] whose bit b is view 32w + b
//   filter     bit-sliced: one 32-bit word carries 32 views, so the median
//              of kv neighbours is a bitwise majority vote computed with a
//              5-plane ripple counter (two passes), and the final pass
//              expands the counter planes into count bytes [nv][V]
#include <mutex>

#include "common.h"

namespace {

constexpr int kMaxRes = 128;
constexpr int kRasterThreads = 1024;

__device__ inline void basis(const float* d, float* t, float* b) {
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

__device__ inline int64_t edge(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t sx,
                               int64_t sy) {
  return (bx - ax) * (sy - ay) - (by - ay) * (sx - ax);
}

__device__ inline bool owns(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  const int64_t dx = bx - ax, dy = by - ay;
  return dy > 0 || (dy == 0 && dx < 0);
}

__device__ inline int64_t fdiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

struct Proj {
  float c[3], rho, irho, t[3], b[3], d[3], scale;
};

__device__ inline void project(const Proj& P, const float* __restrict__ v, int nv, int i,
                               int32_t& U, int32_t& V, float& z) {
  const float q0 = v[i] - P.c[0], q1 = v[nv + i] - P.c[1], q2 = v[2 * nv + i] - P.c[2];
  const float pu = fmaf(P.t[2], q2, fmaf(P.t[1], q1, P.t[0] * q0));
  const float pv = fmaf(P.b[2], q2, fmaf(P.b[1], q1, P.b[0] * q0));
  const float pd = fmaf(P.d[2], q2, fmaf(P.d[1], q1, P.d[0] * q0));
  // u = (t.(x - c) (1/rho) + 1) res / 2
  const float u = (pu * P.irho + 1.f) * P.scale;
  const float w = (pv * P.irho + 1.f) * P.scale;
  U = (int32_t)rintf(u * 256.f);
  V = (int32_t)rintf(w * 256.f);
  z = P.rho - pd;
}

__device__ inline unsigned long long depth_key(float bz, int f) {
  return ((unsigned long long)__float_as_uint(bz) << 32) | (unsigned long long)(uint32_t)f;
}

// General triangle (any extent): edge functions in 64-bit integers.
__device__ void raster_tri_wide(unsigned long long* zb, int res, int f, int64_t x0, int64_t y0,
                                float z0, int64_t x1, int64_t y1, float z1, int64_t x2,
                                int64_t y2, float z2) {
  int64_t area = edge(x0, y0, x1, y1, x2, y2);
  if (area == 0) return;
  if (area < 0) {
    int64_t tx = x1, ty = y1;
    x1 = x2; y1 = y2; x2 = tx; y2 = ty;
    float tz = z1; z1 = z2; z2 = tz;
    area = -area;
  }
  int64_t mnx = min(x0, min(x1, x2)), mxx = max(x0, max(x1, x2));
  int64_t mny = min(y0, min(y1, y2)), mxy = max(y0, max(y1, y2));
  int64_t i_lo = -fdiv(-(mnx - 128), 256), i_hi = fdiv(mxx - 128, 256);
  int64_t j_lo = -fdiv(-(mny - 128), 256), j_hi = fdiv(mxy - 128, 256);
  if (i_lo < 0) i_lo = 0;
  if (j_lo < 0) j_lo = 0;
  if (i_hi > res - 1) i_hi = res - 1;
  if (j_hi > res - 1) j_hi = res - 1;
  const bool o12 = owns(x1, y1, x2, y2), o20 = owns(x2, y2, x0, y0), o01 = owns(x0, y0, x1, y1);
  const float ia = 1.f / (float)area;   // barycentric weights w_e / area
  for (int64_t j = j_lo; j <= j_hi; ++j) {
    const int64_t sy = 256 * j + 128;
    for (int64_t i = i_lo; i <= i_hi; ++i) {
      const int64_t sx = 256 * i + 128;
      const int64_t w0 = edge(x1, y1, x2, y2, sx, sy);
      const int64_t w1 = edge(x2, y2, x0, y0, sx, sy);
      const int64_t w2 = edge(x0, y0, x1, y1, sx, sy);
      const bool in0 = w0 > 0 || (w0 == 0 && o12);
      const bool in1 = w1 > 0 || (w1 == 0 && o20);
      const bool in2 = w2 > 0 || (w2 == 0 && o01);
      if (!(in0 && in1 && in2)) continue;
      const float bz = fmaf((float)w2, z2, fmaf((float)w1, z1, (float)w0 * z0)) * ia;
      atomicMin(&zb[j * res + i], depth_key(bz, f));
    }
  }
}

// Triangle whose bounding box spans fewer than 2^14 fixed-point units on
// both axes (64 pixels): every coordinate difference inside the box (and
// one sample step past it) is below 2^14 + 256, so each edge-function
// product is below 2^29 and the edge functions are exact in 32-bit
// integers.  They are stepped incrementally
// along a row (exact integer updates), and the top-left rule becomes a
// sign test after subtracting 1 from the edges a sample on them does not
// belong to.  Same integers, same depth arithmetic as the wide form.
__device__ inline void raster_tri(unsigned long long* zb, int res, int f, int32_t x0, int32_t y0,
                                  float z0, int32_t x1, int32_t y1, float z1, int32_t x2,
                                  int32_t y2, float z2) {
  const int32_t mnx = min(x0, min(x1, x2)), mxx = max(x0, max(x1, x2));
  const int32_t mny = min(y0, min(y1, y2)), mxy = max(y0, max(y1, y2));
  if ((uint32_t)mxx - (uint32_t)mnx >= 16384u || (uint32_t)mxy - (uint32_t)mny >= 16384u) {
    raster_tri_wide(zb, res, f, x0, y0, z0, x1, y1, z1, x2, y2, z2);
    return;
  }
  int32_t area = (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0);
  if (area == 0) return;
  if (area < 0) {
    int32_t tx = x1, ty = y1;
    x1 = x2; y1 = y2; x2 = tx; y2 = ty;
    float tz = z1; z1 = z2; z2 = tz;
    area = -area;
  }
  // sample columns i with mnx <= 256 i + 128 <= mxx (arithmetic shifts floor)
  const int i_lo = max(0, -((128 - mnx) >> 8)), i_hi = min(res - 1, (mxx - 128) >> 8);
  const int j_lo = max(0, -((128 - mny) >> 8)), j_hi = min(res - 1, (mxy - 128) >> 8);
  if (i_lo > i_hi || j_lo > j_hi) return;
  // w_e(s) = a_e (sx - x_e) + b_e (sy - y_e) for the edge opposite vertex e
  const int32_t a0 = y1 - y2, b0 = x2 - x1;
  const int32_t a1 = y2 - y0, b1 = x0 - x2;
  const int32_t a2 = y0 - y1, b2 = x1 - x0;
  // 0 if a sample on the edge belongs to the triangle, else 1
  // (edge A -> B owns its samples iff B.y > A.y, or B.y == A.y and B.x < A.x)
  const int32_t c0 = (a0 < 0 || (a0 == 0 && b0 < 0)) ? 0 : 1;   // edge v1 -> v2
  const int32_t c1 = (a1 < 0 || (a1 == 0 && b1 < 0)) ? 0 : 1;   // edge v2 -> v0
  const int32_t c2 = (a2 < 0 || (a2 == 0 && b2 < 0)) ? 0 : 1;   // edge v0 -> v1
  const float ia = 1.f / (float)area;   // barycentric weights w_e / area
  const int32_t sx0 = 256 * i_lo + 128;
  for (int j = j_lo; j <= j_hi; ++j) {
    const int32_t sy = 256 * j + 128;
    int32_t w0 = a0 * (sx0 - x1) + b0 * (sy - y1) - c0;
    int32_t w1 = a1 * (sx0 - x2) + b1 * (sy - y2) - c1;
    int32_t w2 = a2 * (sx0 - x0) + b2 * (sy - y0) - c2;
    unsigned long long* row = zb + j * res;
    for (int i = i_lo; i <= i_hi; ++i) {
      if ((w0 | w1 | w2) >= 0) {
        const float bz = fmaf((float)(w2 + c2), z2, fmaf((float)(w1 + c1), z1,
                                                        (float)(w0 + c0) * z0)) * ia;
        atomicMin(&row[i], depth_key(bz, f));
      }
      w0 += 256 * a0;
      w1 += 256 * a1;
      w2 += 256 * a2;
    }
  }
}

// min / max over the 64 lanes of a wave (DPP row shifts, then the two row
// broadcasts; a lane with no source keeps its own value), result in lane 63
template <int CTRL, int ROWS>
__device__ inline float dpp_same(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROWS, 0xf, false));
}

template <bool MAX>
__device__ inline float wave_extreme(float v) {
  auto op = [](float a, float b) { return MAX ? fmaxf(a, b) : fminf(a, b); };
  v = op(v, dpp_same<0x111, 0xf>(v));
  v = op(v, dpp_same<0x112, 0xf>(v));
  v = op(v, dpp_same<0x114, 0xf>(v));
  v = op(v, dpp_same<0x118, 0xf>(v));
  v = op(v, dpp_same<0x142, 0xa>(v));
  v = op(v, dpp_same<0x143, 0xc>(v));
  return v;
}

// frame[0..2] = centre, frame[3] = rho of the posed mesh's bounding box
// (min and max are exact and independent of the reduction order)
__global__ void __launch_bounds__(1024)
frame_kernel(int nv, const float* __restrict__ v, float* __restrict__ frame) {
  __shared__ float ext[6][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // one pass: each thread's vertices, all three axes at once (the loads of
  // an iteration are independent)
  float lo3[3], hi3[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) lo3[a] = hi3[a] = v[a * nv];
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float c = v[a * nv + i];
      lo3[a] = fminf(lo3[a], c);
      hi3[a] = fmaxf(hi3[a], c);
    }
  }
  float r[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = wave_extreme<false>(lo3[a]);
    r[3 + a] = wave_extreme<true>(hi3[a]);
  }
  if (lane == 63) {
#pragma unroll
    for (int q = 0; q < 6; ++q) ext[q][wave] = r[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = ext[a][0];
      hi[a] = ext[3 + a][0];
      for (int w = 1; w < 16; ++w) {
        lo[a] = fminf(lo[a], ext[a][w]);
        hi[a] = fmaxf(hi[a], ext[3 + a][w]);
      }
    }
    float e[3];
    for (int a = 0; a < 3; ++a) {
      frame[a] = (lo[a] + hi[a]) * 0.5f;
      e[a] = hi[a] - lo[a];
    }
    float rr = 1.01f * (0.5f * sqrtf(fmaf(e[2], e[2], fmaf(e[1], e[1], e[0] * e[0]))));
    if (!(rr > 0.f)) rr = 1.f;
    frame[3] = rr;
  }
}

__global__ void __launch_bounds__(kRasterThreads)
raster_kernel(int nv, int nf, const float* __restrict__ verts, const int32_t* __restrict__ faces,
              const float* __restrict__ dirs, int res, const float* __restrict__ frame,
              uint32_t* __restrict__ bits_vm /*[V][nwv]*/, int nwv, int shadow, float bias_px) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* zb = reinterpret_cast<unsigned long long*>(smem);
  uint32_t* mark = reinterpret_cast<uint32_t*>(smem + sizeof(unsigned long long) * res * res);
  const int view = blockIdx.x;
  Proj P;
  P.c[0] = frame[0];
  P.c[1] = frame[1];
  P.c[2] = frame[2];
  P.rho = frame[3];
  P.irho = 1.f / P.rho;
  P.d[0] = dirs[3 * view];
  P.d[1] = dirs[3 * view + 1];
  P.d[2] = dirs[3 * view + 2];
  basis(P.d, P.t, P.b);
  P.scale = 0.5f * (float)res;
  for (int p = threadIdx.x; p < res * res; p += blockDim.x) zb[p] = ~0ull;
  for (int w = threadIdx.x; w < nwv; w += blockDim.x) mark[w] = 0u;
  __syncthreads();
  for (int f = threadIdx.x; f < nf; f += blockDim.x) {
    const int i0 = rga::clampi(faces[3 * f], 0, nv - 1);
    const int i1 = rga::clampi(faces[3 * f + 1], 0, nv - 1);
    const int i2 = rga::clampi(faces[3 * f + 2], 0, nv - 1);
    int32_t x0, y0, x1, y1, x2, y2;
    float z0, z1, z2;
    project(P, verts, nv, i0, x0, y0, z0);
    project(P, verts, nv, i1, x1, y1, z1);
    project(P, verts, nv, i2, x2, y2, z2);
    raster_tri(zb, res, f, x0, y0, z0, x1, y1, z1, x2, y2, z2);
  }
  __syncthreads();
  if (shadow) {
    // shadow-mapping test: the vertex's depth against the depth map's
    // sample in the pixel it projects into, plus bias_px pixel widths; an
    // empty sample occludes nothing
    const float bias = bias_px * (2.f * P.rho) / (float)res;
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
      int32_t U, V;
      float z;
      project(P, verts, nv, i, U, V, z);
      const int px = rga::clampi(U >> 8, 0, res - 1), py = rga::clampi(V >> 8, 0, res - 1);
      const unsigned long long k = zb[py * res + px];
      if (k == ~0ull || z <= __uint_as_float((uint32_t)(k >> 32)) + bias)
        atomicOr(&mark[i >> 5], 1u << (i & 31));
    }
  } else {
    for (int p = threadIdx.x; p < res * res; p += blockDim.x) {
      const unsigned long long k = zb[p];
      if (k == ~0ull) continue;
      const int f = (int)(uint32_t)(k & 0xffffffffull);
      for (int c = 0; c < 3; ++c) {
        const int vi = rga::clampi(faces[3 * f + c], 0, nv - 1);
        atomicOr(&mark[vi >> 5], 1u << (vi & 31));
      }
    }
  }
  __syncthreads();
  for (int w = threadIdx.x; w < nwv; w += blockDim.x) bits_vm[(size_t)view * nwv + w] = mark[w];
}

// view-major [V][nwv] (bit i&31 of word i>>5 = vertex i) -> vertex-major
// [nv][nwV] (bit k&31 of word k>>5 = view k).  Each half-wave transposes one
// 32 x 32 bit block: lane r holds the row of view 32 kw + r, and the ballot
// of bit c over the half-wave is the column of vertex 32 vw + c, which
// lane c keeps and writes.
__global__ void __launch_bounds__(256)
transpose_kernel(int nv, int V, int nwv, int nwV, const uint32_t* __restrict__ vm,
                 uint32_t* __restrict__ out) {
  const int64_t blk = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
  const int64_t total = (int64_t)nwv * nwV;
  const int lane = threadIdx.x & 63, r = lane & 31;
  const bool live = blk < total;            // both halves of a wave run the ballots
  const int vw = live ? (int)(blk / nwV) : 0;  // word of vertices
  const int kw = live ? (int)(blk % nwV) : 0;  // word of views
  const int k = 32 * kw + r;
  const uint32_t a = live && k < V ? vm[(size_t)k * nwv + vw] : 0u;
  uint32_t col = 0u;
#pragma unroll
  for (int c = 0; c < 32; ++c) {
    const uint64_t m = __ballot((a >> c) & 1u);
    const uint32_t half = lane < 32 ? (uint32_t)m : (uint32_t)(m >> 32);
    col = r == c ? half : col;
  }
  const int i = 32 * vw + r;
  if (live && i < nv) out[(size_t)i * nwV + kw] = col;
}

struct Planes {
  uint32_t p[5];
};

__device__ inline void add_word(Planes& s, uint32_t x) {
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const uint32_t c = s.p[k] & x;
    s.p[k] ^= x;
    x = c;
  }
}

// lanes whose 5-bit count >= thr
__device__ inline uint32_t at_least(const Planes& s, int thr) {
  uint32_t ge = 0u, eq = 0xFFFFFFFFu;
#pragma unroll
  for (int k = 4; k >= 0; --k) {
    if ((thr >> k) & 1) {
      eq &= s.p[k];
    } else {
      ge |= eq & s.p[k];
      eq &= ~s.p[k];
    }
  }
  return ge | eq;
}

// Bit planes of the number of neighbours (kv <= 31) whose word has each bit
// set.  All neighbour indices are read first and then all words, so the
// loads overlap instead of forming a chain of dependent round trips.
__device__ inline Planes neighbour_planes(const int32_t* __restrict__ knn, int i, int kv, int nv,
                                          const uint32_t* __restrict__ src, int nwV, int w) {
  const int32_t* row = knn + (size_t)i * kv;
  int idx[31];
#pragma unroll
  for (int j = 0; j < 31; ++j) idx[j] = j < kv ? rga::clampi(row[j], 0, nv - 1) : 0;
  uint32_t x[31];
#pragma unroll
  for (int j = 0; j < 31; ++j) x[j] = j < kv ? src[(size_t)idx[j] * nwV + w] : 0u;
  Planes s = {{0u, 0u, 0u, 0u, 0u}};
#pragma unroll
  for (int j = 0; j < 31; ++j)
    if (j < kv) add_word(s, x[j]);
  return s;
}

__global__ void __launch_bounds__(256)
majority_kernel(int nv, int nwV, const int32_t* __restrict__ knn, int kv,
                const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)nv * nwV) return;
  const int i = (int)(id / nwV), w = (int)(id % nwV);
  const Planes s = neighbour_planes(knn, i, kv, nv, src, nwV, w);
  dst[id] = at_least(s, (kv + 1) / 2);
}

__global__ void __launch_bounds__(256)
count_kernel(int nv, int V, int nwV, const int32_t* __restrict__ knn, int kv,
             const uint32_t* __restrict__ src, uint8_t* __restrict__ count) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)nv * nwV) return;
  const int i = (int)(id / nwV), w = (int)(id % nwV);
  const Planes s = neighbour_planes(knn, i, kv, nv, src, nwV, w);
  uint32_t words[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    uint32_t packed = 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int lanebit = 4 * q + b;
      uint32_t v = 0u;
#pragma unroll
      for (int k = 0; k < 5; ++k) v |= ((s.p[k] >> lanebit) & 1u) << k;
      packed |= v << (8 * b);
    }
    words[q] = packed;
  }
  uint8_t* row = count + (size_t)i * V;
  const int k0 = 32 * w;
  if ((V & 15) == 0 && k0 + 32 <= V) {
    uint4* dst = reinterpret_cast<uint4*>(row + k0);
    dst[0] = make_uint4(words[0], words[1], words[2], words[3]);
    dst[1] = make_uint4(words[4], words[5], words[6], words[7]);
  } else {
    for (int b = 0; b < 32 && k0 + b < V; ++b) row[k0 + b] = (uint8_t)((words[b >> 2] >> (8 * (b & 3))) & 0xFFu);
  }
}

struct VisLayout {
  size_t frame, vm, raw, m1, m2, total;
  int nwv, nwV;
};

VisLayout vis_layout(int nv, int V) {
  VisLayout L{};
  L.nwv = (nv + 31) / 32;
  L.nwV = (V + 31) / 32;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t a = o;
    o = rga::align_up(o + bytes, 256);
    return a;
  };
  L.frame = take(16);
  L.vm = take((size_t)V * L.nwv * 4);
  L.raw = take((size_t)nv * L.nwV * 4);
  L.m1 = take((size_t)nv * L.nwV * 4);
  L.m2 = take((size_t)nv * L.nwV * 4);
  L.total = o;
  return L;
}

}  // namespace

extern "C" size_t mesh_visibility_workspace(int nv, int V) {
  if (nv < 1 || V < 1) return 0;
  return vis_layout(nv, V).total;
}

namespace {

int visibility_impl(void* stream, int nv, int nf, const float* verts, const int32_t* faces, int V,
                    const float* view_dirs, int res, const int32_t* knn, int kv,
                    uint32_t* raw_bits, uint8_t* count, void* ws, size_t ws_bytes, int shadow,
                    float bias_px) {
  if (nv < 1 || nf < 0 || V < 1) return rga::fail(RGA_EINVAL, "mesh_visibility: nv >= 1, nf >= 0, V >= 1");
  if (res < 1 || res > kMaxRes)
    return rga::fail(RGA_EUNSUPPORTED, "mesh_visibility: res must be in 1..%d", kMaxRes);
  if (kv < 1 || kv > 31 || (kv & 1) == 0)
    return rga::fail(RGA_EINVAL, "mesh_visibility: kv must be odd and in 1..31");
  if (!verts || (nf > 0 && !faces) || !view_dirs || !knn || !count || !ws)
    return rga::fail(RGA_EINVAL, "mesh_visibility: null pointer");
  if (!rga::aligned16(ws) || !rga::aligned16(count))
    return rga::fail(RGA_EINVAL, "mesh_visibility: ws and count must be 16-byte aligned");
  VisLayout L = vis_layout(nv, V);
  if (ws_bytes < L.total)
    return rga::fail(RGA_ECAPACITY, "mesh_visibility: workspace %zu < %zu bytes", ws_bytes, L.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  float* frame = reinterpret_cast<float*>(w + L.frame);
  uint32_t* vm = reinterpret_cast<uint32_t*>(w + L.vm);
  uint32_t* raw = raw_bits ? raw_bits : reinterpret_cast<uint32_t*>(w + L.raw);
  uint32_t* m1 = reinterpret_cast<uint32_t*>(w + L.m1);
  uint32_t* m2 = reinterpret_cast<uint32_t*>(w + L.m2);
  const size_t lds = sizeof(unsigned long long) * (size_t)res * res + 4 * (size_t)L.nwv;
  if (lds > 160 * 1024)
    return rga::fail(RGA_EUNSUPPORTED, "mesh_visibility: %d vertices need too much LDS", nv);
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(raster_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  RGA_LAUNCH("vis_frame", frame_kernel, dim3(1), dim3(1024), 0, s, nv, verts, frame);
  RGA_LAUNCH("vis_raster", raster_kernel, dim3(V), dim3(kRasterThreads), lds, s, nv, nf, verts,
             faces, view_dirs, res, frame, vm, L.nwv, shadow, bias_px);
  const int64_t tw = (int64_t)L.nwv * L.nwV;
  RGA_LAUNCH("vis_transpose", transpose_kernel, dim3(rga::ceil_div(tw * 32, 256)), dim3(256), 0, s, nv,
             V, L.nwv, L.nwV, vm, raw);
  const int64_t nw = (int64_t)nv * L.nwV;
  RGA_LAUNCH("vis_majority", majority_kernel, dim3(rga::ceil_div(nw, 256)), dim3(256), 0, s, nv,
             L.nwV, knn, kv, raw, m1);
  RGA_LAUNCH("vis_majority", majority_kernel, dim3(rga::ceil_div(nw, 256)), dim3(256), 0, s, nv,
             L.nwV, knn, kv, m1, m2);
  RGA_LAUNCH("vis_count", count_kernel, dim3(rga::ceil_div(nw, 256)), dim3(256), 0, s, nv, V,
             L.nwV, knn, kv, m2, count);
  RGA_CHECK_LAUNCH("mesh_visibility");
  return RGA_OK;
}

}  // namespace

extern "C" int mesh_visibility(void* stream, int nv, int nf, const float* verts,
                               const int32_t* faces, int V, const float* view_dirs, int res,
                               const int32_t* knn, int kv, uint32_t* raw_bits, uint8_t* count,
                               void* ws, size_t ws_bytes) {
  return visibility_impl(stream, nv, nf, verts, faces, V, view_dirs, res, knn, kv, raw_bits, count,
                         ws, ws_bytes, 0, 0.f);
}

namespace {

// ---- the variant that allocates nothing ----------------------------------
// Its workspace is this file-scope device array.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and is kept per device.
constexpr size_t kNoAllocBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return rga::fail(RGA_EHIP, "mesh_visibility_noalloc: no current device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return rga::fail(RGA_EHIP, "mesh_visibility_noalloc: hipGetSymbolAddress: %s",
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RGA_OK;
}

}  // namespace

extern "C" size_t mesh_visibility_noalloc_limit(void) { return kNoAllocBytes; }

extern "C" int mesh_visibility_noalloc(void* stream, int nv, int nf, const float* verts,
                                       const int32_t* faces, int V, const float* view_dirs,
                                       int res, const int32_t* knn, int kv, uint32_t* raw_bits,
                                       uint8_t* count) {
  if (nv < 1 || nf < 0 || V < 1)
    return rga::fail(RGA_EINVAL, "mesh_visibility_noalloc: nv >= 1, nf >= 0, V >= 1");
  const size_t need = vis_layout(nv, V).total;
  if (need > kNoAllocBytes)
    return rga::fail(RGA_ECAPACITY,
                     "mesh_visibility_noalloc: %d vertices x %d views need %zu B of scratch, "
                     "above its %zu B",
                     nv, V, need, kNoAllocBytes);
  void* ws = nullptr;
  const int rc = scratch_for_current_device(&ws);
  if (rc != RGA_OK) return rc;
  // every byte of the workspace that a kernel reads was written earlier in
  // the same call, so nothing is cleared
  return visibility_impl(stream, nv, nf, verts, faces, V, view_dirs, res, knn, kv, raw_bits, count,
                         ws, kNoAllocBytes, 0, 0.f);
}

extern "C" int mesh_visibility_shadowmap(void* stream, int nv, int nf, const float* verts,
                                         const int32_t* faces, int V, const float* view_dirs,
                                         int res, const int32_t* knn, int kv, float bias_px,
                                         uint32_t* raw_bits, uint8_t* count, void* ws,
                                         size_t ws_bytes) {
  if (!(bias_px >= 0.f && bias_px <= 64.f))
    return rga::fail(RGA_EINVAL, "mesh_visibility_shadowmap: bias_px in [0, 64]");
  return visibility_impl(stream, nv, nf, verts, faces, V, view_dirs, res, knn, kv, raw_bits, count,
                         ws, ws_bytes, 1, bias_px);
}
