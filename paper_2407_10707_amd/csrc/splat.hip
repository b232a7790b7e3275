// Tile-based Gaussian splatting (the 3DGS rasterizer used in Sec. 3.1 of the
// paper): projection, tile binning, depth + tile radix sort, front-to-back
// alpha compositing, and the hand-written adjoint.
//
// Pipeline on one stream, no host synchronisation:
//   preprocess        1 thread / splat: camera transform, covariance, conic,
//                     opacity-aware tile rectangle, packed 48-byte record;
//                     also clears the frame's ranges, counters and sums
//   depth sort        stable LSD radix sort of (depth bits, index) over n:
//                     3 passes of 11-bit digits, each [upsweep of per-block
//                     digit counts, per-digit scan, ranked scatter]; culled
//                     splats carry key 0xFFFFFFFF
//   offsets           exclusive scan of tiles-touched in depth order -> D
//   duplicate         one (tile, splat) entry per touched tile, emitted in
//                     depth order
//   tile sort         stable LSD radix sort of the entries by tile id (one
//                     pass up to 2048 tiles) -> per tile, entries in
//                     (depth bits, index) order
//   ranges            tile boundaries in the sorted entries (written by the
//                     tile sort's scatter when it takes one pass)
//   blend             (tile, 256-entry chunk) work items over a resident
//                     grid; chunk composites, per-tile combine, restart of
//                     the stop chunk; the adjoint over 64-entry sub-chunks
// Stable ranking inside a radix pass uses wave64 ballots (11 ballots give
// the lanes that share a digit) and mbcnt-style lane masks.
#include "common.h"

#include <algorithm>

#include <math.h>

namespace {

constexpr int kTile = 16;
constexpr int kRadixThreads = 256;
constexpr int kItemsD = 8;       // per thread, passes over the duplicates
constexpr int kItemsN = 2;       // per thread, passes over the splats
constexpr int kBlockD = kRadixThreads * kItemsD;
constexpr int kBlockN = kRadixThreads * kItemsN;
constexpr int kChunk = 256;      // splats per blend work item
constexpr int kSub = 64;         // splats per work item of the blend adjoint
constexpr int kSubs = kChunk / kSub;
constexpr int kQueues = 8;       // item queues of the blend adjoint, one 256-byte line each
constexpr float kHalfNegLog2e = -0.72134752f;   // -log2(e) / 2
constexpr float kInvHalfLog2e = 1.38629436f;    // 2 / log2(e) = 2 ln 2
constexpr int kDigitBits = 11;   // radix digit width of the tile sort: 2048 bins
constexpr int kRadix = 1 << kDigitBits;
constexpr int kWideBits = 12;    // one tile pass of 4096 bins for 2049 .. 4096 tiles
constexpr int kDepthBits = 11;   // digit width of the depth sort: 3 passes over 32-bit keys
constexpr int kDepthPasses = (32 + kDepthBits - 1) / kDepthBits;

struct Layout {
  size_t rec, mean2d, conic, depth, rect, touched, fp64, keys0, vals0, keys1, vals1, offs;
  size_t tk0, tv0, tk1, tv1, ranges, hist, binoff, bintot, bsum, boff, count, queue, grad;
  size_t item_off, item_tile, item_chunk, item_sub, cstate, sstate, sub_item, total;
  int tiles_x, tiles_y, nb_n, nb_cap, nb_max, tile_passes;
  int tile_bits;   // digit width of a one-pass tile sort: kDigitBits or kWideBits
  int64_t max_items, max_subs;
};

Layout make_layout(int n, int width, int height, int64_t cap) {
  Layout L{};
  L.tiles_x = (width + kTile - 1) / kTile;
  L.tiles_y = (height + kTile - 1) / kTile;
  const int64_t tiles = (int64_t)L.tiles_x * L.tiles_y;
  L.nb_n = (int)rga::ceil_div(n > 0 ? n : 1, kBlockN);
  L.nb_cap = (int)rga::ceil_div(cap > 0 ? cap : 1, kBlockD);
  L.nb_max = L.nb_n > L.nb_cap ? L.nb_n : L.nb_cap;
  int bits = 0;
  while ((1ll << bits) < tiles) ++bits;
  L.tile_passes = bits <= kWideBits ? 1 : (bits <= 2 * kDigitBits ? 2 : 3);
  L.tile_bits = (bits > kDigitBits && bits <= kWideBits) ? kWideBits : kDigitBits;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = rga::align_up(o + bytes, 256);
    return at;
  };
  const size_t N = (size_t)(n > 0 ? n : 1);
  const size_t C = (size_t)(cap > 0 ? cap : 1);
  L.rec = take(N * 48);
  L.mean2d = take(N * 8);
  L.conic = take(N * 12);
  L.depth = take(N * 4);
  L.rect = take(N * 16);
  L.touched = take(N * 4);
  L.fp64 = take(N);
  L.keys0 = take(N * 4);
  L.vals0 = take(N * 4);
  L.keys1 = take(N * 4);
  L.vals1 = take(N * 4);
  L.offs = take(N * 4);
  L.tk0 = take(C * 4);
  L.tv0 = take(C * 4);
  L.tk1 = take(C * 4);
  L.tv1 = take(C * 4);
  L.ranges = take((size_t)tiles * 8);
  L.hist = take((size_t)L.nb_max * (1 << kWideBits) * 4);
  L.binoff = take((size_t)L.nb_max * (1 << kWideBits) * 4);
  L.bintot = take((1 << kWideBits) * 4);
  L.bsum = take((size_t)L.nb_n * 4);
  L.boff = take((size_t)L.nb_n * 4);
  L.count = take(32);   // int64 [0] = D, [1] = work items, [3] = adjoint items; uint32 [4] = scan ticket
  L.queue = take(kQueues * 256);   // item queues of the blend adjoint, a line each
  L.grad = take(N * 9 * 4);   // adjoint sums: mean2d, conic [5][n], opacity [n], colour [3][n]
  L.max_items = rga::ceil_div(cap > 0 ? cap : 1, kChunk) + tiles;
  L.item_off = take(((size_t)tiles + 1) * 4);
  L.item_tile = take((size_t)L.max_items * 4);
  L.item_chunk = take((size_t)L.max_items * 4);
  L.item_sub = take((size_t)L.max_items * 4);
  L.cstate = take((size_t)L.max_items * 4 * 256 * 4);
  L.sstate = take((size_t)L.max_items * (kSubs - 1) * 4 * 256 * 4);
  L.max_subs = rga::ceil_div(cap > 0 ? cap : 1, kSub) + tiles;
  L.sub_item = take((size_t)L.max_subs * 4);
  L.total = o;
  return L;
}

template <typename T>
__device__ __host__ inline T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

struct CamDev {
  float R[9], t[3], fx, fy, cx, cy;
  int W, H;
};

CamDev to_dev(const rga_camera* c) {
  CamDev d;
  for (int i = 0; i < 9; ++i) d.R[i] = c->R[i];
  for (int i = 0; i < 3; ++i) d.t[i] = c->t[i];
  d.fx = c->fx;
  d.fy = c->fy;
  d.cx = c->cx;
  d.cy = c->cy;
  d.W = c->width;
  d.H = c->height;
  return d;
}

// exp for the scales: Cody-Waite reduction by ln 2, degree-7 Taylor
// polynomial, fixed FP32 operation order (reproducible bit for bit).
__device__ inline float exp_repro(float x) {
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

// Upper bound of ln y (y >= 1) from exact operations: y = m 2^e, m in [1,2),
// ln y <= e ln 2 + (m - 1) / sqrt(m).
__device__ inline float ln_upper(float y) {
  int e;
  const float m = frexpf(y, &e) * 2.f;
  return (float)(e - 1) * 0.693147182f + (m - 1.f) / sqrtf(m);
}

// ---- forward geometry shared by preprocess and its adjoint ----------------
struct Geo {
  float X, Y, Z, xzr, yzr, J00, J11, J02, J12;
  float s[3], q[4], inv, Rq[9], A[9], M[9], V[9], T[6];
  float a, b, c;
};

__device__ inline void geo_forward(const CamDev& cam, const float* __restrict__ x,
                                   const float* __restrict__ A, const float* __restrict__ quat,
                                   const float* __restrict__ log_s, int n, int g, Geo& G,
                                   bool& ok_quat) {
  const float* Rc = cam.R;
  const float x0 = x[g], x1 = x[n + g], x2 = x[2 * n + g];
  G.X = fmaf(Rc[2], x2, fmaf(Rc[1], x1, fmaf(Rc[0], x0, cam.t[0])));
  G.Y = fmaf(Rc[5], x2, fmaf(Rc[4], x1, fmaf(Rc[3], x0, cam.t[1])));
  G.Z = fmaf(Rc[8], x2, fmaf(Rc[7], x1, fmaf(Rc[6], x0, cam.t[2])));
  for (int j = 0; j < 3; ++j) G.s[j] = exp_repro(log_s[j * n + g]);
  const float q0 = quat[g], q1 = quat[n + g], q2 = quat[2 * n + g], q3 = quat[3 * n + g];
  const float qq = fmaf(q3, q3, fmaf(q2, q2, fmaf(q1, q1, q0 * q0)));
  ok_quat = qq > 0.f;
  G.inv = 1.f / sqrtf(ok_quat ? qq : 1.f);
  const float qw = q0 * G.inv, qx = q1 * G.inv, qy = q2 * G.inv, qz = q3 * G.inv;
  G.q[0] = qw;
  G.q[1] = qx;
  G.q[2] = qy;
  G.q[3] = qz;
  const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
  const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
  const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
  G.Rq[0] = 1.f - 2.f * (yy + zz);
  G.Rq[1] = 2.f * (xy - wz);
  G.Rq[2] = 2.f * (xz + wy);
  G.Rq[3] = 2.f * (xy + wz);
  G.Rq[4] = 1.f - 2.f * (xx + zz);
  G.Rq[5] = 2.f * (yz - wx);
  G.Rq[6] = 2.f * (xz - wy);
  G.Rq[7] = 2.f * (yz + wx);
  G.Rq[8] = 1.f - 2.f * (xx + yy);
  for (int k = 0; k < 9; ++k) G.A[k] = A[k * n + g];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      G.M[3 * i + j] = fmaf(G.A[3 * i + 2], G.Rq[6 + j],
                            fmaf(G.A[3 * i + 1], G.Rq[3 + j], G.A[3 * i] * G.Rq[j])) * G.s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      G.V[3 * i + j] = fmaf(Rc[3 * i + 2], G.M[6 + j], fmaf(Rc[3 * i + 1], G.M[3 + j], Rc[3 * i] * G.M[j]));
  G.xzr = G.X / G.Z;
  G.yzr = G.Y / G.Z;
  G.J00 = cam.fx / G.Z;
  G.J11 = cam.fy / G.Z;
  G.J02 = -(G.J00 * G.xzr);
  G.J12 = -(G.J11 * G.yzr);
  for (int j = 0; j < 3; ++j) {
    G.T[j] = fmaf(G.J02, G.V[6 + j], G.J00 * G.V[j]);
    G.T[3 + j] = fmaf(G.J12, G.V[6 + j], G.J11 * G.V[3 + j]);
  }
  G.a = fmaf(G.T[2], G.T[2], fmaf(G.T[1], G.T[1], G.T[0] * G.T[0])) + 0.3f;
  G.b = fmaf(G.T[2], G.T[5], fmaf(G.T[1], G.T[4], G.T[0] * G.T[3]));
  G.c = fmaf(G.T[5], G.T[5], fmaf(G.T[4], G.T[4], G.T[3] * G.T[3])) + 0.3f;
}

// FP64 2x2 covariance of a near-degenerate splat from the same FP32 inputs.
struct Geo64 {
  double M[9], V[9], T[6], J00, J11, J02, J12, a, b, c, det;
};

__device__ inline void geo_forward64(const CamDev& cam, const Geo& G, Geo64& D) {
  const float* Rc = cam.R;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      D.M[3 * i + j] = fma((double)G.A[3 * i + 2], (double)G.Rq[6 + j],
                           fma((double)G.A[3 * i + 1], (double)G.Rq[3 + j],
                               (double)G.A[3 * i] * (double)G.Rq[j])) * (double)G.s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      D.V[3 * i + j] = fma((double)Rc[3 * i + 2], D.M[6 + j],
                           fma((double)Rc[3 * i + 1], D.M[3 + j], (double)Rc[3 * i] * D.M[j]));
  const double Zd = (double)G.Z;
  D.J00 = (double)cam.fx / Zd;
  D.J11 = (double)cam.fy / Zd;
  D.J02 = -(D.J00 * ((double)G.X / Zd));
  D.J12 = -(D.J11 * ((double)G.Y / Zd));
  for (int j = 0; j < 3; ++j) {
    D.T[j] = fma(D.J02, D.V[6 + j], D.J00 * D.V[j]);
    D.T[3 + j] = fma(D.J12, D.V[6 + j], D.J11 * D.V[3 + j]);
  }
  D.a = fma(D.T[2], D.T[2], fma(D.T[1], D.T[1], D.T[0] * D.T[0])) + 0.3;
  D.b = fma(D.T[2], D.T[5], fma(D.T[1], D.T[4], D.T[0] * D.T[3]));
  D.c = fma(D.T[5], D.T[5], fma(D.T[4], D.T[4], D.T[3] * D.T[3])) + 0.3;
  D.det = fma(D.a, D.c, -(D.b * D.b));
}

// ---- preprocess -------------------------------------------------------------
__global__ void __launch_bounds__(256)
preprocess_kernel(int n, CamDev cam, int TX, int TY, const float* __restrict__ x,
                  const float* __restrict__ A, const float* __restrict__ quat,
                  const float* __restrict__ log_s, const float* __restrict__ opac,
                  const uint8_t* __restrict__ front,
                  float4* __restrict__ rec, float* __restrict__ mean2d, float* __restrict__ conic,
                  float* __restrict__ depth, int32_t* __restrict__ rect,
                  int32_t* __restrict__ touched, uint8_t* __restrict__ fp64,
                  uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                  uint32_t* __restrict__ ranges_u32, int64_t nranges, uint32_t* __restrict__ cnt4,
                  float* __restrict__ grad9, uint32_t* __restrict__ queue) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  // the frame's tile ranges start empty, its counters at zero, and so do the
  // adjoint's per-splat sums and item queues
  if (g < nranges) ranges_u32[g] = 0u;
  if (g < 8) cnt4[g] = 0u;
  if (g < kQueues) queue[g * 64] = 0u;
  if (g >= n) return;
#pragma unroll
  for (int q = 0; q < 9; ++q) grad9[(size_t)q * n + g] = 0.f;
  Geo G;
  bool okq;
  geo_forward(cam, x, A, quat, log_s, n, g, G, okq);
  const float o = opac[g];
  bool valid = (G.Z > 0.2f) && front[g] && (o >= 1.f / 255.f) && okq;
  float ca = 0.f, cb = 0.f, cc = 0.f;
  uint8_t used64 = 0;
  if (valid) {
    const float det = fmaf(G.a, G.c, -(G.b * G.b));
    if (det <= (G.a * G.c) * 0x1p-12f) {
      Geo64 D;
      geo_forward64(cam, G, D);
      if (D.det > 0.0) {
        ca = (float)(D.c / D.det);
        cb = (float)(-D.b / D.det);
        cc = (float)(D.a / D.det);
        used64 = 1;
      } else {
        valid = false;
      }
    } else {
      ca = G.c / det;
      cb = -G.b / det;
      cc = G.a / det;
    }
  }
  const float u = fmaf(cam.fx, G.xzr, cam.cx);
  const float v = fmaf(cam.fy, G.yzr, cam.cy);
  int tx0 = 0, ty0 = 0, tx1 = -1, ty1 = -1, cnt = 0;
  float r2_cull = 0.f;
  if (valid) {
    const float r2 = 2.f * ln_upper(255.f * o);
    r2_cull = r2;
    const float hx = sqrtf(r2 * G.a) * 1.001f + 1e-3f;
    const float hy = sqrtf(r2 * G.c) * 1.001f + 1e-3f;
    float fx0 = floorf((u - hx) * 0.0625f), fx1 = floorf((u + hx) * 0.0625f);
    float fy0 = floorf((v - hy) * 0.0625f), fy1 = floorf((v + hy) * 0.0625f);
    const bool finite = (fx0 == fx0) && (fx1 == fx1) && (fy0 == fy0) && (fy1 == fy1);
    fx0 = fmaxf(fx0, 0.f);
    fy0 = fmaxf(fy0, 0.f);
    fx1 = fminf(fx1, (float)(TX - 1));
    fy1 = fminf(fy1, (float)(TY - 1));
    if (finite && fx0 <= fx1 && fy0 <= fy1) {
      tx0 = (int)fx0;
      ty0 = (int)fy0;
      tx1 = (int)fx1;
      ty1 = (int)fy1;
      cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    }
  }
  // the blend evaluates the exponent of alpha in base 2: the record holds
  // the conic scaled by -log2(e) / 2 (cross term by -log2(e)); the blend
  // passes put the colour into its empty slots when they stage it
  rec[3 * g + 0] = make_float4(u, v, ca * kHalfNegLog2e, cb * (2.f * kHalfNegLog2e));
  rec[3 * g + 1] = make_float4(cc * kHalfNegLog2e, o, 0.f, 0.f);
  // for the blend's per-wave culling: the slopes of the exponent's maxima
  // along vertical and horizontal lines, and a lower bound of the exponent
  // any pixel with alpha >= 1/255 can have (r2 bounds 2 ln(255 o) from
  // above; the margin covers the rounding of both evaluations)
  const float thr = valid ? (r2_cull * kHalfNegLog2e) * 1.01f - 0.01f : 0.f;
  rec[3 * g + 2] = make_float4(0.f, valid ? -cb / cc : 0.f, valid ? -cb / ca : 0.f, thr);
  mean2d[g] = valid ? u : 0.f;
  mean2d[n + g] = valid ? v : 0.f;
  conic[g] = ca;
  conic[n + g] = cb;
  conic[2 * n + g] = cc;
  depth[g] = G.Z;
  rect[g] = tx0;
  rect[n + g] = ty0;
  rect[2 * n + g] = tx1;
  rect[3 * n + g] = ty1;
  touched[g] = cnt;
  fp64[g] = used64;
  keys[g] = cnt > 0 ? __float_as_uint(G.Z) : 0xFFFFFFFFu;
  vals[g] = (uint32_t)g;
}

// The back-face rule (a Gaussian whose normal faces away from the camera
// gets zero opacity), for a caller that bins before it shades: the same
// FP32 expression, in the same order, as the shading kernels' decision, so
// the flags agree bit for bit.
__global__ void __launch_bounds__(256)
back_face_kernel(int n, const float* __restrict__ x, const float* __restrict__ nrm, float c0,
                 float c1, float c2, uint8_t* __restrict__ front) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float w0 = c0 - x[g], w1 = c1 - x[n + g], w2 = c2 - x[2 * (size_t)n + g];
  const float m0 = nrm[g], m1 = nrm[n + g], m2 = nrm[2 * (size_t)n + g];
  front[g] = fmaf(m2, w2, fmaf(m1, w1, m0 * w0)) > 0.f ? 1 : 0;
}

// A splat's record for the blend passes, with its colour (slots 6-8, left
// empty by the projection: the binning runs before the colours exist).
struct SplatRec {
  float4 r0, r1, r2;
};
__device__ inline SplatRec load_rec(const float4* __restrict__ rec, const float* __restrict__ color,
                                    int n, uint32_t g) {
  SplatRec R{rec[3 * g], rec[3 * g + 1], rec[3 * g + 2]};
  R.r1.z = color[g];
  R.r1.w = color[(size_t)n + g];
  R.r2.x = color[2 * (size_t)n + g];
  return R;
}

// ---- blend work items -------------------------------------------------------
// Work items: (tile, chunk of kChunk entries) for the forward passes, and
// (item, sub-chunk of kSub entries) for the adjoint, numbered tile by tile
// with one scan over the tiles (the two counts packed in one 64-bit sum),
// by one workgroup of NT threads, each a run of tiles; len(t) is tile t's
// list length.  Each item gets its tile, chunk index and first sub-item; the
// chunk pass lists the sub-items.
template <int NT, class Len>
__device__ void make_work_items(int tiles, Len&& len, uint32_t* __restrict__ item_off,
                                uint32_t* __restrict__ item_tile, uint32_t* __restrict__ item_chunk,
                                uint32_t* __restrict__ item_sub, int64_t max_items,
                                int64_t* __restrict__ counters, uint64_t* part) {
  const int per = (tiles + NT - 1) / NT;
  const int t0 = min(tiles, (int)threadIdx.x * per), t1 = min(tiles, t0 + per);
  uint64_t s = 0;
  for (int t = t0; t < t1; ++t) {
    const int l = len(t);
    s += (uint64_t)((l + kChunk - 1) / kChunk) | ((uint64_t)((l + kSub - 1) / kSub) << 32);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < NT; o <<= 1) {
    const uint64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0ull;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  const uint64_t before = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
  uint32_t off = (uint32_t)before, soff = (uint32_t)(before >> 32);
  for (int t = t0; t < t1; ++t) {
    item_off[t] = off;
    const int l = len(t);
    const int nch = (l + kChunk - 1) / kChunk;
    for (int j = 0; j < nch; ++j) {
      const int64_t b = (int64_t)off + j;
      if (b == max_items) counters[3] = (int64_t)soff;   // lists truncated: existing items' only
      if (b < max_items) {
        item_tile[b] = (uint32_t)t;
        item_chunk[b] = (uint32_t)j;
        item_sub[b] = soff;
      }
      soff += (uint32_t)min(kSubs, (l - j * kChunk + kSub - 1) / kSub);
    }
    off += nch;
  }
  if (threadIdx.x == NT - 1) {
    const uint64_t tot = part[NT - 1];
    item_off[tiles] = (uint32_t)tot;
    counters[1] = (int64_t)(uint32_t)tot;
    if ((int64_t)(uint32_t)tot <= max_items) counters[3] = (int64_t)(tot >> 32);
  }
}

// Where the items go (passed to the tile sort's one-pass scatter).
struct ItemOut {
  uint32_t *off, *tile, *chunk, *sub;
  int64_t max_items;
  int64_t* counters;
};

// ---- radix sort (reduce-then-scan, stable) ----------------------------------
__device__ inline int64_t live_count(const int64_t* cnt_ptr, int64_t fixed, int64_t cap) {
  int64_t c = cnt_ptr ? *cnt_ptr : fixed;
  return c < cap ? c : cap;
}

// Digits of BITS bits: 32-bit depth keys take 3 passes of 11 bits, tile keys
// of up to 2048 tiles 1 pass.

// Per-block digit histogram (LDS integer atomics), digits of BITS bits.
template <int ITEMS, int BITS>
__global__ void __launch_bounds__(kRadixThreads)
radix_upsweep(const uint32_t* __restrict__ keys, const int64_t* cnt_ptr, int64_t fixed,
              int64_t cap, int shift, uint32_t* __restrict__ hist) {
  constexpr int kRadix = 1 << BITS;
  __shared__ uint32_t h[kRadix];
  const int64_t count = live_count(cnt_ptr, fixed, cap);
  const int64_t base = (int64_t)blockIdx.x * (kRadixThreads * ITEMS);
  if (base >= count) return;              // no items: the scan skips this block
  for (int d = threadIdx.x; d < kRadix; d += kRadixThreads) h[d] = 0;
  __syncthreads();
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t i = base + (int64_t)r * kRadixThreads + threadIdx.x;
    if (i < count) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kRadixThreads)
    hist[(size_t)blockIdx.x * kRadix + d] = h[d];
}

// Exclusive scan of each digit's counts over the blocks that hold items
// (the rest of a capacity-sized grid is skipped): 8 digits per workgroup,
// 32 threads per digit each summing a run of blocks (held in registers for
// runs of up to kHeld blocks); the 32 run sums of a digit are scanned with
// wave shuffles (lanes d, d + 8, ..., of each wave) and the four wave totals.
template <int BITS>
__global__ void __launch_bounds__(256)
radix_binscan(const uint32_t* __restrict__ hist, int nb, const int64_t* cnt_ptr, int64_t fixed,
              int64_t cap, int block_items, uint32_t* __restrict__ binoff,
              uint32_t* __restrict__ bintot) {
  constexpr int kRadix = 1 << BITS;
  constexpr int kHeld = 8;
  __shared__ uint32_t wtot[4][8];
  const int dl = threadIdx.x & 7, c = threadIdx.x >> 3;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int d = blockIdx.x * 8 + dl;
  const int64_t count = live_count(cnt_ptr, fixed, cap);
  const int nbl = (int)min((int64_t)nb, (count + block_items - 1) / block_items);
  const int chunk = (nbl + 31) / 32;
  const int j0 = c * chunk, j1 = min(nbl, j0 + chunk);
  uint32_t held[kHeld];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kHeld; ++q) {
    held[q] = j0 + q < j1 ? hist[(size_t)(j0 + q) * kRadix + d] : 0u;
    s += held[q];
  }
  for (int j = j0 + kHeld; j < j1; ++j) s += hist[(size_t)j * kRadix + d];
  uint32_t incl = s;                      // inclusive scan over c within the wave
#pragma unroll
  for (int o = 8; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane >= 56) wtot[wave][dl] = incl;
  __syncthreads();
  uint32_t run = incl - s, total = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t x = wtot[w][dl];
    run += w < wave ? x : 0u;
    total += x;
  }
  if (c == 0) bintot[d] = total;
#pragma unroll
  for (int q = 0; q < kHeld; ++q)
    if (j0 + q < j1) {
      binoff[(size_t)(j0 + q) * kRadix + d] = run;
      run += held[q];
    }
  for (int j = j0 + kHeld; j < j1; ++j) {
    const uint32_t v = hist[(size_t)j * kRadix + d];
    binoff[(size_t)j * kRadix + d] = run;
    run += v;
  }
}

// Stable scatter of one block.  Each wave owns a contiguous run of
// 64 ITEMS items (so the block's order is wave by wave, round by round, lane
// by lane) and keeps them in registers.  Pass 1: per round, items with the
// same digit are matched with one ballot per digit bit (rank = number of
// lower lanes with that digit, group = their number) and each group's
// lowest lane adds the group to the wave's own digit counts in LDS.  Then,
// after one barrier, digit d of wave w starts at
//   (sum of bintot over digits < d) + binoff[block][d] + (counts of d in
//   waves < w),
// written over the wave's counts; after a second barrier each wave scatters
// its rounds with no further barrier: position = running start of the digit
// + rank, and the group's lowest lane advances the running start (the
// wave's LDS operations complete in order).
template <int ITEMS, int BITS>
__global__ void __launch_bounds__(kRadixThreads)
radix_downsweep(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                const int64_t* cnt_ptr, int64_t fixed, int64_t cap, int shift,
                const uint32_t* __restrict__ binoff, const uint32_t* __restrict__ bintot,
                int32_t* __restrict__ ranges, int nranges, ItemOut items) {
  constexpr int kRadix = 1 << BITS;
  constexpr int kWavesR = kRadixThreads / 64;
  constexpr int kPer = kRadix / kRadixThreads;   // digits per thread in the digit scan
  static_assert(kPer >= 1, "at least one digit per thread");
  __shared__ uint32_t run[kWavesR][kRadix];
  __shared__ uint32_t wtot[kWavesR];
  __shared__ uint64_t ipart[kRadixThreads];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t count = live_count(cnt_ptr, fixed, cap);
  const int64_t blk = (int64_t)blockIdx.x * (kRadixThreads * ITEMS);
  // block 0 of a one-pass tile sort writes the ranges and work items even
  // when there are no entries
  if (blk >= count && !(ranges && blockIdx.x == 0)) return;
  uint32_t* wrun = run[wave];
  for (int d = lane; d < kRadix; d += 64) wrun[d] = 0u;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t wbeg = blk + (int64_t)wave * 64 * ITEMS;
  uint32_t key[ITEMS], val[ITEMS], info[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t i = wbeg + 64 * r + lane;
    const bool ok = i < count;
    key[r] = ok ? kin[i] : 0u;
    val[r] = ok ? vin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const bool ok = wbeg + 64 * r + lane < count;
    const uint32_t d = (key[r] >> shift) & (kRadix - 1);
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt);
    const uint32_t group = __popcll(peers);
    if (ok && rank == 0) wrun[d] += group;
    // rank (6 bits), group size (7 bits); all ones = no item
    info[r] = ok ? (rank | (group << 6)) : 0xFFFFFFFFu;
  }
  // digit starts: each thread sums kPer consecutive digit totals, a wave
  // scan, then the waves' totals
  uint32_t tot[kPer];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    tot[q] = bintot[tid * kPer + q];
    s += tot[q];
  }
  uint32_t incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wtot[wave] = incl;
  __syncthreads();
  uint32_t start = incl - s;
  for (int w = 0; w < wave; ++w) start += wtot[w];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int d = tid * kPer + q;
    // a one-pass tile sort: digit d is tile d, and its entries land at
    // [start of the digit, + its total)
    if (ranges && blockIdx.x == 0 && d < nranges) {
      ranges[2 * d] = (int32_t)start;
      ranges[2 * d + 1] = (int32_t)(start + tot[q]);
    }
    uint32_t acc = start + binoff[(size_t)blockIdx.x * kRadix + d];
#pragma unroll
    for (int w = 0; w < kWavesR; ++w) {
      const uint32_t h = run[w][d];
      run[w][d] = acc;
      acc += h;
    }
    start += tot[q];
  }
  __syncthreads();
  // ... and the blend's work items from the tile lengths (the digit totals)
  if (ranges && blockIdx.x == 0)
    make_work_items<kRadixThreads>(nranges, [&](int t) { return (int)bintot[t]; }, items.off,
                                   items.tile, items.chunk, items.sub, items.max_items,
                                   items.counters, ipart);
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    if (info[r] != 0xFFFFFFFFu) {
      const uint32_t d = (key[r] >> shift) & (kRadix - 1);
      const uint32_t rank = info[r] & 63u, group = info[r] >> 6;
      const uint32_t pos = wrun[d] + rank;
      kout[pos] = key[r];
      vout[pos] = val[r];
      if (rank == 0) wrun[d] += group;
    }
  }
}

// ---- exclusive scan of tiles-touched in depth order -> offsets, D ---------
// Exclusive scan of tiles-touched in depth order, in one launch: every block
// sums its items, publishes the sum and takes a ticket; the block that takes
// the last ticket scans the block sums in a fixed order (deterministic) and
// writes the offsets and D.  No block waits for another.  `done` is zeroed
// on the stream before the launch.
__global__ void __launch_bounds__(kRadixThreads)
touched_scan_kernel(int n, const uint32_t* __restrict__ order, const int32_t* __restrict__ touched,
                    uint32_t* __restrict__ bsum, uint32_t* __restrict__ boff,
                    int64_t* __restrict__ count, uint32_t* __restrict__ done) {
  __shared__ uint32_t red[kRadixThreads];
  __shared__ uint64_t part[kRadixThreads];
  __shared__ bool last;
  const int64_t blk = (int64_t)blockIdx.x * kBlockN;
  uint32_t s = 0;
  for (int r = 0; r < kItemsN; ++r) {
    const int64_t i = blk + (int64_t)r * kRadixThreads + threadIdx.x;
    if (i < n) s += (uint32_t)touched[order[i]];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kRadixThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bsum[blockIdx.x] = red[0];
    __threadfence();                                   // publish before the ticket
    last = atomicAdd(done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();                                     // see every block's sum
  const int nb = gridDim.x;
  const int chunk = (nb + kRadixThreads - 1) / kRadixThreads;
  const int j0 = threadIdx.x * chunk, j1 = min(nb, j0 + chunk);
  uint64_t t = 0;
  for (int j = j0; j < j1; ++j) t += bsum[j];
  part[threadIdx.x] = t;
  __syncthreads();
  for (int o = 1; o < kRadixThreads; o <<= 1) {
    const uint64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0ull;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
  for (int j = j0; j < j1; ++j) {
    boff[j] = (uint32_t)(run < 0xFFFFFFFFull ? run : 0xFFFFFFFFull);
    run += bsum[j];
  }
  if (threadIdx.x == kRadixThreads - 1) count[0] = (int64_t)part[kRadixThreads - 1];
}

// One thread per splat in depth order (blocks of kBlockN, as in the
// offsets scan): a workgroup scan of tiles-touched (wave scans, then the
// sixteen wave totals) gives each splat its first entry.
__global__ void __launch_bounds__(kBlockN)
duplicate_kernel(int n, int TX, int64_t cap, const uint32_t* __restrict__ order,
                 const int32_t* __restrict__ touched, const int32_t* __restrict__ rect,
                 const uint32_t* __restrict__ boff, uint32_t* __restrict__ tkeys,
                 uint32_t* __restrict__ tvals) {
  __shared__ uint32_t wt[kBlockN / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i = (int64_t)blockIdx.x * kBlockN + tid;
  uint32_t g = 0u, cnt = 0u;
  if (i < n) {
    g = order[i];
    cnt = (uint32_t)touched[g];
  }
  const uint32_t incl = rga::wave_scan(cnt);
  if (lane == 63) wt[wave] = incl;
  __syncthreads();
  uint32_t before = 0u;
  for (int w = 0; w < wave; ++w) before += wt[w];
  if (cnt == 0u) return;
  uint64_t off = (uint64_t)boff[blockIdx.x] + before + (incl - cnt);
  const int x0 = rect[g], y0 = rect[n + g], x1 = rect[2 * n + g], y1 = rect[3 * n + g];
  for (int ty = y0; ty <= y1; ++ty)
    for (int tx = x0; tx <= x1; ++tx) {
      if ((int64_t)off < cap) {
        tkeys[off] = (uint32_t)(ty * TX + tx);
        tvals[off] = g;
      }
      ++off;
    }
}

__global__ void __launch_bounds__(256)
fill_u32(uint32_t* __restrict__ p, int64_t count, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void __launch_bounds__(256)
tile_ranges_kernel(const uint32_t* __restrict__ tkeys, const int64_t* cnt_ptr, int64_t cap,
                   int32_t* __restrict__ ranges) {
  const int64_t count = live_count(cnt_ptr, 0, cap);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t t = tkeys[i];
  if (i == 0 || tkeys[i - 1] != t) ranges[2 * t] = (int32_t)i;
  if (i == count - 1 || tkeys[i + 1] != t) ranges[2 * t + 1] = (int32_t)(i + 1);
}

// ---- blend ------------------------------------------------------------------
// Work items are (tile, chunk of <= 256 consecutive list entries); heavy
// tiles therefore spread over many workgroups.  Pass 1 composites each chunk
// independently (transmittance starting at 1); the combine pass walks a
// tile's chunks front to back per pixel: a chunk whose end transmittance
// keeps T_in * T_chunk >= 1e-4 cannot contain the stop (T is monotone), so
// it contributes T_in * C_chunk; the first chunk that may contain the stop
// is re-walked sequentially from T_in with the exact stop rule.  The
// combine leaves (C before the chunk, a code for T_in) per (chunk, pixel)
// for the adjoint.  The codes only flip signs, so T_in comes back exactly:
//   code >= 0          whole chunk used, T_in = code
//   -1 <= code < 0     the chunk where the walk stops, T_in = -code
//   code = kPastStop   chunk past the stop
// For the adjoint, which works on sub-chunks of kSub entries so that no
// workgroup walks a long chunk alone, the chunk pass also leaves each
// pixel's (C, T) at the sub-chunk boundaries, measured from the chunk's
// start (T = 1, C = 0), with T negated once the walk has stopped; the
// restart pass overwrites them, for the pixels it re-walks, with absolute
// states: T_in * T_local and C_before + T_in * C_local up to the sub-chunk
// it starts in, then those of its sequential walk.
constexpr float kPastStop = -2.f;

// One front-to-back compositing step for the pixel centre (px, py), written
// with selects instead of divergent branches: an entry is skipped when its
// exponent is positive or its alpha is below 1/255, and the walk stops at
// the first entry that would take T below 1e-4.  Returns the weight
// alpha * T (0 if the entry is skipped or the walk has stopped); `applied`
// tells whether the entry contributed.
__device__ inline float blend_step(const float4& a, const float4& c1, float px, float py, float& T,
                                   bool& stopped, bool& applied, float& alpha, float& dx,
                                   float& dy, float& G, float& araw) {
  dx = a.x - px;
  dy = a.y - py;
  // power log2(e) = -(A dx^2 + 2 B dx dy + C dy^2) log2(e) / 2 from the
  // scaled conic; exp(power) = 2^(power log2 e)
  const float e2 = fmaf(a.z * dx, dx, fmaf(c1.x * dy, dy, (a.w * dx) * dy));
  G = __builtin_amdgcn_exp2f(e2);
  araw = c1.y * G;
  alpha = fminf(0.99f, araw);
  const bool use = !stopped && e2 <= 0.f && alpha >= 1.f / 255.f;
  const float Tn = T * (1.f - alpha);
  const bool stop = use && Tn < 1e-4f;
  stopped = stopped || stop;
  applied = use && !stop;
  const float w = applied ? alpha * T : 0.f;
  T = applied ? Tn : T;
  return w;
}

// The pixels of a tile in the blend passes: wave w covers the 8 x 8 block
// (w & 1, w >> 1) of the 16 x 16 tile, lane l its pixel (l & 7, l >> 3).
__device__ inline void tile_pixel(int t, int TX, int& px, int& py) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  px = (t % TX) * kTile + 8 * (w & 1) + (l & 7);
  py = (t / TX) * kTile + 8 * (w >> 1) + (l >> 3);
}

// Whether a splat record can give alpha >= 1/255 at any pixel centre of
// the rectangle [x0, x1] x [y0, y1]: the base-2 exponent is a concave
// quadratic, so its largest value there is 0 when the mean is inside, else
// the best of the four edges, each maximised along its line in closed form
// (slopes in the record) and clamped to the edge.  The record's threshold
// is a lower bound with a margin, so the test never drops an entry that a
// pixel would use.
__device__ inline bool reaches(const float4& r0, const float4& r1, const float4& r2, float x0,
                               float x1, float y0, float y1) {
  const float A = r0.z, B = r0.w, C = r1.x;
  const float lx = x0 - r0.x, hx = x1 - r0.x, ly = y0 - r0.y, hy = y1 - r0.y;
  auto ex = [&](float dx, float dy) { return fmaf(A * dx, dx, fmaf(C * dy, dy, (B * dx) * dy)); };
  const float e0 = ex(lx, fminf(fmaxf(r2.y * lx, ly), hy));
  const float e1 = ex(hx, fminf(fmaxf(r2.y * hx, ly), hy));
  const float e2 = ex(fminf(fmaxf(r2.z * ly, lx), hx), ly);
  const float e3 = ex(fminf(fmaxf(r2.z * hy, lx), hx), hy);
  const bool inside = lx <= 0.f && hx >= 0.f && ly <= 0.f && hy >= 0.f;
  return inside || !(fmaxf(fmaxf(e0, e1), fmaxf(e2, e3)) < r2.w);
}

// Staging-time culling: the calling thread holds the record of entry
// 64 * qw + lane (valid if `ok`) and tests it against the 8 x 8 pixel block
// of each of the four waves; one ballot per wave gives that wave's mask for
// this quarter, stored in wmask[wave][qw].  All 64 lanes must be active.
__device__ inline void cull_entry(const float4& r0, const float4& r1, const float4& r2, bool ok,
                                  int t, int TX, int qw, uint64_t (*wmask)[kSubs]) {
  const float bx = (float)((t % TX) * kTile) + 0.5f, by = (float)((t / TX) * kTile) + 0.5f;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const float x0 = bx + 8.f * (w & 1), y0 = by + 8.f * (w >> 1);
    const uint64_t m = __ballot(ok && reaches(r0, r1, r2, x0, x0 + 7.f, y0, y0 + 7.f));
    if ((threadIdx.x & 63) == 0) wmask[w][qw] = m;
  }
}

// The blend's work items from the tile ranges, for the cases the tile sort's
// scatter does not build them (no splats, or a tile sort of several passes).
__global__ void __launch_bounds__(1024)
chunk_index_kernel(int tiles, const int32_t* __restrict__ ranges, uint32_t* __restrict__ item_off,
                   uint32_t* __restrict__ item_tile, uint32_t* __restrict__ item_chunk,
                   uint32_t* __restrict__ item_sub, int64_t max_items,
                   int64_t* __restrict__ counters) {
  __shared__ uint64_t part[1024];
  make_work_items<1024>(tiles, [&](int t) { return ranges[2 * t + 1] - ranges[2 * t]; }, item_off,
                        item_tile, item_chunk, item_sub, max_items, counters, part);
}

// One pixel's (C, T code) into a 1024-float state block: C0, C1, C2, code,
// each 256 floats in pixel order.
__device__ inline void put_state(float* q, float C0, float C1, float C2, float code) {
  q[threadIdx.x] = C0;
  q[256 + threadIdx.x] = C1;
  q[512 + threadIdx.x] = C2;
  q[768 + threadIdx.x] = code;
}

// The blend passes run a grid of as many workgroups as fit on the device at
// once (the item count lives on the device, so the grid cannot be sized to
// it without a host sync).  The forward passes take items i, i + grid, ...;
// the adjoint, whose items vary more in cost and which fits fewer
// workgroups per CU, takes the next item from a queue with one atomic (no
// workgroup ever waits for another).  There are kQueues queues, one per
// group of workgroups with equal index mod kQueues (on this part, those of
// one XCD), each a 256-byte line of its own: queue x hands out items x,
// x + kQueues, ..., so the groups share out the items evenly, and the
// atomics of one line are a kQueues-th of the total (on one counter their
// round trips took about 12 ns each, one after another: 90 us per launch).
// The counters are zeroed on the stream before the launch.
__device__ inline int next_item(uint32_t* queue, int* slot) {
  __syncthreads();                // every thread is done with the last item
  if (threadIdx.x == 0) {
    const int nq = gridDim.x < kQueues ? 1 : kQueues;
    const int x = (int)blockIdx.x % nq;
    *slot = x + nq * (int)atomicAdd(queue + 64 * x, 1u);
  }
  __syncthreads();
  return *slot;
}

__global__ void __launch_bounds__(256)
blend_chunk_kernel(int W, int H, int TX, int n, const int32_t* __restrict__ ranges,
                   const uint32_t* __restrict__ sorted, const float4* __restrict__ rec,
                   const float* __restrict__ color,
                   const uint32_t* __restrict__ item_tile, const uint32_t* __restrict__ item_chunk,
                   const int64_t* __restrict__ counters, int64_t max_items,
                   const uint32_t* __restrict__ item_sub, uint32_t* __restrict__ sub_item,
                   int64_t max_subs, float* __restrict__ cstate, float* __restrict__ sstate) {
  __shared__ float4 s0[kChunk], s1[kChunk], s2[kChunk];
  __shared__ uint64_t wmask[4][kSubs];    // per wave and quarter: entries that can reach its pixels
  __shared__ uint32_t lists[4][kChunk];   // the same, as a list per wave
  const int64_t nitems = min(counters[1], max_items);
  for (int b = blockIdx.x; b < nitems; b += gridDim.x) {
  __syncthreads();                        // the previous item's records are done
  const int t = item_tile[b], j = item_chunk[b];
  int px, py;
  tile_pixel(t, TX, px, py);
  const int e0 = ranges[2 * t] + j * kChunk;
  const int cnt = min(kChunk, ranges[2 * t + 1] - e0);
  if ((int)threadIdx.x * kSub < cnt) {    // the adjoint's sub-items of this chunk
    const int64_t u = (int64_t)item_sub[b] + threadIdx.x;
    if (u < max_subs) sub_item[u] = ((uint32_t)b << 2) | threadIdx.x;
  }
  {
    const bool ok = (int)threadIdx.x < cnt;
    float4 r0 = {}, r1 = {}, r2 = {};
    if (ok) {
      const SplatRec R = load_rec(rec, color, n, sorted[e0 + threadIdx.x]);
      r0 = R.r0;
      r1 = R.r1;
      r2 = R.r2;
      s0[threadIdx.x] = r0;
      s1[threadIdx.x] = r1;
      s2[threadIdx.x] = r2;
    }
    cull_entry(r0, r1, r2, ok, t, TX, threadIdx.x >> 6, wmask);
  }
  __syncthreads();
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool sat = !(px < W && py < H);
  const bool outside = sat;
  float* sub = sstate + (size_t)b * (kSubs - 1) * 1024;
  // this wave's entries as a list (quarter after quarter), nq[q] per quarter
  uint32_t* lst = lists[threadIdx.x >> 6];
  int nq[kSubs];
  {
    const int lane = threadIdx.x & 63;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int base = 0;
#pragma unroll
    for (int q = 0; q < kSubs; ++q) {
      const uint64_t m = wmask[threadIdx.x >> 6][q];
      if ((m >> lane) & 1ull) lst[base + __popcll(m & below)] = (uint32_t)(q * kSub + lane);
      nq[q] = __popcll(m);
      base += nq[q];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the wave reads what its lanes wrote
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  bool live = true;                       // some pixel of this wave not saturated
  int pos = 0;
#pragma unroll
  for (int q = 0; q < kSubs; ++q) {
    if (q * kSub >= cnt) break;
    if (q > 0) put_state(sub + (q - 1) * 1024, C0, C1, C2, sat ? -T : T);
    if (live && __ballot(!sat) == 0ull) live = false;
    const int end = live ? pos + nq[q] : pos;
#pragma unroll 4
    for (int i = pos; i < end; ++i) {
      const int k = (int)lst[i];
      const float4 a = s0[k], c1 = s1[k];
      bool applied;
      float alpha, dx, dy, G, araw;
      const float w = blend_step(a, c1, fpx, fpy, T, sat, applied, alpha, dx, dy, G, araw);
      C0 = fmaf(c1.z, w, C0);
      C1 = fmaf(c1.w, w, C1);
      C2 = fmaf(s2[k].x, w, C2);
    }
    pos += nq[q];
  }
  sat = sat && !outside;
  put_state(cstate + (size_t)b * 1024, C0, C1, C2, sat ? -T : T);   // T >= 1e-4 > 0 at a stop
  }
}

// Prefix pass, one workgroup per tile, no splat is touched: per pixel, walk
// the tile's chunk results front to back, leave for every chunk the colour
// before it and its incoming transmittance, find the chunk that may contain
// the stop (saturated, or T_in * T_chunk < 1e-4) and mark it; chunks past it
// are marked past the stop.  Pixels that never stop get their final colour
// here, and so do pixels that stop in the tile's first chunk: that chunk
// was walked from the true incoming T = 1, so its result is already exact.
// The chunk pass leaves T (>= 0) or, where it stopped, -(T at the stop).
// The state codes it leaves are those described above.
__global__ void __launch_bounds__(256)
blend_prefix_kernel(int W, int H, int TX, const uint32_t* __restrict__ item_off,
                    float* __restrict__ cstate, int64_t max_items, float* __restrict__ image,
                    float* __restrict__ Tfinal, const int64_t* __restrict__ counters,
                    int64_t capacity) {
  const int t = blockIdx.x;
  int px, py;
  tile_pixel(t, TX, px, py);
  const bool inside = px < W && py < H;
  const int64_t i0 = min((int64_t)item_off[t], max_items);
  const int nch = (int)(min((int64_t)item_off[t + 1], max_items) - i0);
  float Tin = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  bool active = inside;
  for (int j = 0; j < nch; ++j) {
    float* st = cstate + (size_t)(i0 + j) * 1024;
    const float Cj0 = st[threadIdx.x], Cj1 = st[256 + threadIdx.x], Cj2 = st[512 + threadIdx.x];
    const float Tj = st[768 + threadIdx.x];
    st[threadIdx.x] = C0;
    st[256 + threadIdx.x] = C1;
    st[512 + threadIdx.x] = C2;
    if (!active) {
      st[768 + threadIdx.x] = kPastStop;
      continue;
    }
    if (Tj < 0.f || Tin * Tj < 1e-4f) {
      st[768 + threadIdx.x] = -Tin;
      active = false;
      if (j == 0 && Tj < 0.f && inside) {   // exact already; else the restart pass
        const size_t p = (size_t)py * W + px, HW = (size_t)H * W;
        image[p] = Cj0;
        image[HW + p] = Cj1;
        image[2 * HW + p] = Cj2;
        Tfinal[p] = -Tj;
      }
      continue;
    }
    st[768 + threadIdx.x] = Tin;
    C0 = fmaf(Tin, Cj0, C0);
    C1 = fmaf(Tin, Cj1, C1);
    C2 = fmaf(Tin, Cj2, C2);
    Tin *= Tj;
  }
  if (inside && active) {
    const size_t p = (size_t)py * W + px, HW = (size_t)H * W;
    image[p] = C0;
    image[HW + p] = C1;
    image[2 * HW + p] = C2;
    Tfinal[p] = Tin;
  }
  // more duplicates than the workspace holds: the lists were truncated, so
  // the frame is poisoned (NaN) rather than silently wrong
  if (inside && counters[0] > capacity) {
    const size_t p = (size_t)py * W + px, HW = (size_t)H * W;
    const float nan = __builtin_nanf("");
    image[p] = nan;
    image[HW + p] = nan;
    image[2 * HW + p] = nan;
    Tfinal[p] = nan;
  }
}

// Restart pass, one workgroup per work item after a tile's first, in
// parallel: pixels whose walk stops in this chunk re-walk it from T_in with
// the exact stop rule, starting at the sub-chunk that may hold the stop, and
// write their final colour and transmittance.  (A pixel whose stop test
// does not fire here because of rounding keeps the chunk's end state.)
__global__ void __launch_bounds__(256)
blend_restart_kernel(int W, int H, int TX, int n, const int32_t* __restrict__ ranges,
                     const uint32_t* __restrict__ sorted, const float4* __restrict__ rec,
                     const float* __restrict__ color,
                     const uint32_t* __restrict__ item_tile, const uint32_t* __restrict__ item_chunk,
                     const int64_t* __restrict__ counters, int64_t max_items,
                     const float* __restrict__ cstate, float* __restrict__ sstate,
                     float* __restrict__ image, float* __restrict__ Tfinal, int64_t capacity) {
  __shared__ float4 s0[kChunk], s1[kChunk], s2[kChunk];
  if (counters[0] > capacity) return;     // truncated lists: the prefix pass poisoned the frame
  const int64_t nitems = min(counters[1], max_items);
  for (int b = blockIdx.x; b < nitems; b += gridDim.x) {
  __syncthreads();                        // the previous item's records are done
  const int j = item_chunk[b], t = item_tile[b];
  const float* st = cstate + (size_t)b * 1024;
  const float code = st[768 + threadIdx.x];
  if (j == 0) continue;                    // finished by the prefix pass
  const bool mine = code < 0.f && code >= -1.f;
  if (!__syncthreads_or(mine)) continue;
  int px, py;
  tile_pixel(t, TX, px, py);
  const int e0 = ranges[2 * t] + j * kChunk;
  const int cnt = min(kChunk, ranges[2 * t + 1] - e0);
  // This pixel's colour before the chunk and its states at the sub-chunk
  // boundaries, read while the records are staged.
  float* sub = sstate + (size_t)b * (kSubs - 1) * 1024;
  float B0 = 0.f, B1 = 0.f, B2 = 0.f, bq[kSubs - 1][4];
  if (mine) {
    B0 = st[threadIdx.x];
    B1 = st[256 + threadIdx.x];
    B2 = st[512 + threadIdx.x];
#pragma unroll
    for (int q = 0; q < kSubs - 1; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) bq[q][c] = sub[q * 1024 + c * 256 + threadIdx.x];
  }
  if ((int)threadIdx.x < cnt) {
    const SplatRec R = load_rec(rec, color, n, sorted[e0 + threadIdx.x]);
    s0[threadIdx.x] = R.r0;
    s1[threadIdx.x] = R.r1;
    s2[threadIdx.x] = R.r2;
  }
  __syncthreads();
  if (!mine || !(px < W && py < H)) continue;
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const float Tin = -code;
  float T = Tin, C0 = B0, C1 = B1, C2 = B2;
  bool stopped = false;
  // Skip the sub-chunks that cannot hold the stop (chunk pass not
  // saturated there and T_in * T_local >= 1e-4; T is monotone): start from
  // the product state at the last such boundary, and leave the absolute
  // states for the adjoint.
  int m = 1;                              // next sub-chunk boundary to record
  bool skip = true;
#pragma unroll
  for (int q = 1; q < kSubs; ++q) {
    skip = skip && q * kSub < cnt && !(bq[q - 1][3] < 0.f || Tin * bq[q - 1][3] < 1e-4f);
    if (skip) {
      T = Tin * bq[q - 1][3];
      C0 = fmaf(Tin, bq[q - 1][0], B0);
      C1 = fmaf(Tin, bq[q - 1][1], B1);
      C2 = fmaf(Tin, bq[q - 1][2], B2);
      put_state(sub + (q - 1) * 1024, C0, C1, C2, T);
      m = q + 1;
    }
  }
  for (int k0 = (m - 1) * kSub; k0 < cnt && !stopped; k0 += 32) {
    if (k0 == m * kSub) put_state(sub + (m++ - 1) * 1024, C0, C1, C2, T);
    const int k1 = min(cnt, k0 + 32);
    for (int k = k0; k < k1; ++k) {
      const float4 a = s0[k], c1 = s1[k];
      bool applied;
      float alpha, dx, dy, G, araw;
      const float w = blend_step(a, c1, fpx, fpy, T, stopped, applied, alpha, dx, dy, G, araw);
      C0 = fmaf(c1.z, w, C0);
      C1 = fmaf(c1.w, w, C1);
      C2 = fmaf(s2[k].x, w, C2);
    }
  }
  for (; m < kSubs && m * kSub < cnt; ++m) put_state(sub + (m - 1) * 1024, C0, C1, C2, stopped ? -T : T);
  const size_t p = (size_t)py * W + px, HW = (size_t)H * W;
  image[p] = C0;
  image[HW + p] = C1;
  image[2 * HW + p] = C2;
  Tfinal[p] = T;
  }
}

// ---- adjoint: blend ----------------------------------------------------------
// Per work item (chunk, sub-chunk of kSub entries) and pixel, starting from
// the sub-chunk's incoming state (the chunk's T_in and colour before it for
// the first sub-chunk; for later ones T_in * T_local and C_before +
// T_in * C_local inside a whole chunk, the restart's exact state inside the
// stop chunk), the entries are re-walked front to back with the same
// decisions:
//   dL/dc_i     = alpha_i T_i g
//   dL/dalpha_i = sum_c g_c (c_ic T_i - (C_c - C_<=i,c) / (1 - alpha_i))
// with C the forward colour, then alpha = o exp(power) (unless clamped).
// Per-splat sums over the tile's pixels: the partials of eight entries that
// touch a wave's pixels are summed over the wave together (lane swaps and
// DPP) and stored into the wave's LDS slice; after the sub-chunk the four
// slices are added and each splat gets one set of global atomics per item.
__global__ void __launch_bounds__(256)
blend_bwd_kernel(int W, int H, int TX, int n, const int32_t* __restrict__ ranges,
                 const uint32_t* __restrict__ sorted, const float4* __restrict__ rec,
                 const float* __restrict__ color,
                 const uint32_t* __restrict__ item_tile, const uint32_t* __restrict__ item_chunk,
                 const uint32_t* __restrict__ sub_item, const int64_t* __restrict__ counters,
                 int64_t max_items, int64_t max_subs, uint32_t* __restrict__ queue,
                 const float* __restrict__ cstate, const float* __restrict__ sstate,
                 const float* __restrict__ image, const float* __restrict__ dimage,
                 float* __restrict__ gmean_conic /*[5][n]*/, float* __restrict__ dopac,
                 float* __restrict__ dcolor) {
  __shared__ float4 s0[kSub], s1[kSub], s2[kSub];
  __shared__ uint32_t sg[kSub];
  __shared__ float acc[4][9][kSub];       // per wave: entry sums over its 64 pixels
  __shared__ int slot;
  const int64_t nitems = min(counters[1], max_items);
  const int64_t nsubs = min(counters[3], max_subs);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, myslot = lane >> 3;
  for (;;) {
  const int u = next_item(queue, &slot);
  if (u >= nsubs) break;
  const uint32_t su = sub_item[u];
  const int b = (int)(su >> 2), m = (int)(su & 3u);
  if (b >= nitems) continue;
  const int t = item_tile[b], j = item_chunk[b];
  int px, py;
  tile_pixel(t, TX, px, py);
  const bool inside = px < W && py < H;
  const int e0 = ranges[2 * t] + j * kChunk + m * kSub;
  const int cnt = min(kSub, ranges[2 * t + 1] - e0);
  // Every wave reads the sub-chunk's records (lane = entry) and keeps a mask
  // of the entries that can reach its 8 x 8 block; wave 0 stages them.
  uint64_t mm;
  {
    const bool ok = lane < cnt;
    float4 r0 = {}, r1 = {}, r2 = {};
    if (ok) {
      const uint32_t g = sorted[e0 + lane];
      r0 = rec[3 * g];
      r1 = rec[3 * g + 1];
      r2 = rec[3 * g + 2];
      if (wave == 0) {
        float4 c1 = r1, c2 = r2;
        c1.z = color[g];
        c1.w = color[(size_t)n + g];
        c2.x = color[2 * (size_t)n + g];
        s0[lane] = r0;
        s1[lane] = c1;
        s2[lane] = c2;
        sg[lane] = g;
      }
    }
    const float x0 = (float)((t % TX) * kTile + 8 * (wave & 1)) + 0.5f;
    const float y0 = (float)((t / TX) * kTile + 8 * (wave >> 1)) + 0.5f;
    mm = __ballot(ok && reaches(r0, r1, r2, x0, x0 + 7.f, y0, y0 + 7.f));
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) (&acc[0][0][0])[q * 256 + threadIdx.x] = 0.f;
  const float* st = cstate + (size_t)b * 1024;
  const float code = st[768 + threadIdx.x];
  bool done = !inside || code < -1.f;
  float T = fabsf(code);
  float A0 = st[threadIdx.x], A1 = st[256 + threadIdx.x], A2 = st[512 + threadIdx.x];
  if (m > 0 && !done) {
    const float* q = sstate + ((size_t)b * (kSubs - 1) + (m - 1)) * 1024;
    const float Tr = q[768 + threadIdx.x];
    const float R0 = q[threadIdx.x], R1 = q[256 + threadIdx.x], R2 = q[512 + threadIdx.x];
    if (code >= 0.f) {                    // whole chunk: local state from the chunk start
      A0 = fmaf(code, R0, A0);
      A1 = fmaf(code, R1, A1);
      A2 = fmaf(code, R2, A2);
      T = code * Tr;
    } else {                              // stop chunk: the exact walk's state
      done = Tr < 0.f;
      T = Tr;
      A0 = R0;
      A1 = R1;
      A2 = R2;
    }
  }
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  float Cf0 = 0.f, Cf1 = 0.f, Cf2 = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  if (!done) {
    const size_t p = (size_t)py * W + px, HW = (size_t)H * W;
    Cf0 = image[p];
    Cf1 = image[HW + p];
    Cf2 = image[2 * HW + p];
    g0 = dimage[p];
    g1 = dimage[HW + p];
    g2 = dimage[2 * HW + p];
  }
  __syncthreads();
  // The listed entries, eight at a time and without branching on whether
  // any pixel uses them, fill eight slots of partials, which are then summed
  // over the wave in one go (slot s ends in lanes 8s .. 8s+7) and stored
  // into this wave's LDS slice.
  while (mm && __ballot(!done) != 0ull) {
    float v[8][9];
    int kv = 0;                             // entry of this lane's slot
    int ns = 0;                             // slots filled
#pragma unroll
    for (int s = 0; s < 8; ++s) {
#pragma unroll
      for (int q = 0; q < 9; ++q) v[s][q] = 0.f;
      if (mm) {
        const int k = (int)__builtin_ctzll(mm);
        mm &= mm - 1;
        const float4 a = s0[k], c1 = s1[k];
        const float col2 = s2[k].x;
        const float Tb = T;
        bool applied;
        float alpha, dx, dy, G, araw;
        const float w = blend_step(a, c1, fpx, fpy, T, done, applied, alpha, dx, dy, G, araw);
        A0 = fmaf(c1.z, w, A0);
        A1 = fmaf(c1.w, w, A1);
        A2 = fmaf(col2, w, A2);
        const float inv1m = __builtin_amdgcn_rcpf(1.f - alpha);   // alpha <= 0.99
        const float dal = g0 * (c1.z * Tb - (Cf0 - A0) * inv1m) +
                          g1 * (c1.w * Tb - (Cf1 - A1) * inv1m) +
                          g2 * (col2 * Tb - (Cf2 - A2) * inv1m);
        const bool lin = applied && araw <= 0.99f;   // alpha not clamped
        const float dp = lin ? dal * alpha : 0.f;     // d/d power
        const float q = dp * kInvHalfLog2e;           // unscale the record's conic
        v[s][0] = q * fmaf(0.5f * a.w, dy, a.z * dx);  // d/d mean x
        v[s][1] = q * fmaf(0.5f * a.w, dx, c1.x * dy); // d/d mean y
        v[s][2] = -0.5f * dp * dx * dx;               // d/d conic A
        v[s][3] = -dp * dx * dy;                      // d/d conic B
        v[s][4] = -0.5f * dp * dy * dy;               // d/d conic C
        v[s][5] = lin ? dal * G : 0.f;                // d/d opacity
        v[s][6] = w * g0;                             // d/d colour
        v[s][7] = w * g1;
        v[s][8] = w * g2;
        kv = myslot == s ? k : kv;
        ++ns;
      }
    }
    float r[9];
    rga::slot_sums8(v, r);
    if ((lane & 7) == 0 && myslot < ns) {
#pragma unroll
      for (int q = 0; q < 9; ++q) acc[wave][q][kv] = r[q];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    const int e = threadIdx.x;
    const uint32_t g = sg[e];
    float sum[9];
    bool nz = false;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      sum[q] = (acc[0][q][e] + acc[1][q][e]) + (acc[2][q][e] + acc[3][q][e]);
      nz |= sum[q] != 0.f;
    }
    if (nz) {
#pragma unroll
      for (int q = 0; q < 5; ++q) atomicAdd(&gmean_conic[(size_t)q * n + g], sum[q]);
      atomicAdd(&dopac[g], sum[5]);
      atomicAdd(&dcolor[g], sum[6]);
      atomicAdd(&dcolor[(size_t)n + g], sum[7]);
      atomicAdd(&dcolor[(size_t)2 * n + g], sum[8]);
    }
  }
  }
}

// ---- adjoint: projection --------------------------------------------------
template <typename R>
struct Chain {
  // Inputs: forward quantities in precision R and upstream gradients.
  // Outputs: camera-space gradient gXYZ, dRq (3x3), ds (3).
  static __device__ void run(const CamDev& cam, const R* Tm, const R* Vm, R J00, R J11, R J02,
                             R J12, R X, R Y, R Z, R ca, R cb, R cc, R dca, R dcb, R dcc, R du,
                             R dv, R* gM /*3x3 out*/, R* gXYZ) {
    const R h = dcb * R(0.5);
    const R P00 = dca * ca + h * cb, P01 = dca * cb + h * cc;
    const R P10 = h * ca + dcc * cb, P11 = h * cb + dcc * cc;
    const R S00 = -(ca * P00 + cb * P10);
    const R S01 = -(ca * P01 + cb * P11);
    const R S11 = -(cb * P01 + cc * P11);
    R gT[6];
    for (int j = 0; j < 3; ++j) {
      gT[j] = R(2) * (S00 * Tm[j] + S01 * Tm[3 + j]);
      gT[3 + j] = R(2) * (S01 * Tm[j] + S11 * Tm[3 + j]);
    }
    R gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
    for (int j = 0; j < 3; ++j) {
      gJ00 += gT[j] * Vm[j];
      gJ02 += gT[j] * Vm[6 + j];
      gJ11 += gT[3 + j] * Vm[3 + j];
      gJ12 += gT[3 + j] * Vm[6 + j];
    }
    R gV[9];
    for (int j = 0; j < 3; ++j) {
      gV[j] = J00 * gT[j];
      gV[3 + j] = J11 * gT[3 + j];
      gV[6 + j] = J02 * gT[j] + J12 * gT[3 + j];
    }
    const R fx = (R)cam.fx, fy = (R)cam.fy;
    const R iz = R(1) / Z, iz2 = iz * iz, iz3 = iz2 * iz;
    R gX = gJ02 * (-fx * iz2) + du * fx * iz;
    R gY = gJ12 * (-fy * iz2) + dv * fy * iz;
    R gZ = gJ00 * (-fx * iz2) + gJ02 * (R(2) * fx * X * iz3) + gJ11 * (-fy * iz2) +
           gJ12 * (R(2) * fy * Y * iz3) - du * fx * X * iz2 - dv * fy * Y * iz2;
    gXYZ[0] = gX;
    gXYZ[1] = gY;
    gXYZ[2] = gZ;
    // gM = Rc^T gV
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        gM[3 * i + j] = (R)cam.R[i] * gV[j] + (R)cam.R[3 + i] * gV[3 + j] + (R)cam.R[6 + i] * gV[6 + j];
  }
};

__global__ void __launch_bounds__(256)
preprocess_bwd_kernel(int n, CamDev cam, const float* __restrict__ x, const float* __restrict__ A,
                      const float* __restrict__ quat, const float* __restrict__ log_s,
                      const float* __restrict__ opac, const uint8_t* __restrict__ front,
                      float* __restrict__ grad9, uint32_t* __restrict__ queue,
                      float* __restrict__ dx, float* __restrict__ dquat,
                      float* __restrict__ dlog_s, float* __restrict__ dopac,
                      float* __restrict__ dcolor, float* __restrict__ dA,
                      const int64_t* __restrict__ counters, int64_t capacity) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < kQueues) queue[g * 64] = 0u;
  if (g >= n) return;
  // take the blend adjoint's sums and leave them zero for another backward
  float gs[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    gs[q] = grad9[(size_t)q * n + g];
    grad9[(size_t)q * n + g] = 0.f;
  }
  if (counters[0] > capacity) {
    // the forward's lists were truncated: poison the gradients (NaN)
    const float nan = __builtin_nanf("");
    for (int k = 0; k < 3; ++k) dx[(size_t)k * n + g] = nan;
    for (int k = 0; k < 4; ++k) dquat[(size_t)k * n + g] = nan;
    for (int k = 0; k < 3; ++k) dlog_s[(size_t)k * n + g] = nan;
    for (int k = 0; k < 3; ++k) dcolor[(size_t)k * n + g] = nan;
    dopac[g] = nan;
    if (dA)
      for (int k = 0; k < 9; ++k) dA[(size_t)k * n + g] = nan;
    return;
  }
  dopac[g] = gs[5];
  for (int k = 0; k < 3; ++k) dcolor[(size_t)k * n + g] = gs[6 + k];
  Geo G;
  bool okq;
  geo_forward(cam, x, A, quat, log_s, n, g, G, okq);
  bool valid = (G.Z > 0.2f) && front[g] && (opac[g] >= 1.f / 255.f) && okq;
  float gM[9], gXYZ[3];
  if (valid) {
    const float du = gs[0], dv = gs[1], dca = gs[2], dcb = gs[3], dcc = gs[4];
    const float det = fmaf(G.a, G.c, -(G.b * G.b));
    if (det <= (G.a * G.c) * 0x1p-12f) {
      Geo64 D;
      geo_forward64(cam, G, D);
      if (D.det > 0.0) {
        const double ca = D.c / D.det, cb = -D.b / D.det, cc = D.a / D.det;
        double gM64[9], g64[3];
        Chain<double>::run(cam, D.T, D.V, D.J00, D.J11, D.J02, D.J12, (double)G.X, (double)G.Y,
                           (double)G.Z, ca, cb, cc, dca, dcb, dcc, du, dv, gM64, g64);
        for (int k = 0; k < 9; ++k) gM[k] = (float)gM64[k];
        for (int k = 0; k < 3; ++k) gXYZ[k] = (float)g64[k];
      } else {
        valid = false;
      }
    } else {
      const float ca = G.c / det, cb = -G.b / det, cc = G.a / det;
      Chain<float>::run(cam, G.T, G.V, G.J00, G.J11, G.J02, G.J12, G.X, G.Y, G.Z, ca, cb, cc, dca,
                        dcb, dcc, du, dv, gM, gXYZ);
    }
  }
  if (!valid) {
    for (int k = 0; k < 3; ++k) dx[(size_t)k * n + g] = 0.f;
    for (int k = 0; k < 4; ++k) dquat[(size_t)k * n + g] = 0.f;
    for (int k = 0; k < 3; ++k) dlog_s[(size_t)k * n + g] = 0.f;
    if (dA)
      for (int k = 0; k < 9; ++k) dA[(size_t)k * n + g] = 0.f;
    return;
  }
  // x' -> camera: dx' = Rc^T gXYZ
  for (int k = 0; k < 3; ++k)
    dx[(size_t)k * n + g] = cam.R[k] * gXYZ[0] + cam.R[3 + k] * gXYZ[1] + cam.R[6 + k] * gXYZ[2];
  // M = (A Rq) diag(s)
  float B[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      B[3 * i + j] = G.A[3 * i] * G.Rq[j] + G.A[3 * i + 1] * G.Rq[3 + j] + G.A[3 * i + 2] * G.Rq[6 + j];
  float gB[9];
  for (int j = 0; j < 3; ++j) {
    float gs = 0.f;
    for (int i = 0; i < 3; ++i) {
      gs += gM[3 * i + j] * B[3 * i + j];
      gB[3 * i + j] = gM[3 * i + j] * G.s[j];
    }
    dlog_s[(size_t)j * n + g] = gs * G.s[j];
  }
  // dA = gB Rq^T (the skinning's linear part, for the pose gradient)
  if (dA)
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k)
        dA[(size_t)(3 * i + k) * n + g] =
            gB[3 * i] * G.Rq[3 * k] + gB[3 * i + 1] * G.Rq[3 * k + 1] + gB[3 * i + 2] * G.Rq[3 * k + 2];
  // gRq = A^T gB
  float gR[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      gR[3 * i + j] = G.A[i] * gB[j] + G.A[3 + i] * gB[3 + j] + G.A[6 + i] * gB[6 + j];
  const float w = G.q[0], qx = G.q[1], qy = G.q[2], qz = G.q[3];
  float gw = 2.f * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
  float gx = 2.f * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.f * qx * gR[4] - w * gR[5] +
                    qz * gR[6] + w * gR[7] - 2.f * qx * gR[8]);
  float gy = 2.f * (-2.f * qy * gR[0] + qx * gR[1] + w * gR[2] + qx * gR[3] + qz * gR[5] -
                    w * gR[6] + qz * gR[7] - 2.f * qy * gR[8]);
  float gz = 2.f * (-2.f * qz * gR[0] - w * gR[1] + qx * gR[2] + w * gR[3] - 2.f * qz * gR[4] +
                    qy * gR[5] + qx * gR[6] + qy * gR[7]);
  const float dot = w * gw + qx * gx + qy * gy + qz * gz;
  dquat[g] = (gw - w * dot) * G.inv;
  dquat[(size_t)n + g] = (gx - qx * dot) * G.inv;
  dquat[(size_t)2 * n + g] = (gy - qy * dot) * G.inv;
  dquat[(size_t)3 * n + g] = (gz - qz * dot) * G.inv;
}

// Workgroups of a 256-thread blend kernel that fit on the current device at
// once (the grid of the grid-stride blend passes), cached per device.
template <int K>
int resident_groups(const void* kernel) {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cache[dev] == 0) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess ||
        per < 1)
      per = 1;
    cache[dev] = (cus > 0 ? cus : 1) * per;
  }
  return cache[dev];
}

// ---- storage order of the Gaussians --------------------------------------------
// The Gaussians sorted by their nearest mesh vertex (vidx row 0), stably (ties
// keep their index order), with the binning's radix sort: keys = vertex,
// values = index, 11-bit digits, as many passes as the vertex count needs.
__global__ void __launch_bounds__(256)
vertex_keys_kernel(int n, const int32_t* __restrict__ vidx, int nv, uint32_t* __restrict__ keys,
                   uint32_t* __restrict__ vals) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g < n) {
    keys[g] = (uint32_t)rga::clampi(vidx[g], 0, nv - 1);
    vals[g] = (uint32_t)g;
  }
}

// dst[r][j] = src[r][order[j]] for rows of 4-byte elements
__global__ void __launch_bounds__(256)
gather_columns_kernel(int rows, int n, const uint32_t* __restrict__ src,
                      const int32_t* __restrict__ order, uint32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)rows * n) return;
  const int64_t r = i / n, j = i - r * n;
  dst[i] = src[r * n + rga::clampi(order[j], 0, n - 1)];
}

struct VertexOrderLayout {
  size_t keys0, keys1, vals0, vals1, hist, binoff, bintot, total;
  int nb;
};

VertexOrderLayout vertex_order_layout(int n) {
  VertexOrderLayout L;
  L.nb = (int)rga::ceil_div(n > 0 ? n : 1, kBlockN);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += rga::align_up(bytes, 256);
    return o;
  };
  const size_t items = (size_t)(n > 0 ? n : 1) * sizeof(uint32_t);
  L.keys0 = take(items);
  L.keys1 = take(items);
  L.vals0 = take(items);
  L.vals1 = take(items);
  L.hist = take((size_t)L.nb * kRadix * sizeof(uint32_t));
  L.binoff = take((size_t)L.nb * kRadix * sizeof(uint32_t));
  L.bintot = take((size_t)kRadix * sizeof(uint32_t));
  L.total = off;
  return L;
}

int check_common(const char* fn, int n, const rga_camera* cam, const void* ws, size_t ws_bytes,
                 int64_t cap, Layout& L) {
  if (n < 0) return rga::fail(RGA_EINVAL, "%s: n < 0", fn);
  if (!cam) return rga::fail(RGA_EINVAL, "%s: null camera", fn);
  if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
    return rga::fail(RGA_EINVAL, "%s: image size must be in 1..16384", fn);
  if (cap < 1 || cap > 0x7FFFFFFFll) return rga::fail(RGA_EINVAL, "%s: capacity must be in 1..2^31-1", fn);
  if (n > 0x7FFFFFFF / 16) return rga::fail(RGA_EUNSUPPORTED, "%s: n too large", fn);
  L = make_layout(n, cam->width, cam->height, cap);
  if (!ws) return rga::fail(RGA_EINVAL, "%s: null workspace", fn);
  if (!rga::aligned16(ws)) return rga::fail(RGA_EINVAL, "%s: workspace must be 16-byte aligned", fn);
  if (ws_bytes < L.total)
    return rga::fail(RGA_ECAPACITY, "%s: workspace %zu < %zu bytes", fn, ws_bytes, L.total);
  return RGA_OK;
}

}  // namespace

extern "C" int back_face(void* stream, int n, const float* x, const float* nrm,
                         const float* cam_pos, uint8_t* front) {
  if (n < 0) return rga::fail(RGA_EINVAL, "back_face: n < 0");
  if (n == 0) return RGA_OK;
  if (!x || !nrm || !cam_pos || !front) return rga::fail(RGA_EINVAL, "back_face: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RGA_LAUNCH("back_face", back_face_kernel, dim3(rga::ceil_div(n, 256)), dim3(256), 0, s, n, x,
             nrm, cam_pos[0], cam_pos[1], cam_pos[2], front);
  RGA_CHECK_LAUNCH("back_face");
  return RGA_OK;
}

extern "C" size_t splat_workspace_size(int n, int width, int height, int64_t capacity) {
  if (n < 0 || width < 1 || height < 1 || capacity < 1) return 0;
  return make_layout(n, width, height, capacity).total;
}

extern "C" int splat_state(void* ws, int n, int width, int height, int64_t capacity,
                           rga_splat_state* st) {
  if (!ws || !st || n < 0 || width < 1 || height < 1 || capacity < 1)
    return rga::fail(RGA_EINVAL, "splat_state: bad argument");
  Layout L = make_layout(n, width, height, capacity);
  st->mean2d = at<float>(ws, L.mean2d);
  st->conic = at<float>(ws, L.conic);
  st->depth = at<float>(ws, L.depth);
  st->rect = at<int32_t>(ws, L.rect);
  st->touched = at<int32_t>(ws, L.touched);
  st->fp64 = at<uint8_t>(ws, L.fp64);
  // after the tile sort the entries sit in the buffer of the final pass
  st->sorted = at<int32_t>(ws, (L.tile_passes & 1) ? L.tv1 : L.tv0);
  st->ranges = at<int32_t>(ws, L.ranges);
  st->count = at<int64_t>(ws, L.count);
  st->tiles_x = L.tiles_x;
  st->tiles_y = L.tiles_y;
  return RGA_OK;
}

extern "C" int splat_read_count(void* stream, const void* ws, int n, int width, int height,
                                int64_t capacity, int64_t* D) {
  if (!ws || !D || n < 0 || width < 1 || height < 1 || capacity < 1)
    return rga::fail(RGA_EINVAL, "splat_read_count: bad argument");
  Layout L = make_layout(n, width, height, capacity);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t h = 0;
  if (hipMemcpyAsync(&h, at<int64_t>(const_cast<void*>(ws), L.count), sizeof(int64_t),
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return rga::fail(RGA_EHIP, "splat_read_count: copy failed");
  *D = h;
  return RGA_OK;
}

// Projection, depth sort, duplication, tile sort, tile ranges and the
// blend's work items: everything of the forward that the colours do not enter.
extern "C" int splat_bin(void* stream, int n, const rga_camera* cam, const float* x,
                         const float* A, const float* quat, const float* log_s,
                         const float* opac, const uint8_t* front, void* ws, size_t ws_bytes,
                         int64_t capacity) {
  Layout L;
  int rc = check_common("splat_bin", n, cam, ws, ws_bytes, capacity, L);
  if (rc) return rc;
  if (n > 0 && (!x || !A || !quat || !log_s || !opac || !front))
    return rga::fail(RGA_EINVAL, "splat_bin: null input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const CamDev cd = to_dev(cam);
  const int64_t tiles = (int64_t)L.tiles_x * L.tiles_y;
  int64_t* cnt = at<int64_t>(ws, L.count);
  uint32_t* k0 = at<uint32_t>(ws, L.keys0);
  uint32_t* v0 = at<uint32_t>(ws, L.vals0);
  uint32_t* k1 = at<uint32_t>(ws, L.keys1);
  uint32_t* v1 = at<uint32_t>(ws, L.vals1);
  uint32_t* hist = at<uint32_t>(ws, L.hist);
  uint32_t* binoff = at<uint32_t>(ws, L.binoff);
  uint32_t* bintot = at<uint32_t>(ws, L.bintot);
  int32_t* ranges = at<int32_t>(ws, L.ranges);
  if (n == 0) {
    // ranges := empty; count := 0
    RGA_LAUNCH("splat_fill", fill_u32, dim3(rga::ceil_div(2 * tiles + 4, 256)), dim3(256), 0, s,
               reinterpret_cast<uint32_t*>(ranges), 2 * tiles, 0u);
    RGA_LAUNCH("splat_fill", fill_u32, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t*>(cnt),
               (int64_t)8, 0u);
  } else {
    // the projection also clears the tile ranges and the counters
    const int64_t pre_threads = std::max<int64_t>(std::max<int64_t>(n, 2 * tiles), 8);
    RGA_LAUNCH("splat_preprocess", preprocess_kernel, dim3(rga::ceil_div(pre_threads, 256)),
               dim3(256), 0, s, n, cd, L.tiles_x, L.tiles_y, x, A, quat, log_s, opac, front, at<float4>(ws, L.rec), at<float>(ws, L.mean2d), at<float>(ws, L.conic),
               at<float>(ws, L.depth), at<int32_t>(ws, L.rect), at<int32_t>(ws, L.touched),
               at<uint8_t>(ws, L.fp64), k0, v0, reinterpret_cast<uint32_t*>(ranges), 2 * tiles,
               reinterpret_cast<uint32_t*>(cnt), at<float>(ws, L.grad), at<uint32_t>(ws, L.queue));
    // depth sort: 3 passes of 11 bits over n 32-bit keys (4 passes of 8
    // bits, with 8x smaller digit tables, take longer: the passes are
    // latency-bound launches)
    for (int pass = 0; pass < kDepthPasses; ++pass) {
      const int shift = kDepthBits * pass;
      RGA_LAUNCH("radix_upsweep", (radix_upsweep<kItemsN, kDepthBits>), dim3(L.nb_n), dim3(kRadixThreads), 0, s, k0,
                 (const int64_t*)nullptr, (int64_t)n, (int64_t)n, shift, hist);
      RGA_LAUNCH("radix_binscan", radix_binscan<kDepthBits>, dim3((1 << kDepthBits) / 8), dim3(256), 0, s, hist, L.nb_n,
                 (const int64_t*)nullptr, (int64_t)n, (int64_t)n, kBlockN, binoff, bintot);
      RGA_LAUNCH("radix_downsweep", (radix_downsweep<kItemsN, kDepthBits>), dim3(L.nb_n), dim3(kRadixThreads), 0, s, k0,
                 v0, k1, v1, (const int64_t*)nullptr, (int64_t)n, (int64_t)n, shift, binoff, bintot,
                 (int32_t*)nullptr, 0, ItemOut{});
      uint32_t* t = k0; k0 = k1; k1 = t;
      t = v0; v0 = v1; v1 = t;
    }
    // v0 now holds the splat indices in (depth, index) order
    uint32_t* bsum = at<uint32_t>(ws, L.bsum);
    uint32_t* boff = at<uint32_t>(ws, L.boff);
    RGA_LAUNCH("touched_scan", touched_scan_kernel, dim3(L.nb_n), dim3(kRadixThreads), 0, s, n, v0,
               at<int32_t>(ws, L.touched), bsum, boff, cnt,
               reinterpret_cast<uint32_t*>(cnt) + 4);
    uint32_t* tk0 = at<uint32_t>(ws, L.tk0);
    uint32_t* tv0 = at<uint32_t>(ws, L.tv0);
    uint32_t* tk1 = at<uint32_t>(ws, L.tk1);
    uint32_t* tv1 = at<uint32_t>(ws, L.tv1);
    RGA_LAUNCH("splat_duplicate", duplicate_kernel, dim3(L.nb_n), dim3(kBlockN), 0, s, n,
               L.tiles_x, capacity, v0, at<int32_t>(ws, L.touched), at<int32_t>(ws, L.rect), boff,
               tk0, tv0);
    const ItemOut items{at<uint32_t>(ws, L.item_off), at<uint32_t>(ws, L.item_tile),
                        at<uint32_t>(ws, L.item_chunk), at<uint32_t>(ws, L.item_sub), L.max_items,
                        cnt};
    if (L.tile_passes == 1 && L.tile_bits == kWideBits) {
      // 2049 .. 4096 tiles: one pass of 12-bit digits, whose scatter also
      // writes the tile ranges and the work items
      constexpr int kWide = 1 << kWideBits;
      RGA_LAUNCH("radix_upsweep", (radix_upsweep<kItemsD, kWideBits>), dim3(L.nb_cap),
                 dim3(kRadixThreads), 0, s, tk0, (const int64_t*)cnt, (int64_t)0, capacity, 0, hist);
      RGA_LAUNCH("radix_binscan", radix_binscan<kWideBits>, dim3(kWide / 8), dim3(256), 0, s, hist,
                 L.nb_cap, (const int64_t*)cnt, (int64_t)0, capacity, kBlockD, binoff, bintot);
      RGA_LAUNCH("radix_downsweep", (radix_downsweep<kItemsD, kWideBits>), dim3(L.nb_cap),
                 dim3(kRadixThreads), 0, s, tk0, tv0, tk1, tv1, (const int64_t*)cnt, (int64_t)0,
                 capacity, 0, binoff, bintot, ranges, (int)tiles, items);
      uint32_t* t = tk0; tk0 = tk1; tk1 = t;
      t = tv0; tv0 = tv1; tv1 = t;
    }
    for (int pass = 0; pass < L.tile_passes && L.tile_bits == kDigitBits; ++pass) {
      const int shift = kDigitBits * pass;
      RGA_LAUNCH("radix_upsweep", (radix_upsweep<kItemsD, kDigitBits>), dim3(L.nb_cap), dim3(kRadixThreads), 0, s, tk0,
                 (const int64_t*)cnt, (int64_t)0, capacity, shift, hist);
      RGA_LAUNCH("radix_binscan", radix_binscan<kDigitBits>, dim3(kRadix / 8), dim3(256), 0, s, hist, L.nb_cap,
                 (const int64_t*)cnt, (int64_t)0, capacity, kBlockD, binoff, bintot);
      // with one tile pass its scatter also writes the tile ranges
      const bool one = L.tile_passes == 1;
      RGA_LAUNCH("radix_downsweep", (radix_downsweep<kItemsD, kDigitBits>), dim3(L.nb_cap), dim3(kRadixThreads), 0, s, tk0,
                 tv0, tk1, tv1, (const int64_t*)cnt, (int64_t)0, capacity, shift, binoff, bintot,
                 one ? ranges : (int32_t*)nullptr, one ? (int)tiles : 0, items);
      uint32_t* t = tk0; tk0 = tk1; tk1 = t;
      t = tv0; tv0 = tv1; tv1 = t;
    }
    if (L.tile_passes > 1)
      RGA_LAUNCH("tile_ranges", tile_ranges_kernel, dim3(rga::ceil_div(capacity, 256)), dim3(256), 0,
                 s, tk0, (const int64_t*)cnt, capacity, ranges);
  }
  // work items (tile, chunk) unless the one-pass tile sort built them
  if (n == 0 || L.tile_passes > 1)
    RGA_LAUNCH("chunk_index", chunk_index_kernel, dim3(1), dim3(1024), 0, s, (int)tiles, ranges,
               at<uint32_t>(ws, L.item_off), at<uint32_t>(ws, L.item_tile),
               at<uint32_t>(ws, L.item_chunk), at<uint32_t>(ws, L.item_sub), L.max_items, cnt);
  RGA_CHECK_LAUNCH("splat_bin");
  return RGA_OK;
}

// The colours into the records, chunk composites, front-to-back combine,
// restarts: the rest of the forward, on the lists splat_bin left in ws.
extern "C" int splat_blend(void* stream, int n, const rga_camera* cam, const float* color,
                           void* ws, size_t ws_bytes, int64_t capacity, float* image,
                           float* T_final) {
  Layout L;
  int rc = check_common("splat_blend", n, cam, ws, ws_bytes, capacity, L);
  if (rc) return rc;
  if (!image || !T_final) return rga::fail(RGA_EINVAL, "splat_blend: null output");
  if (n > 0 && !color) return rga::fail(RGA_EINVAL, "splat_blend: null input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int W = cam->width, H = cam->height;
  const int64_t tiles = (int64_t)L.tiles_x * L.tiles_y;
  int64_t* cnt = at<int64_t>(ws, L.count);
  int32_t* ranges = at<int32_t>(ws, L.ranges);
  const uint32_t* sorted = at<uint32_t>(ws, (L.tile_passes & 1) ? L.tv1 : L.tv0);
  const int64_t g_chunk =
      std::min<int64_t>(L.max_items, resident_groups<0>((const void*)blend_chunk_kernel));
  const int64_t g_restart =
      std::min<int64_t>(L.max_items, resident_groups<1>((const void*)blend_restart_kernel));
  RGA_LAUNCH("blend_chunk", blend_chunk_kernel, dim3(g_chunk), dim3(256), 0, s, W, H, L.tiles_x,
             n, ranges, sorted, at<float4>(ws, L.rec), color, at<uint32_t>(ws, L.item_tile),
             at<uint32_t>(ws, L.item_chunk), cnt, L.max_items, at<uint32_t>(ws, L.item_sub),
             at<uint32_t>(ws, L.sub_item), L.max_subs, at<float>(ws, L.cstate),
             at<float>(ws, L.sstate));
  RGA_LAUNCH("blend_prefix", blend_prefix_kernel, dim3(tiles), dim3(256), 0, s, W, H, L.tiles_x,
             at<uint32_t>(ws, L.item_off), at<float>(ws, L.cstate), L.max_items, image, T_final,
             (const int64_t*)cnt, capacity);
  RGA_LAUNCH("blend_restart", blend_restart_kernel, dim3(g_restart), dim3(256), 0, s, W, H,
             L.tiles_x, n, ranges, sorted, at<float4>(ws, L.rec), color, at<uint32_t>(ws, L.item_tile),
             at<uint32_t>(ws, L.item_chunk), cnt, L.max_items, at<float>(ws, L.cstate),
             at<float>(ws, L.sstate), image, T_final, capacity);
  RGA_CHECK_LAUNCH("splat_blend");
  return RGA_OK;
}

extern "C" int splat_forward(void* stream, int n, const rga_camera* cam, const float* x,
                             const float* A, const float* quat, const float* log_s,
                             const float* opac, const float* color, const uint8_t* front,
                             void* ws, size_t ws_bytes, int64_t capacity, float* image,
                             float* T_final) {
  Layout L;
  int rc = check_common("splat_forward", n, cam, ws, ws_bytes, capacity, L);
  if (rc) return rc;
  if (!image || !T_final) return rga::fail(RGA_EINVAL, "splat_forward: null output");
  if (n > 0 && (!x || !A || !quat || !log_s || !opac || !color || !front))
    return rga::fail(RGA_EINVAL, "splat_forward: null input");
  rc = splat_bin(stream, n, cam, x, A, quat, log_s, opac, front, ws, ws_bytes, capacity);
  if (rc) return rc;
  return splat_blend(stream, n, cam, color, ws, ws_bytes, capacity, image, T_final);
}

extern "C" int splat_backward(void* stream, int n, const rga_camera* cam, const float* x,
                              const float* A, const float* quat, const float* log_s,
                              const float* opac, const float* color, const uint8_t* front,
                              void* ws, size_t ws_bytes, int64_t capacity, const float* image,
                              const float* dimage, float* dx, float* dquat, float* dlog_s,
                              float* dopac, float* dcolor, float* dA) {
  Layout L;
  int rc = check_common("splat_backward", n, cam, ws, ws_bytes, capacity, L);
  if (rc) return rc;
  if (n == 0) return RGA_OK;
  if (!x || !A || !quat || !log_s || !opac || !color || !front || !image || !dimage || !dx ||
      !dquat || !dlog_s || !dopac || !dcolor)
    return rga::fail(RGA_EINVAL, "splat_backward: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const CamDev cd = to_dev(cam);
  // The per-splat sums and the item queue were zeroed by splat_forward's
  // projection, and the projection adjoint zeroes them again after use.
  float* grad9 = at<float>(ws, L.grad);
  uint32_t* queue = at<uint32_t>(ws, L.queue);
  const int64_t g_bwd =
      std::min<int64_t>(L.max_subs, resident_groups<2>((const void*)blend_bwd_kernel));
  const uint32_t* sorted = at<uint32_t>(ws, (L.tile_passes & 1) ? L.tv1 : L.tv0);
  RGA_LAUNCH("blend_bwd", blend_bwd_kernel, dim3(g_bwd), dim3(256), 0, s, cam->width,
             cam->height, L.tiles_x, n, at<int32_t>(ws, L.ranges), sorted, at<float4>(ws, L.rec),
             color,
             at<uint32_t>(ws, L.item_tile), at<uint32_t>(ws, L.item_chunk),
             at<uint32_t>(ws, L.sub_item), at<int64_t>(ws, L.count), L.max_items, L.max_subs,
             queue, at<float>(ws, L.cstate), at<float>(ws, L.sstate), image, dimage, grad9,
             grad9 + (size_t)5 * n, grad9 + (size_t)6 * n);
  RGA_LAUNCH("preprocess_bwd", preprocess_bwd_kernel, dim3(rga::ceil_div(n, 256)), dim3(256), 0, s,
             n, cd, x, A, quat, log_s, opac, front, grad9, queue, dx, dquat, dlog_s, dopac, dcolor,
             dA, (const int64_t*)at<int64_t>(ws, L.count), capacity);
  RGA_CHECK_LAUNCH("splat_backward");
  return RGA_OK;
}

extern "C" size_t vertex_order_workspace(int n) {
  if (n < 0) return 0;
  return vertex_order_layout(n).total;
}

extern "C" int vertex_order(void* stream, int n, const int32_t* vidx, int nv, int32_t* order,
                            void* ws, size_t ws_bytes) {
  if (n < 0 || nv < 1) return rga::fail(RGA_EINVAL, "vertex_order: n >= 0 and nv >= 1");
  if (n > 0x7FFFFFFF / 16) return rga::fail(RGA_EUNSUPPORTED, "vertex_order: n too large");
  if (n == 0) return RGA_OK;
  if (!vidx || !order || !ws) return rga::fail(RGA_EINVAL, "vertex_order: null pointer");
  if (!rga::aligned16(ws)) return rga::fail(RGA_EINVAL, "vertex_order: workspace must be 16-byte aligned");
  const VertexOrderLayout L = vertex_order_layout(n);
  if (ws_bytes < L.total)
    return rga::fail(RGA_ECAPACITY, "vertex_order: workspace %zu < %zu bytes", ws_bytes, L.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* k0 = at<uint32_t>(ws, L.keys0);
  uint32_t* k1 = at<uint32_t>(ws, L.keys1);
  uint32_t* v0 = at<uint32_t>(ws, L.vals0);
  uint32_t* v1 = at<uint32_t>(ws, L.vals1);
  uint32_t* hist = at<uint32_t>(ws, L.hist);
  uint32_t* binoff = at<uint32_t>(ws, L.binoff);
  uint32_t* bintot = at<uint32_t>(ws, L.bintot);
  int bits = 0;
  while (bits < 31 && ((uint32_t)(nv - 1) >> bits) != 0u) ++bits;
  const int passes = bits <= kDigitBits ? 1 : (bits <= 2 * kDigitBits ? 2 : 3);
  RGA_LAUNCH("vertex_keys", vertex_keys_kernel, dim3(rga::ceil_div(n, 256)), dim3(256), 0, s, n,
             vidx, nv, k0, v0);
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = kDigitBits * pass;
    const bool last = pass == passes - 1;
    uint32_t* vout = last ? reinterpret_cast<uint32_t*>(order) : v1;
    RGA_LAUNCH("radix_upsweep", (radix_upsweep<kItemsN, kDigitBits>), dim3(L.nb), dim3(kRadixThreads), 0, s, k0,
               (const int64_t*)nullptr, (int64_t)n, (int64_t)n, shift, hist);
    RGA_LAUNCH("radix_binscan", radix_binscan<kDigitBits>, dim3(kRadix / 8), dim3(256), 0, s, hist, L.nb,
               (const int64_t*)nullptr, (int64_t)n, (int64_t)n, kBlockN, binoff, bintot);
    RGA_LAUNCH("radix_downsweep", (radix_downsweep<kItemsN, kDigitBits>), dim3(L.nb), dim3(kRadixThreads), 0, s,
               k0, v0, k1, vout, (const int64_t*)nullptr, (int64_t)n, (int64_t)n, shift, binoff,
               bintot, (int32_t*)nullptr, 0, ItemOut{});
    uint32_t* t = k0; k0 = k1; k1 = t;
    t = v0; v0 = v1; v1 = t;
  }
  RGA_CHECK_LAUNCH("vertex_order");
  return RGA_OK;
}

extern "C" int gather_columns(void* stream, int rows, int n, const void* src, const int32_t* order,
                              void* dst) {
  if (rows < 0 || n < 0) return rga::fail(RGA_EINVAL, "gather_columns: rows >= 0 and n >= 0");
  if ((int64_t)rows * n == 0) return RGA_OK;
  if (!src || !order || !dst) return rga::fail(RGA_EINVAL, "gather_columns: null pointer");
  if (src == dst) return rga::fail(RGA_EINVAL, "gather_columns: src and dst must not overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t total = (int64_t)rows * n;
  if (rga::ceil_div(total, 256) > 0x7FFFFFFF)
    return rga::fail(RGA_EUNSUPPORTED, "gather_columns: rows * n too large");
  RGA_LAUNCH("gather_columns", gather_columns_kernel, dim3(rga::ceil_div(total, 256)), dim3(256), 0,
             s, rows, n, static_cast<const uint32_t*>(src), order, static_cast<uint32_t*>(dst));
  RGA_CHECK_LAUNCH("gather_columns");
  return RGA_OK;
}
