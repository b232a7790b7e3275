// K nearest canonical vertices and the interpolation equation (Sec. 3.1):
// a Gaussian's attributes are the inverse-distance weighted average of the
// attributes of its K_g nearest mesh vertices (K_v nearest for the
// vertex-to-vertex neighbourhood of the visibility filters).
//
//   build   (once per reference set, e.g. the canonical mesh) uniform grid of
//           cubic cells over the points' bounding box, about two points per
//           cell and at most kMaxCells cells: bounds and cell size, per-cell
//           counts (atomics), one-workgroup scan, fill of (x, y, z, index)
//           records in cell order
//   query   queries sorted by grid cell (counting sort); for k <= 4 four
//           lanes per query point, for wider k one wave (below):
//           cells are visited in shells of growing Chebyshev
//           radius r around the query's cell (the cells of one row of a
//           shell are contiguous, so their records are one run); the best k
//           by (distance^2, index) are kept sorted in registers; the search
//           stops once the k-th distance is below the distance to any
//           unvisited cell (r cell widths, with a margin for rounding) or
//           every cell has been visited.  Then the normalised
//           inverse-distance weights.
//   interpolate   gathers by (query, neighbour)
//   adjoint  per (query chunk, channel, vertex range) workgroup: LDS sums,
//           then coalesced atomic adds into the vertex attributes
#include "common.h"

#include <algorithm>
#include <math.h>

namespace {

constexpr int kMaxK = 32;
constexpr int kMaxCells = 8192;          // cells of the grid (its start table: 32 KB)
constexpr int kBlock = 256;

struct KnnLayout {
  size_t bounds, count, start, cell, rank, recs, total;
};

KnnLayout knn_layout(int nr) {
  KnnLayout L{};
  const size_t R = (size_t)(nr > 0 ? nr : 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t a = o;
    o = rga::align_up(o + bytes, 256);
    return a;
  };
  L.bounds = take(16 * 4);
  L.count = take((size_t)kMaxCells * 4);
  L.start = take(((size_t)kMaxCells + 1) * 4);
  L.cell = take(R * 4);
  L.rank = take(R * 4);
  L.recs = take(R * 16);
  L.total = o;
  return L;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// bounds[0..2] origin, [3] 1 / cell size, [4] cell size, [5..7] cells per
// axis (as floats), [8] cell count; cell counts cleared
__global__ void __launch_bounds__(1024)
knn_bounds_kernel(int nr, const float* __restrict__ ref, float* __restrict__ bounds,
                  uint32_t* __restrict__ count) {
  __shared__ float ext[6][1024];
  __shared__ int ncells;
  float lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = ref[a * nr];
    hi[a] = lo[a];
  }
  for (int i = threadIdx.x; i < nr; i += blockDim.x)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float v = ref[a * nr + i];
      lo[a] = fminf(lo[a], v);
      hi[a] = fmaxf(hi[a], v);
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ext[a][threadIdx.x] = lo[a];
    ext[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        ext[a][threadIdx.x] = fminf(ext[a][threadIdx.x], ext[a][threadIdx.x + o]);
        ext[3 + a][threadIdx.x] = fmaxf(ext[3 + a][threadIdx.x], ext[3 + a][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // cubic cells holding about two points each (the box's volume with each
    // side at least 1e-3 of the longest), enlarged until the grid fits
    float e[3], emax = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      e[a] = ext[3 + a][0] - ext[a][0];
      emax = fmaxf(emax, e[a]);
    }
    if (!(emax > 0.f)) emax = 1.f;
    const float floor_e = 1e-3f * emax;
    const float vol = fmaxf(e[0], floor_e) * fmaxf(e[1], floor_e) * fmaxf(e[2], floor_e);
    float h = cbrtf(vol / fminf(fmaxf(0.5f * (float)nr, 1.f), (float)kMaxCells));
    int g[3], cells = 0;
    for (int it = 0; it < 64; ++it) {
      cells = 1;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        g[a] = max(1, min(1024, (int)ceilf(e[a] / h)));
        cells *= g[a];
      }
      if (cells <= kMaxCells) break;
      h *= 1.1f;
    }
    if (cells > kMaxCells) {   // unreachable for finite inputs; one cell then
      g[0] = g[1] = g[2] = 1;
      cells = 1;
      h = emax;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      bounds[a] = ext[a][0];
      bounds[5 + a] = (float)g[a];
    }
    bounds[3] = 1.f / h;
    bounds[4] = h;
    bounds[8] = (float)cells;
    ncells = cells;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncells; c += blockDim.x) count[c] = 0u;
}

__device__ inline int cell_of(float v, float origin, float inv, int G) {
  return rga::clampi((int)floorf((v - origin) * inv), 0, G - 1);
}

__global__ void __launch_bounds__(kBlock)
knn_zero_u32(uint32_t* __restrict__ p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

__global__ void __launch_bounds__(kBlock)
knn_count_kernel(int nr, const float* __restrict__ ref, const float* __restrict__ bounds,
                 uint32_t* __restrict__ count, uint32_t* __restrict__ cell,
                 uint32_t* __restrict__ rank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  const int gx = (int)bounds[5], gy = (int)bounds[6], gz = (int)bounds[7];
  const int cx = cell_of(ref[i], bounds[0], bounds[3], gx);
  const int cy = cell_of(ref[nr + i], bounds[1], bounds[3], gy);
  const int cz = cell_of(ref[2 * nr + i], bounds[2], bounds[3], gz);
  const uint32_t c = (uint32_t)((cz * gy + cy) * gx + cx);
  cell[i] = c;
  rank[i] = atomicAdd(&count[c], 1u);
}

// exclusive scan of the cell counts, one workgroup
__global__ void __launch_bounds__(1024)
knn_scan_kernel(const float* __restrict__ bounds, const uint32_t* __restrict__ count,
                uint32_t* __restrict__ start) {
  __shared__ uint32_t part[1024];
  const int cells = (int)bounds[8];
  const int per = (cells + 1023) / 1024;
  const int c0 = threadIdx.x * per, c1 = min(cells, c0 + per);
  uint32_t s = 0;
  for (int c = c0; c < c1; ++c) s += count[c];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int c = c0; c < c1; ++c) {
    start[c] = run;
    run += count[c];
  }
  if (threadIdx.x == 1023) start[cells] = part[1023];
}

__global__ void __launch_bounds__(kBlock)
knn_fill_kernel(int nr, const float* __restrict__ ref, const uint32_t* __restrict__ start,
                const uint32_t* __restrict__ cell, const uint32_t* __restrict__ rank,
                float4* __restrict__ recs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  recs[start[cell[i]] + rank[i]] = make_float4(ref[i], ref[nr + i], ref[2 * nr + i], __int_as_float(i));
}

// (d, j) before (e, l) in (distance^2, index) order
__device__ inline bool before(float d, int j, float e, int l) { return d < e || (d == e && j < l); }

// Queries are taken in the order of their grid cells (a counting sort:
// per-cell counts with ranks, one-workgroup scan, fill), so that the lanes
// of a wave search the same or neighbouring cells.
__global__ void __launch_bounds__(kBlock)
knn_qcell_kernel(int n, const float* __restrict__ q, const float* __restrict__ bounds,
                 uint32_t* __restrict__ qcount, uint32_t* __restrict__ qcell,
                 uint32_t* __restrict__ qrank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int gx = (int)bounds[5], gy = (int)bounds[6], gz = (int)bounds[7];
  const int cx = cell_of(q[i], bounds[0], bounds[3], gx);
  const int cy = cell_of(q[n + i], bounds[1], bounds[3], gy);
  const int cz = cell_of(q[2 * n + i], bounds[2], bounds[3], gz);
  const uint32_t c = (uint32_t)((cz * gy + cy) * gx + cx);
  qcell[i] = c;
  qrank[i] = atomicAdd(&qcount[c], 1u);
}

__global__ void __launch_bounds__(kBlock)
knn_qfill_kernel(int n, const uint32_t* __restrict__ qstart, const uint32_t* __restrict__ qcell,
                 const uint32_t* __restrict__ qrank, uint32_t* __restrict__ order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) order[qstart[qcell[i]] + qrank[i]] = (uint32_t)i;
}

// Small k (<= 4): four lanes per query (a quad), so that a search of a
// few hundred thousand queries still has several waves per SIMD to hide
// the latency of its dependent loads.  The quad walks the shells row by
// row as one; the records of a row are dealt out to its lanes in turn (so
// a quad reads consecutive records), each lane keeping the best k of its
// own records, sorted, in the last k of four register slots (the slots
// before them hold -inf sentinels that nothing is ever placed before, so
// the worst kept entry is always the last slot).  At the end of each shell the quad merges its four lists:
// k rounds of a minimum over the quad (two DPP exchanges), the lane that
// holds the minimum moving to its next entry; the k-th of the merge drives
// the stop rule and prunes the lanes' candidates.
constexpr int kQuadBatch = 2;            // records per lane loaded together

// (d, j) <- the smallest of the quad's four in (distance^2, index) order
__device__ inline void quad_min(float& d, int& j) {
  float od = __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(d), __float_as_int(d), 0xB1, 0xf, 0xf, false));
  int oj = __builtin_amdgcn_update_dpp(j, j, 0xB1, 0xf, 0xf, false);
  if (before(od, oj, d, j)) {
    d = od;
    j = oj;
  }
  od = __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(d), __float_as_int(d), 0x4E, 0xf, 0xf, false));
  oj = __builtin_amdgcn_update_dpp(j, j, 0x4E, 0xf, 0xf, false);
  if (before(od, oj, d, j)) {
    d = od;
    j = oj;
  }
}

__global__ void __launch_bounds__(kBlock)
knn_query_quad_kernel(int n, const float* __restrict__ q, int k, const float* __restrict__ bounds,
                      const uint32_t* __restrict__ start, const float4* __restrict__ recs,
                      const uint32_t* __restrict__ order, int32_t* __restrict__ idx,
                      float* __restrict__ w) {
  constexpr int S = 4;                    // register slots = the largest k
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int it = (int)(gt >> 2), sub = (int)(gt & 3);
  if (it >= n) return;                    // whole quads leave
  const int i = (int)order[it];
  const int gx = (int)bounds[5], gy = (int)bounds[6], gz = (int)bounds[7];
  const float qx = q[i], qy = q[n + i], qz = q[2 * n + i];
  const int cx = cell_of(qx, bounds[0], bounds[3], gx);
  const int cy = cell_of(qy, bounds[1], bounds[3], gy);
  const int cz = cell_of(qz, bounds[2], bounds[3], gz);
  const float h = bounds[4];
  const int rmax = max(gx, max(gy, gz));
  const int first = S - k;                // slot of the nearest
  float bd[S];
  int bi[S];
#pragma unroll
  for (int t = 0; t < S; ++t) {
    bd[t] = t < first ? -INFINITY : INFINITY;
    bi[t] = t < first ? -1 : 0x7fffffff;
  }
  float md[S], kd = INFINITY;             // the quad's merged best k; its k-th
  int mj[S], kj = 0x7fffffff;
  for (int r = 0; r <= rmax; ++r) {
    const int z0 = max(cz - r, 0), z1 = min(cz + r, gz - 1);
    const int y0 = max(cy - r, 0), y1 = min(cy + r, gy - 1);
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y) {
        const bool face = abs(z - cz) == r || abs(y - cy) == r;
        const int row = (z * gy + y) * gx;
        for (int side = 0; side < (face ? 1 : 2); ++side) {
          int x0, x1;
          if (face) {
            x0 = max(cx - r, 0);
            x1 = min(cx + r, gx - 1);
          } else {
            x0 = x1 = side == 0 ? cx - r : cx + r;
            if (x0 < 0 || x0 > gx - 1) continue;
          }
          const uint32_t e0 = start[row + x0], e1 = start[row + x1 + 1];
          for (uint32_t b = e0; b < e1; b += 4 * kQuadBatch) {   // the same steps in the quad
            const uint32_t e = b + sub;
            float4 pb[kQuadBatch];
#pragma unroll
            for (int u = 0; u < kQuadBatch; ++u)
              pb[u] = e + 4 * u < e1 ? recs[e + 4 * u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < kQuadBatch; ++u) {
              if (e + 4 * u >= e1) continue;
              const float4 p = pb[u];
              const int j = __float_as_int(p.w);
              const float dx = p.x - qx, dy = p.y - qy, dz = p.z - qz;
              const float d = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
              if (!before(d, j, bd[S - 1], bi[S - 1]) || !before(d, j, kd, kj)) continue;
              bool placed = false;
#pragma unroll
              for (int t = S - 1; t >= 0; --t) {
                if (placed) continue;
                if (t > 0 && before(d, j, bd[t - 1], bi[t - 1])) {
                  bd[t] = bd[t - 1];
                  bi[t] = bi[t - 1];
                } else {
                  bd[t] = d;
                  bi[t] = j;
                  placed = true;
                }
              }
            }
          }
        }
      }
    // merge the quad's lists: k rounds of a quad minimum
    int ptr = first;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      md[t] = INFINITY;
      mj[t] = 0x7fffffff;
      if (t >= k) continue;
      float hd = INFINITY;
      int hj = 0x7fffffff;
#pragma unroll
      for (int u = 0; u < S; ++u)
        if (u == ptr) {
          hd = bd[u];
          hj = bi[u];
        }
      float d = hd;
      int j = hj;
      quad_min(d, j);
      if (d == hd && j == hj) ++ptr;
      md[t] = d;
      mj[t] = j;
      kd = d;
      kj = j;
    }
    // unvisited cells are at least r cell widths away (less a margin for
    // the rounding of cell assignment and distances)
    const float reach = (float)r * h;
    if (kd < reach * reach * 0.9999f) break;
  }
  // normalised inverse-distance weights; a query on a vertex takes it alone
  const bool on_vertex = md[0] == 0.f;
  float u[S], s = 0.f;
#pragma unroll
  for (int t = 0; t < S; ++t) {
    u[t] = t < k ? __builtin_amdgcn_rcpf(__builtin_sqrtf(md[t])) : 0.f;
    s += u[t];
  }
  const float is = 1.f / s;
#pragma unroll
  for (int t = 0; t < S; ++t) {
    if (t != sub || t >= k) continue;
    const size_t o = (size_t)t * n + i;
    idx[o] = mj[t];
    w[o] = on_vertex ? (t == 0 ? 1.f : 0.f) : u[t] * is;
  }
}

// Wider searches (k > 4): one wave per query.  The lanes take the cells of
// a shell (the shell's cells among the clipped cube of radius r, 64 at a
// time) and step through their cells' records together, four records per
// lane at a time; a candidate that beats the current k-th is inserted into
// the sorted list held one entry per lane (lane t = the t-th nearest so
// far): its position is the number of list entries before it (one ballot),
// the entries from there on move up one lane.  The stop rule is the quad
// search's, so both return the same neighbours.
constexpr int kWaveBatch = 4;
__global__ void __launch_bounds__(kBlock)
knn_query_wave_kernel(int n, const float* __restrict__ q, int k, const float* __restrict__ bounds,
                      const uint32_t* __restrict__ start, const float4* __restrict__ recs,
                      const uint32_t* __restrict__ order, int32_t* __restrict__ idx,
                      float* __restrict__ w) {
  const int lane = threadIdx.x & 63;
  const int it = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
  if (it >= n) return;                   // whole waves leave
  const int i = __builtin_amdgcn_readfirstlane((int)order[it]);
  const int gx = (int)bounds[5], gy = (int)bounds[6], gz = (int)bounds[7];
  const float qx = q[i], qy = q[n + i], qz = q[2 * n + i];
  const int cx = cell_of(qx, bounds[0], bounds[3], gx);
  const int cy = cell_of(qy, bounds[1], bounds[3], gy);
  const int cz = cell_of(qz, bounds[2], bounds[3], gz);
  const float h = bounds[4];
  const int rmax = max(gx, max(gy, gz));
  float bd = INFINITY;                   // this lane's list entry
  int bi = 0x7fffffff;
  float wd = INFINITY;                   // the k-th entry (wave-uniform)
  int wj = 0x7fffffff;
  const int up = ((lane + 63) & 63) << 2;   // ds_bpermute address of the lane below
  for (int r = 0; r <= rmax; ++r) {
    const int x0 = max(cx - r, 0), x1 = min(cx + r, gx - 1);
    const int y0 = max(cy - r, 0), y1 = min(cy + r, gy - 1);
    const int z0 = max(cz - r, 0), z1 = min(cz + r, gz - 1);
    const int sx = x1 - x0 + 1, sy = y1 - y0 + 1;
    const int box = sx * sy * (z1 - z0 + 1);
    for (int c0 = 0; c0 < box; c0 += 64) {
      const int c = c0 + lane;
      uint32_t e0 = 0, len = 0;
      if (c < box) {
        const int x = x0 + c % sx, yz = c / sx;
        const int y = y0 + yz % sy, z = z0 + yz / sy;
        if (max(abs(x - cx), max(abs(y - cy), abs(z - cz))) == r) {
          const int cell = (z * gy + y) * gx + x;
          e0 = start[cell];
          len = start[cell + 1] - e0;
        }
      }
      for (uint32_t m = 0; __ballot(m < len) != 0ull; m += kWaveBatch) {
        float4 pb[kWaveBatch];
#pragma unroll
        for (int u = 0; u < kWaveBatch; ++u)
          pb[u] = m + u < len ? recs[e0 + m + u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < kWaveBatch; ++u) {
          const bool has = m + u < len;
          const int j = __float_as_int(pb[u].w);
          const float dx = pb[u].x - qx, dy = pb[u].y - qy, dz = pb[u].z - qz;
          const float d = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          uint64_t sm = __ballot(has && before(d, j, wd, wj));
          while (sm) {
            const int src = (int)__builtin_ctzll(sm);
            sm &= sm - 1;
            const float cd = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), src));
            const int cj = __builtin_amdgcn_readlane(j, src);
            if (!before(cd, cj, wd, wj)) continue;   // an earlier insertion raised the bar
            const int pos = __popcll(__ballot(lane < k && before(bd, bi, cd, cj)));
            const float ld = __int_as_float(__builtin_amdgcn_ds_bpermute(up, __float_as_int(bd)));
            const int li = __builtin_amdgcn_ds_bpermute(up, bi);
            if (lane == pos) {
              bd = cd;
              bi = cj;
            } else if (lane > pos) {
              bd = ld;
              bi = li;
            }
            wd = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bd), k - 1));
            wj = __builtin_amdgcn_readlane(bi, k - 1);
          }
        }
      }
    }
    const float reach = (float)r * h;
    if (wd < reach * reach * 0.9999f) break;
  }
  // normalised inverse-distance weights; a query on a vertex takes it alone
  const bool on_vertex = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bd), 0)) == 0.f;
  const float u = lane < k ? __builtin_amdgcn_rcpf(__builtin_sqrtf(bd)) : 0.f;
  const float is = 1.f / rga::wave_sum(u);
  if (lane < k) {
    const size_t o = (size_t)lane * n + i;
    idx[o] = bi;
    w[o] = on_vertex ? (lane == 0 ? 1.f : 0.f) : u * is;
  }
}

template <int KMAX>
__global__ void __launch_bounds__(kBlock)
knn_interp_kernel(int n, int k, const int32_t* __restrict__ idx, const float* __restrict__ w,
                  int C, int nr, const float* __restrict__ attr, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int j[KMAX];
  float wt[KMAX];
#pragma unroll
  for (int t = 0; t < KMAX; ++t) {
    j[t] = t < k ? rga::clampi(idx[(size_t)t * n + i], 0, nr - 1) : 0;
    wt[t] = t < k ? w[(size_t)t * n + i] : 0.f;
  }
  // for small k four channels per step, so that their gathers are in
  // flight together (for wide k the neighbours alone fill the registers)
  constexpr int kStep = KMAX <= 4 ? 4 : 1;
  for (int c0 = 0; c0 < C; c0 += kStep) {
    float v[kStep] = {};
#pragma unroll
    for (int u = 0; u < kStep; ++u) {
      if (c0 + u >= C) continue;
      const float* a = attr + (size_t)(c0 + u) * nr;
#pragma unroll
      for (int t = 0; t < KMAX; ++t)
        if (t < k) v[u] = fmaf(wt[t], a[j[t]], v[u]);
    }
#pragma unroll
    for (int u = 0; u < kStep; ++u)
      if (c0 + u < C) out[(size_t)(c0 + u) * n + i] = v[u];
  }
}

__global__ void __launch_bounds__(kBlock)
knn_zero_kernel(float* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.f;
}

// Adjoint of the average, one workgroup per (chunk of queries, channel,
// range of kVRange vertices): the chunk's w dout terms for vertices in the
// range are summed in LDS (integer compare-and-swap adds), then added to
// dattr with coalesced atomics, one per vertex of the range.  (Global float
// atomics at scattered addresses are far slower on this part.)
constexpr int kVRange = 16384;           // 64 KB of LDS
__global__ void __launch_bounds__(kBlock)
knn_interp_bwd_kernel(int n, int k, const int32_t* __restrict__ idx, const float* __restrict__ w,
                      int nr, const float* __restrict__ dout, float* __restrict__ dattr,
                      int chunk) {
  __shared__ float acc[kVRange];
  const int c = blockIdx.y;
  const int v0 = blockIdx.z * kVRange, vn = min(kVRange, nr - v0);
  const int q0 = blockIdx.x * chunk, q1 = min(n, q0 + chunk);
  for (int j = threadIdx.x; j < vn; j += blockDim.x) acc[j] = 0.f;
  __syncthreads();
  const float* g = dout + (size_t)c * n;
  // Each wave takes its own contiguous quarter of the block's queries, and
  // queries that share a neighbour in consecutive lanes (points stored
  // grouped by vertex) are summed across the wave first: one lane adds per
  // run, and the waves of a block mostly add to different LDS words.
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int per = (q1 - q0 + nw - 1) / nw;
  const int wq0 = q0 + wave * per, wq1 = min(q1, wq0 + per);
  for (int base = wq0; base < wq1; base += 64) {
    const int i = base + lane;
    const bool ok = i < wq1;
    const float gi = ok ? g[i] : 0.f;
    for (int t = 0; t < k; ++t) {
      const int j = ok ? idx[(size_t)t * n + i] - v0 : -1;
      const bool use = ok && gi != 0.f && j >= 0 && j < vn;
      float val = use ? w[(size_t)t * n + i] * gi : 0.f;
      // the LDS float atomic: lanes of one wave that still share a word
      // (neighbours repeating out of order) are serialised in the LDS unit
      // instead of retrying a compare-and-swap (0.129 -> 0.087 ms for 42
      // channels of the avatar's 100k Gaussians)
      if (rga::wave_run_sum(use ? j : -1 - lane, val) && use) atomicAdd(&acc[j], val);
    }
  }
  __syncthreads();
  float* out = dattr + (size_t)c * nr + v0;
  for (int j = threadIdx.x; j < vn; j += blockDim.x) {
    const float a = acc[j];
    if (a != 0.f) atomicAdd(&out[j], a);
  }
}

}  // namespace

extern "C" size_t knn_workspace(int nr) { return knn_layout(nr).total; }

extern "C" int knn_build(void* stream, int nr, const float* ref, void* ws, size_t ws_bytes) {
  if (nr < 1) return rga::fail(RGA_EINVAL, "knn_build: nr >= 1");
  if (!ref || !ws) return rga::fail(RGA_EINVAL, "knn_build: null pointer");
  const KnnLayout L = knn_layout(nr);
  if (ws_bytes < L.total) return rga::fail(RGA_ECAPACITY, "knn_build: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RGA_LAUNCH("knn_bounds", knn_bounds_kernel, dim3(1), dim3(1024), 0, s, nr, ref,
             at<float>(ws, L.bounds), at<uint32_t>(ws, L.count));
  RGA_LAUNCH("knn_count", knn_count_kernel, dim3(rga::ceil_div(nr, kBlock)), dim3(kBlock), 0, s,
             nr, ref, at<float>(ws, L.bounds), at<uint32_t>(ws, L.count),
             at<uint32_t>(ws, L.cell), at<uint32_t>(ws, L.rank));
  RGA_LAUNCH("knn_scan", knn_scan_kernel, dim3(1), dim3(1024), 0, s, at<float>(ws, L.bounds),
             at<uint32_t>(ws, L.count), at<uint32_t>(ws, L.start));
  RGA_LAUNCH("knn_fill", knn_fill_kernel, dim3(rga::ceil_div(nr, kBlock)), dim3(kBlock), 0, s, nr,
             ref, at<uint32_t>(ws, L.start), at<uint32_t>(ws, L.cell), at<uint32_t>(ws, L.rank),
             at<float4>(ws, L.recs));
  RGA_CHECK_LAUNCH("knn_build");
  return RGA_OK;
}

extern "C" size_t knn_query_workspace(int n) {
  if (n < 0) return 0;
  const size_t N = (size_t)(n > 0 ? n : 1);
  return rga::align_up((size_t)kMaxCells * 4, 256) + rga::align_up(((size_t)kMaxCells + 1) * 4, 256) +
         3 * rga::align_up(N * 4, 256);
}

extern "C" int knn_query(void* stream, int n, const float* q, int nr, int k, int32_t* idx,
                         float* w, const void* ws, size_t ws_bytes, void* scratch,
                         size_t scratch_bytes) {
  if (n < 0 || nr < 1) return rga::fail(RGA_EINVAL, "knn_query: n >= 0 and nr >= 1");
  if (k < 1 || k > kMaxK || k > nr)
    return rga::fail(RGA_EINVAL, "knn_query: k must be in 1..min(%d, nr)", kMaxK);
  if (n == 0) return RGA_OK;
  if (!q || !idx || !w || !ws || !scratch) return rga::fail(RGA_EINVAL, "knn_query: null pointer");
  const KnnLayout L = knn_layout(nr);
  if (ws_bytes < L.total) return rga::fail(RGA_ECAPACITY, "knn_query: workspace too small");
  if (scratch_bytes < knn_query_workspace(n))
    return rga::fail(RGA_ECAPACITY, "knn_query: scratch too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* W = const_cast<void*>(ws);
  const size_t N = rga::align_up((size_t)n * 4, 256);
  uint32_t* qcount = static_cast<uint32_t*>(scratch);
  uint32_t* qstart = qcount + rga::align_up((size_t)kMaxCells * 4, 256) / 4;
  uint32_t* qcell = qstart + rga::align_up(((size_t)kMaxCells + 1) * 4, 256) / 4;
  uint32_t* qrank = qcell + N / 4;
  uint32_t* order = qrank + N / 4;
  const dim3 grid(rga::ceil_div(n, kBlock));
  RGA_LAUNCH("knn_qzero", knn_zero_u32, dim3(rga::ceil_div(kMaxCells, kBlock)), dim3(kBlock), 0, s,
             qcount, kMaxCells);
  RGA_LAUNCH("knn_qcell", knn_qcell_kernel, grid, dim3(kBlock), 0, s, n, q, at<float>(W, L.bounds),
             qcount, qcell, qrank);
  RGA_LAUNCH("knn_qscan", knn_scan_kernel, dim3(1), dim3(1024), 0, s, at<float>(W, L.bounds),
             qcount, qstart);
  RGA_LAUNCH("knn_qfill", knn_qfill_kernel, grid, dim3(kBlock), 0, s, n, qstart, qcell, qrank,
             order);
  if (k <= 4)
    RGA_LAUNCH("knn_query", knn_query_quad_kernel, dim3(rga::ceil_div((int64_t)n * 4, kBlock)),
               dim3(kBlock), 0, s, n, q, k, at<float>(W, L.bounds), at<uint32_t>(W, L.start),
               at<float4>(W, L.recs), order, idx, w);
  else
    RGA_LAUNCH("knn_query_wide", knn_query_wave_kernel, dim3(rga::ceil_div(n, kBlock / 64)),
               dim3(kBlock), 0, s, n, q, k, at<float>(W, L.bounds), at<uint32_t>(W, L.start),
               at<float4>(W, L.recs), order, idx, w);
  RGA_CHECK_LAUNCH("knn_query");
  return RGA_OK;
}

extern "C" int knn_interpolate(void* stream, int n, int k, const int32_t* idx, const float* w,
                               int C, int nr, const float* attr, float* out) {
  if (n < 0 || C < 0 || nr < 1 || k < 1 || k > kMaxK)
    return rga::fail(RGA_EINVAL, "knn_interpolate: bad size");
  if (n == 0 || C == 0) return RGA_OK;
  if (!idx || !w || !attr || !out) return rga::fail(RGA_EINVAL, "knn_interpolate: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(rga::ceil_div(n, kBlock));
  if (k <= 4)
    RGA_LAUNCH("knn_interp", knn_interp_kernel<4>, grid, dim3(kBlock), 0, s, n, k, idx, w, C, nr,
               attr, out);
  else
    RGA_LAUNCH("knn_interp", knn_interp_kernel<kMaxK>, grid, dim3(kBlock), 0, s, n, k, idx, w, C,
               nr, attr, out);
  RGA_CHECK_LAUNCH("knn_interpolate");
  return RGA_OK;
}

extern "C" int knn_interpolate_backward(void* stream, int n, int k, const int32_t* idx,
                                        const float* w, int C, int nr, const float* dout,
                                        float* dattr) {
  if (n < 0 || C < 0 || nr < 1 || k < 1 || k > kMaxK || C > 65535)
    return rga::fail(RGA_EINVAL, "knn_interpolate_backward: bad size");
  if (C == 0) return RGA_OK;
  if (!dattr || (n > 0 && (!idx || !w || !dout)))
    return rga::fail(RGA_EINVAL, "knn_interpolate_backward: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t za = (int64_t)C * nr;
  RGA_LAUNCH("knn_interp_zero", knn_zero_kernel, dim3(rga::ceil_div(za, kBlock)), dim3(kBlock), 0,
             s, dattr, za);
  if (n > 0) {
    const int ranges = (int)rga::ceil_div(nr, kVRange);
    const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(rga::ceil_div(n, kBlock),
                                                                   512 / ((int64_t)C * ranges)));
    const int chunk = (int)rga::ceil_div(n, chunks);
    RGA_LAUNCH("knn_interp_bwd", knn_interp_bwd_kernel, dim3(chunks, C, ranges), dim3(kBlock), 0,
               s, n, k, idx, w, nr, dout, dattr, chunk);
  }
  RGA_CHECK_LAUNCH("knn_interpolate_backward");
  return RGA_OK;
}
