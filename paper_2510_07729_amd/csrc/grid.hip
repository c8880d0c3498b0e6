// grid.hip - probe grid, point ordering and k-nearest-probe search (ComGS Sec. 3.1.2,
// efficient querying through SOPs: FRNN search then KNN weights of Eq. 10-11).
//
// Positions are quantised to a 2^15 lattice in FP32; distances are exact integers. Probes
// are counting-sorted into a cube of 2^bits cells per axis addressed by the Morton index of
// the cell, so that cells close in space are close in memory. Points are counting-sorted by
// the same cell index into a processing order, so that consecutive wavefronts shade points
// that share probes. The search visits cells in growing Chebyshev shells and stops when the
// K-th best squared distance is below the squared distance to the nearest unvisited cell.
#include "sop_device.hpp"
#include "sop_internal.hpp"

namespace sopk {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

size_t scan_tmp_elems(size_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* p, int32_t v, size_t n) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// inclusive block scan of one value per thread; returns the exclusive prefix, *total = sum
__device__ __forceinline__ int32_t block_exclusive(int32_t v, int32_t* buf, int32_t* total) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int32_t x = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += x;
    __syncthreads();
  }
  const int32_t incl = buf[t];
  *total = buf[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t* in, size_t n,
                                                            int32_t* sums) {
  __shared__ int32_t buf[kScanThreads];
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  int32_t total;
  block_exclusive(s, buf, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single workgroup: exclusive scan of sums[0..nb) in place, sums[nb] = total
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int32_t* sums, int32_t nb) {
  __shared__ int32_t buf[kScanThreads];
  int32_t carry = 0;
  for (int32_t base = 0; base < nb; base += kScanThreads) {
    const int32_t i = base + (int32_t)threadIdx.x;
    const int32_t v = i < nb ? sums[i] : 0;
    int32_t total;
    const int32_t ex = block_exclusive(v, buf, &total);
    if (i < nb) sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const int32_t* in, int32_t* out,
                                                            size_t n, const int32_t* sums,
                                                            int32_t nb) {
  __shared__ int32_t buf[kScanThreads];
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  int32_t total;
  int32_t run = block_exclusive(s, buf, &total) + sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, size_t n, int32_t* tmp,
                                 hipStream_t s) {
  const int32_t nb = (int32_t)((n + kScanTile - 1) / kScanTile);
  if (nb == 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, out, 0, (size_t)1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_tile_sums, dim3(nb), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_tile_scan, dim3(nb), dim3(kScanThreads), 0, s, in, out, n, tmp, nb);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// probe grid
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cell_of(int qx, int qy, int qz, int shift) {
  return morton3((uint32_t)(qx >> shift), (uint32_t)(qy >> shift), (uint32_t)(qz >> shift));
}

__global__ __launch_bounds__(256) void k_probe_quant(const float* pos, int32_t P, float lo0,
                                                     float lo1, float lo2, float sc,
                                                     int32_t shift, int4* qtmp,
                                                     int32_t* counts, float* pos_copy) {
  const int32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const float x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
  const int qx = quantize1(x, lo0, sc), qy = quantize1(y, lo1, sc), qz = quantize1(z, lo2, sc);
  const uint32_t m = cell_of(qx, qy, qz, shift);
  qtmp[p] = make_int4(qx, qy, qz, (int)m);
  atomicAdd(&counts[m], 1);
  pos_copy[3 * p] = x;
  pos_copy[3 * p + 1] = y;
  pos_copy[3 * p + 2] = z;
}

__global__ __launch_bounds__(256) void k_probe_scatter(const int4* qtmp, int32_t P,
                                                       const int32_t* cell_start,
                                                       int32_t* cursor, int4* qsorted) {
  const int32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const int4 q = qtmp[p];
  const int32_t slot = cell_start[q.w] + atomicAdd(&cursor[q.w], 1);
  qsorted[slot] = make_int4(q.x, q.y, q.z, p);
}

hipError_t launch_probe_grid_build(const float* pos, int32_t P, const float lo[3], float sc,
                                   int32_t bits, int4* qtmp, int32_t* counts,
                                   int32_t* cell_start, int32_t* cursor, int4* qsorted,
                                   float* pos_copy, int32_t* scan_tmp, hipStream_t s) {
  const size_t C = (size_t)1 << (3 * bits);
  hipError_t e = launch_fill_i32(counts, 0, C, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_i32(cursor, 0, C, s)) != hipSuccess) return e;
  if (P > 0) {
    hipLaunchKernelGGL(k_probe_quant, dim3((P + 255) / 256), dim3(256), 0, s, pos, P, lo[0],
                       lo[1], lo[2], sc, 15 - bits, qtmp, counts, pos_copy);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_exclusive_scan(counts, cell_start, C, scan_tmp, s)) != hipSuccess) return e;
  if (P > 0) {
    hipLaunchKernelGGL(k_probe_scatter, dim3((P + 255) / 256), dim3(256), 0, s, qtmp, P,
                       cell_start, cursor, qsorted);
    e = hipGetLastError();
  }
  return e;
}

// ------------------------------------------------------------------------------------------
// point ordering: counting sort by Morton cell
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_point_cells(ProbeGrid g, const float* pts, int64_t N,
                                                     int32_t* point_cell, int32_t* counts) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int qx = quantize1(pts[3 * i], g.lo[0], g.sc);
  const int qy = quantize1(pts[3 * i + 1], g.lo[1], g.sc);
  const int qz = quantize1(pts[3 * i + 2], g.lo[2], g.sc);
  const uint32_t m = cell_of(qx, qy, qz, g.shift);
  point_cell[i] = (int32_t)m;
  atomicAdd(&counts[m], 1);
}

__global__ __launch_bounds__(256) void k_point_scatter(const int32_t* point_cell, int64_t N,
                                                       int32_t* offsets, int32_t* order) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int32_t slot = atomicAdd(&offsets[point_cell[i]], 1);
  order[slot] = (int32_t)i;
}

// Orders the points of each grid cell by the Morton code of their lattice position inside
// the cell (10 bits per axis), ties by point index: consecutive points of the order then
// lie close together at the scale of a few points, not only of a cell, so a batch of them
// shares more neighbouring probes (the adjoint adds each batch's texture gradient once per
// distinct probe). One workgroup per cell, bitonic sort in LDS; a cell of more than
// kRefineMax points keeps the counting sort's order. Also makes the order deterministic.
constexpr int kRefineMax = 4096;
__global__ __launch_bounds__(256) void k_point_refine(ProbeGrid g, const float* pts,
                                                      const int32_t* ends, int32_t* order) {
  __shared__ uint64_t key[kRefineMax];
  const int32_t c = blockIdx.x;
  const int32_t s0 = c == 0 ? 0 : ends[c - 1], s1 = ends[c];
  const int n = s1 - s0;
  if (n <= 1 || n > kRefineMax) return;
  int m = 1;
  while (m < n) m <<= 1;
  const int fine = g.shift < 10 ? g.shift : 10;           // bits per axis inside the cell
  const uint32_t mask = (1u << g.shift) - 1u;
  for (int i = threadIdx.x; i < m; i += 256) {
    uint64_t kv = ~0ull;
    if (i < n) {
      const int32_t p = order[s0 + i];
      const uint32_t qx = (uint32_t)quantize1(pts[3 * (int64_t)p], g.lo[0], g.sc) & mask;
      const uint32_t qy = (uint32_t)quantize1(pts[3 * (int64_t)p + 1], g.lo[1], g.sc) & mask;
      const uint32_t qz = (uint32_t)quantize1(pts[3 * (int64_t)p + 2], g.lo[2], g.sc) & mask;
      const int sh = g.shift - fine;
      kv = ((uint64_t)morton3(qx >> sh, qy >> sh, qz >> sh) << 32) | (uint32_t)p;
    }
    key[i] = kv;
  }
  __syncthreads();
  for (int size = 2; size <= m; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < m / 2; t += 256) {
        const int i = 2 * stride * (t / stride) + (t % stride), j = i + stride;
        const uint64_t x = key[i], y = key[j];
        if ((x > y) == ((i & size) == 0)) {
          key[i] = y;
          key[j] = x;
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < n; i += 256) order[s0 + i] = (int32_t)(key[i] & 0xFFFFFFFFu);
}

hipError_t launch_point_order(const ProbeGrid& g, const float* pts, int64_t N,
                              int32_t* point_cell, int32_t* counts, int32_t* offsets,
                              int32_t* scan_tmp, int32_t* order, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const size_t C = (size_t)1 << (3 * g.bits);
  hipError_t e = launch_fill_i32(counts, 0, C, s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(k_point_cells, dim3(blocks), dim3(256), 0, s, g, pts, N, point_cell,
                     counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_exclusive_scan(counts, offsets, C, scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_point_scatter, dim3(blocks), dim3(256), 0, s, point_cell, N, offsets,
                     order);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // after the scatter offsets[c] holds the end of cell c
  hipLaunchKernelGGL(k_point_refine, dim3((unsigned)C), dim3(256), 0, s, g, pts, offsets, order);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// k nearest probes
// ------------------------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void insert_key(uint64_t (&best)[K], uint64_t key) {
  if (key < best[K - 1]) {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const uint64_t lo = key < best[s] ? key : best[s];
      key = key < best[s] ? best[s] : key;
      best[s] = lo;
    }
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_knn(ProbeGrid g, const float* pts,
                                             const float* normals, int64_t N,
                                             const int32_t* order, uint32_t lim, int32_t* out_idx,
                                             float* out_w) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= N) return;
  int64_t i = t;
  if (order) {
    const int32_t o = order[t];
    if ((uint64_t)o >= (uint64_t)N) return;
    i = o;
  }
  const v3 x = mk3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
  const int q[3] = {quantize1(x.x, g.lo[0], g.sc), quantize1(x.y, g.lo[1], g.sc),
                    quantize1(x.z, g.lo[2], g.sc)};
  const int G = 1 << g.bits;
  const int c[3] = {q[0] >> g.shift, q[1] >> g.shift, q[2] >> g.shift};
  uint64_t best[K];
#pragma unroll
  for (int s = 0; s < K; ++s) best[s] = ~0ull;

  auto visit = [&](int cx, int cy, int cz) {
    const uint32_t m = morton3((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
    const int32_t e0 = g.cell_start[m], e1 = g.cell_start[m + 1];
    for (int32_t e = e0; e < e1; ++e) {
      const int4 pq = g.qsorted[e];
      const int dx = pq.x - q[0], dy = pq.y - q[1], dz = pq.z - q[2];
      const uint32_t d2 = (uint32_t)(dx * dx) + (uint32_t)(dy * dy) + (uint32_t)(dz * dz);
      if (d2 <= lim) insert_key<K>(best, ((uint64_t)d2 << 32) | (uint32_t)pq.w);
    }
  };

  for (int r = 0;; ++r) {
    // cells at Chebyshev distance exactly r from the point's cell
    const int z0 = max(c[2] - r, 0), z1 = min(c[2] + r, G - 1);
    const int y0 = max(c[1] - r, 0), y1 = min(c[1] + r, G - 1);
    const int x0 = max(c[0] - r, 0), x1 = min(c[0] + r, G - 1);
    for (int cz = z0; cz <= z1; ++cz) {
      for (int cy = y0; cy <= y1; ++cy) {
        if (abs(cz - c[2]) == r || abs(cy - c[1]) == r) {
          for (int cx = x0; cx <= x1; ++cx) visit(cx, cy, cz);
        } else {
          if (c[0] - r >= 0) visit(c[0] - r, cy, cz);
          if (c[0] + r <= G - 1) visit(c[0] + r, cy, cz);
        }
      }
    }
    // squared lattice distance to the nearest cell outside the visited cube
    uint64_t lb = ~0ull;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (c[a] - r > 0) {
        const uint64_t d = (uint64_t)(q[a] - ((c[a] - r) << g.shift) + 1);
        lb = d < lb ? d : lb;
      }
      if (c[a] + r + 1 <= G - 1) {
        const uint64_t d = (uint64_t)((((c[a] + r + 1) << g.shift)) - q[a]);
        lb = d < lb ? d : lb;
      }
    }
    if (lb == ~0ull) break;                   // every cell visited
    const uint64_t lb2 = lb * lb;
    if (lb2 > (uint64_t)lim) break;           // nothing further is inside the radius
    if (best[K - 1] != ~0ull && (best[K - 1] >> 32) < lb2) break;
  }

  int32_t* oi = out_idx + i * K;
  float* ow = out_w + i * K;
  if (best[0] != ~0ull && (best[0] >> 32) == 0) {    // exact hit: that probe alone
    oi[0] = (int32_t)(best[0] & 0xFFFFFFFFu);
    ow[0] = 1.0f;
#pragma unroll
    for (int s = 1; s < K; ++s) {
      oi[s] = -1;
      ow[s] = 0.0f;
    }
    return;
  }
  const v3 n = mk3(normals[3 * i], normals[3 * i + 1], normals[3 * i + 2]);
  float wv[K];
  float sum = 0.0f;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    wv[s] = 0.0f;
    if (best[s] != ~0ull) {
      const int p = (int)(best[s] & 0xFFFFFFFFu);
      const v3 d = sub(mk3(g.pos[3 * p], g.pos[3 * p + 1], g.pos[3 * p + 2]), x);
      const float len = sqrtf(dot(d, d));
      const float inv = 1.0f / len;
      const float wb = 0.5f * (1.0f + dot(d, n) * inv) + 0.01f;
      wv[s] = inv * wb;
      sum += wv[s];
    }
  }
  const float isum = 1.0f / sum;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const bool valid = best[s] != ~0ull;
    oi[s] = valid ? (int32_t)(best[s] & 0xFFFFFFFFu) : -1;
    ow[s] = valid ? wv[s] * isum : 0.0f;
  }
}

template <int K>
static hipError_t knn_k(const ProbeGrid& g, const float* pts, const float* normals, int64_t N,
                        const int32_t* order, uint32_t lim, int32_t* idx, float* w,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_knn<K>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, g, pts,
                     normals, N, order, lim, idx, w);
  return hipGetLastError();
}

hipError_t launch_knn(const ProbeGrid& g, const float* pts, const float* normals, int64_t N,
                      const int32_t* order, int32_t k, uint32_t lim, int32_t* idx, float* w,
                      hipStream_t s) {
  if (N == 0) return hipSuccess;
  switch (k) {
#define SOP_KNN_CASE(KK) \
  case KK:               \
    return knn_k<KK>(g, pts, normals, N, order, lim, idx, w, s);
    SOP_KNN_CASE(1) SOP_KNN_CASE(2) SOP_KNN_CASE(3) SOP_KNN_CASE(4) SOP_KNN_CASE(5)
    SOP_KNN_CASE(6) SOP_KNN_CASE(7) SOP_KNN_CASE(8) SOP_KNN_CASE(9) SOP_KNN_CASE(10)
    SOP_KNN_CASE(11) SOP_KNN_CASE(12) SOP_KNN_CASE(13) SOP_KNN_CASE(14) SOP_KNN_CASE(15)
    SOP_KNN_CASE(16)
#undef SOP_KNN_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace sopk
