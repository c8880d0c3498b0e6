// place.hip - probe placement and the losses of the reconstruction step (ComGS Sec. 3.1.2):
// farthest point sampling (FPS) over a surface point cloud with every pick raised along its
// normal, L_sops = L1(L_in, L_tr) + L1(O, O_tr) (probe textures towards the traced ones)
// and L_lam = L1(R, 1) + L1(M, 0) (material regulariser), each with its gradient.
//
// FPS runs as one short kernel per pick: every point, stored as (x, y, z, d) in 16 bytes,
// keeps its squared distance d to the nearest pick so far, and the next pick is the maximum
// of 64-bit keys (distance bits, inverted index) taken with a 64-bit atomic max into one of
// three rotating slots, so no kernel ever waits on another workgroup. The losses are single coalesced passes with
// per-workgroup FP64 partial sums added in a fixed order (the same inputs give the same
// loss bit for bit).
#include "sop_internal.hpp"

namespace sopk {

// squared distance in IEEE single precision, in the fixed order ((dx dx + dy dy) + dz dz)
// and without fused multiply-adds (contraction is switched off here: the compiler would
// otherwise fuse the products into the sums), so that every comparison is reproducible
__device__ __forceinline__ float fps_d2(float4 a, float4 q) {
#pragma clang fp contract(off)
  const float dx = a.x - q.x, dy = a.y - q.y, dz = a.z - q.z;
  return (dx * dx + dy * dy) + dz * dz;
}

// larger distance first, then the lower index (a non-negative float orders as its bits)
__device__ __forceinline__ uint64_t fps_key(float d, int64_t j) {
  return ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)j);
}

__device__ __forceinline__ int64_t fps_index(uint64_t key) {
  return (int64_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFu));
}

__device__ __forceinline__ uint64_t max_u64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Points per thread and sweep of a step: a workgroup takes 256 * kFpsPpt consecutive
// points per sweep; the grid is capped at kFpsMaxBlocks workgroups (larger clouds take
// several sweeps), because the atomics of a pick, one per workgroup on a single slot, are
// serialised and dominate beyond a few hundred.
constexpr int kFpsPpt = 4;
constexpr int64_t kFpsChunk = 256 * kFpsPpt;
constexpr int64_t kFpsMaxBlocks = 256;

// pd[j] = (x_j, y_j, z_j, +inf): the points with their distance to the nearest pick so far
__global__ __launch_bounds__(256) void k_fps_pack(const float* pts, int64_t M, float4* pd) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < M)
    pd[j] = make_float4(pts[3 * j], pts[3 * j + 1], pts[3 * j + 2], __int_as_float(0x7F800000));
}

// Pick k (1 <= k < P): the pick of step k-1 (the start for k = 1, else the winner in slot
// (k-1)%3) lowers every point's distance; the workgroup maxima of the keys go into slot k%3;
// slot (k+1)%3, which no kernel of steps k-1 or k touches, is cleared for step k+1. Each
// thread loads its first points before the winner of the previous step, so the two loads
// overlap.
__device__ __forceinline__ void fps_load(const float4* pd, int64_t M, int64_t j0,
                                         float4 (&p)[kFpsPpt]) {
#pragma unroll
  for (int u = 0; u < kFpsPpt; ++u) {
    const int64_t j = j0 + u * 256;
    p[u] = j < M ? pd[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

__global__ __launch_bounds__(256) void k_fps_step(float4* pd, int64_t M, uint64_t* slots,
                                                  int32_t* chosen, int32_t k, int64_t start) {
  __shared__ uint64_t wave_best[4];
  int64_t base = (int64_t)blockIdx.x * kFpsChunk;       // the same for the whole workgroup
  float4 p[kFpsPpt];
  fps_load(pd, M, base + threadIdx.x, p);
  const int64_t q = k == 1 ? start : fps_index(slots[(k - 1) % 3]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    chosen[k - 1] = (int32_t)q;
    slots[(k + 1) % 3] = 0;
  }
  const float4 c = pd[q];                     // only x, y, z are used (w may be changing)
  uint64_t best = 0;
  for (;;) {
#pragma unroll
    for (int u = 0; u < kFpsPpt; ++u) {
      const int64_t j = base + threadIdx.x + u * 256;
      if (j < M) {
        const float d2 = fps_d2(p[u], c);
        const float d = fminf(p[u].w, d2);
        // only a distance that shrinks is written back (after the first picks most do not)
        if (d2 < p[u].w) reinterpret_cast<float*>(pd + j)[3] = d;
        best = max_u64(best, fps_key(d, j));
      }
    }
    base += (int64_t)gridDim.x * kFpsChunk;
    if (base >= M) break;
    fps_load(pd, M, base + threadIdx.x, p);
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)best, o), hi = __shfl_xor((uint32_t)(best >> 32), o);
    best = max_u64(best, ((uint64_t)hi << 32) | lo);
  }
  if ((threadIdx.x & 63) == 0) wave_best[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t b = max_u64(max_u64(wave_best[0], wave_best[1]),
                               max_u64(wave_best[2], wave_best[3]));
    atomicMax(reinterpret_cast<unsigned long long*>(&slots[k % 3]), (unsigned long long)b);
  }
}

// the last pick, then every probe = fmaf(offset, n, x) of its pick
__global__ __launch_bounds__(256) void k_fps_finish(const float* pts, const float* nrm,
                                                    const uint64_t* slots, int32_t* chosen,
                                                    int32_t P, int64_t start, float offset,
                                                    float* out) {
  const int32_t last = P == 1 ? (int32_t)start : (int32_t)fps_index(slots[(P - 1) % 3]);
  for (int32_t k = blockIdx.x * 256 + threadIdx.x; k < P; k += gridDim.x * 256) {
    const int64_t c = k == P - 1 ? last : chosen[k];
    if (k == P - 1) chosen[k] = last;
#pragma unroll
    for (int a = 0; a < 3; ++a) out[3 * k + a] = fmaf(offset, nrm[3 * c + a], pts[3 * c + a]);
  }
}

hipError_t launch_place_probes(const float* pts, const float* nrm, int64_t M, int32_t P,
                               int64_t start, float offset, float* packed, uint64_t* slots,
                               int32_t* chosen, float* out, hipStream_t s) {
  if (P < 1) return hipSuccess;
  if (M < 1 || M > INT32_MAX || start < 0 || start >= M || !pts || !nrm || !packed || !slots ||
      !chosen || !out)
    return hipErrorInvalidValue;
  float4* pd4 = reinterpret_cast<float4*>(packed);
  hipLaunchKernelGGL(k_fps_pack, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, pts, M,
                     pd4);
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(slots), 0, 6, s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)std::min((M + kFpsChunk - 1) / kFpsChunk, kFpsMaxBlocks);
  for (int32_t k = 1; k < P; ++k)
    hipLaunchKernelGGL(k_fps_step, dim3(blocks), dim3(256), 0, s, pd4, M, slots, chosen, k,
                       start);
  hipLaunchKernelGGL(k_fps_finish, dim3((unsigned)std::min<int64_t>((P + 255) / 256, 1024)),
                     dim3(256), 0, s, pts, nrm, slots, chosen, P, start, offset, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// losses
// ------------------------------------------------------------------------------------------
constexpr int kLossBlocks = 1024;

// sign of x - y from a comparison (exact, whatever the rounding of the difference)
__device__ __forceinline__ float sgn_diff(float x, float y) {
  return x > y ? 1.0f : (x < y ? -1.0f : 0.0f);
}

// per-workgroup FP64 sums of two quantities into part[2 * blockIdx.x + {0, 1}]
__device__ __forceinline__ void block_sum2(double a, double b, double* part) {
  __shared__ double sa[4], sb[4];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    sa[threadIdx.x >> 6] = a;
    sb[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = (sa[0] + sa[1]) + (sa[2] + sa[3]);
    part[2 * blockIdx.x + 1] = (sb[0] + sb[1]) + (sb[2] + sb[3]);
  }
}

// L_sops over T texels (float4: R, G, B, O); grad (may be NULL) is overwritten
__global__ __launch_bounds__(256) void k_sops_loss(const float4* tex, const float4* tgt,
                                                   int64_t T, float g_rgb, float g_o,
                                                   float4* grad, double* part) {
  double a = 0.0, b = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < T;
       t += (int64_t)gridDim.x * 256) {
    const float4 x = tex[t], y = tgt[t];
    const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z, dw = x.w - y.w;
    a += (double)fabsf(dx) + (double)fabsf(dy) + (double)fabsf(dz);
    b += (double)fabsf(dw);
    if (grad)
      grad[t] = make_float4(g_rgb * sgn_diff(x.x, y.x), g_rgb * sgn_diff(x.y, y.y),
                            g_rgb * sgn_diff(x.z, y.z), g_o * sgn_diff(x.w, y.w));
  }
  block_sum2(a, b, part);
}

// L_lam over N points; g_rough / g_metal (may be NULL) are overwritten
__global__ __launch_bounds__(256) void k_lam_loss(const float* rough, const float* metal,
                                                  int64_t N, float g, float* g_rough,
                                                  float* g_metal, double* part) {
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    const float dr = rough[i] - 1.0f, dm = metal[i];
    a += (double)fabsf(dr);
    b += (double)fabsf(dm);
    if (g_rough) g_rough[i] = g * sgn_diff(rough[i], 1.0f);
    if (g_metal) g_metal[i] = g * sgn_diff(metal[i], 0.0f);
  }
  block_sum2(a, b, part);
}

// the partial sums added in a fixed order (thread t takes partials t, t+256, ... in turn,
// then a fixed tree over the threads), each divided by its element count
__global__ __launch_bounds__(256) void k_loss_finish(const double* part, int32_t nblocks,
                                                     double na, double nb, float* loss) {
  __shared__ double sa[256], sb[256];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = tid; i < nblocks; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  sa[tid] = a;
  sb[tid] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      sa[tid] += sa[tid + o];
      sb[tid] += sb[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    loss[0] = na > 0.0 ? (float)(sa[0] / na) : 0.0f;
    loss[1] = nb > 0.0 ? (float)(sb[0] / nb) : 0.0f;
  }
}

static unsigned loss_blocks(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, kLossBlocks));
}

size_t loss_partials(int64_t n) { return 2 * (size_t)loss_blocks(n); }

hipError_t launch_sops_loss(const float* tex, const float* tgt, int64_t T, float* loss,
                            float* grad, double* part, hipStream_t s) {
  if (!loss || !part || (T > 0 && (!tex || !tgt))) return hipErrorInvalidValue;
  const unsigned nb = loss_blocks(T);
  const float g_rgb = T > 0 ? (float)(1.0 / (3.0 * (double)T)) : 0.0f;
  const float g_o = T > 0 ? (float)(1.0 / (double)T) : 0.0f;
  hipLaunchKernelGGL(k_sops_loss, dim3(nb), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(tex), reinterpret_cast<const float4*>(tgt),
                     T, g_rgb, g_o, reinterpret_cast<float4*>(grad), part);
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, part, (int32_t)nb,
                     3.0 * (double)T, (double)T, loss);
  return hipGetLastError();
}

hipError_t launch_lam_loss(const float* rough, const float* metal, int64_t N, float* loss,
                           float* g_rough, float* g_metal, double* part, hipStream_t s) {
  if (!loss || !part || (N > 0 && (!rough || !metal))) return hipErrorInvalidValue;
  const unsigned nb = loss_blocks(N);
  const float g = N > 0 ? (float)(1.0 / (double)N) : 0.0f;
  hipLaunchKernelGGL(k_lam_loss, dim3(nb), dim3(256), 0, s, rough, metal, N, g, g_rough,
                     g_metal, part);
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, part, (int32_t)nb, (double)N,
                     (double)N, loss);
  return hipGetLastError();
}

}  // namespace sopk
