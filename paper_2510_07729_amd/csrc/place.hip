// place.hip - probe placement and the losses of the reconstruction step (ComGS Sec. 3.1.2):
// farthest point sampling (FPS) over a surface point cloud with every pick raised along its
// normal, L_sops = L1(L_in, L_tr) + L1(O, O_tr) (probe textures towards the traced ones)
// and L_lam = L1(R, 1) + L1(M, 0) (material regulariser), each with its gradient.
//
// FPS runs as one kernel of a few dozen workgroups that exchange each pick through memory:
// each keeps its points and their squared distances d to the nearest pick so far in
// registers (or, beyond 32 points per thread, as (x, y, z, d) in 16 bytes of device
// memory), and
// every pick is the maximum of 64-bit keys (distance bits, inverted index). A workgroup
// publishes its own maximum, tagged with the pick number mod 4, in one of three rotating
// rows of per-workgroup words and reads every other workgroup's word of that row until all
// carry the pick's tag: one exchange per pick, with no counter, fence, clear or atomic
// read-modify-write. Every wait is bounded; a workgroup that reaches the bound raises a
// flag, and the probes of that call are then NaN. The losses are single coalesced passes
// with per-workgroup FP64 partial sums added in a fixed order (the same inputs give the
// same loss bit for bit).
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

// Keys of the pick reduction. A non-negative float orders as its bits and 0xFFFFFFFF - j
// puts the lower index first; with j < 2^31 the inverted index always has its top bit set,
// so the distance bits and the low 31 bits of the inverted index fit above a 2-bit tag (the
// pick number mod 4) in the same order.
__device__ __forceinline__ uint64_t fps_tagged(uint64_t key, uint32_t tag) {
  return ((key >> 32) << 33) | ((key & 0x7FFFFFFFull) << 2) | (uint64_t)tag;
}

__device__ __forceinline__ int64_t fps_tagged_index(uint64_t t) {
  return (int64_t)(0x7FFFFFFFu - (uint32_t)((t >> 2) & 0x7FFFFFFFull));
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int o) {
  const uint32_t lo = __shfl_xor((uint32_t)v, o), hi = __shfl_xor((uint32_t)(v >> 32), o);
  return ((uint64_t)hi << 32) | lo;
}

// the published words are read and written at device scope (they bypass the non-coherent
// per-XCD caches); relaxed order suffices because each word carries its own pick's tag and
// nothing else is exchanged through memory
__device__ __forceinline__ uint64_t fps_ld(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void fps_st(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroups of 256 threads, at most kFpsMaxBlocks of them, and one published word per
// workgroup and row, which one lane of the first wavefront of every workgroup reads. Every
// poll of a row reads the same few cache lines from all workgroups, so the traffic of a
// pick grows with the square of the workgroup count: a few dozen workgroups with several
// points per thread (kFpsPts, up to kFpsMaxRegPts in registers) wait far less than one
// point per thread on every compute unit. A wait gives up after kFpsSpin polls (about a
// second; a normal wait is a few microseconds), which only workgroups that are not all
// resident at once can reach: there are far fewer of them than compute units.
constexpr int kFpsMaxBlocks = 64;
constexpr int kFpsPts = 8;
constexpr int kFpsMaxRegPts = 32;
constexpr uint32_t kFpsSpin = 1u << 20;
static_assert(kFpsSyncWords == (size_t)kFpsSyncRows * kFpsMaxBlocks + 1, "fault flag after the rows");

struct FpsArgs {
  const float* pts;  // [M,3]
  float4* pd;        // [M] (x, y, z, d), used when the points do not fit in registers
  int64_t M;
  int32_t P;
  int64_t start;
  uint64_t* rows;    // [3][gridDim.x] published tagged maxima, zero at launch
  int32_t* fault;    // set when a wait gave up, zero at launch
  int32_t* chosen;   // [P]
};

// Thread t of workgroup b owns the points j = b * 256 + t + u * (256 * gridDim.x). Pick k
// (1 <= k < P): the pick of step k-1 lowers every point's distance; the workgroup maximum
// goes into row k % 3 with tag k & 3; the pick is the maximum of that row once every word
// carries the tag. A word of row k % 3 still holds pick k - 3 (tag (k + 1) & 3) or the zero
// of the launch until its workgroup writes pick k, and no workgroup can write pick k + 3
// before every workgroup has read pick k + 1, so a wait never sees a later pick.
template <int U>   // U > 0: U points per thread in registers; U == 0: points in pd
__global__ __launch_bounds__(256) void k_fps(FpsArgs a) {
  __shared__ uint64_t s_part[4], s_win;
  __shared__ float s_xyz[3];
  __shared__ int32_t s_late;
  const int t = threadIdx.x, w = t >> 6;
  const int G = (int)gridDim.x;
  const int64_t T = (int64_t)G * 256, j0 = (int64_t)blockIdx.x * 256 + t;
  float4 p[U > 0 ? U : 1];
  if constexpr (U > 0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * T;
      p[u] = j < a.M ? make_float4(a.pts[3 * j], a.pts[3 * j + 1], a.pts[3 * j + 2],
                                   __int_as_float(0x7F800000))
                     : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  int64_t q = a.start;
  float cx = a.pts[3 * q], cy = a.pts[3 * q + 1], cz = a.pts[3 * q + 2];
  for (int32_t k = 1; k < a.P; ++k) {
    if (blockIdx.x == 0 && t == 0) a.chosen[k - 1] = (int32_t)q;
    const float4 c = make_float4(cx, cy, cz, 0.f);
    uint64_t best = 0;
    if constexpr (U > 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + u * T;
        if (j < a.M) {
          p[u].w = fminf(p[u].w, fps_d2(p[u], c));
          best = max_u64(best, fps_key(p[u].w, j));
        }
      }
    } else {
      for (int64_t j = j0; j < a.M; j += T) {
        const float4 x = a.pd[j];
        const float d2 = fps_d2(x, c);
        // only a distance that shrinks is written back (after the first picks most do not)
        if (d2 < x.w) reinterpret_cast<float*>(a.pd + j)[3] = d2;
        best = max_u64(best, fps_key(fminf(x.w, d2), j));
      }
    }
    for (int o = 32; o > 0; o >>= 1) best = max_u64(best, shfl_xor_u64(best, o));
    if ((t & 63) == 0) s_part[w] = best;
    __syncthreads();
    if (w == 0) {
      const uint32_t tag = (uint32_t)k & 3u;
      uint64_t* row = a.rows + (size_t)(k % 3) * G;
      if (t == 0)
        fps_st(row + blockIdx.x, fps_tagged(max_u64(max_u64(s_part[0], s_part[1]),
                                                    max_u64(s_part[2], s_part[3])), tag));
      // every workgroup's word, and the coordinates of its candidate as soon as it is known
      uint64_t v = 0;
      float x = 0.f, y = 0.f, z = 0.f;
      bool late = false;
      if (t < G) {
        v = fps_ld(row + t);
        for (uint32_t n = 0; (uint32_t)(v & 3u) != tag;) {
          if (++n > kFpsSpin) {
            late = true;
            v = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          v = fps_ld(row + t);
        }
        if (v != 0) {
          const int64_t i = fps_tagged_index(v);
          x = a.pts[3 * i];
          y = a.pts[3 * i + 1];
          z = a.pts[3 * i + 2];
        }
      }
      const bool any_late = __ballot(late) != 0;
      for (int o = 32; o > 0; o >>= 1) {
        const uint64_t v2 = shfl_xor_u64(v, o);
        const float x2 = __shfl_xor(x, o), y2 = __shfl_xor(y, o), z2 = __shfl_xor(z, o);
        if (v2 > v) {
          v = v2;
          x = x2;
          y = y2;
          z = z2;
        }
      }
      if (t == 0) {
        s_win = v;
        s_xyz[0] = x;
        s_xyz[1] = y;
        s_xyz[2] = z;
        s_late = any_late ? 1 : 0;
      }
    }
    __syncthreads();
    if (s_late) {
      if (t == 0) __hip_atomic_store(a.fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    q = fps_tagged_index(s_win);
    cx = s_xyz[0];
    cy = s_xyz[1];
    cz = s_xyz[2];
  }
  if (blockIdx.x == 0 && t == 0) a.chosen[a.P - 1] = (int32_t)q;
}

// pd[j] = (x_j, y_j, z_j, +inf): the points with their distance to the nearest pick so far
__global__ __launch_bounds__(256) void k_fps_pack(const float* pts, int64_t M, float4* pd) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < M)
    pd[j] = make_float4(pts[3 * j], pts[3 * j + 1], pts[3 * j + 2], __int_as_float(0x7F800000));
}

// every probe = fmaf(offset, n, x) of its pick; all NaN when a wait of the picks gave up
__global__ __launch_bounds__(256) void k_fps_finish(const float* pts, const float* nrm,
                                                    const int32_t* chosen, const int32_t* fault,
                                                    int32_t P, float offset, float* out) {
  const bool bad = *fault != 0;
  for (int32_t k = blockIdx.x * 256 + threadIdx.x; k < P; k += gridDim.x * 256) {
    if (bad) {
#pragma unroll
      for (int a = 0; a < 3; ++a) out[3 * k + a] = __int_as_float(0x7FC00000);
      continue;
    }
    const int64_t c = chosen[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) out[3 * k + a] = fmaf(offset, nrm[3 * c + a], pts[3 * c + a]);
  }
}

template <int U>
void launch_fps(const FpsArgs& a, unsigned G, hipStream_t s) {
  hipLaunchKernelGGL(k_fps<U>, dim3(G), dim3(256), 0, s, a);
}

hipError_t launch_place_probes(const float* pts, const float* nrm, int64_t M, int32_t P,
                               int64_t start, float offset, float* packed, uint64_t* sync,
                               int32_t* chosen, float* out, hipStream_t s) {
  if (P < 1) return hipSuccess;
  if (M < 1 || M > INT32_MAX || start < 0 || start >= M || !pts || !nrm || !packed || !sync ||
      !chosen || !out)
    return hipErrorInvalidValue;
  const unsigned G = (unsigned)std::min<int64_t>((M + 256 * kFpsPts - 1) / (256 * kFpsPts),
                                                 kFpsMaxBlocks);
  const int64_t per = (M + 256 * (int64_t)G - 1) / (256 * (int64_t)G);
  int32_t* fault = reinterpret_cast<int32_t*>(sync + kFpsSyncRows * kFpsMaxBlocks);
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(sync), 0, 2 * kFpsSyncWords, s);
  if (e != hipSuccess) return e;
  const FpsArgs a{pts, reinterpret_cast<float4*>(packed), M, P, start, sync, fault, chosen};
  if (per > kFpsMaxRegPts)
    hipLaunchKernelGGL(k_fps_pack, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, pts, M,
                       a.pd);
  if (per <= 1) launch_fps<1>(a, G, s);
  else if (per <= 2) launch_fps<2>(a, G, s);
  else if (per <= 4) launch_fps<4>(a, G, s);
  else if (per <= 8) launch_fps<8>(a, G, s);
  else if (per <= 16) launch_fps<16>(a, G, s);
  else if (per <= kFpsMaxRegPts) launch_fps<kFpsMaxRegPts>(a, G, s);
  else launch_fps<0>(a, G, s);
  hipLaunchKernelGGL(k_fps_finish, dim3((unsigned)std::min<int64_t>((P + 255) / 256, 1024)),
                     dim3(256), 0, s, pts, nrm, chosen, fault, P, offset, out);
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
