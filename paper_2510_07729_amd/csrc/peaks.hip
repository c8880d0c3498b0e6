// peaks.hip - microbenchmarks of the rates the shading and bake kernels are designed
// around, measured on the device they run on (libsop_peaks.so; not part of the SOP
// library). Each benchmark allocates its own buffers, runs one warm-up launch and then
// times `reps` launches with HIP events on a stream of its own.
//
//   int sop_peak_run(int which, int reps, double* rate, double* ms)
//     which: SOP_PEAK_* below; rate receives the measured rate in the unit named by
//     sop_peak_unit(which), ms the mean time of one launch. Returns 0, or -1 for an unknown
//     benchmark, or the HIP error code.
//   const char* sop_peak_name(int which), const char* sop_peak_unit(int which)
//   int sop_peak_count(void)
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

enum {
  kCopy = 0,           // device copy, float4 grid-stride: (read + write) bytes / s
  kFma32,              // dependent FP32 FMA chains, 8 per lane: flop / s
  kFma64,              // the same in FP64
  kAtomicRowsBig,      // float atomics, each wavefront instruction on 64 consecutive floats
                       // of a 64 MiB buffer (the probe-texel gradient's size class)
  kAtomicRowsSmall,    // the same on a 1.5 MiB buffer (the environment gradient's)
  kAtomicScattered,    // float atomics at independent random addresses of 64 MiB
  kLdsGather16,        // 16-byte LDS reads at random addresses of a 16 KiB array
  kLdsRmw16,           // 16-byte LDS read-modify-writes, distinct random texels per lane
  kLdsAtomic,          // LDS float atomics at random addresses
  kGatherL1Random,     // 16-byte global loads at random addresses of a 16 KiB region per
                       // wavefront (one probe map of 64, 1 MiB in all: cache resident);
                       // the 64 lanes touch ~55 different lines
  kGatherL1Rows,       // the same loads with 8 lanes on each 128-byte line: 8 lines each
  kGatherFarRandom,    // random 16-byte loads as kGatherL1Random over 4096 maps (64 MiB,
                       // beyond the L2s)
  kCount
};

const char* kNames[kCount] = {
    "hbm_copy",           "fp32_fma",           "fp64_fma",
    "atomic_f32_rows_64MiB", "atomic_f32_rows_1.5MiB", "atomic_f32_scattered_64MiB",
    "lds_gather_b128",    "lds_rmw_b128",       "lds_atomic_f32",
    "global_gather_b128_random_1MiB", "global_gather_b128_rows_1MiB",
    "global_gather_b128_random_64MiB"};
const char* kUnits[kCount] = {"GB/s",     "TFLOP/s",  "TFLOP/s",  "G lanes/s", "G lanes/s",
                              "G lanes/s", "G lanes/s", "G lanes/s", "G lanes/s", "G lanes/s",
                              "G lanes/s", "G lanes/s"};

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ a,
                                              float4* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    b[i] = a[i];
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__global__ __launch_bounds__(256) void k_fma(T* out, int iters, T seed) {
  T x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = seed + (T)(threadIdx.x + c);
  const T m = (T)0.999999, s = (T)1e-7;
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = fma_t(x[c], m, s);
  T r = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) r += x[c];
  if (r == (T)-1.2345) out[threadIdx.x] = r;   // never true; keeps the chains alive
}

// each wavefront adds to 64 consecutive floats at a random 256-byte-aligned row per step
__global__ __launch_bounds__(256) void k_atomic_rows(float* buf, uint32_t rows, int iters) {
  const uint32_t wave = (blockIdx.x * 256 + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  for (int i = 0; i < iters; ++i) {
    const uint32_t r = hash32(wave * 7919u + (uint32_t)i) % rows;
    unsafeAtomicAdd(buf + (size_t)r * 64 + lane, 1.0f);
  }
}

__global__ __launch_bounds__(256) void k_atomic_scattered(float* buf, uint32_t n, int iters) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  for (int i = 0; i < iters; ++i) unsafeAtomicAdd(buf + hash32(t * 131u + (uint32_t)i) % n, 1.0f);
}

// LDS: a 16 KiB array of float4 (1024 entries, one 32x32 probe map)
template <int MODE>
__global__ __launch_bounds__(256) void k_lds(float* out, int iters) {
  __shared__ float4 m[1024];
  for (int i = threadIdx.x; i < 1024; i += 256) m[i] = make_float4(1.0f, 2.0f, 3.0f, 4.0f);
  __syncthreads();
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int i = 0; i < iters; ++i) {
    const uint32_t h = hash32(t * 2654435761u + (uint32_t)i);
    if (MODE == 0) {
      const float4 v = m[h & 1023u];
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    } else if (MODE == 1) {
      // distinct texels per lane: lane-dependent bits keep the 64 lanes' entries apart
      const uint32_t e = ((h & 15u) << 6) | (threadIdx.x & 63u);
      float4 v = m[e];
      v.x += 1.0f;
      v.y += 1.0f;
      v.z += 1.0f;
      v.w += 1.0f;
      m[e] = v;
    } else {
      atomicAdd(reinterpret_cast<float*>(m) + (h & 4095u), 1.0f);
    }
  }
  __syncthreads();
  if (MODE == 0) {
    if (acc.x == -1.0f) out[t] = acc.y + acc.z + acc.w;   // never true
  } else if (threadIdx.x == 0) {
    out[blockIdx.x] = m[blockIdx.x & 1023u].x;
  }
}

// global 16-byte gathers inside one 16 KiB region per wavefront (L1/L2 resident)
template <bool ROWS>
__global__ __launch_bounds__(256) void k_gather(const float4* __restrict__ maps,
                                                uint32_t n_maps, float* out, int iters) {
  const uint32_t wave = (blockIdx.x * 256 + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  const float4* map = maps + (size_t)(hash32(wave) % n_maps) * 1024;
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int i = 0; i < iters; ++i) {
    const uint32_t h = hash32(wave * 977u + (uint32_t)i);
    // random: each lane its own texel; rows: lanes in groups of 8 on one 128-byte line
    const uint32_t e = ROWS ? (((h >> 3) & 127u) * 8u + (lane & 7u) + (lane >> 3) * 8u * 16u) & 1023u
                            : hash32(h ^ lane) & 1023u;
    const float4 v = map[e];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  if (acc.x == -1.0f) out[blockIdx.x * 256 + threadIdx.x] = acc.y + acc.z + acc.w;
}

struct Timer {
  hipEvent_t a, b;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

}  // namespace

extern "C" int sop_peak_count(void) { return kCount; }
extern "C" const char* sop_peak_name(int which) {
  return which >= 0 && which < kCount ? kNames[which] : "";
}
extern "C" const char* sop_peak_unit(int which) {
  return which >= 0 && which < kCount ? kUnits[which] : "";
}

extern "C" int sop_peak_run(int which, int reps, double* rate, double* ms) {
  if (which < 0 || which >= kCount || reps < 1 || !rate || !ms) return -1;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  hipStream_t s;
  if ((e = hipStreamCreate(&s)) != hipSuccess) return (int)e;
  void* buf = nullptr;
  void* buf2 = nullptr;
  double work = 0.0;   // units per launch
  const unsigned blocks = (unsigned)cus * 16u;
  const size_t copy_n = (size_t)1 << 26;     // float4 elements: 1 GiB per buffer
  const uint32_t big_floats = 16u << 20, small_floats = 384u * 1024u;
  const int iters = 256;
  auto launch = [&]() {
    switch (which) {
      case kCopy:
        hipLaunchKernelGGL(k_copy, dim3(blocks * 4), dim3(256), 0, s, (const float4*)buf,
                           (float4*)buf2, copy_n);
        break;
      case kFma32:
        hipLaunchKernelGGL(k_fma<float>, dim3(blocks), dim3(256), 0, s, (float*)buf, 4096, 1.0f);
        break;
      case kFma64:
        hipLaunchKernelGGL(k_fma<double>, dim3(blocks), dim3(256), 0, s, (double*)buf, 2048, 1.0);
        break;
      case kAtomicRowsBig:
        hipLaunchKernelGGL(k_atomic_rows, dim3(blocks), dim3(256), 0, s, (float*)buf,
                           big_floats / 64u, iters);
        break;
      case kAtomicRowsSmall:
        hipLaunchKernelGGL(k_atomic_rows, dim3(blocks), dim3(256), 0, s, (float*)buf,
                           small_floats / 64u, iters);
        break;
      case kAtomicScattered:
        hipLaunchKernelGGL(k_atomic_scattered, dim3(blocks), dim3(256), 0, s, (float*)buf,
                           big_floats, iters);
        break;
      case kLdsGather16:
        hipLaunchKernelGGL(k_lds<0>, dim3(blocks), dim3(256), 0, s, (float*)buf, 4 * iters);
        break;
      case kLdsRmw16:
        hipLaunchKernelGGL(k_lds<1>, dim3(blocks), dim3(256), 0, s, (float*)buf, 4 * iters);
        break;
      case kLdsAtomic:
        hipLaunchKernelGGL(k_lds<2>, dim3(blocks), dim3(256), 0, s, (float*)buf, 4 * iters);
        break;
      case kGatherL1Random:
        hipLaunchKernelGGL(k_gather<false>, dim3(blocks), dim3(256), 0, s, (const float4*)buf,
                           64u, (float*)buf2, 4 * iters);
        break;
      case kGatherL1Rows:
        hipLaunchKernelGGL(k_gather<true>, dim3(blocks), dim3(256), 0, s, (const float4*)buf,
                           64u, (float*)buf2, 4 * iters);
        break;
      case kGatherFarRandom:
        hipLaunchKernelGGL(k_gather<false>, dim3(blocks), dim3(256), 0, s, (const float4*)buf,
                           4096u, (float*)buf2, 4 * iters);
        break;
    }
  };
  const double lanes = (double)blocks * 256.0;
  switch (which) {
    case kCopy: work = 2.0 * (double)copy_n * 16.0; break;
    case kFma32: work = lanes * 4096.0 * 8.0 * 2.0; break;
    case kFma64: work = lanes * 2048.0 * 8.0 * 2.0; break;
    case kAtomicRowsBig:
    case kAtomicRowsSmall:
    case kAtomicScattered: work = lanes * iters; break;
    default: work = lanes * 4.0 * iters; break;
  }
  size_t bytes = 64u << 20;
  if (which == kCopy) bytes = copy_n * 16;
  e = hipMalloc(&buf, bytes);
  if (e == hipSuccess) e = hipMalloc(&buf2, which == kCopy ? bytes : (size_t)blocks * 256 * 16);
  if (e == hipSuccess) e = hipMemsetAsync(buf, 0, bytes, s);
  if (e == hipSuccess) {
    launch();   // warm-up
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    Timer t;
    (void)hipEventRecord(t.a, s);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(t.b, s);
    e = hipEventSynchronize(t.b);
    float el = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&el, t.a, t.b);
    if (e == hipSuccess) {
      *ms = (double)el / reps;
      const double per_s = work / (*ms * 1e-3);
      *rate = (which == kFma32 || which == kFma64) ? per_s * 1e-12 : per_s * 1e-9;
    }
  }
  if (buf) (void)hipFree(buf);
  if (buf2) (void)hipFree(buf2);
  (void)hipStreamDestroy(s);
  return e == hipSuccess ? 0 : (int)e;
}
