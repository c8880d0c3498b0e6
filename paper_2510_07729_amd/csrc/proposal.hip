// proposal.hip - the learned direction proposal's network on the matrix cores: inference
// (features -> 320 -> 64 -> 64 -> 256 -> softmax), one training step (forward, cross
// entropy, backward, weight gradients) and Adam. An extension of the Monte Carlo estimate of
// Eq. 7 (ComGS Sec. 3.1.2): the network's bin distribution is what the proposal sampler of
// shade.hip draws from.
//
// Matrix products run on v_mfma_f32_16x16x16_bf16 in a transposed formulation, z^T = W^T x^T:
// the output neurons are the M dimension and 16 points are the N dimension, so the
// accumulator of one layer (lane l holds rows 4(l/16)..+3 of column l%16) is, after bias,
// ReLU and rounding, exactly the B operand of the next layer (lane l holds k = 4(l/16)..+3
// of column l%16); no shuffles or LDS round trips between layers. Weights are pre-arranged
// once per call into operand fragments (64 lanes x 4 bf16 = 512 B, one coalesced load).
// Weight gradients contract over points, so they use activations stored transposed
// ([feature][point]) and are a plain GEMM in which each wavefront owns one 16x16 tile of a
// weight matrix (deterministic, no atomics).
#include "sop_device.hpp"
#include "sop_internal.hpp"

namespace sopk {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = SOP_MLP_IN, kHid = SOP_MLP_HIDDEN, kBins = SOP_MLP_BINS;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kIn * kHid, kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kBins;
static_assert(kOffB3 + kBins == SOP_MLP_PARAMS, "parameter layout");

// fragment sets (in fragments of 256 bf16): forward A operands W^T per (m-block, k-block),
// backward A operands W per (m-block = input block, k-block = output block)
constexpr int kF1 = 0;                    // W1^T: 4 x 20
constexpr int kF2 = kF1 + 4 * 20;         // W2^T: 4 x 4
constexpr int kF3 = kF2 + 4 * 4;          // W3^T: 16 x 4
constexpr int kB3 = kF3 + 16 * 4;         // W3:   4 x 16
constexpr int kB2 = kB3 + 4 * 16;         // W2:   4 x 4
constexpr int kFrags = kB2 + 4 * 4;       // 240 fragments

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return 0x7FC0;   // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);                                          // nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 r;
  r[0] = (short)f2bf(a);
  r[1] = (short)f2bf(b);
  r[2] = (short)f2bf(c);
  r[3] = (short)f2bf(d);
  return r;
}

__device__ __forceinline__ bf16x4 load_frag(const uint16_t* frags, int f, int lane) {
  return *reinterpret_cast<const bf16x4*>(frags + ((size_t)f * 64 + lane) * 4);
}

// ------------------------------------------------------------------------------------------
// fragment preparation: one thread per bf16 element
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_frags(const float* __restrict__ P,
                                                   uint16_t* __restrict__ frags) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kFrags * 256) return;
  const int f = e >> 8, lane = (e >> 2) & 63, t = e & 3;
  const int g = lane >> 4, r = lane & 15;
  int src;
  if (f < kF2) {                 // W1^T[out][in]: A[m = out 16mb + r][k = in 16kb + 4g + t]
    const int mb = (f - kF1) / 20, kb = (f - kF1) % 20;
    src = kOffW1 + (16 * kb + 4 * g + t) * kHid + 16 * mb + r;
  } else if (f < kF3) {
    const int mb = (f - kF2) / 4, kb = (f - kF2) % 4;
    src = kOffW2 + (16 * kb + 4 * g + t) * kHid + 16 * mb + r;
  } else if (f < kB3) {
    const int mb = (f - kF3) / 4, kb = (f - kF3) % 4;
    src = kOffW3 + (16 * kb + 4 * g + t) * kBins + 16 * mb + r;
  } else if (f < kB2) {          // W3[in][out]: A[m = in 16mb + r][k = out 16kb + 4g + t]
    const int mb = (f - kB3) / 16, kb = (f - kB3) % 16;
    src = kOffW3 + (16 * mb + r) * kBins + 16 * kb + 4 * g + t;
  } else {
    const int mb = (f - kB2) / 4, kb = (f - kB2) % 4;
    src = kOffW2 + (16 * mb + r) * kHid + 16 * kb + 4 * g + t;
  }
  frags[e] = f2bf(P[src]);
}

// ------------------------------------------------------------------------------------------
// features of the lane's point: the 10 scalars and the B fragment of k-block kb
// ------------------------------------------------------------------------------------------
struct FeatIn {
  float x[10];
};

__device__ __forceinline__ void point_scalars(const MlpArgs& a, int64_t p, FeatIn& fi) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    fi.x[c] = (a.pos[3 * p + c] - a.lo[c]) * a.inv2[c] - 1.0f;
    fi.x[3 + c] = a.nrm[3 * p + c];
  }
  if (a.view) {
#pragma unroll
    for (int c = 0; c < 3; ++c) fi.x[6 + c] = a.view[3 * p + c];
  } else {
    const int64_t f = p / a.ppf;
    float d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] = a.cam[3 * f + c] - a.pos[3 * p + c];
    const float il = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) fi.x[6 + c] = d[c] * il;
  }
  fi.x[9] = a.rough[p];
}

// f_l = 2^(l/2) rounded to float
__device__ __forceinline__ float freq(int l) {
  const float base = (l & 1) ? 1.41421356237309505f : 1.0f;
  return ldexpf(base, l >> 1);
}

// B fragment of features k = 16 kb + 4 g + t for the lane's point: scalar c = kb / 2,
// frequencies l0 = 8 (kb % 2) + 2 g and l0 + 1, (sin, cos, sin, cos)
__device__ __forceinline__ bf16x4 feature_frag(const FeatIn& fi, int kb, int g) {
  const float xv = fi.x[kb >> 1];
  const int l0 = 8 * (kb & 1) + 2 * g;
  float s0, c0, s1, c1;
  sincospif(freq(l0) * xv, &s0, &c0);
  sincospif(freq(l0 + 1) * xv, &s1, &c1);
  return pack4(s0, c0, s1, c1);
}

// ------------------------------------------------------------------------------------------
// forward of one 16-point tile (one wavefront); h1/h2 fragments and pre-activations kept
// ------------------------------------------------------------------------------------------
struct Fwd {
  f32x4 z1[4], z2[4];      // pre-activations (rows 16mb + 4g + t, column = point)
  bf16x4 h1[4], h2[4];     // B fragments of the next layer
  f32x4 z3[16];            // logits
};

__device__ __forceinline__ void forward_tile(const MlpArgs& a, const FeatIn& fi, int lane,
                                             Fwd& F, uint16_t* xT, int64_t col, bool store) {
  const int g = lane >> 4;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) F.z1[mb][t] = a.params[kOffB1 + 16 * mb + 4 * g + t];
#pragma unroll
  for (int kb = 0; kb < 20; ++kb) {        // fully unrolled: fi.x[kb >> 1] stays in registers
    const bf16x4 b = feature_frag(fi, kb, g);
    if (store) {
#pragma unroll
      for (int t = 0; t < 4; ++t) xT[(size_t)(16 * kb + 4 * g + t) * a.ldT + col] = (uint16_t)b[t];
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) F.z1[mb] = mfma16(load_frag(a.frags, kF1 + mb * 20 + kb, lane), b, F.z1[mb]);
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
    F.h1[mb] = pack4(fmaxf(F.z1[mb][0], 0.0f), fmaxf(F.z1[mb][1], 0.0f), fmaxf(F.z1[mb][2], 0.0f),
                     fmaxf(F.z1[mb][3], 0.0f));
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) F.z2[mb][t] = a.params[kOffB2 + 16 * mb + 4 * g + t];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
      F.z2[mb] = mfma16(load_frag(a.frags, kF2 + mb * 4 + kb, lane), F.h1[kb], F.z2[mb]);
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
    F.h2[mb] = pack4(fmaxf(F.z2[mb][0], 0.0f), fmaxf(F.z2[mb][1], 0.0f), fmaxf(F.z2[mb][2], 0.0f),
                     fmaxf(F.z2[mb][3], 0.0f));
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) F.z3[mb][t] = a.params[kOffB3 + 16 * mb + 4 * g + t];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int mb = 0; mb < 16; ++mb)
      F.z3[mb] = mfma16(load_frag(a.frags, kF3 + mb * 4 + kb, lane), F.h2[kb], F.z3[mb]);
}

// max and sum over the 4 lanes that hold one point's logits (lanes r, r+16, r+32, r+48)
__device__ __forceinline__ float point_max(float v) {
  v = fmaxf(v, __shfl_xor(v, 16));
  return fmaxf(v, __shfl_xor(v, 32));
}
__device__ __forceinline__ float point_sum(float v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}

// ------------------------------------------------------------------------------------------
// inference: one wavefront per 16 points
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_infer(MlpArgs a) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t p0 = tile * 16;
  if (p0 >= a.n) return;
  const int64_t p = p0 + r;
  const bool valid = p < a.n;
  FeatIn fi;
  if (valid) point_scalars(a, p, fi);
  else
#pragma unroll
    for (int c = 0; c < 10; ++c) fi.x[c] = 0.0f;
  Fwd F;
  forward_tile(a, fi, lane, F, nullptr, 0, false);
  float mx = -INFINITY;
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) mx = fmaxf(mx, F.z3[mb][t]);
  mx = point_max(mx);
  float se = 0.0f;
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) se += expf(F.z3[mb][t] - mx);
  se = point_sum(se);
  const float inv = 1.0f / se;
  if (!valid) return;
#pragma unroll
  for (int mb = 0; mb < 16; ++mb) {
    const size_t o = (size_t)p * kBins + 16 * mb + 4 * g;
    float4 q = make_float4(expf(F.z3[mb][0] - mx) * inv, expf(F.z3[mb][1] - mx) * inv,
                           expf(F.z3[mb][2] - mx) * inv, expf(F.z3[mb][3] - mx) * inv);
    *reinterpret_cast<float4*>(a.probs + o) = q;
    if (a.logits)
      *reinterpret_cast<float4*>(a.logits + o) =
          make_float4(F.z3[mb][0], F.z3[mb][1], F.z3[mb][2], F.z3[mb][3]);
  }
}

// ------------------------------------------------------------------------------------------
// training: forward + cross entropy + backward of one 16-point tile per wavefront.
// Writes the transposed bf16 operands of the weight-gradient GEMM (zero for padding points),
// accumulates bias gradients and the loss with atomics.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float tile_col_sum(float v) {     // sum over the 16 points
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  return v + __shfl_xor(v, 8);
}

__global__ __launch_bounds__(256) void k_mlp_train(MlpArgs a) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t p0 = tile * 16;
  if (p0 >= a.ldT) return;                        // ldT = batch rounded up to 16
  const int64_t p = p0 + r;
  const bool valid = p < a.n;
  const int64_t col = p;
  FeatIn fi;
  if (valid) point_scalars(a, p, fi);
  else
#pragma unroll
    for (int c = 0; c < 10; ++c) fi.x[c] = 0.0f;
  Fwd F;
  forward_tile(a, fi, lane, F, a.xT, col, true);
  const float vmask = valid ? 1.0f : 0.0f;
  // activations stored transposed (zero for padding points)
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a.h1T[(size_t)(16 * mb + 4 * g + t) * a.ldT + col] = valid ? (uint16_t)F.h1[mb][t] : 0;
      a.h2T[(size_t)(16 * mb + 4 * g + t) * a.ldT + col] = valid ? (uint16_t)F.h2[mb][t] : 0;
    }
  // softmax, normalised targets, loss, dz3 = (q - t) / B
  float mx = -INFINITY;
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) mx = fmaxf(mx, F.z3[mb][t]);
  mx = point_max(mx);
  float se = 0.0f, ts = 0.0f;
  float4 T[16];
#pragma unroll
  for (int mb = 0; mb < 16; ++mb) {
    T[mb] = valid ? *reinterpret_cast<const float4*>(a.targets + (size_t)p * kBins + 16 * mb + 4 * g)
                  : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    ts += T[mb].x + T[mb].y + T[mb].z + T[mb].w;
#pragma unroll
    for (int t = 0; t < 4; ++t) se += expf(F.z3[mb][t] - mx);
  }
  se = point_sum(se);
  ts = point_sum(ts);
  const float lse = mx + logf(se);
  const bool uni = !(ts > 0.0f);
  const float its = uni ? 0.0f : 1.0f / ts;
  const float invB = 1.0f / (float)a.n;
  float loss = 0.0f;
  bf16x4 d3[16];
#pragma unroll
  for (int mb = 0; mb < 16; ++mb) {
    const float tv[4] = {T[mb].x, T[mb].y, T[mb].z, T[mb].w};
    float dz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float tt = uni ? (1.0f / kBins) : tv[t] * its;
      loss -= tt * (F.z3[mb][t] - lse);
      dz[t] = (expf(F.z3[mb][t] - lse) - tt) * invB * vmask;
      const float cs = tile_col_sum(dz[t]);
      if (r == 0) unsafeAtomicAdd(a.grad + kOffB3 + 16 * mb + 4 * g + t, cs);
    }
    d3[mb] = pack4(dz[0], dz[1], dz[2], dz[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      a.dz3T[(size_t)(16 * mb + 4 * g + t) * a.ldT + col] = (uint16_t)d3[mb][t];
  }
  loss = wave_sum(loss * vmask);
  if (lane == 0) unsafeAtomicAdd(a.loss, loss * invB);
  // dh2^T = W3 dz3^T, dz2 = dh2 [z2 > 0]
  f32x4 acc[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kb = 0; kb < 16; ++kb)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = mfma16(load_frag(a.frags, kB3 + mb * 16 + kb, lane), d3[kb], acc[mb]);
  bf16x4 d2[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    float dz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      dz[t] = F.z2[mb][t] > 0.0f ? acc[mb][t] : 0.0f;
      const float cs = tile_col_sum(dz[t]);
      if (r == 0) unsafeAtomicAdd(a.grad + kOffB2 + 16 * mb + 4 * g + t, cs);
    }
    d2[mb] = pack4(dz[0], dz[1], dz[2], dz[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      a.dz2T[(size_t)(16 * mb + 4 * g + t) * a.ldT + col] = (uint16_t)d2[mb][t];
  }
  // dh1^T = W2 dz2^T, dz1 = dh1 [z1 > 0]
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = mfma16(load_frag(a.frags, kB2 + mb * 4 + kb, lane), d2[kb], acc[mb]);
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    float dz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      dz[t] = F.z1[mb][t] > 0.0f ? acc[mb][t] : 0.0f;
      const float cs = tile_col_sum(dz[t]);
      if (r == 0) unsafeAtomicAdd(a.grad + kOffB1 + 16 * mb + 4 * g + t, cs);
    }
    const bf16x4 d1 = pack4(dz[0], dz[1], dz[2], dz[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      a.dz1T[(size_t)(16 * mb + 4 * g + t) * a.ldT + col] = (uint16_t)d1[t];
  }
}

// ------------------------------------------------------------------------------------------
// weight gradients: dW[in][out] = sum_points act[in][pt] dz[out][pt], one 16x16 tile per
// wavefront, K = the (padded) batch
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_wgrad(MlpArgs a) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  // tiles: W1 20 x 4 (80), W2 4 x 4 (16), W3 4 x 16 (64)
  const uint16_t *A, *B;
  int mi, no, out_w, off;
  if (w < 80) {
    mi = w / 4; no = w % 4; A = a.xT; B = a.dz1T; out_w = kHid; off = kOffW1;
  } else if (w < 96) {
    mi = (w - 80) / 4; no = (w - 80) % 4; A = a.h1T; B = a.dz2T; out_w = kHid; off = kOffW2;
  } else if (w < 160) {
    mi = (w - 96) / 16; no = (w - 96) % 16; A = a.h2T; B = a.dz3T; out_w = kBins; off = kOffW3;
  } else {
    return;
  }
  const uint16_t* arow = A + (size_t)(16 * mi + r) * a.ldT + 4 * g;
  const uint16_t* brow = B + (size_t)(16 * no + r) * a.ldT + 4 * g;
  f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t ks = 0; ks < a.ldT; ks += 16) {
    const bf16x4 av = *reinterpret_cast<const bf16x4*>(arow + ks);
    const bf16x4 bv = *reinterpret_cast<const bf16x4*>(brow + ks);
    acc = mfma16(av, bv, acc);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) a.grad[off + (16 * mi + 4 * g + t) * out_w + 16 * no + r] = acc[t];
}

// ------------------------------------------------------------------------------------------
// Adam
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m,
                                              float* __restrict__ v,
                                              const float* __restrict__ gr, int64_t n, float lr,
                                              float b1, float b2, float eps, float ic1,
                                              float ic2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * ic1) / (sqrtf(vi * ic2) + eps);
}

// ------------------------------------------------------------------------------------------
hipError_t launch_mlp_frags(const float* params, uint16_t* frags, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_frags, dim3((kFrags * 256 + 255) / 256), dim3(256), 0, s, params,
                     frags);
  return hipGetLastError();
}

size_t mlp_frag_bytes() { return (size_t)kFrags * 256 * sizeof(uint16_t); }

hipError_t launch_mlp_infer(const MlpArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int64_t tiles = (a.n + 15) / 16;
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_train(const MlpArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int64_t tiles = a.ldT / 16;
  hipLaunchKernelGGL(k_mlp_train, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(40), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr,
                       float b1, float b2, float eps, float ic1, float ic2, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, m, v, g, n,
                     lr, b1, b2, eps, ic1, ic2);
  return hipGetLastError();
}

}  // namespace sopk
