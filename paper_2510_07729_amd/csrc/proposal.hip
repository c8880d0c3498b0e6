// proposal.hip - the learned direction proposal's network on the matrix cores: inference
// (features -> 320 -> 64 -> 64 -> 256 -> softmax), one training step (forward, cross
// entropy, backward, weight gradients) and Adam. An extension of the Monte Carlo estimate of
// Eq. 7 (ComGS Sec. 3.1.2): the network's bin distribution is what the proposal sampler of
// shade.hip draws from.
//
// Matrix products run on v_mfma_f32_16x16x32_bf16 in a transposed formulation, z^T = W^T x^T:
// the output neurons are the M dimension and 16 points are the N dimension, so the
// accumulators of one layer (lane l holds rows 4(l/16)..+3 of column l%16), after bias,
// ReLU and rounding, are the B operands of the next layer (two 16-row blocks per 32-input
// block, in the K order of mlp_device.hpp); no shuffles or LDS round trips between layers.
// Weights are pre-arranged once per call into operand fragments (64 lanes x 8 bf16 = 1 KB,
// one coalesced load).
// Weight gradients contract over points, so they use activations stored transposed
// ([feature][point]) and are a plain GEMM in which each wavefront owns one 16x16 tile of a
// weight matrix (deterministic, no atomics).
#include "mlp_device.hpp"

namespace sopk {

// ------------------------------------------------------------------------------------------
// fragment preparation: one thread per bf16 element
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_frags(const float* __restrict__ P,
                                                   uint16_t* __restrict__ frags) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kFrags * kFragElems) return;
  const int f = e / kFragElems, lane = (e >> 3) & 63, j = e & 7;
  const int g = lane >> 4, r = lane & 15;
  int src;
  if (f < kF2) {                 // W1^T[out][in]: A[m = out 16mb + r][k = in]
    const int mb = (f - kF1) / 10, kb = (f - kF1) % 10;
    src = kOffW1 + kpos_input(kb, g, j) * kHid + 16 * mb + r;
  } else if (f < kF3) {
    const int mb = (f - kF2) / 2, kb = (f - kF2) % 2;
    src = kOffW2 + kpos_input(kb, g, j) * kHid + 16 * mb + r;
  } else if (f < kB3) {
    const int mb = (f - kF3) / 2, kb = (f - kF3) % 2;
    src = kOffW3 + kpos_input(kb, g, j) * kBins + 16 * mb + r;
  } else if (f < kB2) {          // W3[in][out]: A[m = in 16mb + r][k = out]
    const int mb = (f - kB3) / 8, kb = (f - kB3) % 8;
    src = kOffW3 + (16 * mb + r) * kBins + kpos_input(kb, g, j);
  } else {
    const int mb = (f - kB2) / 2, kb = (f - kB2) % 2;
    src = kOffW2 + (16 * mb + r) * kHid + kpos_input(kb, g, j);
  }
  frags[e] = f2bf(P[src]);
}

// ------------------------------------------------------------------------------------------
// inference: one wavefront per 16 points
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_infer(MlpArgs a) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t p0 = tile * 16;
  if (p0 >= a.n) return;
  const int64_t p = p0 + r;
  const bool valid = p < a.n;
  FeatIn fi;
  if (valid) point_scalars(a.pos, a.nrm, a.view, a.cam, a.ppf, a.rough, a.lo, a.inv2, p, fi);
  else
#pragma unroll
    for (int c = 0; c < 10; ++c) fi.x[c] = 0.0f;
  Fwd F;
  forward_tile(a.params, a.frags, fi, lane, F, nullptr, 0, 0, false);
  if (valid && a.logits) {
#pragma unroll
    for (int mb = 0; mb < 16; ++mb)
      *reinterpret_cast<float4*>(a.logits + (size_t)p * kBins + 16 * mb + 4 * g) =
          make_float4(F.z3[mb][0], F.z3[mb][1], F.z3[mb][2], F.z3[mb][3]);
  }
  softmax_tile(F.z3);
  if (!valid) return;
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
    *reinterpret_cast<float4*>(a.probs + (size_t)p * kBins + 16 * mb + 4 * g) =
        make_float4(F.z3[mb][0], F.z3[mb][1], F.z3[mb][2], F.z3[mb][3]);
}

// ------------------------------------------------------------------------------------------
// training: forward + cross entropy + backward of one 16-point tile per wavefront.
// Writes the transposed bf16 operands of the weight-gradient GEMM (zero for padding points)
// and the tile's bias-gradient column sums and loss, which the weight-gradient kernel adds
// up in a fixed order (no atomics: a step is deterministic).
// ------------------------------------------------------------------------------------------
constexpr int kPart = kMlpPart;

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
  if (p0 >= a.ldT) return;                        // ldT = batch rounded up to 32
  const int64_t p = p0 + r;
  const bool valid = p < a.n;
  const int64_t col = p;
  FeatIn fi;
  if (valid) point_scalars(a.pos, a.nrm, a.view, a.cam, a.ppf, a.rough, a.lo, a.inv2, p, fi);
  else
#pragma unroll
    for (int c = 0; c < 10; ++c) fi.x[c] = 0.0f;
  Fwd F;
  forward_tile(a.params, a.frags, fi, lane, F, a.xT, a.ldT, col, true);
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
      if (r == 0) a.part[tile * kPart + 2 * kHid + 16 * mb + 4 * g + t] = cs;
    }
    d3[mb] = pack4(dz[0], dz[1], dz[2], dz[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      a.dz3T[(size_t)(16 * mb + 4 * g + t) * a.ldT + col] = (uint16_t)d3[mb][t];
  }
  loss = wave_sum(loss * vmask);
  if (lane == 0) a.part[tile * kPart + kPart - 1] = loss * invB;
  // dh2^T = W3 dz3^T, dz2 = dh2 [z2 > 0]
  f32x4 acc[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) acc[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    const bf16x8 b = cat8(d3[2 * kb], d3[2 * kb + 1]);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = mfma32(load_frag(a.frags, kB3 + mb * 8 + kb, lane), b, acc[mb]);
  }
  bf16x4 d2[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    float dz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      dz[t] = F.z2[mb][t] > 0.0f ? acc[mb][t] : 0.0f;
      const float cs = tile_col_sum(dz[t]);
      if (r == 0) a.part[tile * kPart + kHid + 16 * mb + 4 * g + t] = cs;
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
  for (int kb = 0; kb < 2; ++kb) {
    const bf16x8 b = cat8(d2[2 * kb], d2[2 * kb + 1]);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = mfma32(load_frag(a.frags, kB2 + mb * 2 + kb, lane), b, acc[mb]);
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    float dz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      dz[t] = F.z1[mb][t] > 0.0f ? acc[mb][t] : 0.0f;
      const float cs = tile_col_sum(dz[t]);
      if (r == 0) a.part[tile * kPart + 16 * mb + 4 * g + t] = cs;
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
    // bias gradients and the loss: the tiles' partial sums added in tile order, so that a
    // training step is deterministic
    const int v = (w - 160) * 64 + lane;
    if (v >= kPart) return;
    const int64_t tiles = a.ldT / 16;
    float sum = 0.0f;
    for (int64_t t = 0; t < tiles; ++t) sum += a.part[t * kPart + v];
    if (v < kHid) a.grad[kOffB1 + v] = sum;
    else if (v < 2 * kHid) a.grad[kOffB2 + v - kHid] = sum;
    else if (v < kPart - 1) a.grad[kOffB3 + v - 2 * kHid] = sum;
    else *a.loss = sum;
    return;
  }
  // K = points: lane l takes points 8(l/16) .. +7 of each 32-point step (ldT is a multiple
  // of 32, padding points are zero)
  const uint16_t* arow = A + (size_t)(16 * mi + r) * a.ldT + 8 * g;
  const uint16_t* brow = B + (size_t)(16 * no + r) * a.ldT + 8 * g;
  f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t ks = 0; ks < a.ldT; ks += 32) {
    const bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<const bf16x8s*>(arow + ks));
    const bf16x8 bv = __builtin_bit_cast(bf16x8, *reinterpret_cast<const bf16x8s*>(brow + ks));
    acc = mfma32(av, bv, acc);
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
  hipLaunchKernelGGL(k_mlp_frags, dim3((kFrags * kFragElems + 255) / 256), dim3(256), 0, s,
                     params, frags);
  return hipGetLastError();
}

size_t mlp_frag_bytes() { return (size_t)kFrags * kFragElems * sizeof(uint16_t); }

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
  // 160 weight tiles, then ceil(kPart / 64) wavefronts of bias/loss sums
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(40 + (kPart + 255) / 256), dim3(256), 0, s, a);
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
