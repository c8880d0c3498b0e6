// mlp_device.hpp - device code of the learned proposal's network shared by the network
// kernels (proposal.hip) and the fused proposal shading kernel (shade.hip): bf16 rounding,
// the matrix-core product, the sinusoidal features written straight into operand fragments,
// the forward of one 16-point tile and the per-point softmax. One definition, so that the
// fused kernel's probabilities are bit for bit those of the inference kernel.
#pragma once
#include "sop_device.hpp"
#include "sop_internal.hpp"

namespace sopk {

constexpr int kIn = SOP_MLP_IN, kHid = SOP_MLP_HIDDEN, kBins = SOP_MLP_BINS;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kIn * kHid, kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kBins;
static_assert(kOffB3 + kBins == SOP_MLP_PARAMS, "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Products run on v_mfma_f32_16x16x32_bf16: a 16 x 32 A block times a 32 x 16 B block, each
// lane holding 8 consecutive positions of K (positions 8(l/16) .. +7). The accumulator of a
// 16-row block holds rows 4(l/16) .. +3 in lane l, so the next layer's B operand for the
// 32 inputs 32 kb .. 32 kb + 31 is the lane's 4 values of block 2 kb followed by its 4 of
// block 2 kb + 1: K position 8 g + j stands for input 32 kb + 4 g + j (j < 4) or
// 32 kb + 16 + 4 g + j - 4 (j >= 4). The A fragments are laid out in the same order.
__device__ __forceinline__ int kpos_input(int kb, int g, int j) {
  return 32 * kb + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

// fragment sets (in fragments of 512 bf16): forward A operands W^T per (m-block, k-block),
// backward A operands W per (m-block = input block, k-block = output block)
constexpr int kF1 = 0;                    // W1^T: 4 x 10
constexpr int kF2 = kF1 + 4 * 10;         // W2^T: 4 x 2
constexpr int kF3 = kF2 + 4 * 2;          // W3^T: 16 x 2
constexpr int kB3 = kF3 + 16 * 2;         // W3:   4 x 8
constexpr int kB2 = kB3 + 4 * 8;          // W2:   4 x 2
constexpr int kFrags = kB2 + 4 * 2;       // 120 fragments
constexpr int kFragElems = 512;

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return 0x7FC0;   // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);                                          // nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// B operand of a 32-input block from the lane's fragments of its two 16-row halves
__device__ __forceinline__ bf16x8 cat8(bf16x4 lo, bf16x4 hi) {
  const bf16x8s v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 r;
  r[0] = (short)f2bf(a);
  r[1] = (short)f2bf(b);
  r[2] = (short)f2bf(c);
  r[3] = (short)f2bf(d);
  return r;
}

__device__ __forceinline__ bf16x8 load_frag(const uint16_t* frags, int f, int lane) {
  return __builtin_bit_cast(
      bf16x8, *reinterpret_cast<const bf16x8s*>(frags + ((size_t)f * 64 + lane) * 8));
}

// ------------------------------------------------------------------------------------------
// features of the lane's point: the 10 scalars and the B fragment of k-block kb
// ------------------------------------------------------------------------------------------
struct FeatIn {
  float x[10];
};

// the 10 scalars of point p: position mapped by lo/inv2, normal, view (or camera), roughness
__device__ __forceinline__ void point_scalars(const float* pos, const float* nrm,
                                              const float* view, const float* cam, int64_t ppf,
                                              const float* rough, const float (&lo)[3],
                                              const float (&inv2)[3], int64_t p, FeatIn& fi) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    fi.x[c] = (pos[3 * p + c] - lo[c]) * inv2[c] - 1.0f;
    fi.x[3 + c] = nrm[3 * p + c];
  }
  if (view) {
#pragma unroll
    for (int c = 0; c < 3; ++c) fi.x[6 + c] = view[3 * p + c];
  } else {
    const int64_t f = p / ppf;
    float d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] = cam[3 * f + c] - pos[3 * p + c];
    const float il = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) fi.x[6 + c] = d[c] * il;
  }
  fi.x[9] = rough[p];
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

__device__ __forceinline__ void forward_tile(const float* params, const uint16_t* frags,
                                             const FeatIn& fi, int lane, Fwd& F, uint16_t* xT,
                                             int64_t ldT, int64_t col, bool store) {
  const int g = lane >> 4;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) F.z1[mb][t] = params[kOffB1 + 16 * mb + 4 * g + t];
#pragma unroll
  for (int kb = 0; kb < 10; ++kb) {        // fully unrolled: fi.x[kb] stays in registers
    const bf16x4 b0 = feature_frag(fi, 2 * kb, g), b1 = feature_frag(fi, 2 * kb + 1, g);
    if (store) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        xT[(size_t)(32 * kb + 4 * g + t) * ldT + col] = (uint16_t)b0[t];
        xT[(size_t)(32 * kb + 16 + 4 * g + t) * ldT + col] = (uint16_t)b1[t];
      }
    }
    const bf16x8 b = cat8(b0, b1);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) F.z1[mb] = mfma32(load_frag(frags, kF1 + mb * 10 + kb, lane), b, F.z1[mb]);
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
    F.h1[mb] = pack4(fmaxf(F.z1[mb][0], 0.0f), fmaxf(F.z1[mb][1], 0.0f), fmaxf(F.z1[mb][2], 0.0f),
                     fmaxf(F.z1[mb][3], 0.0f));
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) F.z2[mb][t] = params[kOffB2 + 16 * mb + 4 * g + t];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    const bf16x8 b = cat8(F.h1[2 * kb], F.h1[2 * kb + 1]);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
      F.z2[mb] = mfma32(load_frag(frags, kF2 + mb * 2 + kb, lane), b, F.z2[mb]);
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
    F.h2[mb] = pack4(fmaxf(F.z2[mb][0], 0.0f), fmaxf(F.z2[mb][1], 0.0f), fmaxf(F.z2[mb][2], 0.0f),
                     fmaxf(F.z2[mb][3], 0.0f));
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) F.z3[mb][t] = params[kOffB3 + 16 * mb + 4 * g + t];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    const bf16x8 b = cat8(F.h2[2 * kb], F.h2[2 * kb + 1]);
#pragma unroll
    for (int mb = 0; mb < 16; ++mb)
      F.z3[mb] = mfma32(load_frag(frags, kF3 + mb * 2 + kb, lane), b, F.z3[mb]);
  }
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

// Bin probabilities of the lane's 64 logits (softmax over the 4 lanes of its point),
// written into z in place: p = exp(z - max) / sum exp(z - max).
__device__ __forceinline__ void softmax_tile(f32x4 (&z)[16]) {
  float mx = -INFINITY;
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) mx = fmaxf(mx, z[mb][t]);
  mx = point_max(mx);
  float se = 0.0f;
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) se += expf(z[mb][t] - mx);
  se = point_sum(se);
  const float inv = 1.0f / se;
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) z[mb][t] = expf(z[mb][t] - mx) * inv;
}

}  // namespace sopk
