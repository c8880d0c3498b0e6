// sop_device.hpp - device functions of the SOP shading path (gfx950, wave64, FP32).
//
// Each function implements one step of ComGS (arXiv 2510.07729) Sec. 3.1.2 in single
// precision, arranged for the GPU: octahedral taps are formed once per direction and shared
// by the K probes, the GGX denominator uses |n x h|^2 instead of 1 - (n.h)^2 so that sharp
// lobes keep their relative precision, and direction sums are reduced across the wavefront
// with DPP row operations.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace sopk {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;

struct v3 {
  float x, y, z;
};
__device__ __forceinline__ v3 mk3(float x, float y, float z) { return v3{x, y, z}; }
__device__ __forceinline__ float dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ v3 add(v3 a, v3 b) { return v3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ v3 sub(v3 a, v3 b) { return v3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ v3 mul(v3 a, float s) { return v3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ v3 cross(v3 a, v3 b) {
  return v3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float sgn1(float x) { return x < 0.0f ? -1.0f : 1.0f; }

// ----------------------------------------------------------------------------------------
// Direction set (Eq. 7: S_r rays from a Hammersley set). Rotation: pcg hash of Jarzynski &
// Olano (JCGT 2020), 24 bits.
// ----------------------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
  uint32_t state = v * 747796405u + 2891336453u;
  uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

// 24 random bits for (point i, draw j, stream k) from the hashed seed seed_h = pcg_hash(seed)
__device__ __forceinline__ uint32_t hash24(uint32_t seed_h, uint32_t i, uint32_t j, uint32_t k) {
  return pcg_hash(pcg_hash(seed_h ^ i) ^ (4u * j + k)) >> 8;
}

__host__ __device__ __forceinline__ uint32_t rotation24(uint32_t seed, bool per_point,
                                                       uint32_t i) {
  return (per_point ? pcg_hash(seed ^ pcg_hash(i)) : pcg_hash(seed)) >> 8;
}

// Orthonormal frame around the normal (Duff et al., JCGT 2017), sign(0) = +1, in FP64.
struct Frame64 {
  double t[3], b[3], n[3];
};
__device__ __forceinline__ Frame64 make_frame64(double nx, double ny, double nz) {
  const double sg = nz < 0.0 ? -1.0 : 1.0;
  const double a = -1.0 / (sg + nz);
  const double b = nx * ny * a;
  Frame64 f;
  f.t[0] = 1.0 + sg * nx * nx * a;
  f.t[1] = sg * b;
  f.t[2] = -sg * nx;
  f.b[0] = b;
  f.b[1] = sg + ny * ny * a;
  f.b[2] = -ny;
  f.n[0] = nx;
  f.n[1] = ny;
  f.n[2] = nz;
  return f;
}

// Direction table entry j of S (local frame, FP64): (sin(theta) cos(phi), sin(theta)
// sin(phi), cos(theta)) with cos(theta) = 1 - (j + 0.5)/S and
// phi = 2 pi ((bitrev(j) >> 8) + rho) mod 2^24 / 2^24. The sample directions are the same
// for every point of a call (one rotation per call), so they are formed once per call.
// With cosine, the cosine-weighted set: sin(theta) = sqrt((j + 0.5)/S), cos(theta) =
// sqrt(1 - (j + 0.5)/S), same phi, and .w = 1/(2 cos(theta)), the sample's weight relative
// to the uniform set's 2 pi/S (the density cos/pi instead of 1/(2 pi)).
__device__ __forceinline__ double4 dir_entry(int j, int S, uint32_t rho, bool cosine = false) {
  double ct, st, wgt = 0.0;
  if (cosine) {
    ct = sqrt((double)(2 * S - 2 * j - 1) / (2.0 * (double)S));
    st = sqrt((double)(2 * j + 1) / (2.0 * (double)S));
    wgt = 0.5 / ct;
  } else {
    ct = (double)(2 * S - 2 * j - 1) / (2.0 * (double)S);
    st = sqrt((1.0 - ct) * (1.0 + ct));
  }
  const uint32_t u24 = ((__builtin_bitreverse32((uint32_t)j) >> 8) + rho) & 0xFFFFFFu;
  double sp, cp;
  sincospi((double)u24 * 0x1p-23, &sp, &cp);
  return make_double4(st * cp, st * sp, ct, wgt);
}

// world direction t*a + b*b + n*ct in FP64
__device__ __forceinline__ void world_dir64(const Frame64& F, double a, double b, double ct,
                                            double w[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) w[c] = fma(F.t[c], a, fma(F.b[c], b, F.n[c] * ct));
}

// ----------------------------------------------------------------------------------------
// Octahedral probe texture (Sec. 3.1.2): +z at the centre, lower hemisphere folded to the
// corners; bilinear taps with mirror wrap across the border.
// ----------------------------------------------------------------------------------------
struct Taps {
  int off[4];    // texel index j*R + i of each tap
  float w[4];    // bilinear weights
  int i0, j0;    // corner tap before the wrap, in [-1, R-1]
};

__device__ __forceinline__ void oct_wrap(int i, int j, int R, int& oi, int& oj) {
  if (i < 0) { i = 0; j = R - 1 - j; }
  else if (i >= R) { i = R - 1; j = R - 1 - j; }
  if (j < 0) { j = 0; i = R - 1 - i; }
  else if (j >= R) { j = R - 1; i = R - 1 - i; }
  oi = i;
  oj = j;
}

__device__ __forceinline__ Taps oct_taps(v3 w, int R, float halfR) {
  const float s = fabsf(w.x) + fabsf(w.y) + fabsf(w.z);
  const float inv = 1.0f / s;
  float px = w.x * inv, py = w.y * inv;
  if (w.z < 0.0f) {
    const float fx = (1.0f - fabsf(py)) * sgn1(px);
    const float fy = (1.0f - fabsf(px)) * sgn1(py);
    px = fx;
    py = fy;
  }
  // clamp to [-0.5, R-0.5] (also maps NaN there): every tap index stays in [-1, R]
  const float hi = 2.0f * halfR - 0.5f;
  const float cu = fminf(fmaxf((px + 1.0f) * halfR - 0.5f, -0.5f), hi);
  const float cv = fminf(fmaxf((py + 1.0f) * halfR - 0.5f, -0.5f), hi);
  const float i0f = floorf(cu), j0f = floorf(cv);
  const float fx = cu - i0f, fy = cv - j0f;
  const int i0 = (int)i0f, j0 = (int)j0f;
  Taps t;
  t.i0 = i0;
  t.j0 = j0;
  int ii, jj;
  oct_wrap(i0, j0, R, ii, jj);
  t.off[0] = jj * R + ii;
  oct_wrap(i0 + 1, j0, R, ii, jj);
  t.off[1] = jj * R + ii;
  oct_wrap(i0, j0 + 1, R, ii, jj);
  t.off[2] = jj * R + ii;
  oct_wrap(i0 + 1, j0 + 1, R, ii, jj);
  t.off[3] = jj * R + ii;
  t.w[0] = (1.0f - fx) * (1.0f - fy);
  t.w[1] = fx * (1.0f - fy);
  t.w[2] = (1.0f - fx) * fy;
  t.w[3] = fx * fy;
  return t;
}

// Same taps from an FP64 direction: the bilinear weights of the probe textures then carry
// no FP32 coordinate rounding (it would be amplified in the texture gradient of entries
// that receive only small weights).
// direction of texture coordinate (u, v) in texel units of an R x R octahedral map, FP64
__device__ __forceinline__ void oct_decode64(double u, double v, int R, double w[3]) {
  double px = 2.0 * u / (double)R - 1.0, py = 2.0 * v / (double)R - 1.0;
  const double z = 1.0 - fabs(px) - fabs(py);
  if (z < 0.0) {
    const double fx = (1.0 - fabs(py)) * (px < 0.0 ? -1.0 : 1.0);
    const double fy = (1.0 - fabs(px)) * (py < 0.0 ? -1.0 : 1.0);
    px = fx;
    py = fy;
  }
  const double il = 1.0 / sqrt(px * px + py * py + z * z);
  w[0] = px * il;
  w[1] = py * il;
  w[2] = z * il;
}

__device__ __forceinline__ Taps oct_taps64(const double w[3], int R) {
  const double s = fabs(w[0]) + fabs(w[1]) + fabs(w[2]);
  const double inv = 1.0 / s;
  double px = w[0] * inv, py = w[1] * inv;
  if (w[2] < 0.0) {
    const double fx = (1.0 - fabs(py)) * (px < 0.0 ? -1.0 : 1.0);
    const double fy = (1.0 - fabs(px)) * (py < 0.0 ? -1.0 : 1.0);
    px = fx;
    py = fy;
  }
  const double halfR = 0.5 * (double)R, hi = (double)R - 0.5;
  const double cu = fmin(fmax((px + 1.0) * halfR - 0.5, -0.5), hi);
  const double cv = fmin(fmax((py + 1.0) * halfR - 0.5, -0.5), hi);
  const double i0f = floor(cu), j0f = floor(cv);
  const double fx = cu - i0f, fy = cv - j0f;
  const int i0 = (int)i0f, j0 = (int)j0f;
  Taps t;
  t.i0 = i0;
  t.j0 = j0;
  int ii, jj;
  oct_wrap(i0, j0, R, ii, jj);
  t.off[0] = jj * R + ii;
  oct_wrap(i0 + 1, j0, R, ii, jj);
  t.off[1] = jj * R + ii;
  oct_wrap(i0, j0 + 1, R, ii, jj);
  t.off[2] = jj * R + ii;
  oct_wrap(i0 + 1, j0 + 1, R, ii, jj);
  t.off[3] = jj * R + ii;
  // weights in FP64: 1 - fx cancels when fx is close to 1
  t.w[0] = (float)((1.0 - fx) * (1.0 - fy));
  t.w[1] = (float)(fx * (1.0 - fy));
  t.w[2] = (float)((1.0 - fx) * fy);
  t.w[3] = (float)(fx * fy);
  return t;
}

__device__ __forceinline__ float4 load_texel(const float4* tex, size_t i) { return tex[i]; }
// channel 3 (occlusion) of texel i alone: 4 bytes (f32 maps) or 2 bytes (f16 maps)
__device__ __forceinline__ float load_occlusion(const float4* tex, size_t i) {
  return reinterpret_cast<const float*>(tex)[4 * i + 3];
}
__device__ __forceinline__ float load_occlusion(const uint2* tex, size_t i) {
  return __half2float(reinterpret_cast<const __half*>(tex)[4 * i + 3]);
}
__device__ __forceinline__ float4 load_texel(const uint2* tex, size_t i) {
  const uint2 u = tex[i];
  const __half2 a = *reinterpret_cast<const __half2*>(&u.x);
  const __half2 b = *reinterpret_cast<const __half2*>(&u.y);
  const float2 fa = __half22float2(a), fb = __half22float2(b);
  return make_float4(fa.x, fa.y, fb.x, fb.y);
}

// ----------------------------------------------------------------------------------------
// Equirectangular environment map (Eq. 8, L_dir): theta from +z down the rows,
// phi = atan2(y, x) along the columns, bilinear, columns wrap, rows clamp.
// ----------------------------------------------------------------------------------------
struct EnvTaps {
  int off[4];
  float w[4];
  int vi, vj;    // corner tap before the wrap and the clamp, plus 2 (>= 0)
};

__device__ __forceinline__ EnvTaps env_taps(v3 w, int H, int W, float u_scale, float v_scale) {
  const float theta = atan2f(sqrtf(w.x * w.x + w.y * w.y), w.z);
  const float phi = atan2f(w.y, w.x);
  // u = (phi + pi) W / (2 pi) = phi * W/(2pi) + W/2, one rounding
  // clamped to [-0.5, W-0.5] x [-0.5, H-0.5] (NaN included) so every tap is in range
  const float cu = fminf(fmaxf(fmaf(phi, u_scale, 0.5f * (float)W) - 0.5f, -0.5f),
                         (float)W - 0.5f);
  const float cv = fminf(fmaxf(theta * v_scale - 0.5f, -0.5f), (float)H - 0.5f);
  const float i0f = floorf(cu), j0f = floorf(cv);
  const float fx = cu - i0f, fy = cv - j0f;
  int i0 = (int)i0f, j0 = (int)j0f;
  const int vi = i0 + 2, vj = j0 + 2;
  int i1 = i0 + 1, j1 = j0 + 1;
  i0 = i0 < 0 ? i0 + W : (i0 >= W ? i0 - W : i0);
  i1 = i1 < 0 ? i1 + W : (i1 >= W ? i1 - W : i1);
  j0 = j0 < 0 ? 0 : (j0 > H - 1 ? H - 1 : j0);
  j1 = j1 < 0 ? 0 : (j1 > H - 1 ? H - 1 : j1);
  EnvTaps t;
  t.vi = vi;
  t.vj = vj;
  t.off[0] = j0 * W + i0;
  t.off[1] = j0 * W + i1;
  t.off[2] = j1 * W + i0;
  t.off[3] = j1 * W + i1;
  t.w[0] = (1.0f - fx) * (1.0f - fy);
  t.w[1] = fx * (1.0f - fy);
  t.w[2] = (1.0f - fx) * fy;
  t.w[3] = fx * fy;
  return t;
}

// Accurate variant. The texel is chosen from the FP32 angles; the fraction inside it is the
// FP64 angle between the direction and the texel's reference direction (the direction
// at cu = i exactly, from a per-call table), through a small-angle arctangent series.
// Both angles then carry ~1e-16 instead of ~1e-7 error, so bilinear weights (and the
// gradients they scatter) are exact to FP32 rounding even when a weight is small.
//   col_ref[i + 1] = (cos, sin) of phi_i = 2 pi (i + 0.5)/W - pi,   i in [-1, W]
//   row_ref[j + 1] = (cos, sin) of theta_j = pi (j + 0.5)/H,        j in [-1, H]
__device__ __forceinline__ double small_atan(double z) {
  // arctan series; |z| <= 0.2 gives |error| < z^15/15 < 3e-12 relative to the texel width
  const double z2 = z * z;
  return z * (1.0 + z2 * (-1.0 / 3 + z2 * (1.0 / 5 + z2 * (-1.0 / 7 + z2 * (1.0 / 9 +
             z2 * (-1.0 / 11 + z2 * (1.0 / 13)))))));
}

// atan2 for the rare wide angles, built on the same series: fold into the first octant,
// then three half-angle steps t -> t / (1 + sqrt(1 + t^2)) take tan(pi/4) to tan(pi/32) <
// 0.1, where the series is exact to ~1e-16. It keeps no polynomial of its own, so the
// common path holds no extra constants.
__device__ __noinline__ double wide_atan2(double y, double x) {
  const double kPi = 3.14159265358979323846;
  if (x == 0.0 && y == 0.0) {
    const double r = signbit(x) ? kPi : 0.0;
    return signbit(y) ? -r : r;
  }
  const double ax = fabs(x), ay = fabs(y);
  const bool steep = ay > ax;
  double t = steep ? ax / ay : ay / ax;                  // in [0, 1]
  t = t / (1.0 + sqrt(fma(t, t, 1.0)));
  t = t / (1.0 + sqrt(fma(t, t, 1.0)));
  t = t / (1.0 + sqrt(fma(t, t, 1.0)));
  double r = 8.0 * small_atan(t);
  if (steep) r = 0.5 * kPi - r;
  if (signbit(x)) r = kPi - r;
  return signbit(y) ? -r : r;
}

__device__ __forceinline__ double angle_from(double c, double s, double x, double y) {
  // signed angle from direction (c, s) to (x, y), both in one plane; the series covers
  // small angles only (dt > 0), the rest (texels wider than a right angle, W < 8 or H < 4)
  // goes through the full arctangent
  const double cr = c * y - s * x, dt = c * x + s * y;
  const double z = cr / dt;
  return (dt > 0.0 && fabs(z) <= 0.2) ? small_atan(z) : wide_atan2(cr, dt);
}

__device__ __forceinline__ EnvTaps env_taps64(const double w[3], int H, int W, float u_scale,
                                              float v_scale, const double2* col_ref,
                                              const double2* row_ref) {
  const float xf = (float)w[0], yf = (float)w[1], zf = (float)w[2];
  const float rhof = sqrtf(xf * xf + yf * yf);
  const float phif = atan2f(yf, xf), thetaf = atan2f(rhof, zf);
  float cuf = fminf(fmaxf(fmaf(phif, u_scale, 0.5f * (float)W) - 0.5f, -0.5f), (float)W - 0.5f);
  float cvf = fminf(fmaxf(thetaf * v_scale - 0.5f, -0.5f), (float)H - 0.5f);
  int i0 = (int)floorf(cuf), j0 = (int)floorf(cvf);   // i0 in [-1, W-1], j0 in [-1, H-1]
  // exact fractions relative to the reference directions of i0 and j0
  const double2 cr = col_ref[i0 + 1];
  double fx = angle_from(cr.x, cr.y, w[0], w[1]) * ((double)W / (2.0 * 3.14159265358979323846));
  double rho2 = w[0] * w[0] + w[1] * w[1];
  double rho = (double)rhof;
  rho = rho > 0.0 ? 0.5 * (rho + rho2 / rho) : 0.0;     // one Newton step to FP64 accuracy
  const double2 rr = row_ref[j0 + 1];
  // angle from theta_ref to theta in the (z, rho) plane, where the direction sits at angle
  // theta from +z and the reference at theta_ref = (cos, sin)
  double fy = angle_from(rr.x, rr.y, w[2], rho) * ((double)H / 3.14159265358979323846);
  // the FP32 choice of texel may be off by one near a boundary
  if (fx < 0.0) { fx += 1.0; i0 -= 1; } else if (fx >= 1.0) { fx -= 1.0; i0 += 1; }
  if (fy < 0.0) { fy += 1.0; j0 -= 1; } else if (fy >= 1.0) { fy -= 1.0; j0 += 1; }
  fx = fmin(fmax(fx, 0.0), 1.0);
  fy = fmin(fmax(fy, 0.0), 1.0);
  // wrap columns (i0 may now be -2 .. W) and clamp rows
  const int vi = i0 + 2, vj = j0 + 2;
  int i1 = i0 + 1, j1 = j0 + 1;
  i0 = i0 < 0 ? i0 + W : (i0 >= W ? i0 - W : i0);
  i1 = i1 < 0 ? i1 + W : (i1 >= W ? i1 - W : i1);
  i0 = min(max(i0, 0), W - 1);
  i1 = min(max(i1, 0), W - 1);
  j0 = j0 < 0 ? 0 : (j0 > H - 1 ? H - 1 : j0);
  j1 = j1 < 0 ? 0 : (j1 > H - 1 ? H - 1 : j1);
  EnvTaps t;
  t.vi = vi;
  t.vj = vj;
  t.off[0] = j0 * W + i0;
  t.off[1] = j0 * W + i1;
  t.off[2] = j1 * W + i0;
  t.off[3] = j1 * W + i1;
  t.w[0] = (float)((1.0 - fx) * (1.0 - fy));
  t.w[1] = (float)(fx * (1.0 - fy));
  t.w[2] = (float)((1.0 - fx) * fy);
  t.w[3] = (float)(fx * fy);
  return t;
}

// ----------------------------------------------------------------------------------------
// BRDF (Eq. 6, read as Lambert + GGX/Smith-Schlick/Schlick). Returns f*cos(theta) per
// channel and, when asked, the pieces the adjoint needs.
// ----------------------------------------------------------------------------------------
struct Material {
  v3 a;          // albedo
  float r, m;    // roughness, metallic
  float alpha, a2, k;
  float NoV;     // clamped n.v
  float one_m_k; // 1 - k
  float g1v;     // Smith G1(NoV)
};

// NoV is formed in FP64 by the caller: for grazing views n.v is a small difference of
// O(1) products.
__device__ __forceinline__ Material make_material(float NoV_clamped, v3 albedo, float r,
                                                  float m) {
  Material M;
  M.a = albedo;
  M.r = r;
  M.m = m;
  M.alpha = r * r;
  M.a2 = M.alpha * M.alpha;
  M.k = 0.5f * M.alpha;
  M.one_m_k = 1.0f - M.k;
  M.NoV = NoV_clamped;
  M.g1v = M.NoV / (M.NoV * M.one_m_k + M.k);
  return M;
}

// Half-vector geometry in FP64. A sharp GGX lobe (alpha ~ 1e-3) turns a direction error
// of 1e-7 into a relative error of ~1e-4 in D, and 1 - (n.h)^2 cancels; both are formed
// here from FP64 directions, then rounded once to FP32.
struct HalfGeom {
  float NoH2;    // (n.h)^2 with h normalised
  float one_m;   // 1 - (n.h)^2
  float VoH;     // v.h
};
__device__ __forceinline__ HalfGeom half_geom(const double n[3], const double v[3],
                                              const double w[3]) {
  const double h0 = w[0] + v[0], h1 = w[1] + v[1], h2 = w[2] + v[2];
  const double hh = fma(h0, h0, fma(h1, h1, h2 * h2));
  const double c = fma(n[0], h0, fma(n[1], h1, n[2] * h2));
  const double vh = fma(v[0], h0, fma(v[1], h1, v[2] * h2));
  const double NoH2 = c * c / hh;
  HalfGeom g;
  g.NoH2 = (float)NoH2;
  g.one_m = (float)(1.0 - NoH2);
  g.VoH = (float)vh * rsqrtf((float)hh);
  return g;
}

struct BrdfTerms {
  float D, G1L, q, one_m, NoH2, x5;   // GGX pieces
  float spec;                         // D * G / (4 NoV) (times cos cancels 1/NoL)
};

__device__ __forceinline__ BrdfTerms brdf_terms(const Material& M, const HalfGeom& hg,
                                                float NoL) {
  BrdfTerms T;
  T.one_m = hg.one_m;
  T.NoH2 = hg.NoH2;
  T.q = fmaf(M.a2, T.NoH2, T.one_m);       // = NoH^2 (alpha^2 - 1) + 1
  T.D = M.a2 / (kPi * T.q * T.q);
  T.G1L = NoL / (NoL * M.one_m_k + M.k);
  const float x = 1.0f - hg.VoH;
  const float x2 = x * x;
  T.x5 = x2 * x2 * x;
  T.spec = T.D * T.G1L * M.g1v / (4.0f * M.NoV);
  return T;
}

// f(w) * cos(theta) for channel albedo ac
__device__ __forceinline__ float fcos(const Material& M, const BrdfTerms& T, float ac,
                                      float ct) {
  const float F0 = 0.04f * (1.0f - M.m) + ac * M.m;
  const float F = F0 + (1.0f - F0) * T.x5;
  return (1.0f - M.m) * ac * kInvPi * ct + T.spec * F;
}

// ----------------------------------------------------------------------------------------
// Wavefront sum with DPP row operations; the total is returned to every lane.
// All 64 lanes must be active.
// ----------------------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_add(float v) {
  const int src = __float_as_int(v);
  const int moved = __builtin_amdgcn_update_dpp(0, src, CTRL, ROW_MASK, 0xF, false);
  return v + __int_as_float(moved);
}

__device__ __forceinline__ float wave_sum(float v) {
  v = dpp_add<0xB1>(v);          // quad_perm [1,0,3,2]
  v = dpp_add<0x4E>(v);          // quad_perm [2,3,0,1]
  v = dpp_add<0x141>(v);         // row_half_mirror
  v = dpp_add<0x140>(v);         // row_mirror
  v = dpp_add<0x142, 0xA>(v);    // row_bcast15 into rows 1,3
  v = dpp_add<0x143, 0xC>(v);    // row_bcast31 into rows 2,3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Workgroups are dispatched to the 8 dies round-robin (block b runs on die b % 8). This
// renumbers them so that each die takes a contiguous range of blocks: consecutive
// (Morton-ordered) points then share one die's L2, which holds the probe maps they read.
__device__ __forceinline__ int64_t die_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

__device__ __forceinline__ int wave_id_uniform() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// ----------------------------------------------------------------------------------------
// Neighbour-search lattice: q = clamp(floor((x - lo) * sc), 0, 32767) in FP32.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ int quantize1(float x, float lo, float sc) {
  const float d = __fsub_rn(x, lo);
  const float s = __fmul_rn(d, sc);
  const float f = floorf(s);
  return f >= 0.0f ? (f > 32767.0f ? 32767 : (int)f) : 0;   // NaN -> 0
}

__host__ __device__ __forceinline__ uint32_t morton_spread(uint32_t v) {
  v &= 0x3FF;
  v = (v | (v << 16)) & 0x030000FF;
  v = (v | (v << 8)) & 0x0300F00F;
  v = (v | (v << 4)) & 0x030C30C3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}
__host__ __device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return morton_spread(x) | (morton_spread(y) << 1) | (morton_spread(z) << 2);
}

}  // namespace sopk
