// bake.hip - probe textures by ray tracing 3D Gaussians (ComGS Sec. 3.1.2: SOP textures
// initialised by ray tracing; the compositing of Eq. 1).
//
// Every Gaussian is turned into its whitening map M = S^-1 R^T (ray in Gaussian units) and
// registered in the cells of a uniform grid that its cut-off ellipsoid (where
// opacity * exp(-m^2/2) can reach alpha_min) overlaps: the cells of its axis-aligned box
// that pass a separating-axis test along the ellipsoid's own axes and an exact test (the
// minimum of the ellipsoid's quadratic form over the cell), all padded for FP32 rounding;
// one wavefront registers one Gaussian.
// Two lanes trace one texel's ray; a wavefront covers an 8x4 texel block of one probe so
// that its rays stay coherent. The ray walks the grid cell by cell (3D DDA); a Gaussian is
// composited in the cell whose t-window [t_enter, t_exit) holds its t*. Within a cell the
// two lanes split the candidates. Each lane first screens its candidates in FP32 (t* in
// the window and m^2 under the cut-off, both with margins far above the FP32 error) and
// keeps the survivors in LDS, then runs the exact FP64 test on those only, so the FP64
// work is done for about one candidate in six and by all lanes together. Accepted keys
// (t*, index) go to a sorted register buffer per lane; the buffers are merged in ascending
// key order while compositing (and the cell is taken again above the largest key that is
// known complete when a buffer overflowed), so the global order is ascending (t*, index).
#include <float.h>

#include "sop_device.hpp"
#include "sop_internal.hpp"

namespace sopk {

constexpr int kGRows = 5;   // float4 rows per Gaussian record

__device__ __forceinline__ int f2ord(float f) {
  const int b = __float_as_int(f);
  return b >= 0 ? b : b ^ 0x7FFFFFFF;
}

// ------------------------------------------------------------------------------------------
// per-Gaussian preparation
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gauss_prep(sop_gaussians g, float alpha_min,
                                                    float4* gdata, float4* aabb,
                                                    int32_t* bounds_ord, float* ext_sum,
                                                    int32_t* n_reg) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= g.count) return;
  float qw = g.rotation[4 * i], qx = g.rotation[4 * i + 1], qy = g.rotation[4 * i + 2],
        qz = g.rotation[4 * i + 3];
  const float ql = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= ql; qx *= ql; qy *= ql; qz *= ql;
  // rotation matrix R (columns are the Gaussian's axes in world space)
  const float R00 = 1 - 2 * (qy * qy + qz * qz), R01 = 2 * (qx * qy - qw * qz),
              R02 = 2 * (qx * qz + qw * qy);
  const float R10 = 2 * (qx * qy + qw * qz), R11 = 1 - 2 * (qx * qx + qz * qz),
              R12 = 2 * (qy * qz - qw * qx);
  const float R20 = 2 * (qx * qz - qw * qy), R21 = 2 * (qy * qz + qw * qx),
              R22 = 1 - 2 * (qx * qx + qy * qy);
  const float s0 = g.scale[3 * i], s1 = g.scale[3 * i + 1], s2 = g.scale[3 * i + 2];
  const float i0 = 1.0f / s0, i1 = 1.0f / s1, i2 = 1.0f / s2;
  const float mx = g.mean[3 * i], my = g.mean[3 * i + 1], mz = g.mean[3 * i + 2];
  const float op = g.opacity[i];
  // M = S^-1 R^T: row k is axis k divided by s_k
  float4* gd = gdata + (size_t)kGRows * i;
  gd[0] = make_float4(R00 * i0, R10 * i0, R20 * i0, mx);
  gd[1] = make_float4(R01 * i1, R11 * i1, R21 * i1, my);
  gd[2] = make_float4(R02 * i2, R12 * i2, R22 * i2, mz);
  gd[3] = make_float4(g.color[3 * i], g.color[3 * i + 1], g.color[3 * i + 2], op);
  gd[4] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // cut-off: alpha >= alpha_min needs m^2 <= 2 ln(opacity / alpha_min)
  const float m2max = op > alpha_min ? 2.0f * logf(op / alpha_min) : -1.0f;
  if (!(m2max >= 0.0f)) {
    aabb[2 * i] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);   // empty (lo > hi): not registered
    aabb[2 * i + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return;
  }
  const float mm = sqrtf(m2max);
  // bounding sphere of the cut-off ellipsoid, padded like the box below
  const float rb = (mm * fmaxf(s0, fmaxf(s1, s2))) * 1.002f + 1e-5f;
  gd[4] = make_float4(rb * rb, rb, mm, op);
  float hx = mm * sqrtf(R00 * R00 * s0 * s0 + R01 * R01 * s1 * s1 + R02 * R02 * s2 * s2);
  float hy = mm * sqrtf(R10 * R10 * s0 * s0 + R11 * R11 * s1 * s1 + R12 * R12 * s2 * s2);
  float hz = mm * sqrtf(R20 * R20 * s0 * s0 + R21 * R21 * s1 * s1 + R22 * R22 * s2 * s2);
  // pad for FP32 decisions near the cut-off and cell boundaries
  hx = hx * 1.002f + 1e-5f;
  hy = hy * 1.002f + 1e-5f;
  hz = hz * 1.002f + 1e-5f;
  const float4 lo = make_float4(mx - hx, my - hy, mz - hz, 0.0f);
  const float4 hi = make_float4(mx + hx, my + hy, mz + hz, 0.0f);
  aabb[2 * i] = lo;
  aabb[2 * i + 1] = hi;
  if (bounds_ord) {
    atomicMin(&bounds_ord[0], f2ord(lo.x));
    atomicMin(&bounds_ord[1], f2ord(lo.y));
    atomicMin(&bounds_ord[2], f2ord(lo.z));
    atomicMax(&bounds_ord[3], f2ord(hi.x));
    atomicMax(&bounds_ord[4], f2ord(hi.y));
    atomicMax(&bounds_ord[5], f2ord(hi.z));
    atomicAdd(ext_sum, (2.0f / 3.0f) * (hx + hy + hz));
    atomicAdd(n_reg, 1);
  }
}

__device__ __forceinline__ bool cell_range(const BakeGrid& G, float4 lo, float4 hi, int c0[3],
                                           int c1[3]) {
  const float l[3] = {lo.x, lo.y, lo.z}, h[3] = {hi.x, hi.y, hi.z};
  if (G.dims[0] <= 0 || G.dims[1] <= 0 || G.dims[2] <= 0) return false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!(l[a] <= h[a])) return false;
    const float f0 = floorf((l[a] - G.origin[a]) * G.inv_cell[a]);
    const float f1 = floorf((h[a] - G.origin[a]) * G.inv_cell[a]);
    c0[a] = (int)fminf(fmaxf(f0, 0.0f), (float)(G.dims[a] - 1));
    c1[a] = (int)fminf(fmaxf(f1, 0.0f), (float)(G.dims[a] - 1));
  }
  return true;
}

// flags Gaussians whose box leaves the grid (possible after an update)
__device__ __forceinline__ bool inside_grid(const BakeGrid& G, float4 lo, float4 hi) {
  return lo.x >= G.origin[0] && lo.y >= G.origin[1] && lo.z >= G.origin[2] &&
         hi.x <= G.origin[0] + G.dims[0] * G.cell[0] &&
         hi.y <= G.origin[1] + G.dims[1] * G.cell[1] &&
         hi.z <= G.origin[2] + G.dims[2] * G.cell[2];
}

// Whether the cut-off ellipsoid of record gd (rows M_k = u_k / s_k, cut-off Mahalanobis
// radius in gd[4].z) can reach cell (cx, cy, cz): separating-axis test along the ellipsoid's
// three axes (its box already bounds the cell range along the grid axes). In the scaled
// frame the ellipsoid spans |M_k (x - mean)| <= m; the cell projects to an interval of
// half-width sum_a |M_k,a| h_a around M_k (centre - mean). Padded like the box, so the test
// is conservative; count and fill take the same decisions.
__device__ __forceinline__ bool cell_overlaps(const BakeGrid& G, const float4* gd, int cx,
                                              int cy, int cz) {
  const float mm = gd[4].z;
  const float h0 = 0.5f * G.cell[0], h1 = 0.5f * G.cell[1], h2 = 0.5f * G.cell[2];
  const float c0 = G.origin[0] + ((float)cx + 0.5f) * G.cell[0] - gd[0].w;
  const float c1 = G.origin[1] + ((float)cy + 0.5f) * G.cell[1] - gd[1].w;
  const float c2 = G.origin[2] + ((float)cz + 0.5f) * G.cell[2] - gd[2].w;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float4 r = gd[k];
    const float proj = r.x * c0 + r.y * c1 + r.z * c2;
    const float ext = fabsf(r.x) * h0 + fabsf(r.y) * h1 + fabsf(r.z) * h2;
    const float len = sqrtf(r.x * r.x + r.y * r.y + r.z * r.z);   // 1 / s_k
    if (fabsf(proj) > mm * 1.002f + 1e-5f * len + ext) return false;
  }
  return true;
}

// Whether the cut-off ellipsoid (padded like the box) meets cell (cx, cy, cz), exactly:
// the minimum of q(x) = (x - mean)^T M^T M (x - mean) over the cell (enlarged by 1e-5) is at
// most the padded cut-off. The minimiser of this convex quadratic over a box has each
// coordinate either free (zero gradient) or at a bound, so the minimum is the smallest q
// over the 26 patterns of fixed coordinates whose free part, solved from the zero-gradient
// equations, lies inside the box (the 27th, all free, is the mean itself, tested first).
// Called after cell_overlaps, which it refines; count and fill take the same decisions.
__device__ __forceinline__ bool cell_meets_ellipsoid(const BakeGrid& G, const float4* gd,
                                                     int cx, int cy, int cz) {
  const int ci[3] = {cx, cy, cz};
  double lo[3], hi[3], mu[3];
  const double pad = 1e-5;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = (double)G.origin[a] + (double)ci[a] * (double)G.cell[a] - pad;
    hi[a] = (double)G.origin[a] + (double)(ci[a] + 1) * (double)G.cell[a] + pad;
    mu[a] = (double)gd[a].w;
  }
  if (mu[0] >= lo[0] && mu[0] <= hi[0] && mu[1] >= lo[1] && mu[1] <= hi[1] &&
      mu[2] >= lo[2] && mu[2] <= hi[2])
    return true;
  double A[3][3];
  {
    const double m[3][3] = {{gd[0].x, gd[0].y, gd[0].z}, {gd[1].x, gd[1].y, gd[1].z},
                            {gd[2].x, gd[2].y, gd[2].z}};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        A[a][b] = m[0][a] * m[0][b] + m[1][a] * m[1][b] + m[2][a] * m[2][b];
  }
  const double mmp = 1.002 * (double)gd[4].z + 1e-6;
  const double r2 = mmp * mmp;
  {                                               // the cell's centre inside: accept
    double y[3], q = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) y[a] = 0.5 * (lo[a] + hi[a]) - mu[a];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) q += y[a] * A[a][b] * y[b];
    if (q <= r2) return true;
  }
  double best = DBL_MAX;
#pragma unroll
  for (int code = 0; code < 26; ++code) {        // 26 = all free, covered above
    const int st[3] = {code % 3, (code / 3) % 3, code / 9};   // 0 free, 1 low, 2 high
    double y[3];                                  // x - mean
#pragma unroll
    for (int a = 0; a < 3; ++a) y[a] = st[a] == 1 ? lo[a] - mu[a] : hi[a] - mu[a];
    const int nf = (st[0] == 0) + (st[1] == 0) + (st[2] == 0);
    bool ok = true;
    if (nf == 1) {
      const int f = st[0] == 0 ? 0 : (st[1] == 0 ? 1 : 2);
      const int b0 = (f + 1) % 3, b1 = (f + 2) % 3;
      y[f] = -(A[f][b0] * y[b0] + A[f][b1] * y[b1]) / A[f][f];
      ok = y[f] >= lo[f] - mu[f] - 1e-12 && y[f] <= hi[f] - mu[f] + 1e-12;
    } else if (nf == 2) {
      const int c = st[0] != 0 ? 0 : (st[1] != 0 ? 1 : 2);
      const int f = (c + 1) % 3, g = (c + 2) % 3;
      const double det = A[f][f] * A[g][g] - A[f][g] * A[g][f];
      const double rf = -A[f][c] * y[c], rg = -A[g][c] * y[c];
      y[f] = (rf * A[g][g] - A[f][g] * rg) / det;
      y[g] = (A[f][f] * rg - A[g][f] * rf) / det;
      ok = y[f] >= lo[f] - mu[f] - 1e-12 && y[f] <= hi[f] - mu[f] + 1e-12 &&
           y[g] >= lo[g] - mu[g] - 1e-12 && y[g] <= hi[g] - mu[g] + 1e-12;
    }
    if (!ok) continue;
    double q = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) q += y[a] * A[a][b] * y[b];
    best = fmin(best, q);
  }
  return best <= r2;
}

// One wavefront per Gaussian; its lanes take the cells of the Gaussian's box in turn.
__device__ __forceinline__ void box_cell(const int c0[3], int nx, int ny, int t, int& x,
                                         int& y, int& z) {
  x = c0[0] + t % nx;
  y = c0[1] + (t / nx) % ny;
  z = c0[2] + t / (nx * ny);
}

// The count pass keeps the acceptance bits of the first 64 kCellMaskWords cells of every box
// (one wavefront ballot per 64 cells), so the fill pass repeats the exact test only beyond
// them.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_gauss_count(BakeGrid G, const float4* aabb,
                                                     int32_t* counts, uint64_t* cellmask,
                                                     int32_t* overflow) {
  const int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= G.G) return;
  const float4 lo = aabb[2 * i], hi = aabb[2 * i + 1];
  int c0[3], c1[3];
  if (!cell_range(G, lo, hi, c0, c1)) return;
  if (lane == 0 && !inside_grid(G, lo, hi)) atomicOr(overflow, 1);
  const float4* gd = G.gdata + (size_t)kGRows * i;
  const int nx = c1[0] - c0[0] + 1, ny = c1[1] - c0[1] + 1, nz = c1[2] - c0[2] + 1;
  const int n = nx * ny * nz;
  for (int t0 = 0; t0 < n; t0 += 64) {       // the same trip count for every lane
    const int t = t0 + lane;
    bool acc = false;
    int32_t c = 0;
    if (t < n) {
      int x, y, z;
      box_cell(c0, nx, ny, t, x, y, z);
      acc = cell_overlaps(G, gd, x, y, z) && cell_meets_ellipsoid(G, gd, x, y, z);
      c = (z * G.dims[1] + y) * G.dims[0] + x;
    }
    const int w = t0 >> 6;
    if (w < kCellMaskWords) {
      const uint64_t m = __ballot(acc);
      if (lane == 0) cellmask[(size_t)kCellMaskWords * i + w] = m;
    }
    if (acc) atomicAdd(&counts[c], 1);
  }
}

__global__ __launch_bounds__(256) void k_gauss_fill(BakeGrid G, const float4* aabb,
                                                    const uint64_t* cellmask,
                                                    const int32_t* cell_start, int32_t* cursor,
                                                    int32_t* entries, int32_t capacity,
                                                    int32_t* overflow) {
  const int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= G.G) return;
  const int32_t ncell = G.dims[0] * G.dims[1] * G.dims[2];
  if (cell_start[ncell] > capacity) {      // more registrations than the plan holds
    if (i == 0 && lane == 0) atomicOr(overflow, 2);
    return;
  }
  const float4 lo = aabb[2 * i], hi = aabb[2 * i + 1];
  int c0[3], c1[3];
  if (!cell_range(G, lo, hi, c0, c1)) return;
  const float4* gd = G.gdata + (size_t)kGRows * i;
  const int nx = c1[0] - c0[0] + 1, ny = c1[1] - c0[1] + 1, nz = c1[2] - c0[2] + 1;
  const int n = nx * ny * nz;
  for (int t0 = 0; t0 < n; t0 += 64) {
    const int t = t0 + lane;
    if (t >= n) continue;
    int x, y, z;
    box_cell(c0, nx, ny, t, x, y, z);
    const int w = t0 >> 6;
    const bool acc = w < kCellMaskWords
                         ? ((cellmask[(size_t)kCellMaskWords * i + w] >> lane) & 1) != 0
                         : cell_overlaps(G, gd, x, y, z) && cell_meets_ellipsoid(G, gd, x, y, z);
    if (!acc) continue;
    const int32_t c = (z * G.dims[1] + y) * G.dims[0] + x;
    const int32_t slot = cell_start[c] + atomicAdd(&cursor[c], 1);
    entries[slot] = i;
  }
}

// ------------------------------------------------------------------------------------------
// per-texel ray traversal
// ------------------------------------------------------------------------------------------

// Response of a Gaussian (rows r0..r2 of S^-1 R^T with the mean in .w) on the ray o + t d
// in FP64: t* = -(Mo . Md) / |Md|^2 and m^2 = |Mo + t* Md|^2 (Mo = M (o - mean)). The
// composite step calls it again for the kept candidates, so alpha is recomputed bit for bit
// instead of being carried through the candidate buffer.
__device__ __forceinline__ double exact_tstar(const float4& r0, const float4& r1,
                                              const float4& r2, const v3& o,
                                              const double (&d64)[3], double& olx, double& oly,
                                              double& olz, double& dlx, double& dly,
                                              double& dlz) {
  const double ox = (double)o.x - (double)r0.w, oy = (double)o.y - (double)r1.w,
               oz = (double)o.z - (double)r2.w;
  olx = fma((double)r0.x, ox, fma((double)r0.y, oy, (double)r0.z * oz));
  oly = fma((double)r1.x, ox, fma((double)r1.y, oy, (double)r1.z * oz));
  olz = fma((double)r2.x, ox, fma((double)r2.y, oy, (double)r2.z * oz));
  dlx = fma((double)r0.x, d64[0], fma((double)r0.y, d64[1], (double)r0.z * d64[2]));
  dly = fma((double)r1.x, d64[0], fma((double)r1.y, d64[1], (double)r1.z * d64[2]));
  dlz = fma((double)r2.x, d64[0], fma((double)r2.y, d64[1], (double)r2.z * d64[2]));
  return -(olx * dlx + oly * dly + olz * dlz) / (dlx * dlx + dly * dly + dlz * dlz);
}

__device__ __forceinline__ float exact_alpha(const BakeGrid& G, double tsd, double olx,
                                             double oly, double olz, double dlx, double dly,
                                             double dlz, float op) {
  const double xx = fma(dlx, tsd, olx), xy = fma(dly, tsd, oly), xz = fma(dlz, tsd, olz);
  const float m2 = (float)(xx * xx + xy * xy + xz * xz);
  return fminf(G.alpha_max, op * expf(-0.5f * m2));
}

constexpr int kLpr = 2;    // lanes that trace one ray
constexpr int kNb = 24;    // sorted candidate keys per lane
constexpr int kCap = 32;   // candidates a lane keeps per screening pass
// screening margins: |t*_32 - t*| < kScreenT (1 + |t*|) and |m^2_32 - m^2| < kScreenM (1 + m^2)
// hold with a wide margin (measured: 4e-7 and 8e-5 on the object workload)
constexpr float kScreenT = 1e-4f;
constexpr float kScreenM = 5e-2f;

// A candidate key (t* bits, Gaussian index) read as the bits of an FP64 number: t* > 0 is a
// finite float, so the number is finite and non-negative and the order of the numbers is
// the order of the 64-bit keys; min/max of two keys are single FP64 instructions.
constexpr double kNone = DBL_MAX;   // above every key

__device__ __forceinline__ double make_key(float ts, int32_t gi) {
  return __longlong_as_double(
      (long long)(((uint64_t)(uint32_t)__float_as_int(ts) << 32) | (uint32_t)gi));
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// minimum over the kLpr consecutive lanes that trace one ray (DPP quad swaps, then the
// half-row and row mirrors for groups of 8 and 16)
__device__ __forceinline__ double ray_min(double x) {
  if constexpr (kLpr >= 2) x = fmin(x, dpp_f64<0xB1>(x));
  if constexpr (kLpr >= 4) x = fmin(x, dpp_f64<0x4E>(x));
  if constexpr (kLpr >= 8) x = fmin(x, dpp_f64<0x141>(x));
  if constexpr (kLpr >= 16) x = fmin(x, dpp_f64<0x140>(x));
  return x;
}

// Blended result of one ray: (R, G, B) = sum T alpha color, O = sum T alpha and
// dt = sum T alpha t* (the depth numerator); every lane of the ray returns the same values.
struct RayResult {
  float r, g, b, o, dt;
};

// Traces the ray o + t d64 through the registered Gaussians. The kLpr consecutive lanes
// that share the ray call it together with their rank g in the ray; mylist is the lane's
// column of the wavefront's LDS candidate list.
__device__ __forceinline__ RayResult trace_ray(const BakeGrid& G, const v3& o,
                                               const double (&d64)[3], int g,
                                               int32_t* mylist) {
  const v3 d = mk3((float)d64[0], (float)d64[1], (float)d64[2]);
  const float dd[3] = {d.x, d.y, d.z}, oo[3] = {o.x, o.y, o.z};

  float T = 1.0f, Cr = 0.0f, Cg = 0.0f, Cb = 0.0f, Dp = 0.0f, Wt = 0.0f;
  const int32_t ncell = G.dims[0] * G.dims[1] * G.dims[2];

  // clip to the grid box
  float t0 = 0.0f, t1 = FLT_MAX;
  float inv[3];
  bool hit = ncell > 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = G.origin[a], hi = G.origin[a] + G.dims[a] * G.cell[a];
    if (dd[a] != 0.0f) {
      inv[a] = 1.0f / dd[a];
      float ta = (lo - oo[a]) * inv[a], tb = (hi - oo[a]) * inv[a];
      if (ta > tb) { const float x = ta; ta = tb; tb = x; }
      t0 = fmaxf(t0, ta);
      t1 = fminf(t1, tb);
    } else {
      inv[a] = 0.0f;
      if (oo[a] < lo || oo[a] > hi) hit = false;
    }
  }
  if (hit && t0 <= t1) {
    int c[3], step[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float pa = oo[a] + t0 * dd[a];
      const float f = floorf((pa - G.origin[a]) * G.inv_cell[a]);
      c[a] = (int)fminf(fmaxf(f, 0.0f), (float)(G.dims[a] - 1));
      step[a] = dd[a] > 0.0f ? 1 : (dd[a] < 0.0f ? -1 : 0);
    }
    float t_lo = -FLT_MAX;                  // the first cell takes every t* before its exit
    bool done = false;
    const int max_steps = G.dims[0] + G.dims[1] + G.dims[2] + 3;
    for (int it = 0; it < max_steps && !done; ++it) {
      // exit parameter of the current cell and the axis that is crossed
      float t_exit = FLT_MAX;
      int axis = -1;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (step[a] != 0) {
          const float b = G.origin[a] + (float)(c[a] + (step[a] > 0 ? 1 : 0)) * G.cell[a];
          const float ta = (b - oo[a]) * inv[a];
          if (ta < t_exit) { t_exit = ta; axis = a; }
        }
      }
      bool last = axis < 0;
      if (!last) {
        const int nc = c[axis] + step[axis];
        last = nc < 0 || nc >= G.dims[axis];
      }
      const float t_hi = last ? FLT_MAX : t_exit;
      const int32_t cell = (c[2] * G.dims[1] + c[1]) * G.dims[0] + c[0];
      const int32_t e0 = min(G.cell_start[cell], G.capacity);
      const int32_t e1 = min(G.cell_start[cell + 1], G.capacity);

      // candidates of this cell in ascending (t*, index): each lane of the ray tests every
      // kLpr-th entry into its own sorted buffer; the buffers are merged when compositing
      double after = -1.0;     // keys <= after are done
      while (e1 > e0 && !done) {            // rounds: the cell again above `after`
        double key[kNb];
#pragma unroll
        for (int s = 0; s < kNb; ++s) key[s] = kNone;
        int32_t e = e0 + g;
        for (;;) {
          // pass 1: an FP32 screen of t* and m^2 with wide margins keeps the candidates the
          // FP64 test could accept (their indices go to this lane's LDS list)
          int n = 0;
          auto screen = [&](const float4& r0, const float4& r1, const float4& r2, float mmv,
                            int32_t gi) {
            const float ox = o.x - r0.w, oy = o.y - r1.w, oz = o.z - r2.w;
            const float ux = fmaf(r0.x, ox, fmaf(r0.y, oy, r0.z * oz));
            const float uy = fmaf(r1.x, ox, fmaf(r1.y, oy, r1.z * oz));
            const float uz = fmaf(r2.x, ox, fmaf(r2.y, oy, r2.z * oz));
            const float wx = fmaf(r0.x, d.x, fmaf(r0.y, d.y, r0.z * d.z));
            const float wy = fmaf(r1.x, d.x, fmaf(r1.y, d.y, r1.z * d.z));
            const float wz = fmaf(r2.x, d.x, fmaf(r2.y, d.y, r2.z * d.z));
            const float ww = fmaf(wx, wx, fmaf(wy, wy, wz * wz));
            const float uw = fmaf(ux, wx, fmaf(uy, wy, uz * wz));
            const float t32 = -uw * __builtin_amdgcn_rcpf(ww);
            const float mt = kScreenT * (1.0f + fabsf(t32));
            if (!(t32 > G.t_min - mt && t32 >= t_lo - mt && t32 < t_hi + mt)) return;
            const float rx = fmaf(wx, t32, ux), ry = fmaf(wy, t32, uy), rz = fmaf(wz, t32, uz);
            const float m2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
            if (!(m2 <= fmaf(mmv * mmv, 1.0f + kScreenM, kScreenM))) return;
            mylist[n * 64] = gi;
            ++n;
          };
          {
            // two record sets take turns: one is tested while the other is in flight
            int32_t giA = 0, giB = 0;
            float4 a0, a1, a2, b0, b1, b2;
            float amm = 0.0f, bmm = 0.0f;
            if (e < e1) {
              giA = G.entries[e];
              const float4* gq = G.gdata + (size_t)kGRows * giA;
              a0 = gq[0]; a1 = gq[1]; a2 = gq[2]; amm = gq[4].z;
            }
            int32_t gnext = e + kLpr < e1 ? G.entries[e + kLpr] : 0;
            while (e < e1 && n < kCap) {
              const bool hasB = e + kLpr < e1;
              if (hasB) {
                giB = gnext;
                const float4* gq = G.gdata + (size_t)kGRows * giB;
                b0 = gq[0]; b1 = gq[1]; b2 = gq[2]; bmm = gq[4].z;
                gnext = e + 2 * kLpr < e1 ? G.entries[e + 2 * kLpr] : 0;
              }
              screen(a0, a1, a2, amm, giA);
              e += kLpr;
              if (!hasB || n >= kCap) break;
              const bool hasA = e + kLpr < e1;
              if (hasA) {
                giA = gnext;
                const float4* gq = G.gdata + (size_t)kGRows * giA;
                a0 = gq[0]; a1 = gq[1]; a2 = gq[2]; amm = gq[4].z;
                gnext = e + 2 * kLpr < e1 ? G.entries[e + 2 * kLpr] : 0;
              }
              screen(b0, b1, b2, bmm, giB);
              e += kLpr;
              if (!hasA) break;
            }
          }
          // pass 2: the exact FP64 test of the kept candidates
          for (int i = 0; i < n; ++i) {
            const int32_t gi = mylist[i * 64];
            const float4* gq = G.gdata + (size_t)kGRows * gi;
            const float4 r0 = gq[0], r1 = gq[1], r2 = gq[2];
            const float op = gq[4].w;
            double olx, oly, olz, dlx, dly, dlz;
            const double tsd = exact_tstar(r0, r1, r2, o, d64, olx, oly, olz, dlx, dly, dlz);
            if (!(tsd > (double)G.t_min && tsd >= (double)t_lo && tsd < (double)t_hi)) continue;
            const float a = exact_alpha(G, tsd, olx, oly, olz, dlx, dly, dlz, op);
            if (!(a >= G.alpha_min)) continue;
            double k = make_key((float)tsd, gi);
            if (k <= after || k >= key[kNb - 1]) continue;
#pragma unroll
            for (int s = 0; s < kNb; ++s) {    // sorted insertion, largest falls out
              const double lo = fmin(k, key[s]);
              k = fmax(k, key[s]);
              key[s] = lo;
            }
          }
          if (!(e < e1)) break;
        }
        // every key of the cell up to `bound` is held by some lane: a full lane dropped only
        // keys above its own largest one
        const double bound = ray_min(key[kNb - 1]);
        for (;;) {
          const double head = key[0];
          const double m = ray_min(head);
          if (m == kNone || m > bound) break;
          const uint64_t mb = (uint64_t)__double_as_longlong(m);
          const int32_t gi = (int32_t)(mb & 0xFFFFFFFFu);
          const float4* gk = G.gdata + (size_t)kGRows * gi;
          const float4 col = gk[3];
          double olx, oly, olz, dlx, dly, dlz;
          const double tsd = exact_tstar(gk[0], gk[1], gk[2], o, d64, olx, oly, olz, dlx, dly,
                                         dlz);
          const float a = exact_alpha(G, tsd, olx, oly, olz, dlx, dly, dlz, col.w);
          const float Tn = T * (1.0f - a);
          if (Tn < G.T_min) { done = true; break; }
          const float ts = __int_as_float((int)(mb >> 32));
          const float wgt = T * a;
          Cr += wgt * col.x;
          Cg += wgt * col.y;
          Cb += wgt * col.z;
          Dp += wgt * ts;
          Wt += wgt;
          T = Tn;
          if (head == m) {                     // the lane that held it moves to its next key
#pragma unroll
            for (int s = 0; s < kNb - 1; ++s) key[s] = key[s + 1];
            key[kNb - 1] = kNone;
          }
        }
        if (bound == kNone) break;             // no lane dropped a key: the cell is finished
        after = bound;
      }
      if (last) break;
      t_lo = t_exit;
      c[axis] += step[axis];
    }
  }
  RayResult res;
  res.r = Cr;
  res.g = Cg;
  res.b = Cb;
  res.o = Wt;
  res.dt = Dp;
  return res;
}

// The kernel needs three wavefronts per SIMD (at most 168 registers; it uses 168): at two
// it runs ~40% slower, so any change here has to keep the register count.
__global__ __launch_bounds__(256) void k_bake(BakeGrid G, const float* probe_pos, int32_t P,
                                              int32_t R, float* texels, float* depth,
                                              const int4* order) {
  // kLpr lanes trace one ray and split each cell's candidates between them; a wavefront
  // holds 64/kLpr rays of one probe, taken in Z order inside 8x8 texel tiles so that they
  // stay coherent; consecutive workgroups take consecutive probes of the order
  const int32_t tiles_x = (R + 7) >> 3;
  const int64_t per_probe = (int64_t)tiles_x * tiles_x * 64;
  const int lane = threadIdx.x & 63;
  const int g = lane & (kLpr - 1);
  const int64_t ray = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 / kLpr) + lane / kLpr;
  if (ray >= (int64_t)P * per_probe) return;      // whole groups leave together
  const int32_t slot = (int32_t)(ray / per_probe);
  const int32_t p = order ? order[slot].w : slot;
  if ((uint32_t)p >= (uint32_t)P) return;
  const int32_t within = (int32_t)(ray % per_probe);
  const int32_t tile = within >> 6, q = within & 63;
  const int32_t ti = (tile % tiles_x) * 8 + ((q & 1) | ((q >> 1) & 2) | ((q >> 2) & 4));
  const int32_t tj = (tile / tiles_x) * 8 + (((q >> 1) & 1) | ((q >> 2) & 2) | ((q >> 3) & 4));
  if (ti >= R || tj >= R) return;
  const size_t texel = (size_t)p * R * R + (size_t)tj * R + ti;

  if (G.overflow && *G.overflow) {
    if (g == 0) {
      const float nan = __int_as_float(0x7FC00000);
      reinterpret_cast<float4*>(texels)[texel] = make_float4(nan, nan, nan, nan);
      if (depth) depth[texel] = nan;
    }
    return;
  }

  __shared__ int32_t screened[4][kCap][64];      // per wavefront: kept candidates per lane
  int32_t* mylist = &screened[threadIdx.x >> 6][0][lane];
  const v3 o = mk3(probe_pos[3 * p], probe_pos[3 * p + 1], probe_pos[3 * p + 2]);
  // ray direction in FP64 (the candidate test below runs in FP64: a Gaussian of scale 0.01
  // one unit away turns a 1e-7 direction error into 1e-5 in its Mahalanobis distance);
  // the grid walk uses its FP32 rounding
  double d64[3];
  {
    double px = 2.0 * (ti + 0.5) / (double)R - 1.0, py = 2.0 * (tj + 0.5) / (double)R - 1.0;
    const double z = 1.0 - fabs(px) - fabs(py);
    if (z < 0.0) {
      const double fx = (1.0 - fabs(py)) * (px < 0.0 ? -1.0 : 1.0);
      const double fy = (1.0 - fabs(px)) * (py < 0.0 ? -1.0 : 1.0);
      px = fx;
      py = fy;
    }
    const double il = 1.0 / sqrt(px * px + py * py + z * z);
    d64[0] = px * il;
    d64[1] = py * il;
    d64[2] = z * il;
  }
  const RayResult res = trace_ray(G, o, d64, g, mylist);
  if (g == 0) {
    reinterpret_cast<float4*>(texels)[texel] = make_float4(res.r, res.g, res.b, res.o);
    if (depth) depth[texel] = res.o > 0.0f ? res.dt / res.o : 0.0f;
  }
}

// Traced shading rays: sample j of point p starts at fmaf(offset, n_p, x_p) (per component,
// FP32) and runs along the sample's world direction, entry j of the shading call's
// direction table turned into the frame of n_p exactly as the shading kernels turn it. A
// wavefront takes 64/kLpr consecutive points of the processing order with one direction,
// so that its rays start close together and leave their surface at the same angle (which
// keeps their lengths alike); the wavefronts of a workgroup take consecutive directions of
// the same points.
__global__ __launch_bounds__(256) void k_trace_samples(BakeGrid G, TraceArgs t) {
  constexpr int kRays = 64 / kLpr;
  const int lane = threadIdx.x & 63;
  const int g = lane & (kLpr - 1);
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t chunks = (t.n + kRays - 1) / kRays;
  if (wave >= chunks * t.S) return;               // whole wavefronts leave together
  const int64_t chunk = wave / t.S;
  const int32_t j = (int32_t)(wave - chunk * t.S);
  const int64_t slot = chunk * kRays + lane / kLpr;
  if (slot >= t.n) return;                         // the lanes of a ray leave together
  int64_t p = slot;
  if (t.order) {
    const int32_t q = t.order[slot];
    if ((uint64_t)q >= (uint64_t)t.n) return;
    p = q;
  }
  if (G.overflow && *G.overflow) {
    if (g == 0) {
      const float nan = __int_as_float(0x7FC00000);
      t.out[p * t.S + j] = make_float4(nan, nan, nan, nan);
    }
    return;
  }

  __shared__ int32_t screened[4][kCap][64];
  int32_t* mylist = &screened[threadIdx.x >> 6][0][lane];
  const float nx = t.nrm[3 * p], ny = t.nrm[3 * p + 1], nz = t.nrm[3 * p + 2];
  const v3 o = mk3(fmaf(t.offset, nx, t.pos[3 * p]), fmaf(t.offset, ny, t.pos[3 * p + 1]),
                   fmaf(t.offset, nz, t.pos[3 * p + 2]));
  const double4 e = t.dir_tab[j];
  double da = e.x, db = e.y;
  if (t.per_point) {
    double sr, cr;
    sincospi((double)rotation24(t.seed, true, (uint32_t)p) * 0x1p-23, &sr, &cr);
    da = e.x * cr - e.y * sr;
    db = e.x * sr + e.y * cr;
  }
  double d64[3];
  world_dir64(make_frame64(nx, ny, nz), da, db, e.z, d64);
  const RayResult res = trace_ray(G, o, d64, g, mylist);
  // the point index is read again rather than held through the trace (registers)
  if (g == 0) {
    const int64_t q = t.order ? (int64_t)__builtin_nontemporal_load(&t.order[slot]) : slot;
    t.out[q * t.S + j] = make_float4(res.r, res.g, res.b, res.o);
  }
}

// ------------------------------------------------------------------------------------------
hipError_t launch_gauss_prep(const sop_gaussians& g, float alpha_min, float4* gdata,
                             float4* aabb, int32_t* bounds_ord, float* ext_sum, int32_t* n_reg,
                             hipStream_t s) {
  if (g.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gauss_prep, dim3((g.count + 255) / 256), dim3(256), 0, s, g, alpha_min,
                     gdata, aabb, bounds_ord, ext_sum, n_reg);
  return hipGetLastError();
}

hipError_t launch_gauss_count(const BakeGrid& G, const float4* aabb, int32_t* counts,
                              uint64_t* cellmask, int32_t* overflow, hipStream_t s) {
  if (G.G == 0) return hipSuccess;
  if (!G.gdata || !aabb || !counts || !cellmask || !overflow) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gauss_count, dim3((G.G + 3) / 4), dim3(256), 0, s, G, aabb, counts,
                     cellmask, overflow);
  return hipGetLastError();
}

hipError_t launch_gauss_fill(const BakeGrid& G, const float4* aabb, const uint64_t* cellmask,
                             const int32_t* cell_start, int32_t* cursor, int32_t* entries,
                             int32_t capacity, int32_t* overflow, hipStream_t s) {
  if (G.G == 0) return hipSuccess;
  if (!G.gdata || !aabb || !cellmask || !cell_start || !cursor || !entries || !overflow)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gauss_fill, dim3((G.G + 3) / 4), dim3(256), 0, s, G, aabb, cellmask,
                     cell_start, cursor, entries, capacity, overflow);
  return hipGetLastError();
}

hipError_t launch_bake(const BakeGrid& G, const float* probe_pos, int32_t P, int32_t R,
                       float* texels, float* depth, const int4* order, hipStream_t s) {
  const int64_t tiles = (int64_t)((R + 7) / 8) * ((R + 7) / 8);
  const int64_t rays = (int64_t)P * tiles * 64;
  const int64_t waves = (rays + (64 / kLpr) - 1) / (64 / kLpr);
  if (waves == 0) return hipSuccess;
  const int64_t blocks = (waves + 3) / 4;
  hipLaunchKernelGGL(k_bake, dim3((unsigned)blocks), dim3(256), 0, s, G, probe_pos, P, R,
                     texels, depth, order);
  return hipGetLastError();
}

hipError_t launch_trace_samples(const BakeGrid& G, const TraceArgs& t, hipStream_t s) {
  const int64_t chunks = (t.n + (64 / kLpr) - 1) / (64 / kLpr);
  const int64_t blocks = (chunks * t.S + 3) / 4;
  if (blocks == 0) return hipSuccess;
  if (blocks > INT32_MAX || !t.pos || !t.nrm || !t.dir_tab || !t.out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trace_samples, dim3((unsigned)blocks), dim3(256), 0, s, G, t);
  return hipGetLastError();
}

}  // namespace sopk
