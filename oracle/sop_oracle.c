/*
 * sop_oracle.c - plain, slow, FP64 reference implementation of the SOP query-and-shade
 * path of ComGS (arXiv 2510.07729). TEST INFRASTRUCTURE ONLY: it exists so that tests, the
 * smoke check and the CPU baseline of the benchmark can check the GPU library against an
 * independent computation. It shares no source with the GPU library and no product code
 * path may call it.
 *
 * Every function follows the definition it cites, step by step, without blocking, fusion
 * or reordering. Floating point is double precision except where a result decides an
 * integer (the neighbour-search lattice), which is computed in IEEE single precision
 * exactly as the definition states. Build: gcc -O2 -ffp-contract=off -fopenmp -shared.
 *
 * Where the paper is silent the oracle takes these readings (each stated again below):
 *   octahedral map with +z at the centre, bilinear taps with mirror wrap at the border;
 *   equirectangular environment map, row 0 at +z; Duff et al. frame; Hammersley set with
 *   xi1 = (j+0.5)/S and an integer rotation of xi2; UE4-style GGX/Lambert BRDF;
 *   shading-point normal in the back-face weight; 3D-Gaussian response at the ray's
 *   point of maximum density for the bake.
 * The BRDF's exact match to the authors' simplified Disney model and the pcg hash's
 * match to its publication are parity unpinned (no values to compare against).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

int orc_version(void) { return 1; }

/* ------------------------------------------------------------------------------------
 * Integer helpers for the direction set (Sec. 3.1.2, Eq. 7: Hammersley point set).
 * ----------------------------------------------------------------------------------*/

/* bit reversal of a 32-bit word, written as the definition: bit b moves to bit 31-b */
uint32_t orc_bitreverse32(uint32_t x) {
  uint32_t r = 0;
  for (int b = 0; b < 32; ++b)
    if (x & (1u << b)) r |= 1u << (31 - b);
  return r;
}

/* PCG hash of Jarzynski & Olano, "Hash Functions for GPU Rendering" (JCGT 2020): one step
 * of the 32-bit PCG LCG followed by the RXS-M-XS output permutation. */
uint32_t orc_pcg_hash(uint32_t v) {
  uint32_t state = v * 747796405u + 2891336453u;
  uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

/* 24-bit rotation of the azimuth sample (reading: one rotation per call, or per point) */
uint32_t orc_rotation24(uint32_t seed, int per_point, uint32_t point_index) {
  uint32_t h = per_point ? orc_pcg_hash(seed ^ orc_pcg_hash(point_index)) : orc_pcg_hash(seed);
  return h >> 8;
}

/* ------------------------------------------------------------------------------------
 * Vector helpers
 * ----------------------------------------------------------------------------------*/
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void normalize3(double v[3]) {
  double l = sqrt(dot3(v, v));
  v[0] /= l; v[1] /= l; v[2] /= l;
}
static double sgn_nonneg(double x) { return x < 0.0 ? -1.0 : 1.0; }

/* ------------------------------------------------------------------------------------
 * Octahedral map (Sec. 3.1.2: probe textures are octahedral textures, Praun & Hoppe 2003;
 * unit-vector form of Cigolle et al. 2014). Reading: +z maps to the centre of the square,
 * the lower hemisphere is folded onto the corners, texel (i,j) has centre (i+0.5, j+0.5).
 * ----------------------------------------------------------------------------------*/
void orc_oct_encode(const double w[3], int R, double uv[2]) {
  double s = fabs(w[0]) + fabs(w[1]) + fabs(w[2]);
  double px = w[0] / s, py = w[1] / s;
  if (w[2] < 0.0) {
    double fx = (1.0 - fabs(py)) * sgn_nonneg(px);
    double fy = (1.0 - fabs(px)) * sgn_nonneg(py);
    px = fx; py = fy;
  }
  uv[0] = (px + 1.0) * 0.5 * R;
  uv[1] = (py + 1.0) * 0.5 * R;
}

void orc_oct_decode(double u, double v, int R, double w[3]) {
  double px = 2.0 * u / R - 1.0, py = 2.0 * v / R - 1.0;
  double z = 1.0 - fabs(px) - fabs(py);
  if (z < 0.0) {
    double fx = (1.0 - fabs(py)) * sgn_nonneg(px);
    double fy = (1.0 - fabs(px)) * sgn_nonneg(py);
    px = fx; py = fy;
  }
  w[0] = px; w[1] = py; w[2] = z;
  normalize3(w);
}

/* Mirror wrap of a texel index outside [0,R): across a vertical border the row is
 * mirrored, across a horizontal border the column is mirrored (the octahedral fold maps
 * border point (1,t) and (1,-t) to the same direction). */
static void oct_wrap(int i, int j, int R, int* oi, int* oj) {
  if (i < 0) { i = 0; j = R - 1 - j; }
  else if (i >= R) { i = R - 1; j = R - 1 - j; }
  if (j < 0) { j = 0; i = R - 1 - i; }
  else if (j >= R) { j = R - 1; i = R - 1 - i; }
  *oi = i; *oj = j;
}

/* The 4 bilinear taps of texture coordinate (u,v): flat texel offsets j*R+i and weights */
void orc_oct_taps(double u, double v, int R, int32_t tap[4], double wt[4]) {
  double cu = u - 0.5, cv = v - 0.5;
  int i0 = (int)floor(cu), j0 = (int)floor(cv);
  double fx = cu - i0, fy = cv - j0;
  int ii, jj;
  oct_wrap(i0, j0, R, &ii, &jj);         tap[0] = jj * R + ii; wt[0] = (1 - fx) * (1 - fy);
  oct_wrap(i0 + 1, j0, R, &ii, &jj);     tap[1] = jj * R + ii; wt[1] = fx * (1 - fy);
  oct_wrap(i0, j0 + 1, R, &ii, &jj);     tap[2] = jj * R + ii; wt[2] = (1 - fx) * fy;
  oct_wrap(i0 + 1, j0 + 1, R, &ii, &jj); tap[3] = jj * R + ii; wt[3] = fx * fy;
}

/* bilinear fetch of a C-channel octahedral texture [R][R][C] in direction w */
void orc_oct_fetch(const double* tex, int R, int C, const double w[3], double* out) {
  double uv[2];
  int32_t tap[4];
  double wt[4];
  orc_oct_encode(w, R, uv);
  orc_oct_taps(uv[0], uv[1], R, tap, wt);
  for (int c = 0; c < C; ++c) {
    double acc = 0.0;
    for (int t = 0; t < 4; ++t) acc += wt[t] * tex[(size_t)tap[t] * C + c];
    out[c] = acc;
  }
}

/* ------------------------------------------------------------------------------------
 * Environment map L_dir (Eq. 8), read as an equirectangular image [H][W][3]: polar angle
 * theta from +z along rows, azimuth phi = atan2(y,x) along columns, bilinear with texel
 * centres at +0.5, columns wrapping, rows clamped.
 * ----------------------------------------------------------------------------------*/
void orc_env_taps(const double w[3], int H, int W, int32_t tap[4], double wt[4]) {
  double theta = atan2(sqrt(w[0] * w[0] + w[1] * w[1]), w[2]);
  double phi = atan2(w[1], w[0]);
  double u = (phi + OR_PI) / (2.0 * OR_PI) * W;
  double v = theta / OR_PI * H;
  double cu = u - 0.5, cv = v - 0.5;
  int i0 = (int)floor(cu), j0 = (int)floor(cv);
  double fx = cu - i0, fy = cv - j0;
  int i1 = i0 + 1, j1 = j0 + 1;
  i0 = ((i0 % W) + W) % W;
  i1 = ((i1 % W) + W) % W;
  j0 = j0 < 0 ? 0 : (j0 > H - 1 ? H - 1 : j0);
  j1 = j1 < 0 ? 0 : (j1 > H - 1 ? H - 1 : j1);
  tap[0] = j0 * W + i0; wt[0] = (1 - fx) * (1 - fy);
  tap[1] = j0 * W + i1; wt[1] = fx * (1 - fy);
  tap[2] = j1 * W + i0; wt[2] = (1 - fx) * fy;
  tap[3] = j1 * W + i1; wt[3] = fx * fy;
}

void orc_env_fetch(const double* env, int H, int W, const double w[3], double out[3]) {
  int32_t tap[4];
  double wt[4];
  orc_env_taps(w, H, W, tap, wt);
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int t = 0; t < 4; ++t) acc += wt[t] * env[(size_t)tap[t] * 3 + c];
    out[c] = acc;
  }
}

/* Environment of a shading call: the equirectangular map above, or with oct an octahedral
 * map [W][W][3] (the paper's own representation of the lighting) read exactly like a probe
 * map: octahedral encode, bilinear taps with mirror wrap. */
void orc_env_taps_any(const double w[3], int H, int W, int oct, int32_t tap[4], double wt[4]) {
  if (!oct) {
    orc_env_taps(w, H, W, tap, wt);
    return;
  }
  double uv[2];
  orc_oct_encode(w, W, uv);
  orc_oct_taps(uv[0], uv[1], W, tap, wt);
}

void orc_env_fetch_any(const double* env, int H, int W, int oct, const double w[3],
                       double out[3]) {
  if (!oct) {
    orc_env_fetch(env, H, W, w, out);
    return;
  }
  orc_oct_fetch(env, W, 3, w, out);
}

/* ------------------------------------------------------------------------------------
 * Local frame around the normal: Duff et al., "Building an Orthonormal Basis, Revisited"
 * (JCGT 2017), branchless form with sign(0) = +1.
 * ----------------------------------------------------------------------------------*/
void orc_frame(const double n[3], double t[3], double b[3]) {
  double sg = n[2] < 0.0 ? -1.0 : 1.0;
  double a = -1.0 / (sg + n[2]);
  double bb = n[0] * n[1] * a;
  t[0] = 1.0 + sg * n[0] * n[0] * a; t[1] = sg * bb; t[2] = -sg * n[0];
  b[0] = bb; b[1] = sg + n[1] * n[1] * a; b[2] = -n[1];
}

/* Direction j of S (Eq. 7, Hammersley set on the hemisphere, uniform in solid angle):
 * cos(theta) = 1 - (j+0.5)/S, phi = 2*pi*u24/2^24 with
 * u24 = ((bitreverse32(j) >> 8) + rho24) mod 2^24. Returns cos(theta). */
double orc_direction(int j, int S, uint32_t rho24, const double n[3], double w[3]) {
  double xi1 = (j + 0.5) / S;
  double ct = 1.0 - xi1;
  double st = sqrt(1.0 - ct * ct);
  uint32_t u24 = ((orc_bitreverse32((uint32_t)j) >> 8) + rho24) & 0xFFFFFFu;
  double phi = 2.0 * OR_PI * (double)u24 / 16777216.0;
  double t[3], b[3];
  orc_frame(n, t, b);
  for (int c = 0; c < 3; ++c)
    w[c] = t[c] * st * cos(phi) + b[c] * st * sin(phi) + n[c] * ct;
  return ct;
}

/* Direction j of S of the cosine-weighted set: the same (xi1, phi) pairs as orc_direction,
 * xi1 = (j+0.5)/S read as the squared radius on the unit disk and lifted to the hemisphere
 * (Malley's method): sin(theta) = sqrt(xi1), cos(theta) = sqrt(1 - xi1), density
 * cos(theta)/pi. Returns cos(theta). */
double orc_direction_cos(int j, int S, uint32_t rho24, const double n[3], double w[3]) {
  double xi1 = (j + 0.5) / S;
  double st = sqrt(xi1);
  double ct = sqrt(1.0 - xi1);
  uint32_t u24 = ((orc_bitreverse32((uint32_t)j) >> 8) + rho24) & 0xFFFFFFu;
  double phi = 2.0 * OR_PI * (double)u24 / 16777216.0;
  double t[3], b[3];
  orc_frame(n, t, b);
  for (int c = 0; c < 3; ++c)
    w[c] = t[c] * st * cos(phi) + b[c] * st * sin(phi) + n[c] * ct;
  return ct;
}

/* ------------------------------------------------------------------------------------
 * BRDF (Eq. 6: the simplified Disney BRDF of Burley 2012; the form is not given, reading:
 * Lambert diffuse weighted by (1-m) plus the GGX microfacet lobe of Walter et al. 2007 with
 * Smith-Schlick geometry k = alpha/2 and Schlick Fresnel, alpha = r^2, as in Karis 2013).
 * ----------------------------------------------------------------------------------*/
double orc_ggx_D(double NoH, double alpha) {
  double a2 = alpha * alpha;
  double q = NoH * NoH * (a2 - 1.0) + 1.0;
  return a2 / (OR_PI * q * q);
}
double orc_smith_G1(double c, double kk) { return c / (c * (1.0 - kk) + kk); }
double orc_schlick_F(double F0, double VoH) {
  double x = 1.0 - VoH;
  return F0 + (1.0 - F0) * x * x * x * x * x;
}

/* f(w_i, w_o) per channel; NoV is clamped at 1e-4 */
void orc_brdf(const double n[3], const double v[3], const double l[3], const double a[3],
              double r, double m, double f[3]) {
  double NoL = dot3(n, l);
  double NoV = dot3(n, v);
  if (NoV < 1e-4) NoV = 1e-4;
  double h[3] = {l[0] + v[0], l[1] + v[1], l[2] + v[2]};
  normalize3(h);
  double NoH = dot3(n, h), VoH = dot3(v, h);
  double alpha = r * r;
  double D = orc_ggx_D(NoH, alpha);
  double G = orc_smith_G1(NoL, alpha / 2.0) * orc_smith_G1(NoV, alpha / 2.0);
  for (int c = 0; c < 3; ++c) {
    double F0 = 0.04 * (1.0 - m) + a[c] * m;
    double F = orc_schlick_F(F0, VoH);
    f[c] = (1.0 - m) * a[c] / OR_PI + D * F * G / (4.0 * NoL * NoV);
  }
}

/* ------------------------------------------------------------------------------------
 * Neighbour search (Sec. 3.1.2, efficient querying: FRNN then KNN; Eq. 10-11 weights).
 * Reading: positions are quantised to a 2^15 lattice in IEEE single precision,
 *   sc = 32768 / max_a (hi_a - lo_a),  q_a = clamp(floor((x_a - lo_a) * sc), 0, 32767),
 * the squared lattice distance is an exact integer, neighbours are the K smallest by
 * (d^2, probe index) among d^2 <= floor((radius*sc)^2); if the smallest d^2 is 0 only that
 * probe is used with weight 1; otherwise w = w_s * w_b normalised, w_s = 1/|d|,
 * w_b = 0.5*(1 + d/|d| . n) + 0.01, d = p_k - x, n the shading normal.
 * ----------------------------------------------------------------------------------*/
float orc_lattice_scale(const float lo[3], const float hi[3]) {
  float ext = hi[0] - lo[0];
  float e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
  if (e1 > ext) ext = e1;
  if (e2 > ext) ext = e2;
  return 32768.0f / ext;
}

void orc_quantize(const float x[3], const float lo[3], float sc, int32_t q[3]) {
  for (int a = 0; a < 3; ++a) {
    volatile float d = x[a] - lo[a];   /* single-precision subtract ...            */
    volatile float s = d * sc;         /* ... then single-precision multiply        */
    float f = floorf(s);
    int32_t v = (f >= 0.0f) ? (f > 32767.0f ? 32767 : (int32_t)f) : 0;
    q[a] = v;
  }
}

uint32_t orc_radius_limit(float radius, float sc) {
  double rq = (double)radius * (double)sc;
  double r2 = rq * rq;
  if (!(r2 < 4294967295.0)) return 0xFFFFFFFFu;
  return (uint32_t)floor(r2);
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* Brute force over all P probes for each of N points. idx[N*K] (-1 pads), w[N*K]. */
void orc_knn(const float* probe_pos, int P, const float lo[3], const float hi[3],
             const float* pts, const float* normals, long N, int K, float radius,
             int32_t* idx, double* w) {
  float sc = orc_lattice_scale(lo, hi);
  uint32_t lim = orc_radius_limit(radius, sc);
  int32_t* pq = (int32_t*)malloc(sizeof(int32_t) * 3 * (P > 0 ? P : 1));
  for (int p = 0; p < P; ++p) orc_quantize(probe_pos + 3 * p, lo, sc, pq + 3 * p);
#pragma omp parallel
  {
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (P > 0 ? P : 1));
#pragma omp for schedule(static)
    for (long i = 0; i < N; ++i) {
      int32_t xq[3];
      orc_quantize(pts + 3 * i, lo, sc, xq);
      int nk = 0;
      for (int p = 0; p < P; ++p) {
        uint64_t d2 = 0;
        for (int a = 0; a < 3; ++a) {
          int64_t d = (int64_t)pq[3 * p + a] - xq[a];
          d2 += (uint64_t)(d * d);
        }
        if (d2 <= lim) keys[nk++] = (d2 << 32) | (uint32_t)p;
      }
      qsort(keys, nk, sizeof(uint64_t), cmp_u64);
      int kk = nk < K ? nk : K;
      for (int s = 0; s < K; ++s) { idx[i * K + s] = -1; w[i * K + s] = 0.0; }
      if (kk == 0) continue;
      if ((keys[0] >> 32) == 0) {           /* exact-hit rule */
        idx[i * K] = (int32_t)(keys[0] & 0xFFFFFFFFu);
        w[i * K] = 1.0;
        continue;
      }
      double sum = 0.0;
      for (int s = 0; s < kk; ++s) {
        int p = (int)(keys[s] & 0xFFFFFFFFu);
        double d[3], n[3];
        for (int a = 0; a < 3; ++a) {
          d[a] = (double)probe_pos[3 * p + a] - (double)pts[3 * i + a];
          n[a] = normals[3 * i + a];
        }
        double len = sqrt(dot3(d, d));
        double ws = 1.0 / len;
        double wb = 0.5 * (1.0 + dot3(d, n) / len) + 0.01;
        idx[i * K + s] = p;
        w[i * K + s] = ws * wb;
        sum += ws * wb;
      }
      for (int s = 0; s < kk; ++s) w[i * K + s] /= sum;
    }
    free(keys);
  }
  free(pq);
}

/* ------------------------------------------------------------------------------------
 * Eq. 9 interpolation: the same world direction indexes every neighbour's texture
 * (reading: no parallax correction). tex is [P][R][R][4] (R,G,B,O) in double.
 * ----------------------------------------------------------------------------------*/
void orc_interp(const double* tex, int R, const int32_t* nb_idx, const double* nb_w, int K,
                const double w[3], double Lin[3], double* O) {
  double uv[2];
  int32_t tap[4];
  double wt[4];
  orc_oct_encode(w, R, uv);
  orc_oct_taps(uv[0], uv[1], R, tap, wt);
  Lin[0] = Lin[1] = Lin[2] = 0.0;
  *O = 0.0;
  for (int s = 0; s < K; ++s) {
    if (nb_idx[s] < 0) continue;
    const double* T = tex + (size_t)nb_idx[s] * R * R * 4;
    for (int t = 0; t < 4; ++t) {
      const double* tx = T + (size_t)tap[t] * 4;
      for (int c = 0; c < 3; ++c) Lin[c] += nb_w[s] * wt[t] * tx[c];
      *O += nb_w[s] * wt[t] * tx[3];
    }
  }
}

/* Eq. 9 for a list of world directions per point: dirs [N][D][3] -> Lin [N][D][3], O [N][D] */
void orc_query(const double* tex, int R, const int32_t* idx, const double* w, int K, long N,
               const double* dirs, int D, double* Lin, double* O) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i)
    for (int j = 0; j < D; ++j)
      orc_interp(tex, R, idx + i * K, w + i * K, K, dirs + (i * D + j) * 3,
                 Lin + (i * D + j) * 3, O + i * D + j);
}

/* ------------------------------------------------------------------------------------
 * Shading (Eq. 6-8): per point,
 *   rgb = (2*pi/S) sum_j f(w_j) L_i(w_j) cos(theta_j),  L_i = (1 - O) L_env + L_in,
 *   irr = (2*pi/S) sum_j L_i(w_j) cos(theta_j).
 * Points: pos/normal/view/albedo [N][3], rough/metal [N]; view may be NULL, then
 * v = normalize(cam[f] - x) with f = i / ppf.
 * ----------------------------------------------------------------------------------*/
typedef struct {
  long N;
  const double* pos; const double* normal; const double* view;
  const double* cam; long ppf;
  const double* albedo; const double* rough; const double* metal;
} orc_points;

static void point_view(const orc_points* p, long i, double v[3]) {
  if (p->view) {
    for (int c = 0; c < 3; ++c) v[c] = p->view[3 * i + c];
  } else {
    long f = i / p->ppf;
    for (int c = 0; c < 3; ++c) v[c] = p->cam[3 * f + c] - p->pos[3 * i + c];
    normalize3(v);
  }
}

/* One point's estimate of Eq. 7. cosine = 0: the uniform Hammersley set, rgb =
 * (2 pi/S) sum f L_i cos; cosine = 1: the cosine-weighted set, whose density cos/pi turns
 * the estimate into rgb = (pi/S) sum f L_i (irradiance (pi/S) sum L_i). */
static void shade_point(const orc_points* pts, long i, const double* tex, int R,
                        const double* env, int H, int W, int env_oct, const int32_t* nb_idx,
                        const double* nb_w, int K, int S, uint32_t seed, int per_point,
                        int cosine, double rgb[3], double irr[3]) {
  double n[3], v[3], a[3];
  for (int c = 0; c < 3; ++c) { n[c] = pts->normal[3 * i + c]; a[c] = pts->albedo[3 * i + c]; }
  point_view(pts, i, v);
  double r = pts->rough[i], m = pts->metal[i];
  uint32_t rho = orc_rotation24(seed, per_point, (uint32_t)i);
  double acc[3] = {0, 0, 0}, acc_e[3] = {0, 0, 0};
  for (int j = 0; j < S; ++j) {
    double w[3];
    double ct = cosine ? orc_direction_cos(j, S, rho, n, w) : orc_direction(j, S, rho, n, w);
    double Lenv[3], Lin[3], O, f[3];
    orc_env_fetch_any(env, H, W, env_oct, w, Lenv);
    orc_interp(tex, R, nb_idx, nb_w, K, w, Lin, &O);
    orc_brdf(n, v, w, a, r, m, f);
    for (int c = 0; c < 3; ++c) {
      double Li = (1.0 - O) * Lenv[c] + Lin[c];
      acc[c] += cosine ? f[c] * Li : f[c] * Li * ct;
      acc_e[c] += cosine ? Li : Li * ct;
    }
  }
  const double scale = cosine ? OR_PI / S : 2.0 * OR_PI / S;
  for (int c = 0; c < 3; ++c) {
    rgb[c] = scale * acc[c];
    if (irr) irr[c] = scale * acc_e[c];
  }
}

void orc_shade(long N, const double* pos, const double* normal, const double* view,
               const double* cam, long ppf, const double* albedo, const double* rough,
               const double* metal, const double* tex, int R, const double* env, int H, int W,
               int env_oct, const int32_t* idx, const double* w, int K, int S, uint32_t seed,
               int per_point, double* rgb, double* irr) {
  orc_points p = {N, pos, normal, view, cam, ppf, albedo, rough, metal};
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < N; ++i)
    shade_point(&p, i, tex, R, env, H, W, env_oct, idx + i * K, w + i * K, K, S, seed, per_point,
                0, rgb + 3 * i, irr ? irr + 3 * i : NULL);
}

/* orc_shade with the cosine-weighted direction set (orc_direction_cos). */
void orc_shade_cosine(long N, const double* pos, const double* normal, const double* view,
                      const double* cam, long ppf, const double* albedo, const double* rough,
                      const double* metal, const double* tex, int R, const double* env, int H,
                      int W, int env_oct, const int32_t* idx, const double* w, int K, int S,
                      uint32_t seed, int per_point, double* rgb, double* irr) {
  orc_points p = {N, pos, normal, view, cam, ppf, albedo, rough, metal};
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < N; ++i)
    shade_point(&p, i, tex, R, env, H, W, env_oct, idx + i * K, w + i * K, K, S, seed, per_point,
                1, rgb + 3 * i, irr ? irr + 3 * i : NULL);
}

/* ------------------------------------------------------------------------------------
 * Adjoint of orc_shade for an upstream gradient g[N][3] (the gradient path through the
 * shading step implied by the learnable materials, environment map and probe textures of
 * Sec. 4.1; the derivation is the chain rule on the definitions above).
 *   d rgb_c / d a_c  = (2pi/S) sum_j L_i,c cos [ (1-m)/pi + D G/(4 NoL NoV) m (1-(1-VoH)^5) ]
 *   d rgb_c / d m    = (2pi/S) sum_j L_i,c cos [ -a_c/pi + D G/(4 NoL NoV)(a_c-0.04)(1-(1-VoH)^5) ]
 *   d rgb_c / d r    = (2pi/S) sum_j L_i,c cos F_c/(4 NoL NoV) (dD/dalpha G + D dG/dalpha) 2r
 *   d rgb_c / d Lin_k[t,c] = (2pi/S) f_c cos w_k b_t
 *   d rgb_c / d O_k[t]     = -(2pi/S) f_c cos Lenv_c w_k b_t
 *   d rgb_c / d env[t',c]  = (2pi/S) f_c cos (1-O) b'_t'
 * Per-point outputs are overwritten; g_tex [P][R][R][4] and g_env [H][W][3] accumulate.
 * The optional m_* outputs receive the sum of |term| of each gradient entry: the natural
 * scale against which the rounding error of a sum of signed terms is measured.
 * ----------------------------------------------------------------------------------*/
void orc_shade_backward(long N, const double* pos, const double* normal, const double* view,
                        const double* cam, long ppf, const double* albedo, const double* rough,
                        const double* metal, const double* tex, int R, const double* env,
                        int H, int W, int env_oct, const int32_t* idx, const double* wts, int K,
                        int S, uint32_t seed, int per_point, const double* grad, double* g_albedo,
                        double* g_rough, double* g_metal, double* g_tex, double* g_env,
                        double* m_albedo, double* m_rough, double* m_metal, double* m_tex,
                        double* m_env) {
  orc_points pts = {N, pos, normal, view, cam, ppf, albedo, rough, metal};
  const double scale = 2.0 * OR_PI / S;
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < N; ++i) {
    double n[3], v[3], a[3], g[3];
    for (int c = 0; c < 3; ++c) {
      n[c] = normal[3 * i + c]; a[c] = albedo[3 * i + c]; g[c] = grad[3 * i + c];
    }
    point_view(&pts, i, v);
    double r = rough[i], m = metal[i];
    double alpha = r * r, kk = alpha / 2.0;
    uint32_t rho = orc_rotation24(seed, per_point, (uint32_t)i);
    const int32_t* nb_idx = idx + i * K;
    const double* nb_w = wts + i * K;
    double ga[3] = {0, 0, 0}, gr = 0.0, gm = 0.0;
    double ma[3] = {0, 0, 0}, mr = 0.0, mm = 0.0;   /* sums of |term| (summation scale) */
    for (int j = 0; j < S; ++j) {
      double w[3];
      double ct = orc_direction(j, S, rho, n, w);
      double Lenv[3], Lin[3], O, f[3];
      orc_env_fetch_any(env, H, W, env_oct, w, Lenv);
      orc_interp(tex, R, nb_idx, nb_w, K, w, Lin, &O);
      orc_brdf(n, v, w, a, r, m, f);
      /* BRDF pieces again for the material derivatives */
      double NoL = dot3(n, w);
      double NoV = dot3(n, v);
      if (NoV < 1e-4) NoV = 1e-4;
      double h[3] = {w[0] + v[0], w[1] + v[1], w[2] + v[2]};
      normalize3(h);
      double NoH = dot3(n, h), VoH = dot3(v, h);
      double D = orc_ggx_D(NoH, alpha);
      double G1L = orc_smith_G1(NoL, kk), G1V = orc_smith_G1(NoV, kk);
      double G = G1L * G1V;
      double q = NoH * NoH * (alpha * alpha - 1.0) + 1.0;
      double dD = 2.0 * alpha / (OR_PI * q * q) - 4.0 * alpha * alpha * alpha * NoH * NoH /
                  (OR_PI * q * q * q);
      double denL = NoL * (1.0 - kk) + kk, denV = NoV * (1.0 - kk) + kk;
      double dG1L = -NoL * (1.0 - NoL) / (denL * denL);   /* d G1 / d k */
      double dG1V = -NoV * (1.0 - NoV) / (denV * denV);
      double dG = 0.5 * (dG1L * G1V + G1L * dG1V);         /* d G / d alpha */
      double x5 = pow(1.0 - VoH, 5.0);
      double spec = 1.0 / (4.0 * NoL * NoV);
      double Li[3];
      for (int c = 0; c < 3; ++c) Li[c] = (1.0 - O) * Lenv[c] + Lin[c];
      for (int c = 0; c < 3; ++c) {
        double F0 = 0.04 * (1.0 - m) + a[c] * m;
        double F = F0 + (1.0 - F0) * x5;
        double common = g[c] * scale * Li[c] * ct;
        double ta = common * ((1.0 - m) / OR_PI + D * G * spec * m * (1.0 - x5));
        double tm = common * (-a[c] / OR_PI + D * G * spec * (a[c] - 0.04) * (1.0 - x5));
        double tr = common * F * spec * (dD * G + D * dG) * 2.0 * r;
        ga[c] += ta; gm += tm; gr += tr;
        ma[c] += fabs(ta); mm += fabs(tm); mr += fabs(tr);
      }
      /* texture adjoints */
      double gl[3], go = 0.0, go_mass = 0.0, ge[3];
      for (int c = 0; c < 3; ++c) {
        gl[c] = g[c] * scale * f[c] * ct;
        go -= g[c] * scale * f[c] * ct * Lenv[c];
        go_mass += fabs(g[c] * scale * f[c] * ct * Lenv[c]);
        ge[c] = g[c] * scale * f[c] * ct * (1.0 - O);
      }
      if (g_tex) {
        double uv[2];
        int32_t tap[4];
        double bt[4];
        orc_oct_encode(w, R, uv);
        orc_oct_taps(uv[0], uv[1], R, tap, bt);
        for (int s = 0; s < K; ++s) {
          if (nb_idx[s] < 0) continue;
          double* G_T = g_tex + (size_t)nb_idx[s] * R * R * 4;
          double* M_T = m_tex ? m_tex + (size_t)nb_idx[s] * R * R * 4 : NULL;
          for (int t = 0; t < 4; ++t) {
            double cw = nb_w[s] * bt[t];
            for (int c = 0; c < 3; ++c) {
#pragma omp atomic
              G_T[(size_t)tap[t] * 4 + c] += cw * gl[c];
              if (M_T) {
#pragma omp atomic
                M_T[(size_t)tap[t] * 4 + c] += fabs(cw * gl[c]);
              }
            }
#pragma omp atomic
            G_T[(size_t)tap[t] * 4 + 3] += cw * go;
            if (M_T) {
#pragma omp atomic
              M_T[(size_t)tap[t] * 4 + 3] += fabs(cw) * go_mass;
            }
          }
        }
      }
      if (g_env) {
        int32_t tap[4];
        double bt[4];
        orc_env_taps_any(w, H, W, env_oct, tap, bt);
        for (int t = 0; t < 4; ++t)
          for (int c = 0; c < 3; ++c) {
#pragma omp atomic
            g_env[(size_t)tap[t] * 3 + c] += bt[t] * ge[c];
            if (m_env) {
#pragma omp atomic
              m_env[(size_t)tap[t] * 3 + c] += fabs(bt[t] * ge[c]);
            }
          }
      }
    }
    if (g_albedo) for (int c = 0; c < 3; ++c) g_albedo[3 * i + c] = ga[c];
    if (g_rough) g_rough[i] = gr;
    if (g_metal) g_metal[i] = gm;
    if (m_albedo) for (int c = 0; c < 3; ++c) m_albedo[3 * i + c] = ma[c];
    if (m_rough) m_rough[i] = mr;
    if (m_metal) m_metal[i] = mm;
  }
}

/* ------------------------------------------------------------------------------------
 * Bake (Sec. 3.1.2: probe textures initialised by ray tracing the Gaussians; Sec. 4.1).
 * Reading: 3D Gaussians respond at the ray parameter of maximum density
 *   t* = (mu - o)^T S^-1 d / (d^T S^-1 d),  m^2 = (o + t* d - mu)^T S^-1 (o + t* d - mu),
 *   alpha = min(alpha_max, opacity * exp(-m^2 / 2)),  Sigma = R diag(s^2) R^T,
 * Gaussians with t* <= t_min or alpha < alpha_min are skipped, the rest are composited
 * front to back in ascending (t*, index) with the transmittance of Eq. 1; compositing
 * stops before a Gaussian that would take T (1 - alpha) below T_min.
 * A ray is flagged ambiguous when a decision lies within a float32 margin of its cut:
 * alpha within 2e-5 (relative) of alpha_min, t* within 1e-5 of t_min, T (1 - alpha)
 * within 1e-3 (relative) of T_min (each about ten times the float32 rounding of that
 * quantity), or two consecutive composited t* closer than 2.5e-7 t* (twice the float32
 * spacing at t*: a GPU that sorts by float32 keys can order them by index instead).
 * ----------------------------------------------------------------------------------*/
static void quat_to_rot(const double q_in[4], double Rm[3][3]) {
  double q[4] = {q_in[0], q_in[1], q_in[2], q_in[3]};
  double l = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int c = 0; c < 4; ++c) q[c] /= l;
  double w = q[0], x = q[1], y = q[2], z = q[3];
  Rm[0][0] = 1 - 2 * (y * y + z * z); Rm[0][1] = 2 * (x * y - w * z); Rm[0][2] = 2 * (x * z + w * y);
  Rm[1][0] = 2 * (x * y + w * z); Rm[1][1] = 1 - 2 * (x * x + z * z); Rm[1][2] = 2 * (y * z - w * x);
  Rm[2][0] = 2 * (x * z - w * y); Rm[2][1] = 2 * (y * z + w * x); Rm[2][2] = 1 - 2 * (x * x + y * y);
}

typedef struct { double t; int32_t idx; double alpha; } orc_hit;

static int cmp_hit(const void* a, const void* b) {
  const orc_hit* x = (const orc_hit*)a;
  const orc_hit* y = (const orc_hit*)b;
  if (x->t < y->t) return -1;
  if (x->t > y->t) return 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

/* Inverse covariance of every Gaussian: Sigma^-1 = R diag(1/s^2) R^T, [G][3][3] */
static double* gaussian_inverse_cov(int G, const double* scale, const double* rot) {
  double* SI = (double*)malloc(sizeof(double) * 9 * (G > 0 ? G : 1));
  for (int g = 0; g < G; ++g) {
    double Rm[3][3];
    quat_to_rot(rot + 4 * g, Rm);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          acc += Rm[r][k] * Rm[c][k] / (scale[3 * g + k] * scale[3 * g + k]);
        SI[9 * g + 3 * r + c] = acc;
      }
  }
  return SI;
}

static void mat3_vec(const double* M, const double x[3], double y[3]) {
  for (int r = 0; r < 3; ++r) y[r] = M[3 * r] * x[0] + M[3 * r + 1] * x[1] + M[3 * r + 2] * x[2];
}

/* one ray: out[0..2] = RGB, out[3] = O, out[4] = depth; returns the ambiguity flag */
static int trace_ray(int G, const double* mean, const double* SI, const double* opacity,
                     const double* color, const double o[3], const double d[3], double t_min,
                     double alpha_min, double alpha_max, double T_min, orc_hit* hits,
                     double out[5], int32_t* n_used) {
  int nh = 0;
  double first_near = HUGE_VAL;   /* smallest t* of a Gaussian whose acceptance is near a cut */
  for (int g = 0; g < G; ++g) {
    const double* M = SI + 9 * g;
    double mo[3] = {mean[3 * g] - o[0], mean[3 * g + 1] - o[1], mean[3 * g + 2] - o[2]};
    double Sd[3];
    mat3_vec(M, d, Sd);
    double t = dot3(mo, Sd) / dot3(d, Sd);
    double x[3] = {o[0] + t * d[0] - mean[3 * g], o[1] + t * d[1] - mean[3 * g + 1],
                   o[2] + t * d[2] - mean[3 * g + 2]};
    double Sx[3];
    mat3_vec(M, x, Sx);
    double m2 = dot3(x, Sx);
    double al = opacity[g] * exp(-0.5 * m2);
    if (al > alpha_max) al = alpha_max;
    /* acceptance is (t > t_min) and (alpha >= alpha_min); it can flip under float32
       rounding when one condition is near its cut and the other holds (or is near too) */
    int near_alpha = fabs(al - alpha_min) <= 2e-5 * alpha_min;
    int near_t = fabs(t - t_min) <= 1e-5;
    int flip = (near_t && al >= alpha_min * (1.0 - 2e-5)) ||
               (near_alpha && t > t_min - 1e-5);
    if (flip && t < first_near) first_near = t;
    if (t <= t_min || al < alpha_min) continue;
    hits[nh].t = t; hits[nh].idx = g; hits[nh].alpha = al;
    ++nh;
  }
  qsort(hits, nh, sizeof(orc_hit), cmp_hit);
  int amb = 0;
  double T = 1.0, C[3] = {0, 0, 0}, Dp = 0.0, Wt = 0.0, t_stop = HUGE_VAL;
  for (int s = 0; s < nh; ++s) {
    double al = hits[s].alpha;
    double Tn = T * (1.0 - al);
    if (fabs(Tn - T_min) <= 1e-3 * T_min) amb = 1;
    if (Tn < T_min) { t_stop = hits[s].t; break; }
    if (s > 0 && hits[s].t - hits[s - 1].t < 2.5e-7 * hits[s].t) amb = 1;
    int g = hits[s].idx;
    for (int c = 0; c < 3; ++c) C[c] += T * al * color[3 * g + c];
    Dp += T * al * hits[s].t;
    Wt += T * al;
    T = Tn;
  }
  if (first_near < t_stop) amb = 1;
  /* Gaussians the definition must resolve on this ray: every accepted one up to and
     including the one that ends the ray */
  if (n_used) {
    int used = 0;
    for (int s = 0; s < nh && hits[s].t <= t_stop; ++s) ++used;
    *n_used = used;
  }
  out[0] = C[0]; out[1] = C[1]; out[2] = C[2];
  out[3] = Wt;
  out[4] = Wt > 0.0 ? Dp / Wt : 0.0;
  return amb;
}

/* Traces n_rays rays given as (probe index, texel index) pairs; texel t = v*R + u of a
 * resolution-R map, direction = octahedral decode of the texel centre.
 * out [n_rays][5] = (R,G,B,O,depth), flags [n_rays] (1 = ambiguous), n_used [n_rays]
 * (optional, may be NULL): accepted Gaussians up to and including the one that ends the ray. */
void orc_bake_rays(int G, const double* mean, const double* scale, const double* rot,
                   const double* opacity, const double* color, const double* probe_pos,
                   int R, long n_rays, const int32_t* ray_probe, const int32_t* ray_texel,
                   double t_min, double alpha_min, double alpha_max, double T_min,
                   double* out, int32_t* flags, int32_t* n_used) {
  double* SI = gaussian_inverse_cov(G, scale, rot);
#pragma omp parallel
  {
    orc_hit* hits = (orc_hit*)malloc(sizeof(orc_hit) * (G > 0 ? G : 1));
#pragma omp for schedule(dynamic, 4)
    for (long r = 0; r < n_rays; ++r) {
      int p = ray_probe[r], t = ray_texel[r];
      double o[3] = {probe_pos[3 * p], probe_pos[3 * p + 1], probe_pos[3 * p + 2]};
      double d[3];
      orc_oct_decode((t % R) + 0.5, (t / R) + 0.5, R, d);
      flags[r] = trace_ray(G, mean, SI, opacity, color, o, d, t_min, alpha_min, alpha_max,
                           T_min, hits, out + 5 * r, n_used ? n_used + r : NULL);
    }
    free(hits);
  }
  free(SI);
}

/* ------------------------------------------------------------------------------------
 * Traced shading (the per-sample tracing that the probes stand in for, Sec. 3.1.2): the
 * estimate of orc_shade (Eq. 6-8 with the Hammersley set of Eq. 7) where O and L_in of
 * sample j come from a ray through the Gaussians instead of the probes. The ray of sample
 * j of point i starts at o = fmaf(offset, n, x) per component in float32 (x and n are the
 * float32 inputs) and runs along w_j; it is blended as a bake ray (trace_ray).
 * rgb [N][3]; irr [N][3], samples [N][S][4] (R,G,B,O) and ray_flags [N][S] (1 = the ray
 * is ambiguous, see trace_ray) may be NULL.
 * ----------------------------------------------------------------------------------*/
void orc_shade_traced(int G, const double* mean, const double* scale, const double* rot,
                      const double* opacity, const double* color, long N, const double* pos,
                      const double* normal, const double* view, const double* cam, long ppf,
                      const double* albedo, const double* rough, const double* metal,
                      const double* env, int H, int W, int env_oct, int S, uint32_t seed,
                      int per_point, float offset, double t_min, double alpha_min, double alpha_max,
                      double T_min, double* rgb, double* irr, double* samples,
                      int32_t* ray_flags) {
  orc_points p = {N, pos, normal, view, cam, ppf, albedo, rough, metal};
  double* SI = gaussian_inverse_cov(G, scale, rot);
#pragma omp parallel
  {
    orc_hit* hits = (orc_hit*)malloc(sizeof(orc_hit) * (G > 0 ? G : 1));
#pragma omp for schedule(dynamic, 1)
    for (long i = 0; i < N; ++i) {
      double n[3], v[3], a[3], o[3];
      for (int c = 0; c < 3; ++c) {
        n[c] = normal[3 * i + c];
        a[c] = albedo[3 * i + c];
        o[c] = (double)fmaf(offset, (float)n[c], (float)pos[3 * i + c]);
      }
      point_view(&p, i, v);
      double r = rough[i], m = metal[i];
      uint32_t rho = orc_rotation24(seed, per_point, (uint32_t)i);
      double acc[3] = {0, 0, 0}, acc_e[3] = {0, 0, 0};
      for (int j = 0; j < S; ++j) {
        double w[3], tr[5], Lenv[3], f[3];
        double ct = orc_direction(j, S, rho, n, w);
        int amb = trace_ray(G, mean, SI, opacity, color, o, w, t_min, alpha_min, alpha_max,
                            T_min, hits, tr, NULL);
        if (ray_flags) ray_flags[i * S + j] = amb;
        if (samples)
          for (int c = 0; c < 4; ++c) samples[(i * S + j) * 4 + c] = tr[c];
        orc_env_fetch_any(env, H, W, env_oct, w, Lenv);
        orc_brdf(n, v, w, a, r, m, f);
        for (int c = 0; c < 3; ++c) {
          double Li = (1.0 - tr[3]) * Lenv[c] + tr[c];
          acc[c] += f[c] * Li * ct;
          acc_e[c] += Li * ct;
        }
      }
      for (int c = 0; c < 3; ++c) {
        rgb[3 * i + c] = 2.0 * OR_PI / S * acc[c];
        if (irr) irr[3 * i + c] = 2.0 * OR_PI / S * acc_e[c];
      }
    }
    free(hits);
  }
  free(SI);
}
