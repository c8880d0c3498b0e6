/*
 * shadow_oracle.c - CPU FP64 oracle of the cast-shadow ratio (test infrastructure only: the
 * tests, the smoke check and the benchmark's CPU baseline use it; the GPU library shares no
 * code with it).
 *
 * ComGS Sec. 3.2 (occlusion caching) and Sec. 3.3 (rendering). For a Lambertian scene point
 * with normal n the shadow that a placed object casts is S = L_o' / L_o (Eq. 17), where
 *   L_o  = f_d * integral of L_i(w) (w.n)+ dw                (Eq. 15)
 *   L_o' = f_d * integral of L_i(w) (1 - O'(w)) (w.n)+ dw    (Eq. 16)
 * per colour channel (f_d cancels). O'(w) is the occlusion the object adds, read from the
 * probes of the shadow region as in Eq. 9 (channel 3 of their maps). L_i is an octahedral
 * environment map [R][R][3] (the paper's own representation of the estimated lighting),
 * read with bilinear filtering and mirror wrap exactly like the probe maps. Both integrals
 * are estimated with the same S samples:
 *   - Hammersley: the hemisphere set of the shading step (Eq. 7), density 1/(2 pi);
 *   - environment importance sampling (Eq. 18): texel t with probability m_t / C (integer
 *     masses from the texel intensities, orc_env_masses), the direction uniform in the
 *     texel's square of the octahedral map, and the density as Eq. 18 states it with its
 *     normalisation read as I_t / sum(I): pdf = (m_t / C) * R^2 / (4 pi), every texel being
 *     given the mean solid angle 4 pi / R^2 (the paper's "roughly uniform texel areas");
 *   - the same draws with their exact density instead: the octahedral square's area element
 *     is dA = dw / s^3 in the square's [-1,1]^2 coordinates (s = |x| + |y| + |z| of the unit
 *     direction: the central projection onto the octahedron face, then the projection of
 *     the face onto the square), so a draw uniform in its texel has
 *     pdf = (m_t / C) * (R^2 / 4) / s^3, and the estimate is unbiased.
 * Samples below the horizon add nothing to either sum. A channel with L_o = 0 has S = 1.
 *
 * The same draws estimate the object's relighting (Sec. 3.3: object relighting and shadow
 * computation are both accelerated by importance sampling with the density of Eq. 18):
 * orc_shade_envis is the shading estimate of Eq. 6-9 (the BRDF, L_i = (1 - O) L_env + L_in
 * from the probes) with these draws and this density in place of the Hammersley set.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define SH_PI 3.14159265358979323846
#define SH_MASS_BITS 14

uint32_t orc_hash24(uint32_t seed, uint32_t i, uint32_t j, uint32_t k);
void orc_brdf(const double n[3], const double v[3], const double l[3], const double a[3],
              double r, double m, double f[3]);
uint32_t orc_rotation24(uint32_t seed, int per_point, uint32_t point_index);
double orc_direction(int j, int S, uint32_t rho24, const double n[3], double w[3]);
void orc_oct_decode(double u, double v, int R, double w[3]);
void orc_oct_fetch(const double* tex, int R, int C, const double w[3], double* out);
void orc_interp(const double* tex, int R, const int32_t* nb_idx, const double* nb_w, int K,
                const double w[3], double Lin[3], double* O);

/* intensity of a texel in IEEE single precision: (r + g) + b, 0 unless positive */
static float texel_intensity(const float* e) {
  float I = (e[0] + e[1]) + e[2];
  return I > 0.0f ? I : 0.0f;
}

/* Integer masses of the environment texels, decided in IEEE single precision:
 * m_t = 1 + floor(I_t * (2^14 / I_max)) with one float32 division and one float32 product
 * (every texel keeps mass >= 1; with I_max = 0 every mass is 1). prefix [R*R + 1] receives
 * the exclusive prefix sums, prefix[R*R] = C, which is returned. */
uint64_t orc_env_masses(const float* env, int R, uint32_t* mass, uint64_t* prefix) {
  const int T = R * R;
  float imax = 0.0f;
  for (int t = 0; t < T; ++t) {
    float I = texel_intensity(env + 3 * t);
    if (I > imax) imax = I;
  }
  const float f = imax > 0.0f ? (float)(1 << SH_MASS_BITS) / imax : 0.0f;
  uint64_t c = 0;
  for (int t = 0; t < T; ++t) {
    float q = texel_intensity(env + 3 * t) * f;
    uint32_t m = 1u + (uint32_t)floorf(q);
    mass[t] = m;
    prefix[t] = c;
    c += m;
  }
  prefix[T] = c;
  return c;
}

/* Draw j of S for point i, stratified over the mass line: x = (j C + ((r C) >> 24)) / S in
 * integers with r = hash24(seed, i, j, 0); the texel t with prefix[t] <= x < prefix[t+1];
 * the position (col + xu, row + xv) in texel units with xu, xv = (hash24(seed, i, j, 1|2)
 * + 1/2) / 2^24; the direction is the octahedral decode of that position. Returns t and
 * the density: of Eq. 18, *pdf = (m_t / C) R^2 / (4 pi), or with exact != 0 the draw's own
 * density (m_t / C) (R^2 / 4) / s^3, s = |w_x| + |w_y| + |w_z|. */
int orc_env_draw(const uint32_t* mass, const uint64_t* prefix, int R, int S, int j,
                 uint32_t seed, uint32_t i, int exact, double w[3], double* pdf) {
  const int T = R * R;
  const uint64_t C = prefix[T];
  const uint64_t r = orc_hash24(seed, i, (uint32_t)j, 0);
  const uint64_t x = ((uint64_t)j * C + ((r * C) >> 24)) / (uint64_t)S;
  int lo = 0, hi = T;                      /* prefix[lo] <= x < prefix[hi] */
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (prefix[mid] <= x) lo = mid; else hi = mid;
  }
  const double xu = ((double)orc_hash24(seed, i, (uint32_t)j, 1) + 0.5) / 16777216.0;
  const double xv = ((double)orc_hash24(seed, i, (uint32_t)j, 2) + 0.5) / 16777216.0;
  orc_oct_decode((double)(lo % R) + xu, (double)(lo / R) + xv, R, w);
  if (exact) {
    const double sl = fabs(w[0]) + fabs(w[1]) + fabs(w[2]);
    *pdf = (double)mass[lo] / (double)C * ((double)T / 4.0) / (sl * sl * sl);
  } else {
    *pdf = (double)mass[lo] / (double)C * (double)T / (4.0 * SH_PI);
  }
  return lo;
}

/* Shadow ratio of N points. normal [N][3]; tex [P][Rp][Rp][4] probe maps (channel 3 = O');
 * idx/nbw [N][K] neighbours (Eq. 9-11); env [Re][Re][3] float32 (its intensities decide
 * the masses). sampler 0 = Hammersley, 1 = environment importance sampling with the
 * density of Eq. 18, 2 = the same draws with their exact density.
 * ratio [N][3]; irr [N][3] (may be NULL) = (1/S) sum E cos+ / pdf (L_o / f_d); texels
 * [N][S] (may be NULL) = the texel of each importance draw (-1 for Hammersley). ids [N]
 * (may be NULL: 0..N-1) are the point indices that key the draws and rotations, so that a
 * subset of a larger set of points can be evaluated with the indices it has there. */
void orc_shadow_ratio(long N, const double* normal, const double* tex, int Rp,
                      const int32_t* idx, const double* nbw, int K, const float* env, int Re,
                      int S, uint32_t seed, int per_point, int sampler, double* ratio,
                      double* irr, int32_t* texels, const uint32_t* ids) {
  const int T = Re * Re;
  double* env64 = (double*)malloc(sizeof(double) * 3 * (size_t)T);
  for (long q = 0; q < 3L * T; ++q) env64[q] = (double)env[q];
  uint32_t* mass = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)T);
  uint64_t* prefix = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)T + 1));
  orc_env_masses(env, Re, mass, prefix);
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < N; ++i) {
    const double n[3] = {normal[3 * i], normal[3 * i + 1], normal[3 * i + 2]};
    const uint32_t id = ids ? ids[i] : (uint32_t)i;
    const uint32_t rho = orc_rotation24(seed, per_point, id);
    double num[3] = {0, 0, 0}, den[3] = {0, 0, 0};
    for (int j = 0; j < S; ++j) {
      double w[3], ct, wt;
      if (sampler == 0) {
        ct = orc_direction(j, S, rho, n, w);
        wt = 2.0 * SH_PI;
        if (texels) texels[i * S + j] = -1;
      } else {
        double pdf;
        int t = orc_env_draw(mass, prefix, Re, S, j, seed, id, sampler == 2, w, &pdf);
        if (texels) texels[i * S + j] = t;
        ct = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
        wt = 1.0 / pdf;
      }
      if (!(ct > 0.0)) continue;
      double E[3], Lin[3], O;
      orc_oct_fetch(env64, Re, 3, w, E);
      orc_interp(tex, Rp, idx + i * K, nbw + i * K, K, w, Lin, &O);
      for (int c = 0; c < 3; ++c) {
        num[c] += E[c] * (1.0 - O) * ct * wt;
        den[c] += E[c] * ct * wt;
      }
    }
    for (int c = 0; c < 3; ++c) {
      ratio[3 * i + c] = den[c] != 0.0 ? num[c] / den[c] : 1.0;
      if (irr) irr[3 * i + c] = den[c] / S;
    }
  }
  free(prefix);
  free(mass);
  free(env64);
}

/* Object relighting with environment importance sampling (Sec. 3.3, Eq. 18): for point i
 * rgb_i = (1/S) sum_j f(w_j) L_i(w_j) (n . w_j)+ / pdf_j, with the draws w_j and densities
 * pdf_j of orc_env_draw on the octahedral environment env [Re][Re][3] (float32: its
 * intensities decide the masses), L_i = (1 - O) L_env + L_in (Eq. 8) with O and L_in from
 * the probe maps tex [P][R][R][4] and the neighbours idx/wts [N][K] (Eq. 9-11), L_env the
 * bilinear octahedral lookup, f the BRDF of the shading step (orc_brdf) for the view v
 * (view [N][3], or cam [F][3] with ppf points per frame when view is NULL). Draws below the
 * horizon add nothing. irr (may be NULL) = (1/S) sum_j L_i (n . w_j)+ / pdf_j; texels (may
 * be NULL) [N][S] receives the texel of every draw; ids (may be NULL: 0..N-1) key the
 * draws, so that a subset of a larger point set keeps its draws. exact != 0 weights every
 * draw by its exact density instead of that of Eq. 18 (orc_env_draw). */
void orc_shade_envis(long N, const double* pos, const double* normal, const double* view,
                     const double* cam, long ppf, const double* albedo, const double* rough,
                     const double* metal, const double* tex, int R, const int32_t* idx,
                     const double* wts, int K, const float* env, int Re, int S, uint32_t seed,
                     const uint32_t* ids, int exact, double* rgb, double* irr,
                     int32_t* texels) {
  const int T = Re * Re;
  double* env64 = (double*)malloc(sizeof(double) * 3 * (size_t)T);
  for (long q = 0; q < 3L * T; ++q) env64[q] = (double)env[q];
  uint32_t* mass = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)T);
  uint64_t* prefix = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)T + 1));
  orc_env_masses(env, Re, mass, prefix);
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < N; ++i) {
    const double n[3] = {normal[3 * i], normal[3 * i + 1], normal[3 * i + 2]};
    const double a[3] = {albedo[3 * i], albedo[3 * i + 1], albedo[3 * i + 2]};
    double v[3];
    if (view) {
      for (int c = 0; c < 3; ++c) v[c] = view[3 * i + c];
    } else {
      const long f = i / ppf;
      for (int c = 0; c < 3; ++c) v[c] = cam[3 * f + c] - pos[3 * i + c];
      const double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      for (int c = 0; c < 3; ++c) v[c] /= l;
    }
    const uint32_t id = ids ? ids[i] : (uint32_t)i;
    double acc[3] = {0, 0, 0}, acc_e[3] = {0, 0, 0};
    for (int j = 0; j < S; ++j) {
      double w[3], pdf;
      const int t = orc_env_draw(mass, prefix, Re, S, j, seed, id, exact, w, &pdf);
      if (texels) texels[i * S + j] = t;
      const double ct = w[0] * n[0] + w[1] * n[1] + w[2] * n[2];
      if (!(ct > 0.0)) continue;
      double E[3], Lin[3], O, f[3];
      orc_oct_fetch(env64, Re, 3, w, E);
      orc_interp(tex, R, idx + i * K, wts + i * K, K, w, Lin, &O);
      orc_brdf(n, v, w, a, rough[i], metal[i], f);
      for (int c = 0; c < 3; ++c) {
        const double Li = (1.0 - O) * E[c] + Lin[c];
        acc[c] += f[c] * Li * ct / pdf;
        acc_e[c] += Li * ct / pdf;
      }
    }
    for (int c = 0; c < 3; ++c) {
      rgb[3 * i + c] = acc[c] / S;
      if (irr) irr[3 * i + c] = acc_e[c] / S;
    }
  }
  free(prefix);
  free(mass);
  free(env64);
}
