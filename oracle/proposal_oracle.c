/*
 * proposal_oracle.c - plain FP64 reference of the learned direction proposal that extends
 * the SOP shading step of ComGS (arXiv 2510.07729). The paper estimates the rendering
 * equation with a fixed Hammersley set (Sec. 3.1.2, Eq. 7); this extension replaces the
 * fixed set by directions drawn from a small network's distribution over hemispherical
 * octahedral bins and weights each sample by its density (importance sampling of Eq. 7),
 * and trains that network on integrand samples the shading step produces.
 *
 * TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU baseline of the benchmark
 * use it to check the GPU library; no product code path calls it, and it shares no source
 * with the GPU library.
 *
 * Readings (the paper does not describe this extension; each choice is stated here):
 *  - features: 16-frequency sinusoidal encoding of 10 scalars (position mapped to [-1,1]
 *    by the scene bounds, normal, view direction, roughness), frequency f_l = 2^(l/2);
 *  - network: ReLU MLP 320 -> 64 -> 64 -> 256, softmax over 16x16 bins; BF16 weights,
 *    features and hidden activations, FP32 (here FP64) accumulation;
 *  - bins: hemispherical octahedral map of the local frame, (u,v) = (x+y, x-y)/(|x|+|y|+z),
 *    16x16 cells over [-1,1]^2, density constant in (u,v) inside a cell;
 *  - defensive mixture with the uniform-bin distribution: q_b = (1-eps) p_b + eps/256,
 *    quantised to 24-bit integer masses so that the bin draws are exact integer decisions;
 *  - stratified draws: sample j takes the j-th of S equal slices of the integer mass line,
 *    its position inside the bin's cell follows its place on the bin's stretch of that line
 *    (u) and a per-point rotated radical inverse of j (v);
 *  - training target of a point: the luminance of f L_i cos integrated over each bin,
 *    estimated with samples placed uniformly in every bin; loss = cross entropy.
 * Build: compiled with sop_oracle.c (gcc -O2 -ffp-contract=off -fopenmp -shared).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PR_PI 3.14159265358979323846
#define PR_FREQS 16
#define PR_SCALARS 10
#define PR_IN 320
#define PR_H 64
#define PR_BINS 256
#define PR_SIDE 16
/* parameter blob: W1 [320][64], b1 [64], W2 [64][64], b2 [64], W3 [64][256], b3 [256] */
#define PR_OFF_W1 0
#define PR_OFF_B1 (PR_OFF_W1 + PR_IN * PR_H)
#define PR_OFF_W2 (PR_OFF_B1 + PR_H)
#define PR_OFF_B2 (PR_OFF_W2 + PR_H * PR_H)
#define PR_OFF_W3 (PR_OFF_B2 + PR_H)
#define PR_OFF_B3 (PR_OFF_W3 + PR_H * PR_BINS)
#define PR_PARAMS (PR_OFF_B3 + PR_BINS)

/* from sop_oracle.c */
uint32_t orc_pcg_hash(uint32_t v);
uint32_t orc_bitreverse32(uint32_t x);
void orc_frame(const double n[3], double t[3], double b[3]);
void orc_env_fetch_any(const double* env, int H, int W, int oct, const double w[3],
                       double out[3]);
void orc_interp(const double* tex, int R, const int32_t* nb_idx, const double* nb_w, int K,
                const double w[3], double Lin[3], double* O);
void orc_brdf(const double n[3], const double v[3], const double l[3], const double a[3],
              double r, double m, double f[3]);

int orc_mlp_param_count(void) { return PR_PARAMS; }

/* ------------------------------------------------------------------------------------
 * bfloat16 round to nearest, ties to even (8 significant bits, FP32 exponent range)
 * ----------------------------------------------------------------------------------*/
double orc_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  double m = frexp(x, &e);              /* x = m 2^e, 0.5 <= |m| < 1 */
  if (e - 1 < -126)                     /* below the normal range: fixed quantum 2^-133 */
    return ldexp(rint(ldexp(x, 133)), -133);
  return ldexp(rint(ldexp(m, 8)), e - 8);   /* rint rounds half to even */
}

static double rnd(double x, int emu) { return emu ? orc_bf16(x) : x; }

/* ------------------------------------------------------------------------------------
 * Features: gamma(x) = (sin(f_l pi x), cos(f_l pi x)), l = 0..15, f_l = 2^(l/2), for the
 * scalars (p_hat, n, v, r); feature 32 c + 2 l is the sine, 32 c + 2 l + 1 the cosine.
 * ----------------------------------------------------------------------------------*/
void orc_pe_features(const double pos[3], const double n[3], const double v[3], double r,
                     const double lo[3], const double hi[3], double feat[PR_IN]) {
  double x[PR_SCALARS];
  for (int c = 0; c < 3; ++c) {
    x[c] = 2.0 * (pos[c] - lo[c]) / (hi[c] - lo[c]) - 1.0;
    x[3 + c] = n[c];
    x[6 + c] = v[c];
  }
  x[9] = r;
  for (int c = 0; c < PR_SCALARS; ++c)
    for (int l = 0; l < PR_FREQS; ++l) {
      double arg = pow(2.0, 0.5 * l) * PR_PI * x[c];
      feat[32 * c + 2 * l] = sin(arg);
      feat[32 * c + 2 * l + 1] = cos(arg);
    }
}

/* ------------------------------------------------------------------------------------
 * Network forward for one feature vector. emu = 1 rounds features, weights and hidden
 * activations to bfloat16 (the GPU's operand precision); sums are exact-order FP64.
 * Outputs (each optional): a0 rounded features, z1/h1, z2/h2 pre- and post-activation,
 * z3 logits, q softmax.
 * ----------------------------------------------------------------------------------*/
void orc_mlp_forward(const double* P, const double feat[PR_IN], int emu, double* a0_out,
                     double* z1_out, double* h1_out, double* z2_out, double* h2_out,
                     double* z3_out, double* q_out) {
  double a0[PR_IN], z1[PR_H], h1[PR_H], z2[PR_H], h2[PR_H], z3[PR_BINS], q[PR_BINS];
  for (int k = 0; k < PR_IN; ++k) a0[k] = rnd(feat[k], emu);
  for (int o = 0; o < PR_H; ++o) {
    double s = 0.0;
    for (int k = 0; k < PR_IN; ++k) s += a0[k] * rnd(P[PR_OFF_W1 + k * PR_H + o], emu);
    z1[o] = s + P[PR_OFF_B1 + o];
    h1[o] = rnd(z1[o] > 0.0 ? z1[o] : 0.0, emu);
  }
  for (int o = 0; o < PR_H; ++o) {
    double s = 0.0;
    for (int k = 0; k < PR_H; ++k) s += h1[k] * rnd(P[PR_OFF_W2 + k * PR_H + o], emu);
    z2[o] = s + P[PR_OFF_B2 + o];
    h2[o] = rnd(z2[o] > 0.0 ? z2[o] : 0.0, emu);
  }
  double mx = -HUGE_VAL;
  for (int o = 0; o < PR_BINS; ++o) {
    double s = 0.0;
    for (int k = 0; k < PR_H; ++k) s += h2[k] * rnd(P[PR_OFF_W3 + k * PR_BINS + o], emu);
    z3[o] = s + P[PR_OFF_B3 + o];
    if (z3[o] > mx) mx = z3[o];
  }
  double sum = 0.0;
  for (int o = 0; o < PR_BINS; ++o) sum += exp(z3[o] - mx);
  for (int o = 0; o < PR_BINS; ++o) q[o] = exp(z3[o] - mx) / sum;
  if (a0_out) memcpy(a0_out, a0, sizeof(a0));
  if (z1_out) memcpy(z1_out, z1, sizeof(z1));
  if (h1_out) memcpy(h1_out, h1, sizeof(h1));
  if (z2_out) memcpy(z2_out, z2, sizeof(z2));
  if (h2_out) memcpy(h2_out, h2, sizeof(h2));
  if (z3_out) memcpy(z3_out, z3, sizeof(z3));
  if (q_out) memcpy(q_out, q, sizeof(q));
}

static void point_features(long i, const double* pos, const double* normal,
                           const double* view, const double* rough, const double lo[3],
                           const double hi[3], double feat[PR_IN]) {
  orc_pe_features(pos + 3 * i, normal + 3 * i, view + 3 * i, rough[i], lo, hi, feat);
}

/* Proposal of N points: probs [N][256] (and logits [N][256] if not NULL). */
void orc_mlp_infer(const double* P, long N, const double* pos, const double* normal,
                   const double* view, const double* rough, const double lo[3],
                   const double hi[3], int emu, double* logits, double* probs) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double feat[PR_IN];
    point_features(i, pos, normal, view, rough, lo, hi, feat);
    orc_mlp_forward(P, feat, emu, NULL, NULL, NULL, NULL, NULL,
                    logits ? logits + PR_BINS * i : NULL, probs ? probs + PR_BINS * i : NULL);
  }
}

/* ------------------------------------------------------------------------------------
 * Cross-entropy loss of a batch and its gradient (chain rule through softmax, the three
 * affine maps and the ReLUs). Targets are raw bin masses T [B][256]; each row is
 * normalised (a row summing to <= 0 means the uniform distribution). loss = mean over the
 * batch of -sum_b t_b log q_b. With emu = 1 the backward operands are rounded to bfloat16
 * where the GPU rounds them: the output-side gradients dz (before they meet a weight or an
 * activation) and the weights; bias gradients use the unrounded dz.
 * mass (optional, [PR_PARAMS]) receives the sum of |terms| of every gradient entry: the
 * same chain rule with every factor replaced by its absolute value and q_b - t_b by
 * q_b + t_b, the scale that bounds the rounding of the sum whatever cancels inside it. A
 * pre-activation within 1e-5 of its own sum of |terms| of zero may fall on either side of
 * the ReLU's kink under another rounding order, so its path counts in the mass either way.
 * ----------------------------------------------------------------------------------*/
void orc_mlp_loss_grad(const double* P, long B, const double* pos, const double* normal,
                       const double* view, const double* rough, const double lo[3],
                       const double hi[3], const double* T, int emu, double* grad,
                       double* loss_out, double* mass) {
  memset(grad, 0, sizeof(double) * PR_PARAMS);
  if (mass) memset(mass, 0, sizeof(double) * PR_PARAMS);
  double loss = 0.0;
  for (long i = 0; i < B; ++i) {
    double feat[PR_IN], a0[PR_IN], z1[PR_H], h1[PR_H], z2[PR_H], h2[PR_H], z3[PR_BINS],
        q[PR_BINS];
    point_features(i, pos, normal, view, rough, lo, hi, feat);
    orc_mlp_forward(P, feat, emu, a0, z1, h1, z2, h2, z3, q);
    double tsum = 0.0, t[PR_BINS];
    for (int b = 0; b < PR_BINS; ++b) tsum += T[PR_BINS * i + b];
    for (int b = 0; b < PR_BINS; ++b) t[b] = tsum > 0.0 ? T[PR_BINS * i + b] / tsum : 1.0 / PR_BINS;
    /* loss with log q = z3 - logsumexp(z3) */
    double mx = -HUGE_VAL, se = 0.0;
    for (int b = 0; b < PR_BINS; ++b) if (z3[b] > mx) mx = z3[b];
    for (int b = 0; b < PR_BINS; ++b) se += exp(z3[b] - mx);
    double lse = mx + log(se);
    for (int b = 0; b < PR_BINS; ++b) loss -= t[b] * (z3[b] - lse) / (double)B;

    double dz3[PR_BINS], dz3r[PR_BINS], m3[PR_BINS];
    for (int b = 0; b < PR_BINS; ++b) {
      dz3[b] = (q[b] - t[b]) / (double)B;
      dz3r[b] = rnd(dz3[b], emu);
      m3[b] = (q[b] + t[b]) / (double)B;
    }
    double dh2[PR_H] = {0}, mh2[PR_H] = {0};
    for (int k = 0; k < PR_H; ++k)
      for (int o = 0; o < PR_BINS; ++o) {
        const double wr = rnd(P[PR_OFF_W3 + k * PR_BINS + o], emu);
        grad[PR_OFF_W3 + k * PR_BINS + o] += h2[k] * dz3r[o];
        dh2[k] += wr * dz3r[o];
        if (mass) {
          mass[PR_OFF_W3 + k * PR_BINS + o] += fabs(h2[k]) * m3[o];
          mh2[k] += fabs(wr) * m3[o];
        }
      }
    for (int o = 0; o < PR_BINS; ++o) {
      grad[PR_OFF_B3 + o] += dz3[o];
      if (mass) mass[PR_OFF_B3 + o] += m3[o];
    }

    double dz2[PR_H], dz2r[PR_H], m2[PR_H];
    for (int k = 0; k < PR_H; ++k) {
      dz2[k] = z2[k] > 0.0 ? dh2[k] : 0.0;
      dz2r[k] = rnd(dz2[k], emu);
      m2[k] = 0.0;
      if (mass) {
        double zm = fabs(P[PR_OFF_B2 + k]);
        for (int i2 = 0; i2 < PR_H; ++i2)
          zm += fabs(h1[i2] * rnd(P[PR_OFF_W2 + i2 * PR_H + k], emu));
        m2[k] = (z2[k] > 0.0 || fabs(z2[k]) <= 1e-5 * zm) ? mh2[k] : 0.0;
      }
    }
    double dh1[PR_H] = {0}, mh1[PR_H] = {0};
    for (int k = 0; k < PR_H; ++k)
      for (int o = 0; o < PR_H; ++o) {
        const double wr = rnd(P[PR_OFF_W2 + k * PR_H + o], emu);
        grad[PR_OFF_W2 + k * PR_H + o] += h1[k] * dz2r[o];
        dh1[k] += wr * dz2r[o];
        if (mass) {
          mass[PR_OFF_W2 + k * PR_H + o] += fabs(h1[k]) * m2[o];
          mh1[k] += fabs(wr) * m2[o];
        }
      }
    for (int o = 0; o < PR_H; ++o) {
      grad[PR_OFF_B2 + o] += dz2[o];
      if (mass) mass[PR_OFF_B2 + o] += m2[o];
    }

    double dz1[PR_H], dz1r[PR_H], m1[PR_H];
    for (int k = 0; k < PR_H; ++k) {
      dz1[k] = z1[k] > 0.0 ? dh1[k] : 0.0;
      dz1r[k] = rnd(dz1[k], emu);
      m1[k] = 0.0;
      if (mass) {
        double zm = fabs(P[PR_OFF_B1 + k]);
        for (int i2 = 0; i2 < PR_IN; ++i2)
          zm += fabs(a0[i2] * rnd(P[PR_OFF_W1 + i2 * PR_H + k], emu));
        m1[k] = (z1[k] > 0.0 || fabs(z1[k]) <= 1e-5 * zm) ? mh1[k] : 0.0;
      }
    }
    for (int k = 0; k < PR_IN; ++k)
      for (int o = 0; o < PR_H; ++o) {
        grad[PR_OFF_W1 + k * PR_H + o] += a0[k] * dz1r[o];
        if (mass) mass[PR_OFF_W1 + k * PR_H + o] += fabs(a0[k]) * m1[o];
      }
    for (int o = 0; o < PR_H; ++o) {
      grad[PR_OFF_B1 + o] += dz1[o];
      if (mass) mass[PR_OFF_B1 + o] += m1[o];
    }
  }
  *loss_out = loss;
}

/* Adam (Kingma & Ba 2015) with bias correction; step counts from 1. */
void orc_adam(long n, double* p, double* m, double* v, const double* g, double lr,
              double beta1, double beta2, double eps, int step) {
  double c1 = 1.0 - pow(beta1, step), c2 = 1.0 - pow(beta2, step);
  for (long i = 0; i < n; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}

/* ------------------------------------------------------------------------------------
 * Sampling over the hemispherical octahedral bins
 * ----------------------------------------------------------------------------------*/

/* counter-based random 24-bit integer of (seed, point, sample, stream) from the PCG hash */
uint32_t orc_hash24(uint32_t seed, uint32_t i, uint32_t j, uint32_t k) {
  return orc_pcg_hash(orc_pcg_hash(orc_pcg_hash(seed) ^ i) ^ (4u * j + k)) >> 8;
}

/* Integer bin masses of the defensive mixture, decided in IEEE single precision:
 * q_b = fma(1 - eps, clamp(p_b, 0, 1), eps/256), c_b = floor(q_b 2^24); all-zero masses
 * fall back to one unit per bin. Returns the total mass. */
uint64_t orc_prop_masses(const float* probs, float eps, uint32_t c[PR_BINS]) {
  float om = 1.0f - eps;
  float add = eps * (1.0f / 256.0f);
  uint64_t total = 0;
  for (int b = 0; b < PR_BINS; ++b) {
    float p = probs[b];
    if (!(p > 0.0f)) p = 0.0f;
    if (p > 1.0f) p = 1.0f;
    float qb = fmaf(om, p, add);
    c[b] = (uint32_t)floorf(qb * 16777216.0f);
    total += c[b];
  }
  if (total == 0) {
    for (int b = 0; b < PR_BINS; ++b) c[b] = 1;
    total = PR_BINS;
  }
  return total;
}

/* local direction at (u,v) in [-1,1]^2: returns the unit vector and l = |(px,py,z)|_2,
 * the inverse of the L1 norm of the unit vector */
static double bin_direction(double u, double v, double wl[3]) {
  double px = 0.5 * (u + v), py = 0.5 * (u - v);
  double z = 1.0 - fabs(px) - fabs(py);
  double l = sqrt(px * px + py * py + z * z);
  wl[0] = px / l; wl[1] = py / l; wl[2] = z / l;
  return l;
}

/* Bin of a local direction with z >= 0 (-1 if below the horizon), and its (u,v). */
int orc_prop_bin(const double wl[3], double uv[2]) {
  if (wl[2] < 0.0) return -1;
  double s = fabs(wl[0]) + fabs(wl[1]) + wl[2];
  double px = wl[0] / s, py = wl[1] / s;
  double u = px + py, v = px - py;
  int bu = (int)floor((u + 1.0) * 8.0), bv = (int)floor((v + 1.0) * 8.0);
  if (bu > 15) bu = 15;
  if (bv > 15) bv = 15;
  if (bu < 0) bu = 0;
  if (bv < 0) bv = 0;
  if (uv) { uv[0] = u; uv[1] = v; }
  return bv * PR_SIDE + bu;
}

/* Solid-angle density of the proposal at a local direction: (c_b/total) * 64 * 2 / s^3,
 * s the L1 norm of the unit direction (d omega = s^3 dA over the (px,py) diamond, and the
 * diamond has half the area of the (u,v) square). */
double orc_prop_pdf(const float* probs, float eps, const double wl[3]) {
  uint32_t c[PR_BINS];
  uint64_t total = orc_prop_masses(probs, eps, c);
  int b = orc_prop_bin(wl, NULL);
  if (b < 0) return 0.0;
  double s = fabs(wl[0]) + fabs(wl[1]) + fabs(wl[2]);
  return (double)c[b] / (double)total * 128.0 / (s * s * s);
}

/* Draw j of S for point i: bin, local direction and density. */
static int prop_draw(const uint32_t c[PR_BINS], uint64_t total, int S, uint32_t seed,
                     uint32_t i, int j, double wl[3], double* pdf) {
  uint32_t r = orc_hash24(seed, i, (uint32_t)j, 0);
  uint64_t x = ((uint64_t)j * total + (((uint64_t)r * total) >> 24)) / (uint64_t)S;
  /* bin with C_b <= x < C_b + c_b, C_b the mass of the bins before b */
  uint64_t cum = 0;
  int b = 0;
  for (; b < PR_BINS; ++b) {
    if (x < cum + c[b]) break;
    cum += c[b];
  }
  if (b == PR_BINS) b = PR_BINS - 1;   /* unreachable: x < total */
  /* position in the cell: u from the draw's place on the bin's stretch of the mass line,
     v from the radical inverse of j rotated per point (a Hammersley set warped through the
     bin distribution) */
  double xu = ((double)(x - cum) + 0.5) / (double)c[b];
  uint32_t v24 = ((orc_bitreverse32((uint32_t)j) >> 8) + orc_hash24(seed, i, 0, 2)) & 0xFFFFFFu;
  double xv = ((double)v24 + 0.5) / 16777216.0;
  double u = -1.0 + ((b % PR_SIDE) + xu) / 8.0, v = -1.0 + ((b / PR_SIDE) + xv) / 8.0;
  double l = bin_direction(u, v, wl);
  *pdf = (double)c[b] / (double)total * 128.0 * l * l * l;
  return b;
}

/* The draws of one point (for tests): bins [S], local directions [S][3], densities [S]. */
void orc_prop_samples(const float* probs, float eps, int S, uint32_t seed, uint32_t i,
                      int32_t* bins, double* wl, double* pdf) {
  uint32_t c[PR_BINS];
  uint64_t total = orc_prop_masses(probs, eps, c);
  for (int j = 0; j < S; ++j) bins[j] = prop_draw(c, total, S, seed, i, j, wl + 3 * j, pdf + j);
}

static void view_of(const double* view, const double* cam, long ppf, const double* pos, long i,
                    double v[3]) {
  if (view) {
    for (int c = 0; c < 3; ++c) v[c] = view[3 * i + c];
  } else {
    long f = i / ppf;
    for (int c = 0; c < 3; ++c) v[c] = cam[3 * f + c] - pos[3 * i + c];
    double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int c = 0; c < 3; ++c) v[c] /= l;
  }
}

/* f L_i cos at a world direction w with local cosine ct (Eq. 6 integrand with Eq. 8) */
static void integrand(const double n[3], const double v[3], const double a[3], double r,
                      double m, const double* tex, int R, const double* env, int H, int W,
                      int env_oct, const int32_t* nb_idx, const double* nb_w, int K,
                      const double w[3],
                      double ct, double out[3], double Li_out[3]) {
  double Lenv[3], Lin[3], O, f[3];
  orc_env_fetch_any(env, H, W, env_oct, w, Lenv);
  orc_interp(tex, R, nb_idx, nb_w, K, w, Lin, &O);
  orc_brdf(n, v, w, a, r, m, f);
  for (int c = 0; c < 3; ++c) {
    double Li = (1.0 - O) * Lenv[c] + Lin[c];
    out[c] = f[c] * Li * ct;
    if (Li_out) Li_out[c] = Li;
  }
}

/* ------------------------------------------------------------------------------------
 * Proposal shading: Lo = (1/S) sum_j f L_i cos / pdf(w_j) with the draws above; the local
 * direction is mapped to the world by the frame of the normal (same frame as the fixed
 * direction set). irr (optional) = (1/S) sum_j L_i cos / pdf.
 * ----------------------------------------------------------------------------------*/
void orc_prop_shade(long N, const double* pos, const double* normal, const double* view,
                    const double* cam, long ppf, const double* albedo, const double* rough,
                    const double* metal, const double* tex, int R, const double* env, int H,
                    int W, int env_oct, const int32_t* idx, const double* wts, int K,
                    const float* probs, float eps, int S, uint32_t seed, double* rgb,
                    double* irr) {
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < N; ++i) {
    double n[3], v[3], a[3], t[3], bt[3];
    for (int c = 0; c < 3; ++c) { n[c] = normal[3 * i + c]; a[c] = albedo[3 * i + c]; }
    view_of(view, cam, ppf, pos, i, v);
    orc_frame(n, t, bt);
    uint32_t cm[PR_BINS];
    uint64_t total = orc_prop_masses(probs + (size_t)PR_BINS * i, eps, cm);
    double acc[3] = {0, 0, 0}, acc_e[3] = {0, 0, 0};
    for (int j = 0; j < S; ++j) {
      double wl[3], pdf, w[3], y[3], Li[3];
      prop_draw(cm, total, S, seed, (uint32_t)i, j, wl, &pdf);
      for (int c = 0; c < 3; ++c) w[c] = t[c] * wl[0] + bt[c] * wl[1] + n[c] * wl[2];
      integrand(n, v, a, rough[i], metal[i], tex, R, env, H, W, env_oct, idx + (size_t)K * i,
                wts + (size_t)K * i, K, w, wl[2], y, Li);
      for (int c = 0; c < 3; ++c) {
        acc[c] += y[c] / pdf;
        acc_e[c] += Li[c] * wl[2] / pdf;
      }
    }
    for (int c = 0; c < 3; ++c) {
      rgb[3 * i + c] = acc[c] / S;
      if (irr) irr[3 * i + c] = acc_e[c] / S;
    }
  }
}

/* ------------------------------------------------------------------------------------
 * Training data: T[i][b] estimates the integral over bin b of lum(f L_i cos), with n_pb
 * samples placed in each bin's (u,v) cell: the (u,v) cell has area 1/64 and
 * d omega = s^3 / 2 dA_uv, so T_b = (1/(128 n_pb)) sum_k lum(y_k) s_k^3. Sample k of bin b
 * is sample j = b n_pb + k of the counter-based generator: u = (k + h(i,j,1))/n_pb inside
 * the cell, v = h(i,j,2) (with the half-unit offset of the 24-bit values).
 * lum = Rec. 709 weights.
 * ----------------------------------------------------------------------------------*/
void orc_dump_integrand(long N, const double* pos, const double* normal, const double* view,
                        const double* cam, long ppf, const double* albedo, const double* rough,
                        const double* metal, const double* tex, int R, const double* env,
                        int H, int W, int env_oct, const int32_t* idx, const double* wts, int K,
                        int n_pb, uint32_t seed, double* T) {
#pragma omp parallel for schedule(dynamic, 8)
  for (long i = 0; i < N; ++i) {
    double n[3], v[3], a[3], t[3], bt[3];
    for (int c = 0; c < 3; ++c) { n[c] = normal[3 * i + c]; a[c] = albedo[3 * i + c]; }
    view_of(view, cam, ppf, pos, i, v);
    orc_frame(n, t, bt);
    for (int b = 0; b < PR_BINS; ++b) {
      double acc = 0.0;
      for (int k = 0; k < n_pb; ++k) {
        uint32_t j = (uint32_t)(b * n_pb + k);
        /* u stratified over the n_pb draws of the bin, v random */
        double xu = (k + ((double)orc_hash24(seed, (uint32_t)i, j, 1) + 0.5) / 16777216.0) / n_pb;
        double xv = ((double)orc_hash24(seed, (uint32_t)i, j, 2) + 0.5) / 16777216.0;
        double u = -1.0 + ((b % PR_SIDE) + xu) / 8.0, vv = -1.0 + ((b / PR_SIDE) + xv) / 8.0;
        double wl[3], w[3], y[3];
        double l = bin_direction(u, vv, wl);
        for (int c = 0; c < 3; ++c) w[c] = t[c] * wl[0] + bt[c] * wl[1] + n[c] * wl[2];
        integrand(n, v, a, rough[i], metal[i], tex, R, env, H, W, env_oct, idx + (size_t)K * i,
                  wts + (size_t)K * i, K, w, wl[2], y, NULL);
        double lum = 0.2126 * y[0] + 0.7152 * y[1] + 0.0722 * y[2];
        acc += lum / (l * l * l);
      }
      T[(size_t)PR_BINS * i + b] = acc / (128.0 * n_pb);
    }
  }
}
