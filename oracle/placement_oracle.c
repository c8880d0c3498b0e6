/*
 * placement_oracle.c - CPU oracle of probe placement and the probe/material losses (test
 * infrastructure only: the tests, the smoke check and the benchmark's CPU baseline use it;
 * the GPU library shares no code with it).
 *
 * Sec. 3.1.2, automatic placement of SOPs: farthest point sampling (FPS) over a surface
 * point cloud, then every chosen point offset along its normal. Reading of the silent
 * details: the first pick is a given start index; every later pick is the point whose
 * distance to the picks so far is largest, squared distances taken in IEEE single
 * precision as ((dx*dx + dy*dy) + dz*dz) with dx = x_j - x_q (so the integer decisions are
 * reproducible), ties to the lowest index; the probe is fmaf(offset, n, x) per component.
 *
 * Sec. 3.1.2, loss of the second step: L_lam = L1(R, 1) + L1(M, 0) (roughness towards 1,
 * metallic towards 0) and L_sops = L1(L_in, L_tr) + L1(O, O_tr) (probe textures towards
 * the traced ones). Reading: L1 is the mean absolute difference over the elements, and its
 * gradient takes sign(x - y) / n with sign(0) = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static float sqdist(const float* a, const float* b) {
  const float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return (dx * dx + dy * dy) + dz * dz;
}

/* FPS of P of the M points pts [M][3] starting at `start`: chosen [P] point indices. */
void orc_fps(const float* pts, long M, int P, long start, int32_t* chosen) {
  float* d = (float*)malloc(sizeof(float) * (size_t)(M > 0 ? M : 1));
  for (long j = 0; j < M; ++j) d[j] = INFINITY;
  long q = start;
  for (int k = 0; k < P; ++k) {
    chosen[k] = (int32_t)q;
    long best = 0;
    float bd = -1.0f;
    for (long j = 0; j < M; ++j) {
      const float s = sqdist(pts + 3 * j, pts + 3 * q);
      if (s < d[j]) d[j] = s;
      if (d[j] > bd) {          /* strict: the lowest index keeps a tie */
        bd = d[j];
        best = j;
      }
    }
    q = best;
  }
  free(d);
}

/* Probe positions of the chosen points: out [P][3] = fmaf(offset, n, x) per component. */
void orc_place(const float* pts, const float* normals, const int32_t* chosen, int P,
               float offset, float* out) {
  for (int k = 0; k < P; ++k)
    for (int c = 0; c < 3; ++c)
      out[3 * k + c] = fmaf(offset, normals[3 * (size_t)chosen[k] + c], pts[3 * (size_t)chosen[k] + c]);
}

static double sgn0(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

/* L_sops over T texels of (R, G, B, O): loss[0] = L1(L_in, L_tr) (mean over 3T values),
 * loss[1] = L1(O, O_tr) (mean over T); grad [T][4] (may be NULL) = d(loss[0] + loss[1]) /
 * d tex. */
void orc_sops_loss(const float* tex, const float* target, long T, double loss[2],
                   double* grad) {
  double a = 0.0, b = 0.0;
  for (long t = 0; t < T; ++t) {
    for (int c = 0; c < 4; ++c) {
      const double diff = (double)tex[4 * t + c] - (double)target[4 * t + c];
      if (c < 3) a += fabs(diff); else b += fabs(diff);
      if (grad) grad[4 * t + c] = sgn0(diff) / (c < 3 ? 3.0 * (double)T : (double)T);
    }
  }
  loss[0] = T > 0 ? a / (3.0 * (double)T) : 0.0;
  loss[1] = T > 0 ? b / (double)T : 0.0;
}

/* L_lam over N points: loss[0] = L1(R, 1), loss[1] = L1(M, 0); g_rough, g_metal [N] (may be
 * NULL) the gradients of loss[0] + loss[1]. */
void orc_lam_loss(const float* rough, const float* metal, long N, double loss[2],
                  double* g_rough, double* g_metal) {
  double a = 0.0, b = 0.0;
  for (long i = 0; i < N; ++i) {
    const double dr = (double)rough[i] - 1.0, dm = (double)metal[i];
    a += fabs(dr);
    b += fabs(dm);
    if (g_rough) g_rough[i] = sgn0(dr) / (double)N;
    if (g_metal) g_metal[i] = sgn0(dm) / (double)N;
  }
  loss[0] = N > 0 ? a / (double)N : 0.0;
  loss[1] = N > 0 ? b / (double)N : 0.0;
}
