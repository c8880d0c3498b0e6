/*
 * sop.h - C ABI of the Surface Octahedral Probe (SOP) query-and-shade library for
 *         AMD Instinct MI355X (gfx950).
 *
 * The library computes the deferred-shading step of ComGS (arXiv 2510.07729), Sec. 3.1.2
 * (material and lighting decomposition):
 *   - every shading point x evaluates the rendering equation (Eq. 6) by the Monte Carlo
 *     estimate of Eq. 7 over S_r Hammersley directions on its hemisphere;
 *   - incident light is the environment map attenuated by occlusion plus indirect light
 *     (Eq. 8);
 *   - occlusion O and indirect radiance L_in come from the octahedral textures of the K
 *     nearest surface octahedral probes, blended with spatial and back-face weights
 *     (Eq. 9-11, efficient querying through SOPs);
 *   - probe textures are initialised by tracing rays through the Gaussians (Sec. 3.1.2,
 *     paragraph introducing SOPs; Sec. 4.1 implementation details).
 * Two entry points go beyond the paper: the adjoint of the shading step
 * (sop_shade_backward) for gradient-based reconstruction (the learnable quantities of
 * Sec. 4.1), and a learned direction proposal (sop_proposal_*).
 *
 * Conventions shared by every entry point
 *   - Array pointers are DEVICE pointers owned by the caller unless a field says "host".
 *     Arrays are contiguous, row-major, 32-bit IEEE float unless a format field says
 *     otherwise, and 4-byte aligned (8-byte for half textures, 16-byte for f32 textures).
 *   - Every call is asynchronous and ordered on the HIP stream it is given; no call
 *     synchronises the host except sop_plan_create, sop_bake_plan_create and the
 *     sop_*_check helpers, which say so.
 *   - sop_knn, sop_query, sop_shade, sop_shade_backward, sop_bake and the proposal calls
 *     never allocate: their scratch memory is the caller's workspace `ws` of `ws_bytes`
 *     bytes (256-byte aligned), sized by the matching *_workspace_size function.
 *   - Every argument is validated on the host before any device work is enqueued. A call
 *     that fails returns a status other than SOP_OK, enqueues nothing and leaves its outputs
 *     untouched; sop_last_error() then returns a message (thread-local) naming the problem.
 *     SOP_ERR_DEVICE reports a HIP runtime error raised while enqueueing.
 *   - Two calls that share a plan, a workspace or an accumulated gradient buffer must not
 *     run concurrently on different streams.
 */
#ifndef SOP_H_
#define SOP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* HIP stream handle (hipStream_t); NULL is the legacy default stream. */
typedef struct ihipStream_t* sop_stream;

typedef enum sop_status {
  SOP_OK = 0,
  SOP_ERR_INVALID_ARGUMENT = 1,   /* NULL/misaligned pointer, size or option out of range   */
  SOP_ERR_UNSUPPORTED = 2,        /* valid request the library does not implement           */
  SOP_ERR_WORKSPACE_TOO_SMALL = 3,/* ws_bytes below the *_workspace_size figure             */
  SOP_ERR_DEVICE = 4,             /* HIP runtime error (message holds hipGetErrorString)    */
  SOP_ERR_OUT_OF_MEMORY = 5       /* plan creation could not allocate device memory         */
} sop_status;

typedef enum sop_texel_format {
  SOP_TEXEL_F32 = 0,              /* 4 x float per texel (16 bytes)                         */
  SOP_TEXEL_F16 = 1               /* 4 x IEEE half per texel (8 bytes)                      */
} sop_texel_format;

/* Library limits. */
#define SOP_MAX_K        16       /* neighbours per shading point                           */
#define SOP_MAX_DIRS     4096     /* directions per shading point                           */
#define SOP_MAX_RES      256      /* octahedral texture side                                */
#define SOP_LATTICE_BITS 15       /* neighbour search quantises positions to 2^15 per axis  */

/* ----------------------------------------------------------------------------------------
 * Inputs
 * --------------------------------------------------------------------------------------*/

/* Probe positions (Sec. 3.1.2, automatic placement of SOPs). bounds_lo/hi are HOST
 * values: the box in which positions are quantised for the neighbour search. Positions
 * outside the box are clamped onto it by the quantisation; hi > lo on every axis. */
typedef struct sop_probe_set {
  int32_t      count;            /* P >= 0                                                */
  const float* pos;              /* device [P,3]; may be NULL when P == 0                 */
  float        bounds_lo[3];     /* host                                                  */
  float        bounds_hi[3];     /* host                                                  */
} sop_probe_set;

/* Probe textures {L_in, O} (Sec. 3.1.2): one octahedral map per probe, +z at the centre of
 * the square. Layout [P][row v][column u][channel], channels (R, G, B, O). */
typedef struct sop_probe_maps {
  int32_t     res;               /* R_t, 2 <= res <= SOP_MAX_RES                          */
  int32_t     format;            /* sop_texel_format                                      */
  const void* texels;            /* device [P,res,res,4]                                  */
} sop_probe_maps;

/* Environment map L_dir (Eq. 8), layout [H][W][3] (RGB):
 *   SOP_ENV_EQUIRECT (0, the default of a zeroed struct): equirectangular, row 0 around +z,
 *     column u covering azimuth phi = 2*pi*u/W - pi; bilinear, columns wrap, rows clamp.
 *   SOP_ENV_OCTAHEDRAL (1): an octahedral map with H = W (the paper's representation of
 *     the estimated lighting, Sec. 3.2), read exactly like a probe map: +z at the centre
 *     of the square, bilinear with mirror wrap. */
typedef enum sop_env_layout {
  SOP_ENV_EQUIRECT = 0,
  SOP_ENV_OCTAHEDRAL = 1
} sop_env_layout;

typedef struct sop_envmap {
  int32_t      height;           /* H >= 1                                                */
  int32_t      width;            /* W >= 1 (== H for SOP_ENV_OCTAHEDRAL, 2..1024)         */
  const float* texels;           /* device [H,W,3]                                        */
  int32_t      layout;           /* sop_env_layout                                        */
} sop_envmap;

/* Shading points (G-buffer texels, Sec. 3.1, multi-target rendering). The view direction
 * is either given per point (`view`, unit vectors toward the viewer) or derived from one
 * camera position per frame: points [f*points_per_frame, (f+1)*points_per_frame) see
 * cam_pos[f]. Normals must be unit length; the BRDF assumes n . view > 0. */
typedef struct sop_points {
  int64_t      count;            /* N >= 0                                                */
  const float* pos;              /* device [N,3]                                          */
  const float* normal;           /* device [N,3]                                          */
  const float* view;             /* device [N,3] or NULL (then cam_pos is used)           */
  const float* cam_pos;          /* device [n_frames,3], used when view == NULL           */
  int64_t      points_per_frame; /* >= 1 when view == NULL                               */
  int32_t      n_frames;         /* N == n_frames * points_per_frame when view == NULL    */
  const float* albedo;           /* device [N,3]                                          */
  const float* roughness;        /* device [N]                                            */
  const float* metallic;         /* device [N]                                            */
} sop_points;

/* Result of the neighbour search (sop_knn), reusable by sop_query/sop_shade/
 * sop_shade_backward so that a forward and its backward search only once. */
typedef struct sop_neighbors {
  int32_t        k;              /* K, 1 <= K <= SOP_MAX_K                                */
  const int32_t* order;          /* device [N]: processing order (a permutation of 0..N-1
                                    grouping points that share probes); NULL = identity  */
  const int32_t* idx;            /* device [N,K]: probe indices, ascending (d^2, index);
                                    -1 pads a short list                                 */
  const float*   weight;         /* device [N,K]: normalised weights, 0 on pads           */
} sop_neighbors;

typedef struct sop_plan sop_plan;             /* probe grid (opaque)                      */

/* ----------------------------------------------------------------------------------------
 * Probe plan: quantised lattice + uniform grid over the probes, the acceleration structure
 * of the fixed-radius / k-nearest search of Sec. 3.1.2 (efficient querying).
 * --------------------------------------------------------------------------------------*/

/* Creates a plan for `probes` and builds its grid on `stream`. Allocates device memory for
 * the grid (O(P) plus the cell table) and synchronises `stream` once. The plan keeps no
 * pointer to probes->pos after the call. Release with sop_plan_destroy. */
sop_status sop_plan_create(const sop_probe_set* probes, sop_stream stream, sop_plan** out);

/* Rebuilds the grid of `plan` for new positions `pos` (device [P,3], same P and bounds as at
 * creation). Asynchronous, allocates nothing. */
sop_status sop_plan_rebuild(sop_plan* plan, const float* pos, sop_stream stream);

/* Frees the plan. Work that uses it must have completed. NULL is accepted. */
sop_status sop_plan_destroy(sop_plan* plan);

/* Number of probes and grid cells of a plan (host values). */
sop_status sop_plan_info(const sop_plan* plan, int32_t* n_probes, int32_t grid_dims[3],
                         float* lattice_scale);

/* ----------------------------------------------------------------------------------------
 * Neighbour search (Eq. 9-11).
 * Positions are quantised to the integer lattice q = clamp(floor((x - lo) * sc), 0, 2^15-1)
 * per axis, in 32-bit float arithmetic, with one isotropic scale
 * sc = 32768 / max_axis(hi - lo). Candidates are the probes with squared lattice distance
 * d^2 <= floor((radius*sc)^2) (radius = +inf: all probes); the K smallest by (d^2, probe
 * index) are kept. If the smallest d^2 is 0, that single probe is used with weight 1.
 * Otherwise w_k = (1/|p_k - x|) * (0.5 * (1 + (p_k - x)/|p_k - x| . n) + 0.01), normalised
 * to sum 1 (Eq. 10-11 with n_p read as the shading normal).
 * --------------------------------------------------------------------------------------*/

/* Writes order[N], idx[N,K] and w[N,K] (see sop_neighbors). order may be NULL. Reads the
 * points' positions and normals only (the other fields of pts may be NULL). */
sop_status sop_knn(const sop_plan* plan, const sop_points* pts, int32_t k, float radius,
                   int32_t* order, int32_t* idx, float* w,
                   void* ws, size_t ws_bytes, sop_stream stream);

/* Eq. 9 as a primitive: for every point i and given world direction dirs[i,j] (unit, device
 * [N,D,3]) returns the interpolated indirect radiance L_in[i,j,0..2] and occlusion O[i,j]
 * (device [N,D,3] and [N,D]). nb may be NULL (the search then runs with k/radius).
 * Each probe texture is read with bilinear filtering and octahedral mirror wrap. */
sop_status sop_query(const sop_plan* plan, const sop_probe_maps* maps, const sop_points* pts,
                     const sop_neighbors* nb, const float* dirs, int32_t n_dirs, int32_t k,
                     float radius, float* L_in, float* O,
                     void* ws, size_t ws_bytes, sop_stream stream);

/* ----------------------------------------------------------------------------------------
 * Shading (Eq. 6-8 with the estimator of Eq. 7).
 * Direction j of S at point i: cos(theta) = 1 - (j + 0.5)/S,
 * phi = 2*pi * (((bitreverse32(j) >> 8) + rho) mod 2^24) / 2^24 in the orthonormal frame of
 * the normal (Duff et al. 2017). rho = pcg_hash(seed) >> 8 (or, per point,
 * pcg_hash(seed ^ pcg_hash(i)) >> 8), pcg_hash as in Jarzynski & Olano 2020.
 * BRDF (a reading of the simplified Disney BRDF the paper names): Lambert (1-m)*a/pi plus GGX
 * D*F*G/(4 NoL NoV), alpha = r^2, Smith-Schlick G with k = alpha/2, Schlick F with
 * F0 = 0.04(1-m) + a*m, NoV = max(n.v, 1e-4).
 * rgb_i = (2*pi/S) * sum_j f(w_j) * L_i(w_j) * cos(theta_j),
 * L_i = (1 - O(w)) * L_env(w) + L_in(w).
 * --------------------------------------------------------------------------------------*/

typedef enum sop_sampler {
  SOP_SAMPLER_HAMMERSLEY = 0,     /* uniform hemisphere Hammersley set (Eq. 7)              */
  SOP_SAMPLER_PROPOSAL = 1,       /* per-point bin distributions given in opts.probs        */
  SOP_SAMPLER_PROPOSAL_NET = 2,   /* bin distributions of the network opts.net, evaluated
                                     inside the shading call (they never reach memory)     */
  SOP_SAMPLER_ENV = 3,            /* environment importance sampling (Eq. 18) on an
                                     octahedral env: the draws and density of
                                     SOP_SHADOW_ENV (see sop_shadow_ratio)                  */
  SOP_SAMPLER_ENV_EXACT = 4,      /* the same draws weighted by their exact density, as
                                     SOP_SHADOW_ENV_EXACT                                  */
  SOP_SAMPLER_COSINE = 5          /* cosine-weighted Hammersley set: the pairs of the
                                     uniform set lifted from the unit disk (Malley's method),
                                     density cos(theta)/pi                                 */
} sop_sampler;

typedef struct sop_mlp sop_mlp;

typedef struct sop_shade_opts {
  int32_t  n_dirs;               /* S, 1 <= S <= SOP_MAX_DIRS                             */
  int32_t  k;                    /* K, 1 <= K <= SOP_MAX_K (ignored when nb != NULL)       */
  float    radius;               /* FRNN radius in world units, +inf = unlimited          */
  uint32_t seed;                 /* rotation seed of the direction set                    */
  int32_t  rotate_per_point;     /* 0: one rotation per call, 1: one per point            */
  int32_t  sampler;              /* sop_sampler                                           */
  float*   out_irradiance;       /* optional device [N,3]: (2pi/S) sum_j L_i cos(theta)   */
  const float* probs;            /* SOP_SAMPLER_PROPOSAL: device [N,256] bin distributions
                                    (one row per point, any non-negative weights; values
                                    are clamped to [0,1], NaN counts as 0)                */
  float    mix_eps;              /* SOP_SAMPLER_PROPOSAL(_NET): weight of the uniform-bin
                                    part of the mixture, 0 <= mix_eps <= 1                 */
  const sop_mlp* net;            /* SOP_SAMPLER_PROPOSAL_NET: the proposal network         */
} sop_shade_opts;

/* Forward shading. Writes rgb[N,3] (and out_irradiance when set). nb may be NULL.
 * With SOP_SAMPLER_COSINE (the cosine fallback next to the uniform set of Eq. 7) direction j
 * has sin(theta_j) = sqrt((j+0.5)/S), cos(theta_j) = sqrt(1-(j+0.5)/S) and the azimuth of
 * the uniform set's direction j (same rotation), and rgb_i = (pi/S) sum_j f(w_j) L_i(w_j),
 * out_irradiance (pi/S) sum_j L_i(w_j); it has no adjoint (sop_shade_backward refuses it).
 * With SOP_SAMPLER_PROPOSAL the S directions of point i are drawn from its bin distribution
 * (see the learned direction proposal below) and rgb_i = (1/S) sum_j f L_i cos / pdf(w_j);
 * out_irradiance is then (1/S) sum_j L_i cos / pdf(w_j). With SOP_SAMPLER_PROPOSAL_NET the
 * distributions are the network's (opts->net), computed in the same kernel exactly as
 * sop_proposal_infer computes them; the result equals that of SOP_SAMPLER_PROPOSAL with
 * sop_proposal_infer's output up to the order of the per-point sums. The proposal samplers
 * have no adjoint: sop_shade_backward accepts only SOP_SAMPLER_HAMMERSLEY. The proposal
 * samplers (and sop_dump_integrand) take an equirectangular env only
 * (SOP_ERR_UNSUPPORTED for SOP_ENV_OCTAHEDRAL). With SOP_SAMPLER_ENV (object relighting by
 * importance sampling, Sec. 3.3) the env must be SOP_ENV_OCTAHEDRAL (else
 * SOP_ERR_UNSUPPORTED); draw j of point i (its index in pts) is the draw of the
 * SOP_SHADOW_ENV sampler with density pdf_j = (m_t / C) R_e^2 / (4 pi), and
 * rgb_i = (1/S) sum_j f L_i (n . w_j)+ / pdf_j, out_irradiance (1/S) sum_j L_i (n . w_j)+ /
 * pdf_j; draws below the horizon add nothing. SOP_SAMPLER_ENV_EXACT takes the same draws
 * with the density of SOP_SHADOW_ENV_EXACT. Neither has an adjoint. */
sop_status sop_shade(const sop_plan* plan, const sop_probe_maps* maps, const sop_envmap* env,
                     const sop_points* pts, const sop_neighbors* nb,
                     const sop_shade_opts* opts, float* rgb,
                     void* ws, size_t ws_bytes, sop_stream stream);

/* Adjoint of sop_shade for the upstream gradient grad_rgb[N,3]. Recomputes every sample
 * (nothing is stored by the forward). Per-point gradients are OVERWRITTEN:
 * g_albedo[N,3], g_rough[N], g_metal[N] (each may be NULL). Texture gradients are
 * ACCUMULATED (+=) and may be NULL: g_env[H,W,3] and g_tex[P,res,res,4] (always f32, also
 * for half textures; channel 3 is dL/dO). Geometry (positions, normals, views) and the
 * neighbour weights receive no gradient. Accumulation order is not fixed, so g_env/g_tex
 * may differ between runs by float rounding. */
sop_status sop_shade_backward(const sop_plan* plan, const sop_probe_maps* maps,
                              const sop_envmap* env, const sop_points* pts,
                              const sop_neighbors* nb, const sop_shade_opts* opts,
                              const float* grad_rgb, float* g_albedo, float* g_rough,
                              float* g_metal, float* g_env, float* g_tex,
                              void* ws, size_t ws_bytes, sop_stream stream);

/* Deterministic adjoint: the gradients of sop_shade_backward with g_env and g_tex that do
 * not depend on how the work was scheduled, bit for bit equal from run to run (the per-point
 * gradients of sop_shade_backward already are). Same arguments and semantics (g_env and
 * g_tex accumulate, +=), plus `acc`, device scratch of acc_bytes >=
 * sop_shade_backward_acc_size(plan's P, maps->res, env->height, env->width) bytes, 256-byte
 * aligned, owned by the caller (its contents on entry do not matter; NULL is accepted only
 * when g_env and g_tex are both NULL). Every contribution c to an output value is added
 * exactly, as an integer multiple of 2^-96, into four 64-bit words per value (integer
 * addition does not depend on order); the exact sum is rounded once (through FP64) and
 * added to the value. Contributions with |c| < 2^-96 are dropped (the bits below 2^-96 of
 * the others are truncated towards zero); a contribution with |c| >= 2^32 or not finite
 * sets every g_env and g_tex value of the call to NaN. Up to 2^31 contributions per value.
 * For callers that need reproducible gradients; it is slower than sop_shade_backward
 * (64-bit atomics, up to two per contribution, and a final pass over the words).
 * Errors as sop_shade_backward, plus SOP_ERR_WORKSPACE_TOO_SMALL for a short acc. */
sop_status sop_shade_backward_deterministic(const sop_plan* plan, const sop_probe_maps* maps,
                                            const sop_envmap* env, const sop_points* pts,
                                            const sop_neighbors* nb,
                                            const sop_shade_opts* opts, const float* grad_rgb,
                                            float* g_albedo, float* g_rough, float* g_metal,
                                            float* g_env, float* g_tex, void* ws,
                                            size_t ws_bytes, void* acc, size_t acc_bytes,
                                            sop_stream stream);

/* Accumulator bytes of sop_shade_backward_deterministic for P probes of res x res texels and
 * an env_height x env_width environment: 32 bytes per g_tex and g_env value plus alignment
 * (0 on a negative argument). */
size_t sop_shade_backward_acc_size(int32_t n_probes, int32_t res, int32_t env_height,
                                   int32_t env_width);

typedef enum sop_op {
  SOP_OP_KNN = 0,
  SOP_OP_QUERY = 1,
  SOP_OP_SHADE = 2,
  SOP_OP_SHADE_BACKWARD = 3,
  SOP_OP_DUMP_INTEGRAND = 4,     /* sop_dump_integrand (sized by sop_workspace_size)        */
  SOP_OP_PROPOSAL_INFER = 5,     /* sop_proposal_infer (sized by sop_proposal_workspace_size) */
  SOP_OP_PROPOSAL_TRAIN = 6      /* sop_proposal_train_step (sop_proposal_workspace_size)   */
} sop_op;

/* Workspace bytes that `op` needs for n_points points with k neighbours, n_dirs directions
 * and an environment map of env_height x env_width texels (shading ops keep per-call
 * direction and environment reference tables there) on `plan`, assuming the neighbour
 * search runs inside the call (nb == NULL); with_neighbors != 0 gives the smaller figure
 * for calls that receive nb. For SOP_OP_SHADE_BACKWARD it includes, for environments of up
 * to 4096 x 2048 texels, 64 bytes per 2x2 texel block in each of 4 block offsets
 * (~21 bytes per texel), where the environment adjoint is gathered before it is added to
 * g_env. Returns 0 on an invalid argument. */
size_t sop_workspace_size(const sop_plan* plan, sop_op op, int64_t n_points, int32_t k,
                          int32_t n_dirs, int32_t env_height, int32_t env_width,
                          int32_t with_neighbors);

/* ----------------------------------------------------------------------------------------
 * Bake: probe textures by ray tracing through 3D Gaussians (Sec. 3.1.2, the SOP texture
 * initialisation by ray tracing; Sec. 4.1). For texel (u,v) of probe p the ray starts at
 * p along the octahedral decode of the texel centre. Each Gaussian responds at the ray
 * parameter t* of maximum density; alpha = min(alpha_max, opacity * exp(-m^2/2)) with m the
 * Mahalanobis distance at t*; Gaussians with t* <= t_min or alpha < alpha_min are skipped.
 * The rest are blended front to back in ascending (t*, index) as in Eq. 1: T starts at 1,
 * blending stops before a Gaussian that would take T*(1-alpha) below T_min.
 * Outputs (R,G,B) = sum T*alpha*color, O = sum T*alpha, depth = sum T*alpha*t* / O (0 when
 * O == 0), the unbiased depth D/W of Sec. 3.1.
 * --------------------------------------------------------------------------------------*/

typedef struct sop_gaussians {
  int32_t      count;            /* G >= 0                                                */
  const float* mean;             /* device [G,3]                                          */
  const float* scale;            /* device [G,3]: standard deviations, > 0                */
  const float* rotation;         /* device [G,4]: quaternion (w,x,y,z), normalised here   */
  const float* opacity;          /* device [G], in [0,1]                                  */
  const float* color;            /* device [G,3]                                          */
} sop_gaussians;

typedef struct sop_bake_opts {
  float t_min;                   /* default 0; >= 0 (rays start at the probe)             */
  float alpha_min;               /* default 1/255                                         */
  float alpha_max;               /* default 0.99                                          */
  float T_min;                   /* default 1e-4                                          */
  float cell_scale;              /* grid cell side relative to the mean cut-off box of the
                                    Gaussians; 0 selects the library default (0.25)       */
} sop_bake_opts;

typedef struct sop_bake_plan sop_bake_plan;   /* Gaussian grid (opaque)                   */

/* Precomputes per-Gaussian frames and registers every Gaussian in the cells of a uniform
 * grid overlapped by its cut-off ellipsoid (where its response can reach alpha_min).
 * Allocates device memory sized by a counting pass and synchronises `stream` once. */
sop_status sop_bake_plan_create(const sop_gaussians* g, const sop_bake_opts* opts,
                                sop_stream stream, sop_bake_plan** out);

/* Re-registers Gaussians with the same count G into the existing grid, asynchronously and
 * without allocating. If the new registration exceeds the capacity fixed at creation,
 * sop_bake writes NaN to every output texel and sop_bake_plan_check reports it. */
sop_status sop_bake_plan_update(sop_bake_plan* plan, const sop_gaussians* g,
                                sop_stream stream);

/* Synchronises `stream` and returns SOP_ERR_WORKSPACE_TOO_SMALL if the last update of the
 * plan overflowed its grid capacity, else SOP_OK. */
sop_status sop_bake_plan_check(const sop_bake_plan* plan, sop_stream stream);

sop_status sop_bake_plan_destroy(sop_bake_plan* plan);

/* Traces every texel of P probes at resolution res. texels: device [P,res,res,4] f32
 * (R,G,B,O); depth: device [P,res,res] f32 or NULL. No workspace. order_by (may be NULL) is
 * a probe plan over the same P probes: the probes are then traced in its cell-major Morton
 * order, which keeps the Gaussians that concurrently traced rays meet in one die's cache;
 * outputs stay in the caller's probe order and do not depend on it. */
sop_status sop_bake(const sop_bake_plan* plan, const float* probe_pos, int32_t n_probes,
                    int32_t res, float* texels, float* depth, const sop_plan* order_by,
                    sop_stream stream);

/* ----------------------------------------------------------------------------------------
 * Traced shading: the per-sample ray tracing that the probes stand in for (Sec. 3.1.2:
 * occlusion and indirect light are read from the probes instead of tracing the Gaussians
 * for every sample; the composition table of Sec. 4.2 compares the two). The estimate
 * of sop_shade with the Hammersley sampler (same directions, BRDF and sums), where O(w_j)
 * and L_in(w_j) of sample j of point i come from one ray through the Gaussians of `gauss`:
 * the ray starts at o_i = fmaf(offset, n_i, x_i) (per component, IEEE single precision),
 * runs along w_j and is blended exactly as sop_bake blends a texel's ray, with the plan's
 * t_min, alpha_min, alpha_max and T_min: L_in = sum T alpha color, O = sum T alpha.
 *   - order_by (may be NULL): a plan whose grid orders the points so that rays of nearby
 *     points are traced together. Any plan over the same bounds serves; one built over
 *     the shading points themselves has the finest cells for them. The results do not
 *     depend on it.
 *   - opts: n_dirs, seed, rotate_per_point and out_irradiance are used and the sampler
 *     must be SOP_SAMPLER_HAMMERSLEY (else SOP_ERR_UNSUPPORTED); k, radius, probs and net
 *     are ignored.
 *   - offset: finite and >= 0, world units along the normal.
 *   - samples (may be NULL): device [N,S,4] f32, 16-byte aligned; receives (L_in rgb, O)
 *     of every sample in the caller's point order. When NULL the workspace holds them.
 * Writes rgb[N,3] (and out_irradiance). If the last update of `gauss` overflowed its grid,
 * the samples and so rgb are NaN (sop_bake_plan_check reports it). Workspace:
 * sop_shade_traced_workspace_size with the same order_by, N, S, environment and samples. */
sop_status sop_shade_traced(const sop_bake_plan* gauss, const sop_plan* order_by,
                            const sop_envmap* env, const sop_points* pts,
                            const sop_shade_opts* opts, float offset, float* rgb,
                            float* samples, void* ws, size_t ws_bytes, sop_stream stream);

/* Workspace bytes of sop_shade_traced for n_points points, n_dirs directions and an
 * env_height x env_width environment; with_samples != 0 when the call passes `samples`
 * (otherwise the workspace also holds the 16 * n_points * n_dirs bytes of samples).
 * order_by as in the call (may be NULL). Returns 0 on an invalid argument. */
size_t sop_shade_traced_workspace_size(const sop_plan* order_by, int64_t n_points,
                                       int32_t n_dirs, int32_t env_height, int32_t env_width,
                                       int32_t with_samples);

/* ----------------------------------------------------------------------------------------
 * Cast-shadow ratio (Sec. 3.2, occlusion caching; Sec. 3.3, rendering). For a Lambertian
 * scene point with normal n the shadow of a placed object is S = L_o' / L_o (Eq. 17) with
 * L_o = f_d * integral L_i(w) (w.n)+ dw (Eq. 15) and
 * L_o' = f_d * integral L_i(w) (1 - O'(w)) (w.n)+ dw (Eq. 16), per colour channel (f_d
 * cancels). O' is the object's occlusion, read from the probes of the shadow region
 * exactly as sop_query reads O (channel 3 of their maps; their RGB is not used). L_i is an
 * octahedral environment map, bilinear with mirror wrap like the probe maps. Both
 * integrals are estimated with the same S samples (samples below the horizon add nothing):
 *   SOP_SHADOW_HAMMERSLEY: the direction set of sop_shade, density 1/(2 pi);
 *   SOP_SHADOW_ENV: environment importance sampling (Eq. 18). Texel t has intensity
 *     I_t = (r + g) + b (0 unless positive) and mass m_t = 1 + floor(I_t * (2^14 / I_max))
 *     (one IEEE single-precision division and one product; every mass is 1 when
 *     I_max = 0), C = sum m_t. Draw j of point i: x = (j C + ((h(i,j,0) C) >> 24)) / S in
 *     integers, the texel t with M_t <= x < M_t + m_t (M_t = mass of the texels before t),
 *     the direction = octahedral decode of (column + (h(i,j,1) + 1/2)/2^24,
 *     row + (h(i,j,2) + 1/2)/2^24) in texel units, and the density of Eq. 18 with its
 *     normalisation read as I_t / sum(I): pdf = (m_t / C) R^2 / (4 pi), which gives every
 *     texel the mean solid angle 4 pi / R^2 (the estimate then carries the map's area
 *     distortion as a bias). Here h(i,j,k) = pcg(pcg(pcg(seed) ^ i) ^ (4 j + k)) >> 8 (pcg
 *     as for the directions).
 *   SOP_SHADOW_ENV_EXACT: the same draws with their exact density,
 *     pdf = (m_t / C) (R^2 / 4) / s^3 with s = |x| + |y| + |z| of the unit direction (the
 *     octahedral square's area element is dw / s^3): an unbiased estimate.
 * ratio_c = sum_j L_c (1 - O') cos+ / pdf  /  sum_j L_c cos+ / pdf, and 1 where the
 * denominator is 0.
 * --------------------------------------------------------------------------------------*/

/* Octahedral environment map: +z at the centre of the square, layout [row v][column u][3]
 * like sop_probe_maps (channels R, G, B). */
typedef struct sop_env_oct {
  int32_t      res;              /* R_e, 2 <= R_e <= 1024                                  */
  const float* texels;           /* device [R_e,R_e,3]                                     */
} sop_env_oct;

typedef enum sop_shadow_sampler {
  SOP_SHADOW_HAMMERSLEY = 0,     /* hemisphere Hammersley set (Eq. 7)                      */
  SOP_SHADOW_ENV = 1,            /* environment importance sampling (Eq. 18)               */
  SOP_SHADOW_ENV_EXACT = 2       /* the same draws with their exact density                */
} sop_shadow_sampler;

typedef struct sop_shadow_opts {
  int32_t  n_dirs;               /* S, 1 <= S <= SOP_MAX_DIRS                              */
  int32_t  k;                    /* K, 1 <= K <= SOP_MAX_K (ignored when nb != NULL)        */
  float    radius;               /* FRNN radius in world units, +inf = unlimited           */
  uint32_t seed;                 /* direction rotation / draw seed                         */
  int32_t  rotate_per_point;     /* Hammersley: 0 one rotation per call, 1 one per point   */
  int32_t  sampler;              /* sop_shadow_sampler                                     */
  float*   out_irradiance;       /* optional device [N,3]: (1/S) sum_j L cos+ / pdf, the
                                    unshadowed L_o / f_d                                   */
} sop_shadow_opts;

/* Writes ratio[N,3]. The probes of `plan` and `maps` are those of the shadow region; the
 * points' positions and normals are used (the other point fields may be NULL). nb may be
 * NULL (the search then runs with opts->k and opts->radius). Workspace:
 * sop_shadow_workspace_size. */
sop_status sop_shadow_ratio(const sop_plan* plan, const sop_probe_maps* maps,
                            const sop_env_oct* env, const sop_points* pts,
                            const sop_neighbors* nb, const sop_shadow_opts* opts, float* ratio,
                            void* ws, size_t ws_bytes, sop_stream stream);

/* Workspace bytes of sop_shadow_ratio (direction table, texel masses and their prefix sums,
 * and the neighbour search unless with_neighbors != 0). Returns 0 on an invalid argument. */
size_t sop_shadow_workspace_size(const sop_plan* plan, int64_t n_points, int32_t k,
                                 int32_t n_dirs, int32_t env_res, int32_t with_neighbors);

/* ----------------------------------------------------------------------------------------
 * Probe placement (Sec. 3.1.2, automatic placement of SOPs): farthest point sampling over
 * a surface point cloud with normals, then every pick raised along its normal. The first
 * pick is `start`; pick k is the point whose squared distance to its nearest earlier pick
 * is largest, the squared distance taken in IEEE single precision as
 * ((dx*dx + dy*dy) + dz*dz), dx = x_j - x_q, without fused multiply-adds; ties go to the
 * lowest index. Probe k = fmaf(offset, n_c, x_c) per component of its pick c.
 * --------------------------------------------------------------------------------------*/

/* pts, normals: device [M,3], 1 <= M <= 2^31 - 1; 1 <= n_probes <= M; 0 <= start < M;
 * offset finite. Writes probe_pos [n_probes,3] and, when not NULL, chosen [n_probes] (the
 * picks' indices). Enqueues a fill, all the picks as one launch of at most 64 workgroups
 * that exchange every pick through device memory, and the probe positions. Every
 * device-side wait between those workgroups is bounded (about a second): should one give
 * up, which needs some of them to be kept from running while the others wait (e.g. a
 * device filled by other work), probe_pos is all NaN. Workspace:
 * sop_place_workspace_size(M, n_probes). */
sop_status sop_place_probes(const float* pts, const float* normals, int64_t n_points,
                            int32_t n_probes, int64_t start, float offset, int32_t* chosen,
                            float* probe_pos, void* ws, size_t ws_bytes, sop_stream stream);

size_t sop_place_workspace_size(int64_t n_points, int32_t n_probes);

/* ----------------------------------------------------------------------------------------
 * Losses of the reconstruction step (Sec. 3.1.2): L_sops = L1(L_in, L_tr) + L1(O, O_tr)
 * supervises the probe textures with the traced ones, and L_lam = L1(R, 1) + L1(M, 0)
 * regularises the materials. L1 is the mean absolute difference over the elements (RGB
 * channels together, O apart); gradients take sign(x - y) / n with sign(0) = 0. Each call
 * writes its two terms to loss[0], loss[1] (device, float) from per-workgroup partial sums
 * in double precision added in a fixed order (the same inputs give the same loss).
 * --------------------------------------------------------------------------------------*/

/* tex, target: device [T,4] (R,G,B,O) f32, 16-byte aligned (for instance [P,R_t,R_t,4]
 * maps: T = P R_t^2). loss[0] = L1(L_in, L_tr), loss[1] = L1(O, O_tr); grad (may be NULL,
 * [T,4]) is OVERWRITTEN with d(loss[0] + loss[1]) / d tex. Workspace:
 * sop_loss_workspace_size(T). */
sop_status sop_sops_loss(const float* tex, const float* target, int64_t n_texels, float* loss,
                         float* grad, void* ws, size_t ws_bytes, sop_stream stream);

/* rough, metal: device [N]. loss[0] = L1(R, 1), loss[1] = L1(M, 0); g_rough, g_metal (may be
 * NULL, [N]) are OVERWRITTEN with the gradients of loss[0] + loss[1]. Workspace:
 * sop_loss_workspace_size(N). */
sop_status sop_lam_loss(const float* rough, const float* metal, int64_t n_points, float* loss,
                        float* g_rough, float* g_metal, void* ws, size_t ws_bytes,
                        sop_stream stream);

size_t sop_loss_workspace_size(int64_t n_elements);

/* ----------------------------------------------------------------------------------------
 * Learned direction proposal: an extension of the Monte Carlo estimate of Eq. 7 (the paper
 * uses a fixed Hammersley set; here the directions can instead be importance sampled from a
 * per-point distribution that a small network predicts, trained on integrand samples that
 * the shading step itself produces).
 *
 * Bins: the local hemisphere of the shading frame (the frame of the direction set above)
 * is mapped to the square (u,v) = ((x+y), (x-y)) / (|x|+|y|+z) in [-1,1]^2, cut into 16x16
 * cells; bin b = 16*row + col with col = floor((u+1)*8), row = floor((v+1)*8). Inside a
 * cell the density is uniform in (u,v); in solid angle it is
 *   pdf(w) = (c_b / C) * 128 / s^3,   s = |x| + |y| + z of the unit local direction.
 * Masses: q_b = fmaf(1 - eps, clamp(p_b, 0, 1), eps/256) in IEEE single precision,
 * c_b = floor(q_b * 2^24), C = sum_b c_b (all-zero masses fall back to c_b = 1).
 * Draw j of S at point i: x_j = (j*C + ((r*C) >> 24)) / S in integer arithmetic with
 * r = h(i,j,0); the bin is the smallest b with C_b + c_b > x_j (C_b = c_0 + ... + c_{b-1});
 * the position in the cell is u = (x_j - C_b + 0.5) / c_b (the draw's place on the bin's
 * stretch of the mass line) and v = ((((bitreverse32(j) >> 8) + h(i,0,2)) mod 2^24) + 0.5)
 * / 2^24 (a radical inverse of j rotated per point), where
 * h(i,j,k) = pcg(pcg(pcg(seed) ^ i) ^ (4j + k)) >> 8 and pcg is the hash of the direction
 * set above.
 *
 * Network: features are sin(pi f_l x) and cos(pi f_l x) (feature 32c + 2l and 32c + 2l + 1),
 * f_l = 2^(l/2), l = 0..15, of the 10 scalars x = (2 (pos - lo)/(hi - lo) - 1, n, v, r);
 * z1 = x W1 + b1, h1 = relu(z1), z2 = h1 W2 + b2, h2 = relu(z2), z3 = h2 W3 + b3,
 * p = softmax(z3). Features, weights and hidden activations are rounded to bfloat16
 * (round to nearest even) and multiplied on the matrix cores with FP32 accumulation;
 * biases, logits and the softmax stay FP32.
 * --------------------------------------------------------------------------------------*/
#define SOP_MLP_FREQS 16
#define SOP_MLP_IN 320
#define SOP_MLP_HIDDEN 64
#define SOP_MLP_BINS 256
#define SOP_MLP_PARAMS 41344          /* W1[320][64] b1[64] W2[64][64] b2[64] W3[64][256] b3[256] */

struct sop_mlp {
  float* params;                 /* device [SOP_MLP_PARAMS] f32, row-major W[in][out]; read by
                                    inference, updated in place by a training step        */
  float  bounds_lo[3];           /* host: scene box mapped to [-1,1]^3 for the features   */
  float  bounds_hi[3];
};

typedef struct sop_adam {
  float   lr, beta1, beta2, eps;
  int32_t step;                  /* 1-based index of this update (bias correction)        */
} sop_adam;

/* Workspace bytes of SOP_OP_PROPOSAL_INFER / SOP_OP_PROPOSAL_TRAIN for n_points points
 * (0 on an invalid argument). */
size_t sop_proposal_workspace_size(sop_op op, int64_t n_points);

/* probs [N,256] (device f32, rows sum to 1) and optionally logits [N,256] (NULL to skip)
 * of the proposal network for the points' position, normal, view and roughness. */
sop_status sop_proposal_infer(const sop_mlp* mlp, const sop_points* pts, float* probs,
                              float* logits, void* ws, size_t ws_bytes, sop_stream stream);

/* One training step on a batch of B points with raw bin targets T [B,256] (device f32,
 * non-negative; each row is normalised, a row summing to <= 0 counts as uniform):
 * loss = mean_i sum_b -t_ib log p_ib, written to *loss (device f32). The gradient of the
 * loss (in the parameter layout) is written to grad (device [SOP_MLP_PARAMS], may be NULL).
 * When opt is not NULL the parameters are then updated in place by Adam with the state
 * adam_m / adam_v (device [SOP_MLP_PARAMS] each). In the backward pass the output-side
 * gradients are rounded to bfloat16 before they meet a weight or an activation. The step
 * uses no atomics: the same inputs give the same loss, gradient and parameters bit for
 * bit. */
sop_status sop_proposal_train_step(const sop_mlp* mlp, const sop_points* pts,
                                   const float* targets, const sop_adam* opt, float* adam_m,
                                   float* adam_v, float* loss, float* grad, void* ws,
                                   size_t ws_bytes, sop_stream stream);

/* Adam (Kingma & Ba 2015) on n parameters: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). All device f32. */
sop_status sop_adam_update(float* params, float* adam_m, float* adam_v, const float* grad,
                           int64_t n, const sop_adam* opt, sop_stream stream);

/* Training targets of the proposal: T[i,b] = (1/(128 n)) sum_k lum(f L_i cos)(w_bk) / l_bk^3
 * estimates the integral over bin b of the luminance (Rec. 709 weights) of the integrand of
 * Eq. 6 at point i, with n = samples_per_bin directions placed in bin b's cell at
 * u = (k + (h(i,j,1) + 0.5) / 2^24) / n, v = (h(i,j,2) + 0.5) / 2^24, j = b n + k, and
 * l_bk the L2 norm of the
 * (px,py,z) point of the direction. Uses opts->seed (and k/radius when nb is NULL);
 * targets: device [N,256] f32. */
sop_status sop_dump_integrand(const sop_plan* plan, const sop_probe_maps* maps,
                              const sop_envmap* env, const sop_points* pts,
                              const sop_neighbors* nb, const sop_shade_opts* opts,
                              int32_t samples_per_bin, float* targets,
                              void* ws, size_t ws_bytes, sop_stream stream);

/* ----------------------------------------------------------------------------------------
 * Shading for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): sop_shade with its workspace taken from a fixed
 * device array inside the library, SOP_NOALLOC_SCRATCH_BYTES per device, held by every
 * device that runs the library until the process ends. The caller still passes inputs and
 * outputs. Same arguments, results and errors as sop_shade; a call whose workspace
 * (sop_workspace_size with op SOP_OP_SHADE) exceeds the array returns
 * SOP_ERR_WORKSPACE_TOO_SMALL before any device work (pass nb, or fewer points). The stream
 * must belong to the current device. The first call on a device looks up that device's
 * copy of the array once; no call allocates. Calls that overlap on one device (two streams,
 * or two threads) share the array and race: serialise them.
 * --------------------------------------------------------------------------------------*/
#define SOP_NOALLOC_SCRATCH_BYTES (32u << 20)

sop_status sop_shade_noalloc(const sop_plan* plan, const sop_probe_maps* maps,
                             const sop_envmap* env, const sop_points* pts,
                             const sop_neighbors* nb, const sop_shade_opts* opts, float* rgb,
                             sop_stream stream);

/* ----------------------------------------------------------------------------------------
 * Misc
 * --------------------------------------------------------------------------------------*/
/* Text of a status code; any int is accepted (values that name no status give
 * "unknown status"), so the parameter is an int rather than the enum. */
const char* sop_status_string(int status);
const char* sop_last_error(void);
int32_t     sop_version(void);          /* major*10000 + minor*100 + patch */

#ifdef __cplusplus
}
#endif
#endif /* SOP_H_ */
