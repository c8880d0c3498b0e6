// api.cpp - host side of the SOP C ABI: argument validation before any device work,
// plan objects, workspace carving and stream-ordered dispatch of the kernels.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "sop_internal.hpp"

using sopk::Bump;

namespace {

thread_local std::string g_err;

sop_status fail(sop_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

sop_status hip_fail(hipError_t e, const char* where) {
  return fail(SOP_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define SOP_HIP(expr, where)                      \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// lattice scale: 32768 / max_axis(hi - lo) in IEEE single precision
float lattice_scale(const float lo[3], const float hi[3]) {
  float ext = hi[0] - lo[0];
  const float e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
  if (e1 > ext) ext = e1;
  if (e2 > ext) ext = e2;
  return 32768.0f / ext;
}

uint32_t radius_limit(float radius, float sc) {
  const double rq = (double)radius * (double)sc;
  const double r2 = rq * rq;
  if (!(r2 < 4294967295.0)) return 0xFFFFFFFFu;
  return (uint32_t)std::floor(r2);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// probe plan
// ------------------------------------------------------------------------------------------
struct sop_plan {
  int32_t P = 0;
  float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  float sc = 0.0f;
  int32_t bits = 1;
  size_t C = 0;
  int4* qsorted = nullptr;
  int4* qtmp = nullptr;
  int32_t* counts = nullptr;
  int32_t* cell_start = nullptr;
  int32_t* cursor = nullptr;
  float* pos = nullptr;
  int32_t* scan_tmp = nullptr;

  sopk::ProbeGrid view() const {
    sopk::ProbeGrid g;
    g.P = P;
    g.bits = bits;
    g.shift = 15 - bits;
    for (int a = 0; a < 3; ++a) g.lo[a] = lo[a];
    g.sc = sc;
    g.qsorted = qsorted;
    g.cell_start = cell_start;
    g.pos = pos;
    return g;
  }
  void release() {
    void* ptrs[] = {qsorted, qtmp, counts, cell_start, cursor, pos, scan_tmp};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    qsorted = qtmp = nullptr;
    counts = cell_start = cursor = scan_tmp = nullptr;
    pos = nullptr;
  }
};

static int32_t grid_bits_for(int32_t P) {
  // about one grid cell per probe along a surface: cbrt(P) cells per axis, doubled
  const double c = std::cbrt((double)(P > 1 ? P : 1));
  int b = (int)std::lround(std::log2(c)) + 1;
  if (b < 1) b = 1;
  if (b > 7) b = 7;
  return b;
}

static sop_status validate_probe_set(const sop_probe_set* probes) {
  if (!probes) return fail(SOP_ERR_INVALID_ARGUMENT, "probes is NULL");
  if (probes->count < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "probes->count < 0");
  if (probes->count > 0 && (!probes->pos || !aligned(probes->pos, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "probes->pos is NULL or misaligned");
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(probes->bounds_lo[a]) || !std::isfinite(probes->bounds_hi[a]) ||
        !(probes->bounds_hi[a] > probes->bounds_lo[a]))
      return fail(SOP_ERR_INVALID_ARGUMENT, "bounds must be finite with hi > lo on every axis");
  }
  return SOP_OK;
}

extern "C" sop_status sop_plan_create(const sop_probe_set* probes, sop_stream stream,
                                      sop_plan** out) {
  if (!out) return fail(SOP_ERR_INVALID_ARGUMENT, "out is NULL");
  sop_status st = validate_probe_set(probes);
  if (st != SOP_OK) return st;
  sop_plan* pl = new (std::nothrow) sop_plan();
  if (!pl) return fail(SOP_ERR_OUT_OF_MEMORY, "host allocation failed");
  pl->P = probes->count;
  for (int a = 0; a < 3; ++a) {
    pl->lo[a] = probes->bounds_lo[a];
    pl->hi[a] = probes->bounds_hi[a];
  }
  pl->sc = lattice_scale(pl->lo, pl->hi);
  pl->bits = grid_bits_for(pl->P);
  pl->C = (size_t)1 << (3 * pl->bits);
  const size_t P1 = pl->P > 0 ? (size_t)pl->P : 1;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  alloc((void**)&pl->qsorted, P1 * sizeof(int4));
  alloc((void**)&pl->qtmp, P1 * sizeof(int4));
  alloc((void**)&pl->counts, pl->C * sizeof(int32_t));
  alloc((void**)&pl->cell_start, (pl->C + 1) * sizeof(int32_t));
  alloc((void**)&pl->cursor, pl->C * sizeof(int32_t));
  alloc((void**)&pl->pos, P1 * 3 * sizeof(float));
  alloc((void**)&pl->scan_tmp, sopk::scan_tmp_elems(pl->C) * sizeof(int32_t));
  if (e != hipSuccess) {
    pl->release();
    delete pl;
    (void)hipGetLastError();
    return fail(SOP_ERR_OUT_OF_MEMORY, std::string("plan allocation: ") + hipGetErrorString(e));
  }
  e = sopk::launch_probe_grid_build(probes->pos, pl->P, pl->lo, pl->sc, pl->bits, pl->qtmp,
                                    pl->counts, pl->cell_start, pl->cursor, pl->qsorted, pl->pos,
                                    pl->scan_tmp, (hipStream_t)stream);
  if (e != hipSuccess) {
    pl->release();
    delete pl;
    return hip_fail(e, "sop_plan_create");
  }
  *out = pl;
  return SOP_OK;
}

extern "C" sop_status sop_plan_rebuild(sop_plan* plan, const float* pos, sop_stream stream) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (plan->P > 0 && (!pos || !aligned(pos, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "pos is NULL or misaligned");
  SOP_HIP(sopk::launch_probe_grid_build(pos, plan->P, plan->lo, plan->sc, plan->bits,
                                        plan->qtmp, plan->counts, plan->cell_start,
                                        plan->cursor, plan->qsorted, plan->pos, plan->scan_tmp,
                                        (hipStream_t)stream),
          "sop_plan_rebuild");
  return SOP_OK;
}

extern "C" sop_status sop_plan_destroy(sop_plan* plan) {
  if (!plan) return SOP_OK;
  plan->release();
  delete plan;
  return SOP_OK;
}

extern "C" sop_status sop_plan_info(const sop_plan* plan, int32_t* n_probes,
                                    int32_t grid_dims[3], float* lattice_scale_out) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (n_probes) *n_probes = plan->P;
  if (grid_dims)
    for (int a = 0; a < 3; ++a) grid_dims[a] = 1 << plan->bits;
  if (lattice_scale_out) *lattice_scale_out = plan->sc;
  return SOP_OK;
}

// ------------------------------------------------------------------------------------------
// workspace
// ------------------------------------------------------------------------------------------
namespace {

struct KnnScratch {
  int32_t* point_cell;
  int32_t* counts;
  int32_t* offsets;
  int32_t* scan_tmp;
};

KnnScratch carve_knn(Bump& b, const sop_plan* plan, int64_t N) {
  KnnScratch k;
  k.point_cell = b.take<int32_t>((size_t)N);
  k.counts = b.take<int32_t>(plan->C);
  k.offsets = b.take<int32_t>(plan->C + 1);
  k.scan_tmp = b.take<int32_t>(sopk::scan_tmp_elems(plan->C));
  return k;
}

struct NbScratch {
  int32_t* order;
  int32_t* idx;
  float* w;
};

NbScratch carve_nb(Bump& b, int64_t N, int32_t k) {
  NbScratch s;
  s.order = b.take<int32_t>((size_t)N);
  s.idx = b.take<int32_t>((size_t)N * k);
  s.w = b.take<float>((size_t)N * k);
  return s;
}

// texel masses, their prefix sums and scan scratch of an environment of T texels (the
// environment importance sampler)
struct EnvCdf {
  uint32_t* mass;
  uint64_t* prefix;
  uint64_t* tiles;
  float* imax;
  int32_t* guide;
};

EnvCdf carve_env_cdf(Bump& b, size_t T) {
  EnvCdf c;
  c.mass = b.take<uint32_t>(T);
  c.prefix = b.take<uint64_t>(T + 1);
  c.tiles = b.take<uint64_t>((T + 1023) / 1024 + 1);
  c.imax = b.take<float>(1);
  c.guide = b.take<int32_t>((size_t)sopk::kEnvGuide + 1);
  return c;
}

// Workspace layout: [direction table (shade ops)] [order, idx, w] [search scratch]
// the float adjoint's environment blocks (sopk::env_block_cols), for environments up to
// sopk::kEnvBlkMaxTexels texels; larger ones are added with runs straight into g_env
bool env_blocks_fit(int32_t env_h, int32_t env_w) {
  return env_h > 0 && env_w > 0 && (int64_t)env_h * env_w <= sopk::kEnvBlkMaxTexels;
}
size_t env_block_floats(int32_t env_h, int32_t env_w) {
  return (size_t)4 * sopk::env_block_cols(env_w) * sopk::env_block_rows(env_h) *
         sopk::kEnvBlkFloats;
}

size_t ws_needed(const sop_plan* plan, sop_op op, int64_t N, int32_t k, bool with_nb,
                 int32_t n_dirs, int32_t env_h = 0, int32_t env_w = 0) {
  Bump b{nullptr, 0, 0};
  if (op == SOP_OP_KNN) {
    (void)b.take<int32_t>((size_t)N);   // order when the caller passes none
    carve_knn(b, plan, N);
    return b.used;
  }
  if (op == SOP_OP_SHADE || op == SOP_OP_SHADE_BACKWARD || op == SOP_OP_DUMP_INTEGRAND) {
    if (op == SOP_OP_SHADE) {
      (void)b.take<uint16_t>(sopk::mlp_frag_bytes() / sizeof(uint16_t));
      (void)b.take<double4>((size_t)n_dirs);   // directions along the hemisphere's Z curve
      carve_env_cdf(b, (size_t)env_h * (size_t)env_w);   // environment sampler
    }
    (void)b.take<double4>((size_t)n_dirs);
    (void)b.take<double2>((size_t)env_w + 2);
    (void)b.take<double2>((size_t)env_h + 2);
  }
  if (!with_nb) {
    carve_nb(b, N, k);
    carve_knn(b, plan, N);
  }
  if (op == SOP_OP_SHADE_BACKWARD) (void)b.take<double4>((size_t)n_dirs);   // Z-curve order
  if (op == SOP_OP_SHADE_BACKWARD && env_blocks_fit(env_h, env_w))
    (void)b.take<float>(env_block_floats(env_h, env_w));
  return b.used;
}

sop_status validate_points(const sop_points* pts) {
  if (!pts) return fail(SOP_ERR_INVALID_ARGUMENT, "pts is NULL");
  if (pts->count < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "pts->count < 0");
  if (pts->count > INT32_MAX) return fail(SOP_ERR_UNSUPPORTED, "more than 2^31-1 points");
  if (pts->count == 0) return SOP_OK;
  const void* req[] = {pts->pos, pts->normal, pts->albedo, pts->roughness, pts->metallic};
  for (const void* p : req)
    if (!p || !aligned(p, 4))
      return fail(SOP_ERR_INVALID_ARGUMENT, "a point array is NULL or misaligned");
  if (pts->view) {
    if (!aligned(pts->view, 4)) return fail(SOP_ERR_INVALID_ARGUMENT, "view misaligned");
  } else {
    if (!pts->cam_pos || !aligned(pts->cam_pos, 4) || pts->points_per_frame < 1 ||
        pts->n_frames < 1 || (int64_t)pts->n_frames * pts->points_per_frame != pts->count)
      return fail(SOP_ERR_INVALID_ARGUMENT,
                  "view is NULL: need cam_pos and n_frames * points_per_frame == count");
  }
  return SOP_OK;
}

sop_status validate_maps(const sop_plan* plan, const sop_probe_maps* maps) {
  if (!maps) return fail(SOP_ERR_INVALID_ARGUMENT, "maps is NULL");
  if (maps->res < 2 || maps->res > SOP_MAX_RES)
    return fail(SOP_ERR_INVALID_ARGUMENT, "maps->res out of [2, 256]");
  if (maps->format != SOP_TEXEL_F32 && maps->format != SOP_TEXEL_F16)
    return fail(SOP_ERR_INVALID_ARGUMENT, "unknown texel format");
  const size_t al = maps->format == SOP_TEXEL_F32 ? 16 : 8;
  if (plan->P > 0 && (!maps->texels || !aligned(maps->texels, al)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "maps->texels is NULL or misaligned");
  return SOP_OK;
}

sop_status validate_env(const sop_envmap* env) {
  if (!env) return fail(SOP_ERR_INVALID_ARGUMENT, "env is NULL");
  if (env->height < 1 || env->width < 1 || env->height > (1 << 16) || env->width > (1 << 16))
    return fail(SOP_ERR_INVALID_ARGUMENT, "env size out of range");
  if (!env->texels || !aligned(env->texels, 4))
    return fail(SOP_ERR_INVALID_ARGUMENT, "env->texels is NULL or misaligned");
  if (env->layout != SOP_ENV_EQUIRECT && env->layout != SOP_ENV_OCTAHEDRAL)
    return fail(SOP_ERR_INVALID_ARGUMENT, "unknown env layout");
  if (env->layout == SOP_ENV_OCTAHEDRAL &&
      (env->height != env->width || env->width < 2 || env->width > 1024))
    return fail(SOP_ERR_INVALID_ARGUMENT, "an octahedral env needs height == width in [2, 1024]");
  return SOP_OK;
}

sop_status validate_nb(const sop_neighbors* nb) {
  if (nb->k < 1 || nb->k > SOP_MAX_K) return fail(SOP_ERR_INVALID_ARGUMENT, "nb->k out of [1,16]");
  if (!nb->idx || !nb->weight || !aligned(nb->idx, 4) || !aligned(nb->weight, 4))
    return fail(SOP_ERR_INVALID_ARGUMENT, "nb->idx/weight NULL or misaligned");
  if (nb->order && !aligned(nb->order, 4))
    return fail(SOP_ERR_INVALID_ARGUMENT, "nb->order misaligned");
  return SOP_OK;
}

sop_status validate_k_radius(int32_t k, float radius) {
  if (k < 1 || k > SOP_MAX_K) return fail(SOP_ERR_INVALID_ARGUMENT, "k out of [1, 16]");
  if (std::isnan(radius) || !(radius > 0.0f))
    return fail(SOP_ERR_INVALID_ARGUMENT, "radius must be > 0 (or +inf)");
  return SOP_OK;
}

sop_status validate_ws(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return SOP_OK;
  if (!ws || !aligned(ws, 256))
    return fail(SOP_ERR_INVALID_ARGUMENT, "workspace is NULL or not 256-byte aligned");
  if (ws_bytes < need)
    return fail(SOP_ERR_WORKSPACE_TOO_SMALL,
                "workspace too small: need " + std::to_string(need) + " bytes");
  return SOP_OK;
}

// neighbour search into caller- or workspace-provided buffers
hipError_t run_knn(const sop_plan* plan, const sop_points* pts, int32_t k, float radius,
                   int32_t* order, int32_t* idx, float* w, KnnScratch ks, hipStream_t s) {
  const sopk::ProbeGrid g = plan->view();
  hipError_t e = sopk::launch_point_order(g, pts->pos, pts->count, ks.point_cell, ks.counts,
                                          ks.offsets, ks.scan_tmp, order, s);
  if (e != hipSuccess) return e;
  return sopk::launch_knn(g, pts->pos, pts->normal, pts->count, order, k,
                          radius_limit(radius, plan->sc), idx, w, s);
}

}  // namespace

extern "C" size_t sop_workspace_size(const sop_plan* plan, sop_op op, int64_t n_points,
                                     int32_t k, int32_t n_dirs, int32_t env_height,
                                     int32_t env_width, int32_t with_neighbors) {
  if (!plan || n_points < 0 || k < 1 || k > SOP_MAX_K) return 0;
  if (op < SOP_OP_KNN || op > SOP_OP_DUMP_INTEGRAND) return 0;
  if (env_height < 0 || env_width < 0) return 0;
  size_t need = ws_needed(plan, op, n_points, k, with_neighbors != 0, n_dirs > 0 ? n_dirs : 1,
                          env_height, env_width);
  return need > 0 ? need : 256;
}

// ------------------------------------------------------------------------------------------
// neighbour search and query
// ------------------------------------------------------------------------------------------
extern "C" sop_status sop_knn(const sop_plan* plan, const sop_points* pts, int32_t k,
                              float radius, int32_t* order, int32_t* idx, float* w, void* ws,
                              size_t ws_bytes, sop_stream stream) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  // the search reads positions and normals only
  if (!pts) return fail(SOP_ERR_INVALID_ARGUMENT, "pts is NULL");
  if (pts->count < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "pts->count < 0");
  if (pts->count > INT32_MAX) return fail(SOP_ERR_UNSUPPORTED, "more than 2^31-1 points");
  if (pts->count > 0 && (!pts->pos || !pts->normal || !aligned(pts->pos, 4) ||
                         !aligned(pts->normal, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "pts->pos/normal NULL or misaligned");
  sop_status st = validate_k_radius(k, radius);
  if (st != SOP_OK) return st;
  if (pts->count > 0 && (!idx || !w || !aligned(idx, 4) || !aligned(w, 4) ||
                         (order && !aligned(order, 4))))
    return fail(SOP_ERR_INVALID_ARGUMENT, "idx/w NULL or misaligned");
  const size_t need = ws_needed(plan, SOP_OP_KNN, pts->count, k, false, 1);
  if ((st = validate_ws(ws, ws_bytes, need)) != SOP_OK) return st;
  if (pts->count == 0) return SOP_OK;
  Bump b{(char*)ws, 0, ws_bytes};
  int32_t* ws_order = b.take<int32_t>((size_t)pts->count);
  KnnScratch ks = carve_knn(b, plan, pts->count);
  SOP_HIP(run_knn(plan, pts, k, radius, order ? order : ws_order, idx, w, ks,
                  (hipStream_t)stream),
          "sop_knn");
  return SOP_OK;
}

namespace {

sopk::ShadeArgs base_args(const sop_plan* plan, const sop_probe_maps* maps, const sop_points* pts) {
  sopk::ShadeArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = pts->count;
  a.pos = pts->pos;
  a.nrm = pts->normal;
  a.view = pts->view;
  a.cam = pts->cam_pos;
  a.ppf = pts->points_per_frame > 0 ? pts->points_per_frame : 1;
  a.albedo = pts->albedo;
  a.rough = pts->roughness;
  a.metal = pts->metallic;
  a.P = plan->P;
  a.tex = maps->texels;
  a.R = maps->res;
  a.halfR = 0.5f * (float)maps->res;
  return a;
}

// resolves the neighbour lists: the caller's, or a search into the workspace
sop_status resolve_nb(const sop_plan* plan, const sop_points* pts, const sop_neighbors* nb,
                      int32_t k, float radius, Bump& b, hipStream_t s,
                      const int32_t** order, const int32_t** idx, const float** w,
                      int32_t* k_out) {
  if (nb) {
    *order = nb->order;
    *idx = nb->idx;
    *w = nb->weight;
    *k_out = nb->k;
    return SOP_OK;
  }
  NbScratch ns = carve_nb(b, pts->count, k);
  KnnScratch ks = carve_knn(b, plan, pts->count);
  SOP_HIP(run_knn(plan, pts, k, radius, ns.order, ns.idx, ns.w, ks, s), "neighbour search");
  *order = ns.order;
  *idx = ns.idx;
  *w = ns.w;
  *k_out = k;
  return SOP_OK;
}

}  // namespace

extern "C" sop_status sop_query(const sop_plan* plan, const sop_probe_maps* maps,
                                const sop_points* pts, const sop_neighbors* nb,
                                const float* dirs, int32_t n_dirs, int32_t k, float radius,
                                float* L_in, float* O, void* ws, size_t ws_bytes,
                                sop_stream stream) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  sop_status st = validate_points(pts);
  if (st != SOP_OK) return st;
  if ((st = validate_maps(plan, maps)) != SOP_OK) return st;
  if (nb) {
    if ((st = validate_nb(nb)) != SOP_OK) return st;
  } else if ((st = validate_k_radius(k, radius)) != SOP_OK) {
    return st;
  }
  if (n_dirs < 1 || n_dirs > SOP_MAX_DIRS)
    return fail(SOP_ERR_INVALID_ARGUMENT, "n_dirs out of [1, 4096]");
  if (pts->count > 0 && (!dirs || !L_in || !O || !aligned(dirs, 4) || !aligned(L_in, 4) ||
                         !aligned(O, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "dirs/L_in/O NULL or misaligned");
  const size_t need =
      ws_needed(plan, SOP_OP_QUERY, pts->count, nb ? nb->k : k, nb != nullptr, n_dirs);
  if ((st = validate_ws(ws, ws_bytes, need)) != SOP_OK) return st;
  if (pts->count == 0) return SOP_OK;
  const hipStream_t s = (hipStream_t)stream;
  sopk::ShadeArgs a = base_args(plan, maps, pts);
  int32_t kk;
  Bump b{(char*)ws, 0, ws_bytes};
  if ((st = resolve_nb(plan, pts, nb, k, radius, b, s, &a.order, &a.nb_idx, &a.nb_w, &kk)) !=
      SOP_OK)
    return st;
  SOP_HIP(sopk::launch_query(a, kk, maps->format, dirs, n_dirs, L_in, O, s), "sop_query");
  return SOP_OK;
}

// ------------------------------------------------------------------------------------------
// shading
// ------------------------------------------------------------------------------------------
namespace {

sop_status validate_shade(const sop_plan* plan, const sop_probe_maps* maps,
                          const sop_envmap* env, const sop_points* pts,
                          const sop_neighbors* nb, const sop_shade_opts* o,
                          bool allow_proposal) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (!o) return fail(SOP_ERR_INVALID_ARGUMENT, "opts is NULL");
  sop_status st = validate_points(pts);
  if (st != SOP_OK) return st;
  if ((st = validate_maps(plan, maps)) != SOP_OK) return st;
  if ((st = validate_env(env)) != SOP_OK) return st;
  if (nb) {
    if ((st = validate_nb(nb)) != SOP_OK) return st;
  } else if ((st = validate_k_radius(o->k, o->radius)) != SOP_OK) {
    return st;
  }
  if (o->n_dirs < 1 || o->n_dirs > SOP_MAX_DIRS)
    return fail(SOP_ERR_INVALID_ARGUMENT, "n_dirs out of [1, 4096]");
  if ((o->sampler == SOP_SAMPLER_PROPOSAL || o->sampler == SOP_SAMPLER_PROPOSAL_NET) &&
      env->layout == SOP_ENV_OCTAHEDRAL && allow_proposal)
    return fail(SOP_ERR_UNSUPPORTED, "the proposal samplers take an equirectangular env");
  if (o->sampler == SOP_SAMPLER_PROPOSAL) {
    if (!allow_proposal)
      return fail(SOP_ERR_UNSUPPORTED, "the proposal sampler has no adjoint");
    if (pts->count > 0 && (!o->probs || !aligned(o->probs, 16)))
      return fail(SOP_ERR_INVALID_ARGUMENT, "probs is NULL or not 16-byte aligned");
    if (!(o->mix_eps >= 0.0f && o->mix_eps <= 1.0f))
      return fail(SOP_ERR_INVALID_ARGUMENT, "mix_eps out of [0, 1]");
  } else if (o->sampler == SOP_SAMPLER_PROPOSAL_NET) {
    if (!allow_proposal)
      return fail(SOP_ERR_UNSUPPORTED, "the proposal sampler has no adjoint");
    if (!o->net) return fail(SOP_ERR_INVALID_ARGUMENT, "net is NULL");
    if (!o->net->params || !aligned(o->net->params, 16))
      return fail(SOP_ERR_INVALID_ARGUMENT, "net->params is NULL or not 16-byte aligned");
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(o->net->bounds_lo[c]) || !std::isfinite(o->net->bounds_hi[c]) ||
          !(o->net->bounds_hi[c] > o->net->bounds_lo[c]))
        return fail(SOP_ERR_INVALID_ARGUMENT, "net bounds must be finite with hi > lo");
    if (!(o->mix_eps >= 0.0f && o->mix_eps <= 1.0f))
      return fail(SOP_ERR_INVALID_ARGUMENT, "mix_eps out of [0, 1]");
  } else if (o->sampler == SOP_SAMPLER_ENV || o->sampler == SOP_SAMPLER_ENV_EXACT) {
    if (!allow_proposal)
      return fail(SOP_ERR_UNSUPPORTED, "the environment sampler has no adjoint");
    if (env->layout != SOP_ENV_OCTAHEDRAL)
      return fail(SOP_ERR_UNSUPPORTED, "the environment sampler takes an octahedral env");
  } else if (o->sampler == SOP_SAMPLER_COSINE) {
    if (!allow_proposal)
      return fail(SOP_ERR_UNSUPPORTED, "the cosine sampler has no adjoint");
  } else if (o->sampler != SOP_SAMPLER_HAMMERSLEY) {
    return fail(SOP_ERR_UNSUPPORTED, "unknown sampler");
  }
  if (o->out_irradiance && !aligned(o->out_irradiance, 4))
    return fail(SOP_ERR_INVALID_ARGUMENT, "out_irradiance misaligned");
  return SOP_OK;
}

void set_dirs(sopk::ShadeArgs& a, const sop_envmap* env, const sop_shade_opts* o) {
  a.env = env->texels;
  a.H = env->height;
  a.W = env->width;
  a.u_scale = (float)((double)env->width / (2.0 * M_PI));
  a.v_scale = (float)((double)env->height / M_PI);
  a.S = o->n_dirs;
  a.inv2S = (float)(1.0 / (2.0 * o->n_dirs));
  a.scale = (float)(2.0 * M_PI / o->n_dirs);
  a.seed = o->seed;
  a.per_point = o->rotate_per_point ? 1 : 0;
  a.env_oct = env->layout == SOP_ENV_OCTAHEDRAL ? 1 : 0;
}

// the call's direction table, first piece of the workspace
sop_status setup_dirs(sopk::ShadeArgs& a, Bump& b, const sop_shade_opts* o, hipStream_t s) {
  double4* tab = b.take<double4>((size_t)o->n_dirs);
  double2* col = b.take<double2>((size_t)a.W + 2);
  double2* row = b.take<double2>((size_t)a.H + 2);
  a.dir_tab = tab;
  // the reference directions serve the equirectangular lookup only
  a.col_ref = a.env_oct ? nullptr : col;
  a.row_ref = a.env_oct ? nullptr : row;
  SOP_HIP(sopk::launch_dir_table(o->n_dirs, o->seed, o->rotate_per_point ? 1 : 0, a.H, a.W, tab,
                                 a.env_oct ? nullptr : col, a.env_oct ? nullptr : row, s),
          "direction table");
  return SOP_OK;
}

}  // namespace

extern "C" sop_status sop_shade(const sop_plan* plan, const sop_probe_maps* maps,
                                const sop_envmap* env, const sop_points* pts,
                                const sop_neighbors* nb, const sop_shade_opts* opts,
                                float* rgb, void* ws, size_t ws_bytes, sop_stream stream) {
  sop_status st = validate_shade(plan, maps, env, pts, nb, opts, true);
  if (st != SOP_OK) return st;
  if (pts->count > 0 && (!rgb || !aligned(rgb, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "rgb is NULL or misaligned");
  const int32_t k = nb ? nb->k : opts->k;
  const size_t need = ws_needed(plan, SOP_OP_SHADE, pts->count, k, nb != nullptr, opts->n_dirs,
                                env->height, env->width);
  if ((st = validate_ws(ws, ws_bytes, need)) != SOP_OK) return st;
  if (pts->count == 0) return SOP_OK;
  const hipStream_t s = (hipStream_t)stream;
  sopk::ShadeArgs a = base_args(plan, maps, pts);
  set_dirs(a, env, opts);
  a.rgb = rgb;
  a.irr = opts->out_irradiance;
  int32_t kk;
  Bump b{(char*)ws, 0, ws_bytes};
  uint16_t* frags = b.take<uint16_t>(sopk::mlp_frag_bytes() / sizeof(uint16_t));
  double4* sorted = b.take<double4>((size_t)opts->n_dirs);
  const EnvCdf cdf = carve_env_cdf(b, (size_t)env->height * (size_t)env->width);
  if ((st = setup_dirs(a, b, opts, s)) != SOP_OK) return st;
  if ((st = resolve_nb(plan, pts, nb, opts->k, opts->radius, b, s, &a.order, &a.nb_idx,
                       &a.nb_w, &kk)) != SOP_OK)
    return st;
  if (opts->sampler == SOP_SAMPLER_PROPOSAL_NET) {
    a.mix_eps = opts->mix_eps;
    a.mlp_params = opts->net->params;
    a.mlp_frags = frags;
    for (int c = 0; c < 3; ++c) {
      a.mlp_lo[c] = opts->net->bounds_lo[c];
      a.mlp_inv2[c] = 2.0f / (opts->net->bounds_hi[c] - opts->net->bounds_lo[c]);
    }
    SOP_HIP(sopk::launch_mlp_frags(opts->net->params, frags, s), "sop_shade");
    SOP_HIP(sopk::launch_shade_prop_net(a, kk, maps->format, s), "sop_shade");
  } else if (opts->sampler == SOP_SAMPLER_PROPOSAL) {
    a.probs = opts->probs;
    a.mix_eps = opts->mix_eps;
    SOP_HIP(sopk::launch_shade_prop(a, kk, maps->format, s), "sop_shade");
  } else if (opts->sampler == SOP_SAMPLER_ENV || opts->sampler == SOP_SAMPLER_ENV_EXACT) {
    a.env_res = env->width;
    a.env_pdf_exact = opts->sampler == SOP_SAMPLER_ENV_EXACT ? 1 : 0;
    a.env_mass = cdf.mass;
    a.env_prefix = cdf.prefix;
    a.env_guide = cdf.guide;
    SOP_HIP(sopk::launch_env_cdf(env->texels, env->width * env->height, cdf.mass, cdf.prefix,
                                 cdf.tiles, cdf.imax, cdf.guide, s),
            "sop_shade");
    SOP_HIP(sopk::launch_shade_envis(a, kk, maps->format, s), "sop_shade");
  } else {
    a.cosine = opts->sampler == SOP_SAMPLER_COSINE ? 1 : 0;
    SOP_HIP(sopk::launch_dir_sort(opts->n_dirs, opts->seed, opts->rotate_per_point ? 1 : 0,
                                  sorted, s, a.cosine),
            "sop_shade");
    a.dir_sorted = sorted;
    SOP_HIP(sopk::launch_shade_fwd(a, kk, maps->format, s), "sop_shade");
  }
  return SOP_OK;
}

extern "C" sop_status sop_dump_integrand(const sop_plan* plan, const sop_probe_maps* maps,
                                         const sop_envmap* env, const sop_points* pts,
                                         const sop_neighbors* nb, const sop_shade_opts* opts,
                                         int32_t samples_per_bin, float* targets, void* ws,
                                         size_t ws_bytes, sop_stream stream) {
  sop_status st = validate_shade(plan, maps, env, pts, nb, opts, true);
  if (st != SOP_OK) return st;
  if (samples_per_bin < 1 || samples_per_bin > 64)
    return fail(SOP_ERR_INVALID_ARGUMENT, "samples_per_bin out of [1, 64]");
  if (pts->count > 0 && (!targets || !aligned(targets, 16)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "targets is NULL or not 16-byte aligned");
  const int32_t k = nb ? nb->k : opts->k;
  const size_t need = ws_needed(plan, SOP_OP_DUMP_INTEGRAND, pts->count, k, nb != nullptr,
                                opts->n_dirs, env->height, env->width);
  if ((st = validate_ws(ws, ws_bytes, need)) != SOP_OK) return st;
  if (pts->count == 0) return SOP_OK;
  const hipStream_t s = (hipStream_t)stream;
  if (env->layout != SOP_ENV_EQUIRECT)
    return fail(SOP_ERR_UNSUPPORTED, "sop_dump_integrand takes an equirectangular env");
  sopk::ShadeArgs a = base_args(plan, maps, pts);
  set_dirs(a, env, opts);
  a.npb = samples_per_bin;
  a.targets = targets;
  int32_t kk;
  Bump b{(char*)ws, 0, ws_bytes};
  if ((st = setup_dirs(a, b, opts, s)) != SOP_OK) return st;
  if ((st = resolve_nb(plan, pts, nb, opts->k, opts->radius, b, s, &a.order, &a.nb_idx,
                       &a.nb_w, &kk)) != SOP_OK)
    return st;
  SOP_HIP(sopk::launch_dump_integrand(a, kk, maps->format, s), "sop_dump_integrand");
  return SOP_OK;
}

namespace {

// Layout of the deterministic adjoint's accumulator: the texture words (4 per g_tex value),
// the environment words (4 per g_env value), the flag; each region 256-byte aligned.
struct DetLayout {
  int64_t nt = 0, ne = 0;
  size_t off_env = 0, off_flag = 0, bytes = 0;
};

bool det_layout(int64_t P, int32_t res, int32_t env_h, int32_t env_w, DetLayout* d) {
  if (P < 0 || res < 0 || env_h < 0 || env_w < 0) return false;
  d->nt = P * (int64_t)res * res * 4;
  d->ne = (int64_t)env_h * env_w * 3;
  const size_t a = 256;
  d->off_env = ((size_t)d->nt * 4 * 8 + a - 1) / a * a;
  d->off_flag = d->off_env + ((size_t)d->ne * 4 * 8 + a - 1) / a * a;
  d->bytes = d->off_flag + a;
  return true;
}

sop_status shade_backward_impl(const sop_plan* plan, const sop_probe_maps* maps,
                               const sop_envmap* env, const sop_points* pts,
                               const sop_neighbors* nb, const sop_shade_opts* opts,
                               const float* grad_rgb, float* g_albedo, float* g_rough,
                               float* g_metal, float* g_env, float* g_tex, void* ws,
                               size_t ws_bytes, void* acc, size_t acc_bytes, bool det,
                               sop_stream stream, const char* fn) {
  sop_status st = validate_shade(plan, maps, env, pts, nb, opts, false);
  if (st != SOP_OK) return st;
  if (pts->count > 0 && (!grad_rgb || !aligned(grad_rgb, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "grad_rgb is NULL or misaligned");
  const void* outs[] = {g_albedo, g_rough, g_metal, g_env, g_tex};
  for (const void* p : outs)
    if (p && !aligned(p, 4)) return fail(SOP_ERR_INVALID_ARGUMENT, "a gradient is misaligned");
  const int32_t k = nb ? nb->k : opts->k;
  const size_t need = ws_needed(plan, SOP_OP_SHADE_BACKWARD, pts->count, k, nb != nullptr,
                                opts->n_dirs, env->height, env->width);
  if ((st = validate_ws(ws, ws_bytes, need)) != SOP_OK) return st;
  DetLayout dl;
  if (det && (g_env || g_tex)) {
    if (!det_layout(plan->P, maps->res, env->height, env->width, &dl))
      return fail(SOP_ERR_INVALID_ARGUMENT, "accumulator layout");
    if (!acc || !aligned(acc, 256))
      return fail(SOP_ERR_INVALID_ARGUMENT, "acc is NULL or not 256-byte aligned");
    if (acc_bytes < dl.bytes)
      return fail(SOP_ERR_WORKSPACE_TOO_SMALL,
                  "acc smaller than sop_shade_backward_acc_size(P, res, env_h, env_w)");
  }
  if (pts->count == 0) return SOP_OK;
  const hipStream_t s = (hipStream_t)stream;
  sopk::ShadeArgs a = base_args(plan, maps, pts);
  set_dirs(a, env, opts);
  a.grad = grad_rgb;
  a.g_albedo = g_albedo;
  a.g_rough = g_rough;
  a.g_metal = g_metal;
  a.g_env = g_env;
  a.g_tex = g_tex;
  int32_t kk;
  Bump b{(char*)ws, 0, ws_bytes};
  if ((st = setup_dirs(a, b, opts, s)) != SOP_OK) return st;
  if ((st = resolve_nb(plan, pts, nb, opts->k, opts->radius, b, s, &a.order, &a.nb_idx,
                       &a.nb_w, &kk)) != SOP_OK)
    return st;
  unsigned long long* wt = nullptr;
  unsigned long long* we = nullptr;
  int32_t* flag = nullptr;
  if (det && (g_env || g_tex)) {
    char* base = (char*)acc;
    wt = reinterpret_cast<unsigned long long*>(base);
    we = reinterpret_cast<unsigned long long*>(base + dl.off_env);
    flag = reinterpret_cast<int32_t*>(base + dl.off_flag);
    // zero the words in use and the flag (a fill kernel, no memset node)
    if (g_tex)
      SOP_HIP(sopk::launch_fill_i32(reinterpret_cast<int32_t*>(wt), 0, (size_t)dl.nt * 8, s), fn);
    if (g_env)
      SOP_HIP(sopk::launch_fill_i32(reinterpret_cast<int32_t*>(we), 0, (size_t)dl.ne * 8, s), fn);
    SOP_HIP(sopk::launch_fill_i32(flag, 0, 1, s), fn);
    a.det_tex = g_tex ? wt : nullptr;
    a.det_env = g_env ? we : nullptr;
    a.det_flag = flag;
    a.det_nt = dl.nt;
    a.det_ne = dl.ne;
  }
  double4* sorted = b.take<double4>((size_t)opts->n_dirs);
  SOP_HIP(sopk::launch_dir_sort(opts->n_dirs, opts->seed, opts->rotate_per_point ? 1 : 0,
                                sorted, s),
          fn);
  a.dir_sorted = sorted;
  const bool blocks = !det && g_env && env_blocks_fit(env->height, env->width) &&
                      sopk::shade_bwd_batched(maps->res, kk);
  if (blocks) {
    const size_t nf = env_block_floats(env->height, env->width);
    a.env_blk = b.take<float>(nf);
    a.env_bw = sopk::env_block_cols(env->width);
    a.env_bh = sopk::env_block_rows(env->height);
    SOP_HIP(sopk::launch_fill_i32(reinterpret_cast<int32_t*>(a.env_blk), 0, nf, s), fn);
  }
  SOP_HIP(sopk::launch_shade_bwd(a, kk, maps->format, s), fn);
  if (blocks)
    SOP_HIP(sopk::launch_env_blk_finish(a.env_blk, a.env_bw, a.env_bh, env->height,
                                        env->width, env->layout == SOP_ENV_OCTAHEDRAL, g_env,
                                        s),
            fn);
  if (det && g_tex) SOP_HIP(sopk::launch_det_finish(wt, dl.nt, flag, g_tex, s), fn);
  if (det && g_env) SOP_HIP(sopk::launch_det_finish(we, dl.ne, flag, g_env, s), fn);
  return SOP_OK;
}

}  // namespace

extern "C" sop_status sop_shade_backward(const sop_plan* plan, const sop_probe_maps* maps,
                                         const sop_envmap* env, const sop_points* pts,
                                         const sop_neighbors* nb, const sop_shade_opts* opts,
                                         const float* grad_rgb, float* g_albedo,
                                         float* g_rough, float* g_metal, float* g_env,
                                         float* g_tex, void* ws, size_t ws_bytes,
                                         sop_stream stream) {
  return shade_backward_impl(plan, maps, env, pts, nb, opts, grad_rgb, g_albedo, g_rough,
                             g_metal, g_env, g_tex, ws, ws_bytes, nullptr, 0, false, stream,
                             "sop_shade_backward");
}

extern "C" size_t sop_shade_backward_acc_size(int32_t n_probes, int32_t res,
                                              int32_t env_height, int32_t env_width) {
  DetLayout dl;
  if (!det_layout(n_probes, res, env_height, env_width, &dl)) return 0;
  return dl.bytes;
}

extern "C" sop_status sop_shade_backward_deterministic(
    const sop_plan* plan, const sop_probe_maps* maps, const sop_envmap* env,
    const sop_points* pts, const sop_neighbors* nb, const sop_shade_opts* opts,
    const float* grad_rgb, float* g_albedo, float* g_rough, float* g_metal, float* g_env,
    float* g_tex, void* ws, size_t ws_bytes, void* acc, size_t acc_bytes, sop_stream stream) {
  return shade_backward_impl(plan, maps, env, pts, nb, opts, grad_rgb, g_albedo, g_rough,
                             g_metal, g_env, g_tex, ws, ws_bytes, acc, acc_bytes, true, stream,
                             "sop_shade_backward_deterministic");
}

// ------------------------------------------------------------------------------------------
// learned direction proposal: network inference, training step, Adam
// ------------------------------------------------------------------------------------------
namespace {

sop_status validate_mlp(const sop_mlp* m) {
  if (!m) return fail(SOP_ERR_INVALID_ARGUMENT, "mlp is NULL");
  if (!m->params || !aligned(m->params, 16))
    return fail(SOP_ERR_INVALID_ARGUMENT, "mlp->params is NULL or not 16-byte aligned");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(m->bounds_lo[a]) || !std::isfinite(m->bounds_hi[a]) ||
        !(m->bounds_hi[a] > m->bounds_lo[a]))
      return fail(SOP_ERR_INVALID_ARGUMENT, "mlp bounds must be finite with hi > lo");
  return SOP_OK;
}

// the network reads position, normal, view (or camera) and roughness
sop_status validate_mlp_points(const sop_points* pts) {
  if (!pts) return fail(SOP_ERR_INVALID_ARGUMENT, "pts is NULL");
  if (pts->count < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "pts->count < 0");
  if (pts->count > INT32_MAX) return fail(SOP_ERR_UNSUPPORTED, "more than 2^31-1 points");
  if (pts->count == 0) return SOP_OK;
  const void* req[] = {pts->pos, pts->normal, pts->roughness};
  for (const void* p : req)
    if (!p || !aligned(p, 4))
      return fail(SOP_ERR_INVALID_ARGUMENT, "a point array is NULL or misaligned");
  if (pts->view) {
    if (!aligned(pts->view, 4)) return fail(SOP_ERR_INVALID_ARGUMENT, "view misaligned");
  } else if (!pts->cam_pos || !aligned(pts->cam_pos, 4) || pts->points_per_frame < 1 ||
             pts->n_frames < 1 ||
             (int64_t)pts->n_frames * pts->points_per_frame != pts->count) {
    return fail(SOP_ERR_INVALID_ARGUMENT,
                "view is NULL: need cam_pos and n_frames * points_per_frame == count");
  }
  return SOP_OK;
}

sop_status validate_adam(const sop_adam* o) {
  if (!(o->lr >= 0.0f) || !std::isfinite(o->lr) || !(o->beta1 >= 0.0f && o->beta1 < 1.0f) ||
      !(o->beta2 >= 0.0f && o->beta2 < 1.0f) || !(o->eps > 0.0f) || !std::isfinite(o->eps) ||
      o->step < 1)
    return fail(SOP_ERR_INVALID_ARGUMENT, "Adam options out of range");
  return SOP_OK;
}

sopk::MlpArgs mlp_args(const sop_mlp* m, const sop_points* pts) {
  sopk::MlpArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = pts->count;
  a.pos = pts->pos;
  a.nrm = pts->normal;
  a.view = pts->view;
  a.cam = pts->cam_pos;
  a.ppf = pts->points_per_frame > 0 ? pts->points_per_frame : 1;
  a.rough = pts->roughness;
  for (int c = 0; c < 3; ++c) {
    a.lo[c] = m->bounds_lo[c];
    a.inv2[c] = 2.0f / (m->bounds_hi[c] - m->bounds_lo[c]);
  }
  a.params = m->params;
  return a;
}

// Workspace: [weight fragments] then, for training, the transposed bf16 operands
// x^T [320][B16], h1^T, h2^T, dz1^T, dz2^T [64][B16], dz3^T [256][B16], a gradient buffer
// and the per-tile partial sums [B16 / 16][385]
size_t proposal_ws(sop_op op, int64_t n) {
  Bump b{nullptr, 0, 0};
  (void)b.take<uint16_t>(sopk::mlp_frag_bytes() / sizeof(uint16_t));
  if (op == SOP_OP_PROPOSAL_TRAIN) {
    const size_t ld = (size_t)((n + 31) / 32) * 32;   // the weight-gradient GEMM takes K in 32s
    (void)b.take<uint16_t>((size_t)SOP_MLP_IN * ld);
    for (int i = 0; i < 4; ++i) (void)b.take<uint16_t>((size_t)SOP_MLP_HIDDEN * ld);
    (void)b.take<uint16_t>((size_t)SOP_MLP_BINS * ld);
    (void)b.take<float>(SOP_MLP_PARAMS);
    (void)b.take<float>((ld / 16) * sopk::kMlpPart);
  }
  return b.used;
}

}  // namespace

extern "C" size_t sop_proposal_workspace_size(sop_op op, int64_t n_points) {
  if (n_points < 0 || n_points > INT32_MAX) return 0;
  if (op != SOP_OP_PROPOSAL_INFER && op != SOP_OP_PROPOSAL_TRAIN) return 0;
  return proposal_ws(op, n_points);
}

extern "C" sop_status sop_proposal_infer(const sop_mlp* mlp, const sop_points* pts,
                                         float* probs, float* logits, void* ws,
                                         size_t ws_bytes, sop_stream stream) {
  sop_status st = validate_mlp(mlp);
  if (st != SOP_OK) return st;
  if ((st = validate_mlp_points(pts)) != SOP_OK) return st;
  if (pts->count > 0 && (!probs || !aligned(probs, 16) || (logits && !aligned(logits, 16))))
    return fail(SOP_ERR_INVALID_ARGUMENT, "probs is NULL or probs/logits not 16-byte aligned");
  if ((st = validate_ws(ws, ws_bytes, proposal_ws(SOP_OP_PROPOSAL_INFER, pts->count))) != SOP_OK)
    return st;
  if (pts->count == 0) return SOP_OK;
  const hipStream_t s = (hipStream_t)stream;
  Bump b{(char*)ws, 0, ws_bytes};
  uint16_t* frags = b.take<uint16_t>(sopk::mlp_frag_bytes() / sizeof(uint16_t));
  sopk::MlpArgs a = mlp_args(mlp, pts);
  a.frags = frags;
  a.probs = probs;
  a.logits = logits;
  SOP_HIP(sopk::launch_mlp_frags(mlp->params, frags, s), "sop_proposal_infer");
  SOP_HIP(sopk::launch_mlp_infer(a, s), "sop_proposal_infer");
  return SOP_OK;
}

extern "C" sop_status sop_adam_update(float* params, float* adam_m, float* adam_v,
                                      const float* grad, int64_t n, const sop_adam* opt,
                                      sop_stream stream) {
  if (!opt) return fail(SOP_ERR_INVALID_ARGUMENT, "opt is NULL");
  if (n < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "n < 0");
  sop_status st = validate_adam(opt);
  if (st != SOP_OK) return st;
  if (n == 0) return SOP_OK;
  const void* req[] = {params, adam_m, adam_v, grad};
  for (const void* p : req)
    if (!p || !aligned(p, 4))
      return fail(SOP_ERR_INVALID_ARGUMENT, "an Adam array is NULL or misaligned");
  const double ic1 = 1.0 / (1.0 - std::pow((double)opt->beta1, opt->step));
  const double ic2 = 1.0 / (1.0 - std::pow((double)opt->beta2, opt->step));
  SOP_HIP(sopk::launch_adam(params, adam_m, adam_v, grad, n, opt->lr, opt->beta1, opt->beta2,
                            opt->eps, (float)ic1, (float)ic2, (hipStream_t)stream),
          "sop_adam_update");
  return SOP_OK;
}

extern "C" sop_status sop_proposal_train_step(const sop_mlp* mlp, const sop_points* pts,
                                              const float* targets, const sop_adam* opt,
                                              float* adam_m, float* adam_v, float* loss,
                                              float* grad, void* ws, size_t ws_bytes,
                                              sop_stream stream) {
  sop_status st = validate_mlp(mlp);
  if (st != SOP_OK) return st;
  if ((st = validate_mlp_points(pts)) != SOP_OK) return st;
  if (pts->count > 0 && (!targets || !aligned(targets, 16)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "targets is NULL or not 16-byte aligned");
  if (!loss || !aligned(loss, 4)) return fail(SOP_ERR_INVALID_ARGUMENT, "loss is NULL or misaligned");
  if (grad && !aligned(grad, 4)) return fail(SOP_ERR_INVALID_ARGUMENT, "grad misaligned");
  if (opt) {
    if ((st = validate_adam(opt)) != SOP_OK) return st;
    if (!adam_m || !adam_v || !aligned(adam_m, 4) || !aligned(adam_v, 4))
      return fail(SOP_ERR_INVALID_ARGUMENT, "adam_m/adam_v NULL or misaligned");
  }
  if ((st = validate_ws(ws, ws_bytes, proposal_ws(SOP_OP_PROPOSAL_TRAIN, pts->count))) != SOP_OK)
    return st;
  if (pts->count == 0) return SOP_OK;
  const hipStream_t s = (hipStream_t)stream;
  Bump b{(char*)ws, 0, ws_bytes};
  sopk::MlpArgs a = mlp_args(mlp, pts);
  const size_t ld = (size_t)((pts->count + 31) / 32) * 32;   // K steps of 32 in the weight gradients
  uint16_t* frags = b.take<uint16_t>(sopk::mlp_frag_bytes() / sizeof(uint16_t));
  a.frags = frags;
  a.xT = b.take<uint16_t>((size_t)SOP_MLP_IN * ld);
  a.h1T = b.take<uint16_t>((size_t)SOP_MLP_HIDDEN * ld);
  a.h2T = b.take<uint16_t>((size_t)SOP_MLP_HIDDEN * ld);
  a.dz1T = b.take<uint16_t>((size_t)SOP_MLP_HIDDEN * ld);
  a.dz2T = b.take<uint16_t>((size_t)SOP_MLP_HIDDEN * ld);
  a.dz3T = b.take<uint16_t>((size_t)SOP_MLP_BINS * ld);
  float* ws_grad = b.take<float>(SOP_MLP_PARAMS);
  a.part = b.take<float>((ld / 16) * sopk::kMlpPart);
  a.ldT = (int64_t)ld;
  a.targets = targets;
  a.loss = loss;
  a.grad = grad ? grad : ws_grad;          // every entry and the loss are written
  SOP_HIP(sopk::launch_mlp_frags(mlp->params, frags, s), "sop_proposal_train_step");
  SOP_HIP(sopk::launch_mlp_train(a, s), "sop_proposal_train_step");
  if (opt) return sop_adam_update(mlp->params, adam_m, adam_v, a.grad, SOP_MLP_PARAMS, opt, stream);
  return SOP_OK;
}

// ------------------------------------------------------------------------------------------
// bake
// ------------------------------------------------------------------------------------------
struct sop_bake_plan {
  int32_t G = 0;
  sop_bake_opts opts{};
  float4* gdata = nullptr;
  float4* aabb = nullptr;
  uint64_t* cellmask = nullptr;   // [G][kCellMaskWords] acceptance bits of the count pass
  int32_t* counts = nullptr;
  int32_t* cell_start = nullptr;
  int32_t* cursor = nullptr;
  int32_t* entries = nullptr;
  int32_t capacity = 0;
  int32_t* scan_tmp = nullptr;
  int32_t* misc = nullptr;   // [0..5] bounds (ordered ints), [6] n_reg, [7] overflow, [8] ext (float)
  sopk::BakeGrid grid{};
  size_t ncell = 0;

  void release() {
    void* ptrs[] = {gdata, aabb, cellmask, counts, cell_start, cursor, entries, scan_tmp, misc};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    gdata = aabb = nullptr;
    cellmask = nullptr;
    counts = cell_start = cursor = entries = scan_tmp = misc = nullptr;
  }
};

namespace {

float ord2f(int32_t v) {
  const int32_t b = v >= 0 ? v : v ^ 0x7FFFFFFF;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

sop_status validate_gaussians(const sop_gaussians* g) {
  if (!g) return fail(SOP_ERR_INVALID_ARGUMENT, "gaussians is NULL");
  if (g->count < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "gaussians->count < 0");
  if (g->count == 0) return SOP_OK;
  const void* req[] = {g->mean, g->scale, g->rotation, g->opacity, g->color};
  for (const void* p : req)
    if (!p || !aligned(p, 4))
      return fail(SOP_ERR_INVALID_ARGUMENT, "a Gaussian array is NULL or misaligned");
  return SOP_OK;
}

sop_bake_opts resolve_bake_opts(const sop_bake_opts* o) {
  sop_bake_opts r;
  r.t_min = 0.0f;
  r.alpha_min = 1.0f / 255.0f;
  r.alpha_max = 0.99f;
  r.T_min = 1e-4f;
  r.cell_scale = 0.0f;
  if (o) r = *o;
  return r;
}

hipError_t register_gaussians(sop_bake_plan* pl, hipStream_t s) {
  hipError_t e = sopk::launch_fill_i32(pl->counts, 0, pl->ncell, s);
  if (e == hipSuccess) e = sopk::launch_fill_i32(pl->cursor, 0, pl->ncell, s);
  if (e == hipSuccess)
    e = sopk::launch_gauss_count(pl->grid, pl->aabb, pl->counts, pl->cellmask, pl->misc + 7, s);
  if (e == hipSuccess)
    e = sopk::launch_exclusive_scan(pl->counts, pl->cell_start, pl->ncell, pl->scan_tmp, s);
  return e;
}

}  // namespace

extern "C" sop_status sop_bake_plan_create(const sop_gaussians* g, const sop_bake_opts* opts,
                                           sop_stream stream, sop_bake_plan** out) {
  if (!out) return fail(SOP_ERR_INVALID_ARGUMENT, "out is NULL");
  sop_status st = validate_gaussians(g);
  if (st != SOP_OK) return st;
  const sop_bake_opts o = resolve_bake_opts(opts);
  if (!(o.alpha_min > 0.0f) || !(o.alpha_max >= o.alpha_min) || !(o.alpha_max < 1.0f) ||
      !(o.T_min > 0.0f) || !(o.t_min >= 0.0f) || !std::isfinite(o.t_min) ||
      !(o.cell_scale >= 0.0f))
    return fail(SOP_ERR_INVALID_ARGUMENT, "bake options out of range");
  const hipStream_t s = (hipStream_t)stream;
  sop_bake_plan* pl = new (std::nothrow) sop_bake_plan();
  if (!pl) return fail(SOP_ERR_OUT_OF_MEMORY, "host allocation failed");
  pl->G = g->count;
  pl->opts = o;
  const size_t G1 = g->count > 0 ? (size_t)g->count : 1;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  alloc((void**)&pl->gdata, G1 * 5 * sizeof(float4));
  alloc((void**)&pl->aabb, G1 * 2 * sizeof(float4));
  alloc((void**)&pl->cellmask, G1 * sopk::kCellMaskWords * sizeof(uint64_t));
  alloc((void**)&pl->misc, 16 * sizeof(int32_t));
  auto bail = [&](sop_status code, const std::string& msg) {
    pl->release();
    delete pl;
    return fail(code, msg);
  };
  if (e != hipSuccess) return bail(SOP_ERR_OUT_OF_MEMORY, "bake plan allocation");
  // each pointer of the device view is set as soon as its buffer exists
  pl->grid.gdata = pl->gdata;
  pl->grid.overflow = pl->misc + 7;
  int32_t init[16] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN, 0, 0,
                      0, 0, 0, 0, 0, 0, 0, 0};
  e = hipMemcpyAsync(pl->misc, init, sizeof(init), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = sopk::launch_gauss_prep(*g, o.alpha_min, pl->gdata, pl->aabb, pl->misc,
                                reinterpret_cast<float*>(pl->misc + 8), pl->misc + 6, s);
  int32_t host[16];
  if (e == hipSuccess) e = hipMemcpyAsync(host, pl->misc, sizeof(host), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(SOP_ERR_DEVICE, std::string("bake plan: ") + hipGetErrorString(e));

  // grid geometry: the box around all cut-off boxes, cells about one Gaussian box wide
  sopk::BakeGrid& G = pl->grid;
  G.G = g->count;
  const int32_t n_reg = host[6];
  float ext_sum;
  std::memcpy(&ext_sum, &host[8], 4);
  if (n_reg > 0) {
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = ord2f(host[a]);
      hi[a] = ord2f(host[3 + a]);
      const float pad = 1e-4f * (hi[a] - lo[a]) + 1e-5f;
      lo[a] -= pad;
      hi[a] += pad;
    }
    const double cs = o.cell_scale > 0.0f ? (double)o.cell_scale : 0.25;
    double h = cs * (double)ext_sum / n_reg;
    if (!(h > 0)) h = 1.0;
    for (;;) {
      size_t cells = 1;
      for (int a = 0; a < 3; ++a) {
        const double n = std::ceil((hi[a] - lo[a]) / h);
        G.dims[a] = (int32_t)std::max(1.0, std::min(n, 1024.0));
        cells *= (size_t)G.dims[a];
      }
      if (cells <= ((size_t)1 << 24)) break;
      h *= 1.25;
    }
    for (int a = 0; a < 3; ++a) {
      G.origin[a] = lo[a];
      G.cell[a] = (hi[a] - lo[a]) / (float)G.dims[a];
      G.inv_cell[a] = 1.0f / G.cell[a];
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      G.dims[a] = 0;
      G.origin[a] = 0.0f;
      G.cell[a] = 1.0f;
      G.inv_cell[a] = 1.0f;
    }
  }
  G.t_min = o.t_min;
  G.alpha_min = o.alpha_min;
  G.alpha_max = o.alpha_max;
  G.T_min = o.T_min;
  pl->ncell = (size_t)G.dims[0] * G.dims[1] * G.dims[2];
  const size_t C1 = pl->ncell > 0 ? pl->ncell : 1;
  alloc((void**)&pl->counts, C1 * sizeof(int32_t));
  alloc((void**)&pl->cell_start, (C1 + 1) * sizeof(int32_t));
  alloc((void**)&pl->cursor, C1 * sizeof(int32_t));
  alloc((void**)&pl->scan_tmp, sopk::scan_tmp_elems(C1) * sizeof(int32_t));
  if (e != hipSuccess) return bail(SOP_ERR_OUT_OF_MEMORY, "bake grid allocation");
  G.cell_start = pl->cell_start;
  int32_t total = 0;
  e = register_gaussians(pl, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&total, pl->cell_start + pl->ncell, sizeof(int32_t),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(SOP_ERR_DEVICE, std::string("bake grid: ") + hipGetErrorString(e));
  const int64_t cap = (int64_t)total + total / 4 + 1024;
  if (cap > INT32_MAX) return bail(SOP_ERR_UNSUPPORTED, "too many grid registrations");
  pl->capacity = (int32_t)cap;
  alloc((void**)&pl->entries, (size_t)pl->capacity * sizeof(int32_t));
  if (e != hipSuccess) return bail(SOP_ERR_OUT_OF_MEMORY, "bake entries allocation");
  G.entries = pl->entries;
  G.capacity = pl->capacity;
  e = sopk::launch_gauss_fill(G, pl->aabb, pl->cellmask, pl->cell_start, pl->cursor,
                              pl->entries, pl->capacity, pl->misc + 7, s);
  if (e != hipSuccess) return bail(SOP_ERR_DEVICE, std::string("bake fill: ") + hipGetErrorString(e));
  *out = pl;
  return SOP_OK;
}

extern "C" sop_status sop_bake_plan_update(sop_bake_plan* plan, const sop_gaussians* g,
                                           sop_stream stream) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  sop_status st = validate_gaussians(g);
  if (st != SOP_OK) return st;
  if (g->count != plan->G)
    return fail(SOP_ERR_INVALID_ARGUMENT, "update needs the Gaussian count of the plan");
  const hipStream_t s = (hipStream_t)stream;
  SOP_HIP(sopk::launch_fill_i32(plan->misc + 7, 0, 1, s), "sop_bake_plan_update");
  SOP_HIP(sopk::launch_gauss_prep(*g, plan->opts.alpha_min, plan->gdata, plan->aabb, nullptr,
                                  nullptr, nullptr, s),
          "sop_bake_plan_update");
  if (plan->ncell == 0) {
    if (plan->G > 0) SOP_HIP(sopk::launch_fill_i32(plan->misc + 7, 4, 1, s), "sop_bake_plan_update");
    return SOP_OK;
  }
  SOP_HIP(register_gaussians(plan, s), "sop_bake_plan_update");
  SOP_HIP(sopk::launch_gauss_fill(plan->grid, plan->aabb, plan->cellmask, plan->cell_start,
                                  plan->cursor, plan->entries, plan->capacity, plan->misc + 7,
                                  s),
          "sop_bake_plan_update");
  return SOP_OK;
}

extern "C" sop_status sop_bake_plan_check(const sop_bake_plan* plan, sop_stream stream) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  int32_t flag = 0;
  SOP_HIP(hipMemcpyAsync(&flag, plan->misc + 7, sizeof(int32_t), hipMemcpyDeviceToHost,
                         (hipStream_t)stream),
          "sop_bake_plan_check");
  SOP_HIP(hipStreamSynchronize((hipStream_t)stream), "sop_bake_plan_check");
  if (flag)
    return fail(SOP_ERR_WORKSPACE_TOO_SMALL,
                "Gaussian update exceeded the grid built at plan creation (flag " +
                    std::to_string(flag) + ")");
  return SOP_OK;
}

extern "C" sop_status sop_bake_plan_destroy(sop_bake_plan* plan) {
  if (!plan) return SOP_OK;
  plan->release();
  delete plan;
  return SOP_OK;
}

extern "C" sop_status sop_bake(const sop_bake_plan* plan, const float* probe_pos,
                               int32_t n_probes, int32_t res, float* texels, float* depth,
                               const sop_plan* order_by, sop_stream stream) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (n_probes < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "n_probes < 0");
  if (order_by && order_by->P != n_probes)
    return fail(SOP_ERR_INVALID_ARGUMENT, "order_by holds a different number of probes");
  if (res < 2 || res > SOP_MAX_RES) return fail(SOP_ERR_INVALID_ARGUMENT, "res out of [2, 256]");
  if (n_probes > 0 && (!probe_pos || !texels || !aligned(probe_pos, 4) || !aligned(texels, 16) ||
                       (depth && !aligned(depth, 4))))
    return fail(SOP_ERR_INVALID_ARGUMENT, "probe_pos/texels NULL or misaligned");
  if (n_probes == 0) return SOP_OK;
  SOP_HIP(sopk::launch_bake(plan->grid, probe_pos, n_probes, res, texels, depth,
                            order_by ? order_by->qsorted : nullptr, (hipStream_t)stream),
          "sop_bake");
  return SOP_OK;
}

// ------------------------------------------------------------------------------------------
// traced shading
// ------------------------------------------------------------------------------------------
namespace {

// Workspace layout: [direction table, environment references] [order, order scratch]
// [samples when the caller passes none]
size_t traced_ws(const sop_plan* order_by, int64_t N, int32_t S, int32_t H, int32_t W,
                 bool with_samples) {
  Bump b{nullptr, 0, 0};
  (void)b.take<double4>((size_t)S);
  (void)b.take<double2>((size_t)W + 2);
  (void)b.take<double2>((size_t)H + 2);
  if (order_by) {
    (void)b.take<int32_t>((size_t)N);
    carve_knn(b, order_by, N);
  }
  if (!with_samples) (void)b.take<float4>((size_t)N * S);
  return b.used;
}

}  // namespace

extern "C" size_t sop_shade_traced_workspace_size(const sop_plan* order_by, int64_t n_points,
                                                  int32_t n_dirs, int32_t env_height,
                                                  int32_t env_width, int32_t with_samples) {
  if (n_points < 0 || n_dirs < 1 || n_dirs > SOP_MAX_DIRS || env_height < 0 || env_width < 0)
    return 0;
  const size_t need =
      traced_ws(order_by, n_points, n_dirs, env_height, env_width, with_samples != 0);
  return need > 0 ? need : 256;
}

extern "C" sop_status sop_shade_traced(const sop_bake_plan* gauss, const sop_plan* order_by,
                                       const sop_envmap* env, const sop_points* pts,
                                       const sop_shade_opts* opts, float offset, float* rgb,
                                       float* samples, void* ws, size_t ws_bytes,
                                       sop_stream stream) {
  if (!gauss) return fail(SOP_ERR_INVALID_ARGUMENT, "gauss is NULL");
  if (!opts) return fail(SOP_ERR_INVALID_ARGUMENT, "opts is NULL");
  sop_status st = validate_points(pts);
  if (st != SOP_OK) return st;
  if ((st = validate_env(env)) != SOP_OK) return st;
  if (opts->n_dirs < 1 || opts->n_dirs > SOP_MAX_DIRS)
    return fail(SOP_ERR_INVALID_ARGUMENT, "n_dirs out of [1, 4096]");
  if (opts->sampler != SOP_SAMPLER_HAMMERSLEY)
    return fail(SOP_ERR_UNSUPPORTED, "traced shading uses the Hammersley sampler only");
  if (!(offset >= 0.0f) || !std::isfinite(offset))
    return fail(SOP_ERR_INVALID_ARGUMENT, "offset must be finite and >= 0");
  if (pts->count > 0 && (!rgb || !aligned(rgb, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "rgb is NULL or misaligned");
  if (samples && !aligned(samples, 16))
    return fail(SOP_ERR_INVALID_ARGUMENT, "samples not 16-byte aligned");
  if (opts->out_irradiance && !aligned(opts->out_irradiance, 4))
    return fail(SOP_ERR_INVALID_ARGUMENT, "out_irradiance misaligned");
  const int64_t N = pts->count;
  const int32_t S = opts->n_dirs;
  // one wavefront per 32 points and direction, four per workgroup
  if ((N + 31) / 32 > ((int64_t)INT32_MAX * 4) / S)
    return fail(SOP_ERR_UNSUPPORTED, "too many samples for one launch");
  const size_t need = traced_ws(order_by, N, S, env->height, env->width, samples != nullptr);
  if ((st = validate_ws(ws, ws_bytes, need)) != SOP_OK) return st;
  if (N == 0) return SOP_OK;
  const hipStream_t s = (hipStream_t)stream;
  sopk::ShadeArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = N;
  a.pos = pts->pos;
  a.nrm = pts->normal;
  a.view = pts->view;
  a.cam = pts->cam_pos;
  a.ppf = pts->points_per_frame > 0 ? pts->points_per_frame : 1;
  a.albedo = pts->albedo;
  a.rough = pts->roughness;
  a.metal = pts->metallic;
  set_dirs(a, env, opts);
  a.rgb = rgb;
  a.irr = opts->out_irradiance;
  Bump b{(char*)ws, 0, ws_bytes};
  if ((st = setup_dirs(a, b, opts, s)) != SOP_OK) return st;
  int32_t* order = nullptr;
  if (order_by) {
    order = b.take<int32_t>((size_t)N);
    KnnScratch ks = carve_knn(b, order_by, N);
    SOP_HIP(sopk::launch_point_order(order_by->view(), pts->pos, N, ks.point_cell, ks.counts,
                                     ks.offsets, ks.scan_tmp, order, s),
            "sop_shade_traced");
  }
  float4* buf = samples ? reinterpret_cast<float4*>(samples) : b.take<float4>((size_t)N * S);
  sopk::TraceArgs t;
  t.n = N;
  t.S = S;
  t.pos = pts->pos;
  t.nrm = pts->normal;
  t.order = order;
  t.dir_tab = a.dir_tab;
  t.seed = opts->seed;
  t.per_point = opts->rotate_per_point ? 1 : 0;
  t.offset = offset;
  t.out = buf;
  SOP_HIP(sopk::launch_trace_samples(gauss->grid, t, s), "sop_shade_traced");
  a.order = order;
  a.traced = buf;
  SOP_HIP(sopk::launch_shade_traced(a, s), "sop_shade_traced");
  return SOP_OK;
}

// ------------------------------------------------------------------------------------------
// cast-shadow ratio
// ------------------------------------------------------------------------------------------
namespace {

// Workspace layout: [direction table] [texel masses] [mass prefix sums] [tile sums]
// [intensity maximum] [order, idx, w] [search scratch]
size_t shadow_ws(const sop_plan* plan, int64_t N, int32_t k, int32_t S, int32_t Re,
                 bool with_nb) {
  Bump b{nullptr, 0, 0};
  (void)b.take<double4>((size_t)S);
  (void)b.take<uint32_t>((size_t)Re * Re);
  (void)b.take<uint64_t>((size_t)Re * Re + 1);
  (void)b.take<uint64_t>(((size_t)Re * Re + 1023) / 1024);
  (void)b.take<float>(1);
  (void)b.take<int32_t>((size_t)sopk::kEnvGuide + 1);
  if (!with_nb) {
    carve_nb(b, N, k);
    carve_knn(b, plan, N);
  }
  return b.used;
}

}  // namespace

extern "C" size_t sop_shadow_workspace_size(const sop_plan* plan, int64_t n_points, int32_t k,
                                            int32_t n_dirs, int32_t env_res,
                                            int32_t with_neighbors) {
  if (!plan || n_points < 0 || n_dirs < 1 || n_dirs > SOP_MAX_DIRS || env_res < 2 ||
      env_res > 1024)
    return 0;
  if (!with_neighbors && (k < 1 || k > SOP_MAX_K)) return 0;
  const size_t need = shadow_ws(plan, n_points, k, n_dirs, env_res, with_neighbors != 0);
  return need > 0 ? need : 256;
}

extern "C" sop_status sop_shadow_ratio(const sop_plan* plan, const sop_probe_maps* maps,
                                       const sop_env_oct* env, const sop_points* pts,
                                       const sop_neighbors* nb, const sop_shadow_opts* opts,
                                       float* ratio, void* ws, size_t ws_bytes,
                                       sop_stream stream) {
  if (!plan) return fail(SOP_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (!opts) return fail(SOP_ERR_INVALID_ARGUMENT, "opts is NULL");
  if (!pts) return fail(SOP_ERR_INVALID_ARGUMENT, "pts is NULL");
  if (pts->count < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "pts->count < 0");
  if (pts->count > INT32_MAX) return fail(SOP_ERR_UNSUPPORTED, "more than 2^31-1 points");
  if (pts->count > 0 && (!pts->pos || !pts->normal || !aligned(pts->pos, 4) ||
                         !aligned(pts->normal, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "pts->pos/normal NULL or misaligned");
  sop_status st = validate_maps(plan, maps);
  if (st != SOP_OK) return st;
  if (!env) return fail(SOP_ERR_INVALID_ARGUMENT, "env is NULL");
  if (env->res < 2 || env->res > 1024)
    return fail(SOP_ERR_INVALID_ARGUMENT, "env->res out of [2, 1024]");
  if (!env->texels || !aligned(env->texels, 4))
    return fail(SOP_ERR_INVALID_ARGUMENT, "env->texels is NULL or misaligned");
  if (nb) {
    if ((st = validate_nb(nb)) != SOP_OK) return st;
  } else if ((st = validate_k_radius(opts->k, opts->radius)) != SOP_OK) {
    return st;
  }
  if (opts->n_dirs < 1 || opts->n_dirs > SOP_MAX_DIRS)
    return fail(SOP_ERR_INVALID_ARGUMENT, "n_dirs out of [1, 4096]");
  if (opts->sampler != SOP_SHADOW_HAMMERSLEY && opts->sampler != SOP_SHADOW_ENV &&
      opts->sampler != SOP_SHADOW_ENV_EXACT)
    return fail(SOP_ERR_UNSUPPORTED, "unknown shadow sampler");
  if (pts->count > 0 && (!ratio || !aligned(ratio, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "ratio is NULL or misaligned");
  if (opts->out_irradiance && !aligned(opts->out_irradiance, 4))
    return fail(SOP_ERR_INVALID_ARGUMENT, "out_irradiance misaligned");
  const int32_t k = nb ? nb->k : opts->k;
  const size_t need = shadow_ws(plan, pts->count, k, opts->n_dirs, env->res, nb != nullptr);
  if ((st = validate_ws(ws, ws_bytes, need)) != SOP_OK) return st;
  if (pts->count == 0) return SOP_OK;
  const hipStream_t s = (hipStream_t)stream;
  sopk::ShadeArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = pts->count;
  a.pos = pts->pos;
  a.nrm = pts->normal;
  a.P = plan->P;
  a.tex = maps->texels;
  a.R = maps->res;
  a.env = env->texels;
  a.env_res = env->res;
  a.S = opts->n_dirs;
  a.seed = opts->seed;
  a.per_point = opts->rotate_per_point ? 1 : 0;
  a.shadow_sampler = opts->sampler;
  a.env_pdf_exact = opts->sampler == SOP_SHADOW_ENV_EXACT ? 1 : 0;
  a.rgb = ratio;
  a.irr = opts->out_irradiance;
  Bump b{(char*)ws, 0, ws_bytes};
  double4* tab = b.take<double4>((size_t)opts->n_dirs);
  const int32_t T = env->res * env->res;
  uint32_t* mass = b.take<uint32_t>((size_t)T);
  uint64_t* prefix = b.take<uint64_t>((size_t)T + 1);
  uint64_t* tile_tmp = b.take<uint64_t>(((size_t)T + 1023) / 1024);
  float* imax = b.take<float>(1);
  int32_t* guide = b.take<int32_t>((size_t)sopk::kEnvGuide + 1);
  if (opts->sampler == SOP_SHADOW_HAMMERSLEY) {
    a.dir_tab = tab;
    // the table's environment references are not used here (width/height 0)
    SOP_HIP(sopk::launch_dir_table(opts->n_dirs, opts->seed, a.per_point, 0, 0, tab, nullptr,
                                   nullptr, s),
            "sop_shadow_ratio");
  } else {
    a.env_mass = mass;
    a.env_prefix = prefix;
    a.env_guide = guide;
    SOP_HIP(sopk::launch_env_cdf(env->texels, T, mass, prefix, tile_tmp, imax, guide, s),
            "sop_shadow_ratio");
  }
  int32_t kk;
  if ((st = resolve_nb(plan, pts, nb, opts->k, opts->radius, b, s, &a.order, &a.nb_idx,
                       &a.nb_w, &kk)) != SOP_OK)
    return st;
  SOP_HIP(sopk::launch_shadow_ratio(a, kk, maps->format, s), "sop_shadow_ratio");
  return SOP_OK;
}

// ------------------------------------------------------------------------------------------
// probe placement and the losses of the reconstruction step
// ------------------------------------------------------------------------------------------
namespace {

// Workspace layout: [points with their distance to the nearest pick, 4 floats each] [the
// words the picks are exchanged through and a fault flag] [picks, used when the caller
// passes no array for them]
size_t place_ws(int64_t M, int32_t P) {
  Bump b{nullptr, 0, 0};
  (void)b.take<float>(4 * (size_t)M);
  (void)b.take<uint64_t>(sopk::kFpsSyncWords);
  (void)b.take<int32_t>((size_t)P);
  return b.used;
}

}  // namespace

extern "C" size_t sop_place_workspace_size(int64_t n_points, int32_t n_probes) {
  if (n_points < 1 || n_points > INT32_MAX || n_probes < 1 || n_probes > n_points) return 0;
  return place_ws(n_points, n_probes);
}

extern "C" sop_status sop_place_probes(const float* pts, const float* normals,
                                       int64_t n_points, int32_t n_probes, int64_t start,
                                       float offset, int32_t* chosen, float* probe_pos,
                                       void* ws, size_t ws_bytes, sop_stream stream) {
  if (n_points < 1 || n_points > INT32_MAX)
    return fail(SOP_ERR_INVALID_ARGUMENT, "n_points out of [1, 2^31-1]");
  if (n_probes < 1 || n_probes > n_points)
    return fail(SOP_ERR_INVALID_ARGUMENT, "n_probes out of [1, n_points]");
  if (start < 0 || start >= n_points)
    return fail(SOP_ERR_INVALID_ARGUMENT, "start out of [0, n_points)");
  if (!std::isfinite(offset)) return fail(SOP_ERR_INVALID_ARGUMENT, "offset is not finite");
  if (!pts || !normals || !probe_pos || !aligned(pts, 4) || !aligned(normals, 4) ||
      !aligned(probe_pos, 4) || (chosen && !aligned(chosen, 4)))
    return fail(SOP_ERR_INVALID_ARGUMENT, "pts/normals/probe_pos NULL or misaligned");
  sop_status st = validate_ws(ws, ws_bytes, place_ws(n_points, n_probes));
  if (st != SOP_OK) return st;
  Bump b{(char*)ws, 0, ws_bytes};
  float* packed = b.take<float>(4 * (size_t)n_points);
  uint64_t* sync = b.take<uint64_t>(sopk::kFpsSyncWords);
  int32_t* picks = b.take<int32_t>((size_t)n_probes);
  SOP_HIP(sopk::launch_place_probes(pts, normals, n_points, n_probes, start, offset, packed, sync,
                                    chosen ? chosen : picks, probe_pos, (hipStream_t)stream),
          "sop_place_probes");
  return SOP_OK;
}

extern "C" size_t sop_loss_workspace_size(int64_t n_elements) {
  if (n_elements < 0) return 0;
  Bump b{nullptr, 0, 0};
  (void)b.take<double>(sopk::loss_partials(n_elements));
  return b.used;
}

extern "C" sop_status sop_sops_loss(const float* tex, const float* target, int64_t n_texels,
                                    float* loss, float* grad, void* ws, size_t ws_bytes,
                                    sop_stream stream) {
  if (n_texels < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "n_texels < 0");
  if (!loss || !aligned(loss, 4)) return fail(SOP_ERR_INVALID_ARGUMENT, "loss NULL or misaligned");
  if (n_texels > 0 && (!tex || !target || !aligned(tex, 16) || !aligned(target, 16) ||
                       (grad && !aligned(grad, 16))))
    return fail(SOP_ERR_INVALID_ARGUMENT, "tex/target/grad NULL or not 16-byte aligned");
  sop_status st = validate_ws(ws, ws_bytes, sop_loss_workspace_size(n_texels));
  if (st != SOP_OK) return st;
  SOP_HIP(sopk::launch_sops_loss(tex, target, n_texels, loss, grad, (double*)ws,
                                 (hipStream_t)stream),
          "sop_sops_loss");
  return SOP_OK;
}

extern "C" sop_status sop_lam_loss(const float* rough, const float* metal, int64_t n_points,
                                   float* loss, float* g_rough, float* g_metal, void* ws,
                                   size_t ws_bytes, sop_stream stream) {
  if (n_points < 0) return fail(SOP_ERR_INVALID_ARGUMENT, "n_points < 0");
  if (!loss || !aligned(loss, 4)) return fail(SOP_ERR_INVALID_ARGUMENT, "loss NULL or misaligned");
  if (n_points > 0 && (!rough || !metal || !aligned(rough, 4) || !aligned(metal, 4) ||
                       (g_rough && !aligned(g_rough, 4)) || (g_metal && !aligned(g_metal, 4))))
    return fail(SOP_ERR_INVALID_ARGUMENT, "rough/metal/gradients NULL or misaligned");
  sop_status st = validate_ws(ws, ws_bytes, sop_loss_workspace_size(n_points));
  if (st != SOP_OK) return st;
  SOP_HIP(sopk::launch_lam_loss(rough, metal, n_points, loss, g_rough, g_metal, (double*)ws,
                                (hipStream_t)stream),
          "sop_lam_loss");
  return SOP_OK;
}

// ------------------------------------------------------------------------------------------
// shading without allocation: the workspace is a fixed device array of this library
// ------------------------------------------------------------------------------------------
namespace {

// Every device that runs the library holds its own copy until the process ends. In host
// code the name below only stands in for the array: its device address (per device) comes
// from hipGetSymbolAddress and is the only form passed to kernels.
__device__ __align__(256) unsigned char scratch[SOP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's copy of `scratch`, looked up once per device
sop_status current_scratch(void** out) {
  int dev = -1;
  SOP_HIP(hipGetDevice(&dev), "sop_shade_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SOP_ERR_UNSUPPORTED, "sop_shade_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SOP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
            "sop_shade_noalloc: scratch address");
    if (!p) return fail(SOP_ERR_DEVICE, "sop_shade_noalloc: scratch address is NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SOP_OK;
}

}  // namespace

extern "C" sop_status sop_shade_noalloc(const sop_plan* plan, const sop_probe_maps* maps,
                                        const sop_envmap* env, const sop_points* pts,
                                        const sop_neighbors* nb, const sop_shade_opts* opts,
                                        float* rgb, sop_stream stream) {
  sop_status st = validate_shade(plan, maps, env, pts, nb, opts, true);
  if (st != SOP_OK) return st;
  const int32_t k = nb ? nb->k : opts->k;
  const size_t need = ws_needed(plan, SOP_OP_SHADE, pts->count, k, nb != nullptr, opts->n_dirs,
                                env->height, env->width);
  if (need > (size_t)SOP_NOALLOC_SCRATCH_BYTES)
    return fail(SOP_ERR_WORKSPACE_TOO_SMALL,
                "sop_shade_noalloc: this call needs " + std::to_string(need) +
                    " bytes of scratch, the fixed array holds " +
                    std::to_string((size_t)SOP_NOALLOC_SCRATCH_BYTES) +
                    " (pass neighbour lists or fewer points)");
  void* ws = nullptr;
  if ((st = current_scratch(&ws)) != SOP_OK) return st;
  // sop_shade writes every scratch word it reads later in the same call (direction tables,
  // neighbour-search counters are cleared by its own kernels), so the previous call's
  // contents do not matter
  return sop_shade(plan, maps, env, pts, nb, opts, rgb, ws, (size_t)SOP_NOALLOC_SCRATCH_BYTES,
                   stream);
}

// ------------------------------------------------------------------------------------------
extern "C" const char* sop_status_string(int status) {
  switch (status) {
    case SOP_OK: return "ok";
    case SOP_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SOP_ERR_UNSUPPORTED: return "unsupported";
    case SOP_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case SOP_ERR_DEVICE: return "device error";
    case SOP_ERR_OUT_OF_MEMORY: return "out of memory";
  }
  return "unknown status";
}

extern "C" const char* sop_last_error(void) { return g_err.c_str(); }

extern "C" int32_t sop_version(void) { return 100; }
