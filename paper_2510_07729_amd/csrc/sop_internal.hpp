// sop_internal.hpp - types and kernel launchers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sop.h"

namespace sopk {

// Device view of a probe grid: the probes' lattice coordinates sorted by the Morton index
// of their cell, with cell ranges, over a cube of 2^bits cells per axis covering the
// 2^15 lattice (cell side 2^(15-bits) lattice units).
struct ProbeGrid {
  int32_t P;
  int32_t bits;
  int32_t shift;          // 15 - bits
  float lo[3];
  float sc;               // lattice scale (cells per world unit * 2^shift)
  const int4* qsorted;    // [P] (qx, qy, qz, probe index), cell-major
  const int32_t* cell_start;  // [8^bits + 1]
  const float* pos;       // [P,3] probe positions, original order
};

// Bump allocator over a caller workspace (256-byte aligned pieces).
struct Bump {
  char* base;
  size_t used, cap;
  template <typename T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
    used += bytes;
    return p;
  }
};

// grid.hip ---------------------------------------------------------------------------------
size_t scan_tmp_elems(size_t n);
hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s);
// out[0..n] = exclusive scan of in[0..n), out[n] = total; tmp holds scan_tmp_elems(n) ints
hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, size_t n, int32_t* tmp,
                                 hipStream_t s);
hipError_t launch_probe_grid_build(const float* pos, int32_t P, const float lo[3], float sc,
                                   int32_t bits, int4* qtmp, int32_t* counts,
                                   int32_t* cell_start, int32_t* cursor, int4* qsorted,
                                   float* pos_copy, int32_t* scan_tmp, hipStream_t s);
// points -> processing order grouped by grid cell (counting sort by Morton cell)
hipError_t launch_point_order(const ProbeGrid& g, const float* pts, int64_t N,
                              int32_t* point_cell, int32_t* counts, int32_t* offsets,
                              int32_t* scan_tmp, int32_t* order, hipStream_t s);
hipError_t launch_knn(const ProbeGrid& g, const float* pts, const float* normals, int64_t N,
                      const int32_t* order, int32_t k, uint32_t radius_limit, int32_t* idx,
                      float* w, hipStream_t s);

// shade.hip --------------------------------------------------------------------------------
struct ShadeArgs {
  int64_t n;
  const float* pos;
  const float* nrm;
  const float* view;
  const float* cam;
  int64_t ppf;
  const float* albedo;
  const float* rough;
  const float* metal;
  const int32_t* order;
  const int32_t* nb_idx;
  const float* nb_w;
  int32_t P;
  const void* tex;
  int32_t R;
  float halfR;
  const float* env;
  int32_t H, W;
  float u_scale, v_scale;
  int32_t S;
  const double4* dir_tab;   // [S] local directions of the call (see dir_entry)
  const double4* dir_sorted;  // [S] the same directions along a Z curve over the hemisphere
  const double2* col_ref;   // [W+2] environment column reference directions
  const double2* row_ref;   // [H+2] environment row reference directions
  float inv2S;
  float scale;            // 2 pi / S
  uint32_t seed;
  int32_t per_point;
  float* rgb;
  float* irr;
  const float4* traced;     // [n,S] (L_in rgb, O) per sample (traced shading)
  int32_t env_oct;          // env is an octahedral map [W,W,3] (else equirectangular [H,W,3])
  int32_t cosine;           // forward: dir_sorted is the cosine-weighted set (weights in .w)
  // cast-shadow ratio: octahedral environment in env, its texel masses and their prefix
  const uint32_t* env_mass; // [Re*Re]
  const uint64_t* env_prefix;  // [Re*Re + 1], env_prefix[Re*Re] = total mass
  const int32_t* env_guide;    // [kEnvGuide + 1] guide of the mass line (launch_env_cdf)
  int32_t env_res;
  int32_t shadow_sampler;   // 0 Hammersley, 1 environment importance sampling
  int32_t env_pdf_exact;    // importance draws weighted by their exact density (else Eq. 18's)
  // learned proposal sampler / training targets
  const float* probs;       // [n,256] bin distributions
  float mix_eps;
  float* targets;           // [n,256] bin integrals (integrand dump)
  const float* mlp_params;  // fused proposal: network parameters, bf16 fragments, feature box
  const uint16_t* mlp_frags;
  float mlp_lo[3], mlp_inv2[3];
  int32_t npb;              // draws per bin (integrand dump)
  // adjoint
  const float* grad;
  float* g_albedo;
  float* g_rough;
  float* g_metal;
  float* g_env;
  float* g_tex;
  // deterministic adjoint: exact accumulation of the texture and environment gradients in
  // 64-bit words, word k of value i at [k * n + i] (NULL: float atomics into g_tex / g_env)
  unsigned long long* det_tex;
  unsigned long long* det_env;
  int32_t* det_flag;        // set when a contribution cannot be represented
  int64_t det_nt, det_ne;   // values of g_tex and of g_env
  // float adjoint of the environment: 2x2-texel blocks (see env_block_count), NULL: float
  // atomics straight into g_env
  float* env_blk;
  int32_t env_bw, env_bh;   // blocks per row and per column of one parity class
};

// learned proposal network (proposal.hip)
// per 16-point training tile: column sums of dz1, dz2 (SOP_MLP_HIDDEN each), dz3
// (SOP_MLP_BINS) and the tile's loss
constexpr int kMlpPart = 2 * SOP_MLP_HIDDEN + SOP_MLP_BINS + 1;
struct MlpArgs {
  int64_t n;                 // points (inference) or batch size (training)
  const float* pos;
  const float* nrm;
  const float* view;         // or NULL: camera mode
  const float* cam;
  int64_t ppf;
  const float* rough;
  float lo[3], inv2[3];      // features: (pos - lo) * inv2 - 1, inv2 = 2 / (hi - lo)
  const float* params;       // [SOP_MLP_PARAMS] f32
  const uint16_t* frags;     // bf16 operand fragments of the weights
  float* probs;              // inference outputs [n,256]
  float* logits;
  // training
  const float* targets;      // [n,256]
  float* loss;               // [1]
  float* grad;               // [SOP_MLP_PARAMS]
  float* part;               // [ldT / 16][kMlpPart]: per-tile bias-gradient sums and loss
  uint16_t *xT, *h1T, *h2T, *dz1T, *dz2T, *dz3T;   // [rows][ldT] bf16, transposed operands
  int64_t ldT;               // batch rounded up to 16
};
size_t mlp_frag_bytes();
hipError_t launch_mlp_frags(const float* params, uint16_t* frags, hipStream_t s);
hipError_t launch_mlp_infer(const MlpArgs& a, hipStream_t s);
hipError_t launch_mlp_train(const MlpArgs& a, hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr,
                       float b1, float b2, float eps, float ic1, float ic2, hipStream_t s);

// per-call direction table: dir_entry(j, S, rho) with rho of the call (0 when per point)
hipError_t launch_dir_table(int32_t S, uint32_t seed, int32_t per_point, int32_t H, int32_t W,
                            double4* tab, double2* col_ref, double2* row_ref, hipStream_t s);
// the call's directions in the order of a Z curve over the hemisphere (shading forward)
hipError_t launch_dir_sort(int32_t S, uint32_t seed, int32_t per_point, double4* sorted,
                           hipStream_t s, int32_t cosine = 0);
hipError_t launch_shade_fwd(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s);
hipError_t launch_shade_bwd(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s);
// whether launch_shade_bwd takes the batched kernel (the one that reads a.env_blk)
bool shade_bwd_batched(int32_t res, int32_t k);
// out[i] += the exact sum held in words[k * n + i] (k = 0..3), rounded once; NaN if *flag
hipError_t launch_det_finish(const unsigned long long* words, int64_t n, const int32_t* flag,
                             float* out, hipStream_t s);
// Environment adjoint in blocks. A sample's bilinear footprint is the 2x2 texels whose
// corner is its (unwrapped) base tap (i0, j0); with the corner shifted by 2 (so that every
// corner the lookups make is >= 0), blocks of parity class (i0 & 1, j0 & 1) tile the
// plane so that the footprint is exactly one block: 12 floats (4 texels x 3 channels) in
// a 64-byte record. Classes x rows x columns of blocks for an H x W environment:
constexpr int kEnvBlkFloats = 16;
inline int32_t env_block_cols(int32_t W) { return W / 2 + 3; }
inline int32_t env_block_rows(int32_t H) { return H / 2 + 3; }
// the largest environment (texels) whose adjoint goes through blocks (~540 MB of them)
constexpr int64_t kEnvBlkMaxTexels = (int64_t)4096 * 2048;
// g_env += the blocks' values at their wrapped (equirectangular) or mirrored (octahedral)
// texels
hipError_t launch_env_blk_finish(const float* blk, int32_t bw, int32_t bh, int32_t H,
                                 int32_t W, bool octahedral, float* g_env, hipStream_t s);
hipError_t launch_shade_prop(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s);
hipError_t launch_dump_integrand(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s);
// cast-shadow ratio: texel masses and prefix of an octahedral environment [T <= 2^20
// texels]; tile_tmp holds ceil(T/1024) values, imax one
// The sampler's texel for a point x of the mass line is the largest t with prefix[t] <= x.
// guide[g] is that texel for x = g << shift (shift = max(0, bit length of the total - 16),
// so g < 2^16 + 1 cells cover the line): the texel of any x in cell g lies in
// [guide[g], guide[g + 1]], a few texels instead of the whole map.
constexpr int kEnvGuide = 65536;
hipError_t launch_env_cdf(const float* env, int32_t T, uint32_t* mass, uint64_t* prefix,
                          uint64_t* tile_tmp, float* imax, int32_t* guide, hipStream_t s);
// relighting with environment importance sampling (a.env octahedral, a.env_mass/prefix)
hipError_t launch_shade_envis(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s);
// ratio [n,3] in a.rgb (optional unshadowed estimate in a.irr)
hipError_t launch_shadow_ratio(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s);
// traced shading: the estimate of launch_shade_fwd with a.traced for L_in and O
hipError_t launch_shade_traced(const ShadeArgs& a, hipStream_t s);
hipError_t launch_shade_prop_net(const ShadeArgs& a, int32_t k, int32_t format,
                                 hipStream_t s);
hipError_t launch_query(const ShadeArgs& a, int32_t k, int32_t format, const float* dirs,
                        int32_t D, float* Lin, float* O, hipStream_t s);

// bake.hip ---------------------------------------------------------------------------------
struct BakeGrid {
  int32_t G;
  int32_t dims[3];
  float origin[3];
  float cell[3];           // cell size per axis
  float inv_cell[3];
  const float4* gdata;     // [G][5]: (M row0 | mu.x) (M row1 | mu.y) (M row2 | mu.z)
                           //          (color rgb | opacity) (r^2, r, cut-off radius,
                           //          opacity) with r the bounding sphere's radius
  const int32_t* cell_start;  // [cells + 1]
  const int32_t* entries;     // [capacity] Gaussian indices, cell-major
  int32_t capacity;
  const int32_t* overflow;    // device flag
  float t_min, alpha_min, alpha_max, T_min;
};

hipError_t launch_gauss_prep(const sop_gaussians& g, float alpha_min, float4* gdata,
                             float4* aabb, int32_t* bounds_ord, float* ext_sum, int32_t* n_reg,
                             hipStream_t s);
// 64-bit words of cell acceptance bits the count pass keeps per Gaussian for the fill pass
constexpr int kCellMaskWords = 4;
hipError_t launch_gauss_count(const BakeGrid& G, const float4* aabb, int32_t* counts,
                              uint64_t* cellmask, int32_t* overflow, hipStream_t s);
hipError_t launch_gauss_fill(const BakeGrid& G, const float4* aabb, const uint64_t* cellmask,
                             const int32_t* cell_start, int32_t* cursor, int32_t* entries,
                             int32_t capacity, int32_t* overflow, hipStream_t s);
// traced shading: one ray per (point, direction) sample
struct TraceArgs {
  int64_t n;                // points
  int32_t S;                // directions per point
  const float* pos;         // [n,3]
  const float* nrm;         // [n,3]
  const int32_t* order;     // [n] processing order (a permutation) or NULL
  const double4* dir_tab;   // [S] local directions of the call (see dir_entry)
  const double4* dir_sorted;  // [S] the same directions along a Z curve over the hemisphere
  uint32_t seed;            // direction rotation seed
  int32_t per_point;        // 1: one rotation per point
  float offset;             // ray origin fmaf(offset, n, x)
  float4* out;              // [n,S] (L_in rgb, O), caller's point order
};
hipError_t launch_trace_samples(const BakeGrid& G, const TraceArgs& t, hipStream_t s);
hipError_t launch_bake(const BakeGrid& G, const float* probe_pos, int32_t P, int32_t R,
                       float* texels, float* depth, const int4* order, hipStream_t s);

// place.hip --------------------------------------------------------------------------------
// farthest point sampling of P of M points from `start`, chosen [P], probes out [P,3] =
// fmaf(offset, n, x); scratch: packed [4M] floats (points with their distances, for clouds
// too large for registers) and sync [kFpsSyncWords] (the rows the picks are exchanged
// through, at most 64 workgroups, then a fault flag)
constexpr int kFpsSyncRows = 3;
constexpr size_t kFpsSyncWords = kFpsSyncRows * 64 + 1;
hipError_t launch_place_probes(const float* pts, const float* nrm, int64_t M, int32_t P,
                               int64_t start, float offset, float* packed, uint64_t* sync,
                               int32_t* chosen, float* out, hipStream_t s);
// doubles of partial sums the loss launches need for n elements
size_t loss_partials(int64_t n);
hipError_t launch_sops_loss(const float* tex, const float* tgt, int64_t T, float* loss,
                            float* grad, double* part, hipStream_t s);
hipError_t launch_lam_loss(const float* rough, const float* metal, int64_t N, float* loss,
                           float* g_rough, float* g_metal, double* part, hipStream_t s);

}  // namespace sopk
