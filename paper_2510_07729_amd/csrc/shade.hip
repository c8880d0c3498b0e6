// shade.hip - deferred shading with surface octahedral probes (ComGS Sec. 3.1.2):
// Monte Carlo estimate of the rendering equation (Eq. 6-7) over S Hammersley directions,
// incident light (1 - O) L_env + L_in (Eq. 8), O and L_in interpolated from the K nearest
// probes (Eq. 9-11), and the adjoint of that estimate.
//
// Layouts: the forward gives each point 8 lanes of a wavefront that take its directions in
// the order of a Z curve over the hemisphere (k_shade_fwd_cl); the adjoint and the other
// estimates give one wavefront to a point, lane l taking directions l, l+64, ..., with the
// point's data and its neighbour list wave-uniform (scalar loads). The octahedral taps of a
// direction are formed once and reused for all K probes, and per-point sums are reduced
// across lanes. The backward pass recomputes every sample instead of storing per-sample
// fetches.
#include "mlp_device.hpp"
#include "sop_device.hpp"
#include "sop_internal.hpp"

namespace sopk {

constexpr int kWavesPerBlock = 4;

struct PointState {
  int64_t p;
  double n64[3], v64[3];
  v3 n, v;
  Material M;
  Frame64 F;
  double cr, sr;   // per-point rotation of the direction table (1, 0 when per call)
};

// Point of processing slot wv. Uniform: one point per wavefront (the index is made
// wave-uniform so that the point's data comes through scalar loads); otherwise each lane
// group loads its own point.
template <bool Uniform = true>
__device__ __forceinline__ bool load_point(const ShadeArgs& a, int64_t wv, PointState& ps) {
  int64_t p = wv;
  if (a.order) {
    int32_t o = a.order[wv];
    if (Uniform) o = __builtin_amdgcn_readfirstlane(o);
    if ((uint64_t)o >= (uint64_t)a.n) return false;
    p = o;
  }
  ps.p = p;
  ps.n = mk3(a.nrm[3 * p], a.nrm[3 * p + 1], a.nrm[3 * p + 2]);
  ps.n64[0] = ps.n.x;
  ps.n64[1] = ps.n.y;
  ps.n64[2] = ps.n.z;
  if (a.view) {
    ps.v = mk3(a.view[3 * p], a.view[3 * p + 1], a.view[3 * p + 2]);
    ps.v64[0] = ps.v.x;
    ps.v64[1] = ps.v.y;
    ps.v64[2] = ps.v.z;
  } else {
    const int64_t f = p / a.ppf;
    double d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] = (double)a.cam[3 * f + c] - (double)a.pos[3 * p + c];
    const double il = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) ps.v64[c] = d[c] * il;
    ps.v = mk3((float)ps.v64[0], (float)ps.v64[1], (float)ps.v64[2]);
  }
  double nv = ps.n64[0] * ps.v64[0] + ps.n64[1] * ps.v64[1] + ps.n64[2] * ps.v64[2];
  const float NoV = (float)(nv < 1e-4 ? 1e-4 : nv);
  const v3 alb = mk3(a.albedo[3 * p], a.albedo[3 * p + 1], a.albedo[3 * p + 2]);
  ps.M = make_material(NoV, alb, a.rough[p], a.metal[p]);
  ps.F = make_frame64(ps.n64[0], ps.n64[1], ps.n64[2]);
  if (a.per_point) {
    const uint32_t rho = rotation24(a.seed, true, (uint32_t)p);
    sincospi((double)rho * 0x1p-23, &ps.sr, &ps.cr);
  } else {
    ps.cr = 1.0;
    ps.sr = 0.0;
  }
  return true;
}

// Neighbour list of a point: KT > 0 keeps K entries in registers (scalar), KT == 0 reads the
// list inside the loop for a run-time K.
template <int KT>
struct Neighbors {
  int32_t idx[KT];
  float w[KT];
  __device__ __forceinline__ void load(const ShadeArgs& a, int64_t p, int32_t) {
#pragma unroll
    for (int s = 0; s < KT; ++s) {
      int32_t id = a.nb_idx[p * KT + s];
      idx[s] = ((uint32_t)id < (uint32_t)a.P) ? id : -1;   // drop out-of-range entries
      w[s] = a.nb_w[p * KT + s];
    }
  }
  __device__ __forceinline__ int count(int32_t) const { return KT; }
  __device__ __forceinline__ int32_t id(int s, const ShadeArgs&, int64_t, int32_t) const {
    return idx[s];
  }
  __device__ __forceinline__ float wt(int s, const ShadeArgs&, int64_t, int32_t) const {
    return w[s];
  }
};

template <>
struct Neighbors<0> {
  __device__ __forceinline__ void load(const ShadeArgs&, int64_t, int32_t) {}
  __device__ __forceinline__ int count(int32_t k) const { return k; }
  __device__ __forceinline__ int32_t id(int s, const ShadeArgs& a, int64_t p, int32_t k) const {
    const int32_t v = a.nb_idx[p * k + s];
    return ((uint32_t)v < (uint32_t)a.P) ? v : -1;
  }
  __device__ __forceinline__ float wt(int s, const ShadeArgs& a, int64_t p, int32_t k) const {
    return a.nb_w[p * k + s];
  }
};

// per-sample quantities shared by forward and backward
struct Sample {
  double w64[3];
  v3 w;
  float ct;
  EnvTaps et;
  Taps tt;
  float Le[3];
  float Lin[3];
  float O;
};

// environment taps of direction w64: equirectangular (FP64-corrected per-call references) or,
// with EO, octahedral (the probe maps' lookup at the map's side). The layout is a template
// parameter so that the equirectangular kernels carry no code of the other lookup.
template <bool EO>
__device__ __forceinline__ EnvTaps env_taps_of(const ShadeArgs& a, const double w64[3]) {
  if constexpr (EO) {
    const Taps t = oct_taps64(w64, a.W);
    EnvTaps e;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      e.off[i] = t.off[i];
      e.w[i] = t.w[i];
    }
    e.vi = t.i0 + 2;
    e.vj = t.j0 + 2;
    return e;
  }
  else {
    return env_taps64(w64, a.H, a.W, a.u_scale, a.v_scale, a.col_ref, a.row_ref);
  }
}

// environment fetch of a sample whose direction (w64, w, ct) is set
template <bool EO>
__device__ __forceinline__ void eval_env(const ShadeArgs& a, Sample& s) {
  s.et = env_taps_of<EO>(a, s.w64);
  s.Le[0] = s.Le[1] = s.Le[2] = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float* e = a.env + 3 * (size_t)s.et.off[t];
    s.Le[0] += s.et.w[t] * e[0];
    s.Le[1] += s.et.w[t] * e[1];
    s.Le[2] += s.et.w[t] * e[2];
  }
}

// the value of v in the other lane of the lane's pair: lanes l and l ^ D (D = 1: DPP
// quad permutation; D = 16: across rows, through the LDS crossbar)
template <int D>
__device__ __forceinline__ int pair_swap(int v) {
  if constexpr (D == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
  else return __shfl_xor(v, D);
}
template <int D>
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(pair_swap<D>(__float_as_int(v)));
}

// environment and probe fetches of a sample whose direction (w64, w, ct) is set.
// PAIR = D > 0 (lanes l and l ^ D shade the same point): when every pair of the wavefront
// is active, the two lanes split the taps of both their samples so that each
// load instruction reads, per pair, two texels of one row of one sample (one cache line
// unless the row crosses a line boundary) instead of one texel of each of two directions:
// the even lane takes taps 0 and 2, the odd lane taps 1 and 3, of both samples; each lane
// adds its two taps of its own sample and its two taps of the partner's, and the
// partner's part changes lanes once per sample. The sum per sample is the same (its terms
// are grouped in two halves instead of one running sum).
template <int KT, typename TexT, bool EO = false, int PAIR = 0>
__device__ __forceinline__ void eval_at(const ShadeArgs& a, const PointState& ps,
                                        const Neighbors<KT>& nb, int32_t k, Sample& s) {
  s.et = env_taps_of<EO>(a, s.w64);
  s.Le[0] = s.Le[1] = s.Le[2] = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float* e = a.env + 3 * (size_t)s.et.off[t];
    s.Le[0] += s.et.w[t] * e[0];
    s.Le[1] += s.et.w[t] * e[1];
    s.Le[2] += s.et.w[t] * e[2];
  }
  s.tt = oct_taps64(s.w64, a.R);
  s.Lin[0] = s.Lin[1] = s.Lin[2] = 0.0f;
  s.O = 0.0f;
  const TexT* tex = reinterpret_cast<const TexT*>(a.tex);
  const size_t RR = (size_t)a.R * a.R;
  const int kn = KT > 0 ? KT : nb.count(k);
  if constexpr (PAIR > 0) {
    // lanes whose bit PAIR is clear (the pairs' low lanes)
    constexpr uint64_t kLow = PAIR == 1 ? 0x5555555555555555ull : 0x0000FFFF0000FFFFull;
    static_assert(PAIR == 1 || PAIR == 16, "pairs are lanes l, l ^ 1 or l, l ^ 16");
    const uint64_t act = __ballot(1);
    if (((act ^ (act >> PAIR)) & kLow) == 0) {   // uniform: all pairs whole
      const bool odd = (__lane_id() & PAIR) != 0;
      // partner's taps: the even lane needs 0 and 2, the odd lane 1 and 3
      const int q0 = pair_swap<PAIR>(odd ? s.tt.off[0] : s.tt.off[1]);
      const int q1 = pair_swap<PAIR>(odd ? s.tt.off[2] : s.tt.off[3]);
      const float u0 = pair_swap<PAIR>(odd ? s.tt.w[0] : s.tt.w[1]);
      const float u1 = pair_swap<PAIR>(odd ? s.tt.w[2] : s.tt.w[3]);
      // loads 1..4: row 0 of the even sample, row 0 of the odd sample, then row 1 of each
      const int ad0 = odd ? q0 : s.tt.off[0];
      const int ad1 = odd ? s.tt.off[1] : q0;
      const int ad2 = odd ? q1 : s.tt.off[2];
      const int ad3 = odd ? s.tt.off[3] : q1;
      // weights of loads 1, 3 (even sample) and 2, 4 (odd sample) in this lane
      const float c0 = odd ? u0 : s.tt.w[0];
      const float c1 = odd ? s.tt.w[1] : u0;
      const float c2 = odd ? u1 : s.tt.w[2];
      const float c3 = odd ? s.tt.w[3] : u1;
      float4 ev = make_float4(0.0f, 0.0f, 0.0f, 0.0f), od = ev;
#pragma unroll
      for (int s2 = 0; s2 < kn; ++s2) {
        const int32_t id = nb.id(s2, a, ps.p, k);
        if (id < 0) continue;
        const float wk = nb.wt(s2, a, ps.p, k);
        const TexT* T = tex + (size_t)id * RR;
        const float4 x0 = load_texel(T, (size_t)ad0), x1 = load_texel(T, (size_t)ad1);
        const float4 x2 = load_texel(T, (size_t)ad2), x3 = load_texel(T, (size_t)ad3);
        const float e0 = wk * c0, e1 = wk * c1, e2 = wk * c2, e3 = wk * c3;
        ev.x += e0 * x0.x + e2 * x2.x;
        ev.y += e0 * x0.y + e2 * x2.y;
        ev.z += e0 * x0.z + e2 * x2.z;
        ev.w += e0 * x0.w + e2 * x2.w;
        od.x += e1 * x1.x + e3 * x3.x;
        od.y += e1 * x1.y + e3 * x3.y;
        od.z += e1 * x1.z + e3 * x3.z;
        od.w += e1 * x1.w + e3 * x3.w;
      }
      const float4 keep = odd ? od : ev, send = odd ? ev : od;
      s.Lin[0] = keep.x + pair_swap<PAIR>(send.x);
      s.Lin[1] = keep.y + pair_swap<PAIR>(send.y);
      s.Lin[2] = keep.z + pair_swap<PAIR>(send.z);
      s.O = keep.w + pair_swap<PAIR>(send.w);
      return;
    }
  }
#pragma unroll
  for (int s2 = 0; s2 < kn; ++s2) {
    const int32_t id = nb.id(s2, a, ps.p, k);
    if (id < 0) continue;
    const float wk = nb.wt(s2, a, ps.p, k);
    const TexT* T = tex + (size_t)id * RR;
    // the four taps are requested together, then used
    float4 x[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = load_texel(T, (size_t)s.tt.off[t]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float c = wk * s.tt.w[t];
      s.Lin[0] += c * x[t].x;
      s.Lin[1] += c * x[t].y;
      s.Lin[2] += c * x[t].z;
      s.O += c * x[t].w;
    }
  }
}

template <int KT, typename TexT, bool EO = false>
__device__ __forceinline__ void eval_sample(const ShadeArgs& a, const PointState& ps,
                                            const Neighbors<KT>& nb, int32_t k, int j,
                                            Sample& s) {
  // the adjoint walks the directions along the Z curve over the hemisphere (dir_sorted):
  // a wavefront's 64 lanes then look into one compact region, and its gathers share more
  // cache lines than in the table's own order (the sum over directions is order-free)
  const double4 e = a.dir_sorted ? a.dir_sorted[j] : a.dir_tab[j];
  const double da = e.x * ps.cr - e.y * ps.sr;
  const double db = e.x * ps.sr + e.y * ps.cr;
  world_dir64(ps.F, da, db, e.z, s.w64);
  s.w = mk3((float)s.w64[0], (float)s.w64[1], (float)s.w64[2]);
  s.ct = (float)e.z;
  eval_at<KT, TexT, EO, 1>(a, ps, nb, k, s);
}

// Sum over the L lanes of a lane group (L = 64: the whole wavefront, with DPP).
template <int L>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (L == 64) {
    return wave_sum(v);
  } else {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o);
    return v;
  }
}

// Processing slot of the lane's group: L lanes per point, 64/L points per wavefront (small
// direction counts would otherwise leave lanes idle and pay a wavefront's fixed per-point
// cost for one point).
template <int L>
__device__ __forceinline__ int64_t group_slot(int lane) {
  return (die_block() * kWavesPerBlock + wave_id_uniform()) * (64 / L) + lane / L;
}

// Neighbour entries of a lane's point in ascending probe index (dropped entries, -1, last),
// so that lanes of nearby points, whose lists mostly hold the same probes, read the same
// probe at the same step. Eq. 9 is a sum over the entries: their order is free.
template <int KT>
__device__ __forceinline__ void order_by_probe(Neighbors<KT>& nb) {
  if constexpr (KT > 0) {
#pragma unroll
    for (int pass = 0; pass < KT; ++pass)
#pragma unroll
      for (int i = pass & 1; i + 1 < KT; i += 2) {
        const bool sw = (uint32_t)nb.idx[i] > (uint32_t)nb.idx[i + 1];
        const int32_t i0 = nb.idx[i], i1 = nb.idx[i + 1];
        const float w0 = nb.w[i], w1 = nb.w[i + 1];
        nb.idx[i] = sw ? i1 : i0;
        nb.idx[i + 1] = sw ? i0 : i1;
        nb.w[i] = sw ? w1 : w0;
        nb.w[i + 1] = sw ? w0 : w1;
      }
  }
}

// Shading forward in the cluster layout: a wavefront takes 8 consecutive points of the
// processing order, 8 lanes per point, and lane q of a point takes directions q, q + 8, ...
// of the call's direction table sorted along a Z curve over the hemisphere (dir_sorted),
// so that at every step the 8 directions of a point are close together, and the 8 points,
// whose normals are close (the processing order groups them by probe-grid cell) and whose
// neighbour lists mostly coincide (ordered by probe index), look the same way, and the
// per-point work (neighbour lists, frame, material, the final sums) is shared by 8 lanes
// instead of 64. On the object workload this layout takes 0.95 ms against 1.19 ms for one
// point per wavefront; its texture units stay ~86% busy (32 16-byte gathers per sample),
// so the texture path remains the bound. The sum over a point's
// directions is order-free (Eq. 7); the 8 lanes' partial sums meet by shuffles.
constexpr int kFwdLanes = 8;          // lanes per point (points per wavefront: 64 / kFwdLanes)
template <int KT, typename TexT, bool EO = false, bool COS = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_shade_fwd_cl(ShadeArgs a, int32_t k) {
  constexpr int PPW = 64 / kFwdLanes;
  const int lane = threadIdx.x & 63, q = lane % kFwdLanes;
  const int64_t wv = die_block() * kWavesPerBlock + wave_id_uniform();
  if (wv * PPW >= a.n) return;                          // uniform over the wavefront
  const int64_t slot = wv * PPW + lane / kFwdLanes;
  PointState ps;
  const bool valid = slot < a.n && load_point<false>(a, slot, ps);
  float acc[3] = {0.0f, 0.0f, 0.0f}, acc_e[3] = {0.0f, 0.0f, 0.0f};
  if (valid) {
    Neighbors<KT> nb;
    nb.load(a, ps.p, k);
    order_by_probe<KT>(nb);
    const float al[3] = {ps.M.a.x, ps.M.a.y, ps.M.a.z};
    for (int i = q; i < a.S; i += kFwdLanes) {
      const double4 e = a.dir_sorted[i];
      Sample s;
      const double da = e.x * ps.cr - e.y * ps.sr;
      const double db = e.x * ps.sr + e.y * ps.cr;
      world_dir64(ps.F, da, db, e.z, s.w64);
      s.w = mk3((float)s.w64[0], (float)s.w64[1], (float)s.w64[2]);
      s.ct = (float)e.z;
      eval_at<KT, TexT, EO, 1>(a, ps, nb, k, s);
      const BrdfTerms bt = brdf_terms(ps.M, half_geom(ps.n64, ps.v64, s.w64), s.ct);
      // the cosine-weighted set weighs each sample by 1/(2 cos) relative to 2 pi/S
      const float wj = COS ? (float)e.w : 1.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float Li = (1.0f - s.O) * s.Le[c] + s.Lin[c];
        if constexpr (COS) {
          acc[c] += fcos(ps.M, bt, al[c], s.ct) * Li * wj;
          acc_e[c] += Li * s.ct * wj;
        } else {
          acc[c] += fcos(ps.M, bt, al[c], s.ct) * Li;
          acc_e[c] += Li * s.ct;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int o = 1; o < kFwdLanes; o <<= 1) {
      acc[c] += __shfl_xor(acc[c], o);
      acc_e[c] += __shfl_xor(acc_e[c], o);
    }
  if (!valid || q != 0) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) a.rgb[3 * ps.p + c] = acc[c] * a.scale;
  if (a.irr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.irr[3 * ps.p + c] = acc_e[c] * a.scale;
  }
}

// Traced shading: the estimate of the shading forward with L_in and O of every sample read from its
// traced ray (a.traced, [n,S] in the caller's point order) instead of the probes.
template <int L, bool EO = false>
__global__ __launch_bounds__(256) void k_shade_traced(ShadeArgs a) {
  const int lane = threadIdx.x & 63, li = lane % L;
  const int64_t slot = group_slot<L>(lane);
  if ((die_block() * kWavesPerBlock + wave_id_uniform()) * (64 / L) >= a.n) return;
  PointState ps;
  const bool valid = slot < a.n && load_point<L == 64>(a, slot, ps);
  if (L == 64 && !valid) return;
  float acc[3] = {0.0f, 0.0f, 0.0f}, acc_e[3] = {0.0f, 0.0f, 0.0f};
  if (valid) {
    const float4* tr = a.traced + ps.p * a.S;
    for (int j = li; j < a.S; j += L) {
      const double4 e = a.dir_tab[j];
      const double da = e.x * ps.cr - e.y * ps.sr;
      const double db = e.x * ps.sr + e.y * ps.cr;
      double w64[3];
      world_dir64(ps.F, da, db, e.z, w64);
      const float ct = (float)e.z;
      const EnvTaps et = env_taps_of<EO>(a, w64);
      float Le[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float* ep = a.env + 3 * (size_t)et.off[t];
        Le[0] += et.w[t] * ep[0];
        Le[1] += et.w[t] * ep[1];
        Le[2] += et.w[t] * ep[2];
      }
      const float4 q = tr[j];
      const float Lin[3] = {q.x, q.y, q.z};
      const BrdfTerms bt = brdf_terms(ps.M, half_geom(ps.n64, ps.v64, w64), ct);
      const float al[3] = {ps.M.a.x, ps.M.a.y, ps.M.a.z};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float Li = (1.0f - q.w) * Le[c] + Lin[c];
        acc[c] += fcos(ps.M, bt, al[c], ct) * Li;
        acc_e[c] += Li * ct;
      }
    }
  }
  float r[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = group_sum<L>(acc[c]) * a.scale;
  if (valid && li == 0) {
    a.rgb[3 * ps.p] = r[0];
    a.rgb[3 * ps.p + 1] = r[1];
    a.rgb[3 * ps.p + 2] = r[2];
  }
  if (a.irr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = group_sum<L>(acc_e[c]) * a.scale;
    if (valid && li == 0) {
      a.irr[3 * ps.p] = r[0];
      a.irr[3 * ps.p + 1] = r[1];
      a.irr[3 * ps.p + 2] = r[2];
    }
  }
}

// ------------------------------------------------------------------------------------------
// Cast-shadow ratio (Sec. 3.2 occlusion caching, Eq. 15-17) on an octahedral environment,
// with the Hammersley set or environment importance sampling (Eq. 18).
// ------------------------------------------------------------------------------------------

// intensity of an environment texel in IEEE single precision: (r + g) + b, 0 unless > 0
__device__ __forceinline__ float env_intensity(const float* e) {
  const float I = (e[0] + e[1]) + e[2];
  return I > 0.0f ? I : 0.0f;
}

// Texel masses m_t = 1 + floor(I_t * (2^14 / I_max)) (one IEEE division, one product; all 1
// when I_max = 0) and their exclusive prefix sums, prefix[T] = the total, in four coalesced
// passes: the maximum (one workgroup), masses and a scan inside tiles of 1024 texels, a
// scan of the tile totals (one workgroup; T <= 2^20), and the tile offsets added.
constexpr int kCdfTile = 1024;

// cell width (log2) of the guide of a mass line of total C: 2^16 cells at most
__device__ __forceinline__ int env_guide_shift(uint64_t C) {
  const int bits = C ? 64 - __clzll((long long)C) : 0;
  return bits > 16 ? bits - 16 : 0;
}

// the texel whose stretch of the mass line holds x < C: the largest t with prefix[t] <= x,
// searched between the guide entries of x's cell
__device__ __forceinline__ int env_pick(const uint64_t* __restrict__ prefix,
                                        const int32_t* __restrict__ guide, int32_t T,
                                        uint64_t C, uint64_t x) {
  const uint64_t g = x >> env_guide_shift(C);
  int lo = guide[g], hi = min(guide[g + 1] + 1, T);
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// guide[g] = the texel of x = g << shift, by a full search (kEnvGuide + 1 entries)
__global__ __launch_bounds__(256) void k_env_guide(const uint64_t* __restrict__ prefix,
                                                   int32_t T, int32_t* __restrict__ guide) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g > kEnvGuide) return;
  const uint64_t C = prefix[T];
  const uint64_t v = (uint64_t)g << env_guide_shift(C);
  int lo = 0, hi = T;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= v) lo = mid; else hi = mid;
  }
  guide[g] = lo;
}

__global__ __launch_bounds__(1024) void k_env_max(const float* env, int32_t T, float* imax) {
  __shared__ float smax[1024];
  const int tid = threadIdx.x;
  float m = 0.0f;
  for (int t = tid; t < T; t += 1024) m = fmaxf(m, env_intensity(env + 3 * (size_t)t));
  smax[tid] = m;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o) smax[tid] = fmaxf(smax[tid], smax[tid + o]);
    __syncthreads();
  }
  if (tid == 0) *imax = smax[0];
}

// inclusive scan of one value per thread over a 1024-thread workgroup (Hillis-Steele)
__device__ __forceinline__ uint64_t block_scan_1024(uint64_t v, uint64_t* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint64_t add = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  return sh[tid];
}

__global__ __launch_bounds__(1024) void k_env_tiles(const float* env, int32_t T,
                                                    const float* imax, uint32_t* mass,
                                                    uint64_t* prefix, uint64_t* tile_sum) {
  __shared__ uint64_t sh[1024];
  const float im = *imax;
  const float f = im > 0.0f ? __fdiv_rn(16384.0f, im) : 0.0f;
  const int t = blockIdx.x * kCdfTile + threadIdx.x;
  uint32_t m = 0;
  if (t < T) {
    m = 1u + (uint32_t)floorf(__fmul_rn(env_intensity(env + 3 * (size_t)t), f));
    mass[t] = m;
  }
  const uint64_t inc = block_scan_1024(m, sh);
  if (t < T) prefix[t] = inc - m;
  if (threadIdx.x == 1023) tile_sum[blockIdx.x] = inc;
}

__global__ __launch_bounds__(1024) void k_env_tile_scan(int32_t ntiles, uint64_t* tile_sum,
                                                        uint64_t* prefix, int32_t T) {
  __shared__ uint64_t sh[1024];
  const int b = threadIdx.x;
  const uint64_t v = b < ntiles ? tile_sum[b] : 0;
  const uint64_t inc = block_scan_1024(v, sh);
  if (b < ntiles) tile_sum[b] = inc - v;           // offset of tile b
  if (b == 1023) prefix[T] = inc;
}

__global__ __launch_bounds__(1024) void k_env_add(int32_t T, const uint64_t* tile_off,
                                                  uint64_t* prefix) {
  const int t = blockIdx.x * kCdfTile + threadIdx.x;
  if (t < T && blockIdx.x > 0) prefix[t] += tile_off[blockIdx.x];
}

// 1 / pdf of an environment importance draw of texel mass m (total C, T texels) in the unit
// direction w: Eq. 18's density (m / C) T / (4 pi), or with exact the draw's own density
// (m / C) (T / 4) / s^3, s = |w_x| + |w_y| + |w_z| (the octahedral square's area element).
__device__ __forceinline__ float env_inv_pdf(const double w[3], uint32_t m, uint64_t C,
                                             int32_t T, bool exact) {
  if (exact) {
    const double sl = fabs(w[0]) + fabs(w[1]) + fabs(w[2]);
    return (float)(4.0 * (sl * sl * sl) * (double)C / ((double)m * (double)T));
  }
  return (float)(12.566370614359172 * (double)C / ((double)m * (double)T));
}

// L lanes per point (64/L points per wavefront, in processing order; L = 64 for S > 32),
// lane l of a point takes directions l, l+L, ...; the estimates of Eq. 15 and 16 share
// every sample, and the ratio is formed after the lane-group sums.
template <int KT, typename TexT, int L>
__global__ __launch_bounds__(256) void k_shadow_ratio(ShadeArgs a, int32_t k) {
  const int lane = threadIdx.x & 63, li = lane % L;
  if ((die_block() * kWavesPerBlock + wave_id_uniform()) * (64 / L) >= a.n) return;
  const int64_t slot = group_slot<L>(lane);
  bool valid = slot < a.n;
  int64_t p = valid ? slot : 0;
  if (valid && a.order) {
    int32_t o = a.order[slot];
    if (L == 64) o = __builtin_amdgcn_readfirstlane(o);
    if ((uint64_t)o >= (uint64_t)a.n) valid = false;
    else p = o;
  }
  if (L == 64 && !valid) return;
  double n64[3] = {0.0, 0.0, 1.0};
  if (valid) {
    n64[0] = a.nrm[3 * p];
    n64[1] = a.nrm[3 * p + 1];
    n64[2] = a.nrm[3 * p + 2];
  }
  Neighbors<KT> nb;
  if (valid) nb.load(a, p, k);
  const int kn = KT > 0 ? KT : nb.count(k);
  const bool importance = a.shadow_sampler != 0;
  Frame64 F;
  double cr = 1.0, sr = 0.0;
  if (!importance) {
    F = make_frame64(n64[0], n64[1], n64[2]);
    if (a.per_point) sincospi((double)rotation24(a.seed, true, (uint32_t)p) * 0x1p-23, &sr, &cr);
  }
  const int32_t Re = a.env_res;
  const int32_t T = Re * Re;
  const uint64_t C = a.env_prefix ? a.env_prefix[T] : 0;
  const uint32_t sh = pcg_hash(a.seed);
  const TexT* tex = reinterpret_cast<const TexT*>(a.tex);
  const size_t RR = (size_t)a.R * a.R;
  float num[3] = {0.0f, 0.0f, 0.0f}, den[3] = {0.0f, 0.0f, 0.0f};
  for (int j = li; valid && j < a.S; j += L) {
    double w64[3];
    float ct, wt;
    if (!importance) {
      const double4 e = a.dir_tab[j];
      world_dir64(F, e.x * cr - e.y * sr, e.x * sr + e.y * cr, e.z, w64);
      ct = (float)e.z;
      wt = 6.283185307179586f;
    } else {
      // the j-th of S slices of the mass line, then the texel whose stretch holds x
      const uint64_t r = hash24(sh, (uint32_t)p, (uint32_t)j, 0);
      const uint64_t x = ((uint64_t)j * C + ((r * C) >> 24)) / (uint64_t)a.S;
      const int lo = env_pick(a.env_prefix, a.env_guide, T, C, x);
      const double xu = ((double)hash24(sh, (uint32_t)p, (uint32_t)j, 1) + 0.5) * 0x1p-24;
      const double xv = ((double)hash24(sh, (uint32_t)p, (uint32_t)j, 2) + 0.5) * 0x1p-24;
      oct_decode64((double)(lo % Re) + xu, (double)(lo / Re) + xv, Re, w64);
      const double cd = w64[0] * n64[0] + w64[1] * n64[1] + w64[2] * n64[2];
      if (!(cd > 0.0)) continue;
      ct = (float)cd;
      wt = env_inv_pdf(w64, a.env_mass[lo], C, T, a.env_pdf_exact != 0);
    }
    const Taps te = oct_taps64(w64, Re);
    float E[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float* ep = a.env + 3 * (size_t)te.off[t];
      E[0] += te.w[t] * ep[0];
      E[1] += te.w[t] * ep[1];
      E[2] += te.w[t] * ep[2];
    }
    const Taps tt = oct_taps64(w64, a.R);
    float O = 0.0f;
#pragma unroll
    for (int s2 = 0; s2 < kn; ++s2) {
      const int32_t id = nb.id(s2, a, p, k);
      if (id < 0) continue;
      const float wk = nb.wt(s2, a, p, k);
      const TexT* Tp = tex + (size_t)id * RR;
      // only the occlusion channel is read (a quarter of each texel)
      float q[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) q[t] = load_occlusion(Tp, (size_t)tt.off[t]);
#pragma unroll
      for (int t = 0; t < 4; ++t) O += wk * tt.w[t] * q[t];
    }
    const float cw = ct * wt;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      num[c] += E[c] * (1.0f - O) * cw;
      den[c] += E[c] * cw;
    }
  }
  float rn[3], rd[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    rn[c] = group_sum<L>(num[c]);
    rd[c] = group_sum<L>(den[c]);
  }
  if (valid && li == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.rgb[3 * p + c] = rd[c] != 0.0f ? rn[c] / rd[c] : 1.0f;
    if (a.irr) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.irr[3 * p + c] = rd[c] / (float)a.S;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Object relighting with environment importance sampling (Sec. 3.3: relighting and shadows
// are both estimated with the density of Eq. 18): the shading estimate of Eq. 6-9 with the
// draws of the cast-shadow ratio's Eq. 18 sampler on an octahedral environment,
// rgb = (1/S) sum_j f L_i cos+ / pdf_j with pdf_j = (m_t / C) R_e^2 / (4 pi), or the draw's
// exact density (env_inv_pdf); draws below the horizon add nothing. L lanes per point (64/L points per wavefront), lane l of a point
// taking draws l, l + L, ...
// ------------------------------------------------------------------------------------------
template <int KT, typename TexT, int L>
__global__ __launch_bounds__(256) void k_shade_envis(ShadeArgs a, int32_t k) {
  const int lane = threadIdx.x & 63, li = lane % L;
  if ((die_block() * kWavesPerBlock + wave_id_uniform()) * (64 / L) >= a.n) return;
  const int64_t slot = group_slot<L>(lane);
  PointState ps;
  const bool valid = slot < a.n && load_point<L == 64>(a, slot, ps);
  if (L == 64 && !valid) return;
  float acc[3] = {0.0f, 0.0f, 0.0f}, acc_e[3] = {0.0f, 0.0f, 0.0f};
  if (valid) {
    Neighbors<KT> nb;
    nb.load(a, ps.p, k);
    const int32_t Re = a.env_res, T = Re * Re;
    const uint64_t C = a.env_prefix[T];
    const uint32_t sh = pcg_hash(a.seed), pi = (uint32_t)ps.p;
    const float al[3] = {ps.M.a.x, ps.M.a.y, ps.M.a.z};
    for (int j = li; j < a.S; j += L) {
      // the j-th of S slices of the mass line, then the texel whose stretch holds x
      const uint64_t r = hash24(sh, pi, (uint32_t)j, 0);
      const uint64_t x = ((uint64_t)j * C + ((r * C) >> 24)) / (uint64_t)a.S;
      const int lo = env_pick(a.env_prefix, a.env_guide, T, C, x);
      const double xu = ((double)hash24(sh, pi, (uint32_t)j, 1) + 0.5) * 0x1p-24;
      const double xv = ((double)hash24(sh, pi, (uint32_t)j, 2) + 0.5) * 0x1p-24;
      Sample s;
      oct_decode64((double)(lo % Re) + xu, (double)(lo / Re) + xv, Re, s.w64);
      const double cd = s.w64[0] * ps.n64[0] + s.w64[1] * ps.n64[1] + s.w64[2] * ps.n64[2];
      if (!(cd > 0.0)) continue;
      s.w = mk3((float)s.w64[0], (float)s.w64[1], (float)s.w64[2]);
      s.ct = (float)cd;
      eval_at<KT, TexT, true>(a, ps, nb, k, s);
      const float wt = env_inv_pdf(s.w64, a.env_mass[lo], C, T, a.env_pdf_exact != 0);
      const BrdfTerms bt = brdf_terms(ps.M, half_geom(ps.n64, ps.v64, s.w64), s.ct);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float Li = (1.0f - s.O) * s.Le[c] + s.Lin[c];
        acc[c] += fcos(ps.M, bt, al[c], s.ct) * Li * wt;
        acc_e[c] += Li * s.ct * wt;
      }
    }
  }
  const float scale = 1.0f / (float)a.S;
  float r3[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r3[c] = group_sum<L>(acc[c]) * scale;
  if (valid && li == 0) {
    a.rgb[3 * ps.p] = r3[0];
    a.rgb[3 * ps.p + 1] = r3[1];
    a.rgb[3 * ps.p + 2] = r3[2];
  }
  if (a.irr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) r3[c] = group_sum<L>(acc_e[c]) * scale;
    if (valid && li == 0) {
      a.irr[3 * ps.p] = r3[0];
      a.irr[3 * ps.p + 1] = r3[1];
      a.irr[3 * ps.p + 2] = r3[2];
    }
  }
}

// ------------------------------------------------------------------------------------------
// Learned direction proposal: importance-sampled estimate of Eq. 7. Directions are drawn
// from 16x16 bins over the hemispherical octahedral square of the local frame,
// (u,v) = (x+y, x-y)/(|x|+|y|+z), with integer bin masses (decided in IEEE single
// precision, so every bin choice is exact), and each sample is weighted by 1/pdf,
// pdf = (c_b / C) * 128 * l^3 with l = |(px,py,z)|.
// ------------------------------------------------------------------------------------------

// unit local direction of square point (u,v); returns l = |(px, py, z)|
__device__ __forceinline__ double bin_dir(double u, double v, double wl[3]) {
  const double px = 0.5 * (u + v), py = 0.5 * (u - v);
  const double z = 1.0 - fabs(px) - fabs(py);
  const double l = sqrt(fma(px, px, fma(py, py, z * z)));
  const double il = 1.0 / l;
  wl[0] = px * il;
  wl[1] = py * il;
  wl[2] = z * il;
  return l;
}

// local direction of the point (xu, xv) in [0,1)^2 of bin b's cell
__device__ __forceinline__ double cell_point(double xu, double xv, int b, double wl[3]) {
  const double u = -1.0 + ((double)(b & 15) + xu) * 0.125;
  const double v = -1.0 + ((double)(b >> 4) + xv) * 0.125;
  return bin_dir(u, v, wl);
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d, int width) {
  const uint32_t lo = __shfl_up((uint32_t)v, d, width);
  const uint32_t hi = __shfl_up((uint32_t)(v >> 32), d, width);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src, int width) {
  const uint32_t lo = __shfl((uint32_t)v, src, width), hi = __shfl((uint32_t)(v >> 32), src, width);
  return ((uint64_t)hi << 32) | lo;
}

// Cumulative integer masses cum[0..256] of the point's bins into the group's LDS row; the L
// lanes of the group take 256/L consecutive bins each. Lanes with load = false (a group past
// the end) contribute nothing and take the uniform fallback.
template <int L>
__device__ __forceinline__ uint64_t bin_masses(const ShadeArgs& a, int64_t p, bool load,
                                               int li, uint64_t* cum) {
  constexpr int BPL = SOP_MLP_BINS / L;
  const float om = 1.0f - a.mix_eps, add = a.mix_eps * (1.0f / 256.0f);
  uint32_t c[BPL];
#pragma unroll
  for (int q4 = 0; q4 < BPL / 4; ++q4) {
    float4 pr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (load)
      pr = *reinterpret_cast<const float4*>(a.probs + (size_t)p * SOP_MLP_BINS + BPL * li + 4 * q4);
    const float pv[4] = {pr.x, pr.y, pr.z, pr.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float q = pv[t];
      q = q > 0.0f ? fminf(q, 1.0f) : 0.0f;                // NaN and negatives count as 0
      c[4 * q4 + t] = (uint32_t)floorf(__builtin_fmaf(om, q, add) * 16777216.0f);
    }
  }
  uint64_t own = 0;
#pragma unroll
  for (int t = 0; t < BPL; ++t) own += c[t];
  uint64_t incl = own;
#pragma unroll
  for (int d = 1; d < L; d <<= 1) {
    const uint64_t o = shfl_up_u64(incl, d, L);
    if (li >= d) incl += o;
  }
  uint64_t total = shfl_u64(incl, L - 1, L);
  if (total == 0) {                                         // nothing to sample: one unit per bin
#pragma unroll
    for (int t = 0; t < BPL; ++t) c[t] = 1;
    incl = (uint64_t)BPL * (li + 1);
    own = BPL;
    total = SOP_MLP_BINS;
  }
  uint64_t run = incl - own;
  if (li == 0) cum[0] = 0;
#pragma unroll
  for (int t = 0; t < BPL; ++t) {
    run += c[t];
    cum[BPL * li + t + 1] = run;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return total;
}

// bin of mass coordinate x < total: the largest b with cum[b] <= x
template <typename CumT>
__device__ __forceinline__ int find_bin(const CumT* cum, uint64_t x) {
  int b = 0;
#pragma unroll
  for (int step = 128; step >= 1; step >>= 1)
    if (cum[b + step] <= x) b += step;
  return b;
}

template <int KT, typename TexT, int L>
// three wavefronts per SIMD, like the forward kernel
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_shade_prop(ShadeArgs a, int32_t k) {
  constexpr int PPW = 64 / L;
  __shared__ uint64_t s_cum[kWavesPerBlock][PPW][SOP_MLP_BINS + 1];
  const int lane = threadIdx.x & 63, li = lane % L;
  const int64_t slot = group_slot<L>(lane);
  if ((die_block() * kWavesPerBlock + wave_id_uniform()) * PPW >= a.n) return;
  uint64_t* cum = s_cum[threadIdx.x >> 6][lane / L];
  PointState ps;
  const bool valid = slot < a.n && load_point<L == 64>(a, slot, ps);
  if (L == 64 && !valid) return;
  const uint64_t total = bin_masses<L>(a, valid ? ps.p : 0, valid, li, cum);
  Neighbors<KT> nb;
  float acc[3] = {0.0f, 0.0f, 0.0f}, acc_e[3] = {0.0f, 0.0f, 0.0f};
  if (valid) {
    nb.load(a, ps.p, k);
    const uint32_t sh = pcg_hash(a.seed), pi = (uint32_t)ps.p;
    const uint32_t rot_v = hash24(sh, pi, 0, 2);
    const double inv_total = 1.0 / (double)total;
    const float al[3] = {ps.M.a.x, ps.M.a.y, ps.M.a.z};
    for (int j = li; j < a.S; j += L) {
      const uint64_t r = hash24(sh, pi, (uint32_t)j, 0);
      const uint64_t x = ((uint64_t)j * total + ((r * total) >> 24)) / (uint64_t)a.S;
      const int b = find_bin(cum, x);
      const uint64_t cb = cum[b + 1] - cum[b];
      // u: place of the draw on the bin's stretch of the mass line; v: radical inverse of j
      // rotated per point
      const double xu = ((double)(x - cum[b]) + 0.5) / (double)cb;
      const uint32_t v24 = ((__builtin_bitreverse32((uint32_t)j) >> 8) + rot_v) & 0xFFFFFFu;
      const double xv = ((double)v24 + 0.5) * 0x1p-24;
      double wl[3];
      const double l = cell_point(xu, xv, b, wl);
      const float inv_pdf = (float)(1.0 / ((double)cb * inv_total * 128.0 * l * l * l));
      Sample s;
      world_dir64(ps.F, wl[0], wl[1], wl[2], s.w64);
      s.w = mk3((float)s.w64[0], (float)s.w64[1], (float)s.w64[2]);
      s.ct = (float)wl[2];
      eval_at<KT, TexT>(a, ps, nb, k, s);
      const BrdfTerms bt = brdf_terms(ps.M, half_geom(ps.n64, ps.v64, s.w64), s.ct);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float Li = (1.0f - s.O) * s.Le[c] + s.Lin[c];
        acc[c] += fcos(ps.M, bt, al[c], s.ct) * Li * inv_pdf;
        acc_e[c] += Li * s.ct * inv_pdf;
      }
    }
  }
  const float scale = 1.0f / (float)a.S;
  float r3[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r3[c] = group_sum<L>(acc[c]) * scale;
  if (valid && li == 0) {
    a.rgb[3 * ps.p] = r3[0];
    a.rgb[3 * ps.p + 1] = r3[1];
    a.rgb[3 * ps.p + 2] = r3[2];
  }
  if (a.irr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) r3[c] = group_sum<L>(acc_e[c]) * scale;
    if (valid && li == 0) {
      a.irr[3 * ps.p] = r3[0];
      a.irr[3 * ps.p + 1] = r3[1];
      a.irr[3 * ps.p + 2] = r3[2];
    }
  }
}

// Proposal shading with the network evaluated in the same kernel: a wavefront takes 16
// points, runs the network on the matrix cores (the logits of point l%16 end in the four
// lanes l%16 + 16g), turns them into bin masses exactly as the inference kernel and the
// sampler above do, and then shades the 16 points with lane l%16 + 16g taking draws
// g, g+4, ... of point l%16. The bin probabilities never leave the chip.
template <int KT, typename TexT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_shade_prop_net(ShadeArgs a, int32_t k) {
  __shared__ uint32_t s_cum[kWavesPerBlock][16][SOP_MLP_BINS + 1];
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int64_t tile = die_block() * kWavesPerBlock + wave_id_uniform();
  if (tile * 16 >= a.n) return;
  const int64_t slot = tile * 16 + r;
  uint32_t* cum = s_cum[threadIdx.x >> 6][r];
  PointState ps;
  const bool valid = slot < a.n && load_point<false>(a, slot, ps);

  // network forward of the 16 points and their bin probabilities
  f32x4 prob[16];
  {
    FeatIn fi;
    if (valid)
      point_scalars(a.pos, a.nrm, a.view, a.cam, a.ppf, a.rough, a.mlp_lo, a.mlp_inv2, ps.p, fi);
    else
#pragma unroll
      for (int c = 0; c < 10; ++c) fi.x[c] = 0.0f;
    Fwd F;
    forward_tile(a.mlp_params, a.mlp_frags, fi, lane, F, nullptr, 0, 0, false);
    softmax_tile(F.z3);
#pragma unroll
    for (int mb = 0; mb < 16; ++mb) prob[mb] = F.z3[mb];
  }
  // integer masses into the point's LDS row (bin b = 16 mb + 4 g + t), then the prefix over
  // bins: lane g of the point takes bins [64 g, 64 g + 64)
  const float om = 1.0f - a.mix_eps, add = a.mix_eps * (1.0f / 256.0f);
#pragma unroll
  for (int mb = 0; mb < 16; ++mb)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float q = prob[mb][t];
      q = q > 0.0f ? fminf(q, 1.0f) : 0.0f;
      cum[16 * mb + 4 * g + t + 1] = (uint32_t)floorf(__builtin_fmaf(om, q, add) * 16777216.0f);
    }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t own = 0;
  for (int b = 64 * g; b < 64 * g + 64; ++b) own += cum[b + 1];
  uint32_t incl = own;
  {
    const uint32_t o1 = __shfl_up(incl, 16);
    if (g >= 1) incl += o1;
    const uint32_t o2 = __shfl_up(incl, 32);
    if (g >= 2) incl += o2;
  }
  uint32_t total = __shfl(incl, 48 + r);
  const bool fallback = total == 0;
  if (fallback) total = SOP_MLP_BINS;
  uint32_t run = fallback ? 64u * g : incl - own;
  if (g == 0) cum[0] = 0;
  for (int b = 64 * g; b < 64 * g + 64; ++b) {
    run += fallback ? 1u : cum[b + 1];
    cum[b + 1] = run;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  Neighbors<KT> nb;
  float acc[3] = {0.0f, 0.0f, 0.0f}, acc_e[3] = {0.0f, 0.0f, 0.0f};
  if (valid) {
    nb.load(a, ps.p, k);
    const uint32_t sh = pcg_hash(a.seed), pi = (uint32_t)ps.p;
    const uint32_t rot_v = hash24(sh, pi, 0, 2);
    const double inv_total = 1.0 / (double)total;
    const float al[3] = {ps.M.a.x, ps.M.a.y, ps.M.a.z};
    for (int j = g; j < a.S; j += 4) {
      const uint64_t rr = hash24(sh, pi, (uint32_t)j, 0);
      const uint64_t x = ((uint64_t)j * total + ((rr * total) >> 24)) / (uint64_t)a.S;
      const int b = find_bin(cum, x);
      const uint64_t cb = cum[b + 1] - cum[b];
      const double xu = ((double)(x - cum[b]) + 0.5) / (double)cb;
      const uint32_t v24 = ((__builtin_bitreverse32((uint32_t)j) >> 8) + rot_v) & 0xFFFFFFu;
      const double xv = ((double)v24 + 0.5) * 0x1p-24;
      double wl[3];
      const double l = cell_point(xu, xv, b, wl);
      const float inv_pdf = (float)(1.0 / ((double)cb * inv_total * 128.0 * l * l * l));
      Sample s;
      world_dir64(ps.F, wl[0], wl[1], wl[2], s.w64);
      s.w = mk3((float)s.w64[0], (float)s.w64[1], (float)s.w64[2]);
      s.ct = (float)wl[2];
      eval_at<KT, TexT, false, 16>(a, ps, nb, k, s);
      const BrdfTerms bt = brdf_terms(ps.M, half_geom(ps.n64, ps.v64, s.w64), s.ct);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float Li = (1.0f - s.O) * s.Le[c] + s.Lin[c];
        acc[c] += fcos(ps.M, bt, al[c], s.ct) * Li * inv_pdf;
        acc_e[c] += Li * s.ct * inv_pdf;
      }
    }
  }
  const float scale = 1.0f / (float)a.S;
  float r3[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r3[c] = point_sum(acc[c]) * scale;
  if (valid && g == 0) {
    a.rgb[3 * ps.p] = r3[0];
    a.rgb[3 * ps.p + 1] = r3[1];
    a.rgb[3 * ps.p + 2] = r3[2];
  }
  if (a.irr) {
#pragma unroll
    for (int c = 0; c < 3; ++c) r3[c] = point_sum(acc_e[c]) * scale;
    if (valid && g == 0) {
      a.irr[3 * ps.p] = r3[0];
      a.irr[3 * ps.p + 1] = r3[1];
      a.irr[3 * ps.p + 2] = r3[2];
    }
  }
}

// Training targets of the proposal: T[i][b] = (1/(128 n)) sum_k lum(f L_i cos) / l^3 over n
// draws placed in bin b's cell (draw j = b n + k, u stratified over the n draws, v random),
// summed per bin in the wave's LDS row.
template <int KT, typename TexT>
__global__ __launch_bounds__(256) void k_dump_integrand(ShadeArgs a, int32_t k) {
  __shared__ float s_acc[kWavesPerBlock][SOP_MLP_BINS];
  const int64_t wv = die_block() * kWavesPerBlock + wave_id_uniform();
  if (wv >= a.n) return;
  const int lane = threadIdx.x & 63;
  float* accb = s_acc[threadIdx.x >> 6];
  PointState ps;
  if (!load_point(a, wv, ps)) return;
  Neighbors<KT> nb;
  nb.load(a, ps.p, k);
#pragma unroll
  for (int t = 0; t < 4; ++t) accb[4 * lane + t] = 0.0f;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t sh = pcg_hash(a.seed), pi = (uint32_t)ps.p;
  const int npb = a.npb, total = SOP_MLP_BINS * npb;
  const float al[3] = {ps.M.a.x, ps.M.a.y, ps.M.a.z};
  for (int j0 = 0; j0 < total; j0 += 64) {
    const int j = j0 + lane;
    if (j < total) {
      const int b = j / npb, kk = j - b * npb;
      // u stratified over the bin's draws, v random
      const double xu =
          ((double)kk + ((double)hash24(sh, pi, (uint32_t)j, 1) + 0.5) * 0x1p-24) / (double)npb;
      const double xv = ((double)hash24(sh, pi, (uint32_t)j, 2) + 0.5) * 0x1p-24;
      double wl[3];
      const double l = cell_point(xu, xv, b, wl);
      Sample s;
      world_dir64(ps.F, wl[0], wl[1], wl[2], s.w64);
      s.w = mk3((float)s.w64[0], (float)s.w64[1], (float)s.w64[2]);
      s.ct = (float)wl[2];
      eval_at<KT, TexT>(a, ps, nb, k, s);
      const BrdfTerms bt = brdf_terms(ps.M, half_geom(ps.n64, ps.v64, s.w64), s.ct);
      float y[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        y[c] = fcos(ps.M, bt, al[c], s.ct) * ((1.0f - s.O) * s.Le[c] + s.Lin[c]);
      const float lum = 0.2126f * y[0] + 0.7152f * y[1] + 0.0722f * y[2];
      atomicAdd(accb + b, lum * (float)(1.0 / (l * l * l)));
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const float sc = 1.0f / (128.0f * (float)npb);
  const float4 v = make_float4(accb[4 * lane] * sc, accb[4 * lane + 1] * sc,
                               accb[4 * lane + 2] * sc, accb[4 * lane + 3] * sc);
  *reinterpret_cast<float4*>(a.targets + (size_t)ps.p * SOP_MLP_BINS + 4 * lane) = v;
}

// Adjoint of one sample. With g the upstream gradient of the point and s = 2 pi / S:
//   d/da_c  = s sum g_c L_i,c [ (1-m) cos/pi + spec m (1 - x^5) ]
//   d/dm    = s sum_c g_c L_i,c [ -a_c cos/pi + spec (a_c - 0.04)(1 - x^5) ]
//   d/dr    = s sum_c g_c L_i,c F_c/(4 NoV) (dD/dalpha G + D dG/dalpha) 2 r
//   d/dLin_k[t,c] = s g_c fcos_c w_k b_t,   d/dO_k[t] = -s sum_c g_c fcos_c Le_c w_k b_t
//   d/denv[t',c]  = s g_c fcos_c (1 - O) b'_t'
// where spec = D G1(NoL) G1(NoV) / (4 NoV) and x = 1 - v.h. Material terms are added to
// ga/gr/gm (without the factor s); gl (RGB) and go (O) are the texture factors before the
// w_k b_t weights, ge the environment factors before b'.
struct SampleAdj {
  float gl[3], go, ge[3];
};

template <int KT, typename TexT, bool EO = false>
__device__ __forceinline__ void sample_adjoint(const ShadeArgs& a, const PointState& ps,
                                               const Neighbors<KT>& nb, int32_t k, int j,
                                               const float g[3], float ga[3], float& gr,
                                               float& gm, Sample& s, SampleAdj& r) {
  const Material& M = ps.M;
  const float al[3] = {M.a.x, M.a.y, M.a.z};
  eval_sample<KT, TexT, EO>(a, ps, nb, k, j, s);
  const BrdfTerms bt = brdf_terms(M, half_geom(ps.n64, ps.v64, s.w64), s.ct);
  const float om5 = 1.0f - bt.x5;
  // dD/dalpha = 2 alpha (1 - NoH^2 - alpha^2 NoH^2) / (pi q^3)
  const float dD = 2.0f * M.alpha * (bt.one_m - M.a2 * bt.NoH2) / (kPi * bt.q * bt.q * bt.q);
  const float denL = s.ct * M.one_m_k + M.k, denV = M.NoV * M.one_m_k + M.k;
  const float dG1L = -s.ct * (1.0f - s.ct) / (denL * denL);
  const float dG1V = -M.NoV * (1.0f - M.NoV) / (denV * denV);
  const float G = bt.G1L * M.g1v;
  const float dG = 0.5f * (dG1L * M.g1v + bt.G1L * dG1V);
  const float i4nv = 1.0f / (4.0f * M.NoV);
  const float drough = i4nv * (dD * G + bt.D * dG) * 2.0f * M.r;
  r.go = 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float Li = (1.0f - s.O) * s.Le[c] + s.Lin[c];
    const float F0 = 0.04f * (1.0f - M.m) + al[c] * M.m;
    const float F = F0 + (1.0f - F0) * bt.x5;
    const float fc = (1.0f - M.m) * al[c] * kInvPi * s.ct + bt.spec * F;
    const float cm = g[c] * Li;
    ga[c] += cm * ((1.0f - M.m) * kInvPi * s.ct + bt.spec * M.m * om5);
    gm += cm * (-al[c] * kInvPi * s.ct + bt.spec * (al[c] - 0.04f) * om5);
    gr += cm * F * drough;
    const float gf = g[c] * fc * a.scale;
    r.gl[c] = gf;
    r.go -= gf * s.Le[c];
    r.ge[c] = gf * (1.0f - s.O);
  }
}

// Exact accumulation for the deterministic adjoint. A float v is m 2^e with an integer
// m < 2^24, so v 2^96 is the integer m 2^(e+96) whenever e >= -96 (below that the bits under
// 2^-96 are dropped, towards zero); for |v| < 2^32 it has at most 128 bits, and its 24
// significant bits fall into at most two of the four 32-bit chunks k = 0..3. Each chunk is
// added, with the sign of v, to the 64-bit word k of the value (integer addition: the order
// of the additions does not change the sum; up to 2^31 terms per value fit). A value that
// is not finite or has |v| >= 2^32 sets *flag instead.
__device__ __forceinline__ void det_add(unsigned long long* words, int64_t n, int64_t i,
                                        float v, int32_t* flag) {
  const uint32_t b = __float_as_uint(v);
  const uint32_t ex = (b >> 23) & 0xFFu;
  if (ex == 0xFFu) {
    atomicOr(flag, 1);
    return;
  }
  uint32_t m = b & 0x7FFFFFu;
  int sh;
  if (ex == 0) {
    sh = -149 + 96;                   // subnormal: m 2^-149
  } else {
    m |= 0x800000u;
    sh = (int)ex - 150 + 96;          // m 2^(ex - 150), times 2^96
  }
  if (m == 0) return;
  if (sh > 104) {                     // |v| >= 2^32
    atomicOr(flag, 1);
    return;
  }
  if (sh < 0) {
    if (sh <= -24) return;
    m >>= -sh;
    sh = 0;
    if (m == 0) return;
  }
  const unsigned __int128 X = (unsigned __int128)m << sh;
  const bool neg = (b >> 31) != 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned long long c = (unsigned long long)(uint32_t)(X >> (32 * k));
    if (c) atomicAdd(words + (size_t)k * n + i, neg ? 0ull - c : c);
  }
}

// adds v to value i of a gradient: a float atomic into out, or (DET) exactly into words
template <bool DET>
__device__ __forceinline__ void add_grad(float* out, unsigned long long* words, int64_t n,
                                         int64_t i, float v, int32_t* flag) {
  if constexpr (DET)
    det_add(words, n, i, v, flag);
  else
    unsafeAtomicAdd(out + i, v);
}

template <bool DET = false>
__device__ __forceinline__ void scatter_env(const ShadeArgs& a, const Sample& s,
                                            const SampleAdj& r) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t o = (int64_t)s.et.off[t] * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      add_grad<DET>(a.g_env, a.det_env, a.det_ne, o + c, s.et.w[t] * r.ge[c], a.det_flag);
  }
}

// General adjoint: one wavefront per point, texture gradients scattered with atomics.
// Used when the grouped kernel below does not apply (res > 32, more than 16384 probes).
template <int KT, typename TexT, bool EO = false, bool DET = false>
__global__ __launch_bounds__(256) void k_shade_bwd(ShadeArgs a, int32_t k) {
  const int64_t wv = die_block() * kWavesPerBlock + wave_id_uniform();
  if (wv >= a.n) return;
  const int lane = threadIdx.x & 63;
  PointState ps;
  if (!load_point(a, wv, ps)) return;
  Neighbors<KT> nb;
  nb.load(a, ps.p, k);
  const float g[3] = {a.grad[3 * ps.p], a.grad[3 * ps.p + 1], a.grad[3 * ps.p + 2]};
  const size_t RR = (size_t)a.R * a.R;
  const int kc = KT > 0 ? KT : nb.count(k);

  float ga[3] = {0.0f, 0.0f, 0.0f}, gr = 0.0f, gm = 0.0f;
  for (int j0 = 0; j0 < a.S; j0 += 64) {
    const int j = j0 + lane;
    if (j < a.S) {
      Sample s;
      SampleAdj r;
      sample_adjoint<KT, TexT, EO>(a, ps, nb, k, j, g, ga, gr, gm, s, r);
      if (a.g_tex) {
        for (int s2 = 0; s2 < kc; ++s2) {
          const int32_t id = nb.id(s2, a, ps.p, k);
          if (id < 0) continue;
          const float wk = nb.wt(s2, a, ps.p, k);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const float cw = wk * s.tt.w[t];
            const int64_t o = ((int64_t)id * (int64_t)RR + s.tt.off[t]) * 4;
            add_grad<DET>(a.g_tex, a.det_tex, a.det_nt, o + 0, cw * r.gl[0], a.det_flag);
            add_grad<DET>(a.g_tex, a.det_tex, a.det_nt, o + 1, cw * r.gl[1], a.det_flag);
            add_grad<DET>(a.g_tex, a.det_tex, a.det_nt, o + 2, cw * r.gl[2], a.det_flag);
            add_grad<DET>(a.g_tex, a.det_tex, a.det_nt, o + 3, cw * r.go, a.det_flag);
          }
        }
      }
      if (a.g_env) scatter_env<DET>(a, s, r);
    }
  }
  const float r0 = wave_sum(ga[0]) * a.scale, r1 = wave_sum(ga[1]) * a.scale,
              r2 = wave_sum(ga[2]) * a.scale;
  const float rr = wave_sum(gr) * a.scale, rm = wave_sum(gm) * a.scale;
  if (lane == 0) {
    if (a.g_albedo) {
      a.g_albedo[3 * ps.p] = r0;
      a.g_albedo[3 * ps.p + 1] = r1;
      a.g_albedo[3 * ps.p + 2] = r2;
    }
    if (a.g_rough) a.g_rough[ps.p] = rr;
    if (a.g_metal) a.g_metal[ps.p] = rm;
  }
}

// ------------------------------------------------------------------------------------------
// Batched adjoint: a workgroup of kBatch wavefronts takes kBatch points that are
// consecutive in the processing order (they share most of their probes), one wavefront per
// point. Every point's texture adjoint H_p (its samples' factors spread over their 4 taps)
// is accumulated densely in LDS. Then, for each distinct probe k of the batch, each thread
// forms sum_p w_{p,k} H_p over the flattened texel-channel values it owns
// (v = t + kBatchThreads * i) and adds it to g_tex[k] with atomics that are coalesced
// (consecutive lanes, consecutive words). This replaces K*4*4 scattered atomics per
// sample by about (distinct probes / kBatch) * res^2 * 4 coalesced atomics per point.
// The environment adjoint of a sample is its bilinear footprint, 4 texels x 3 channels.
// Scattered one float per lane, every atomic instruction touches 64 cache lines; instead
// each wavefront stages the footprints of 32 samples in LDS and adds each with
// consecutive lanes: as one 64-byte block record (env_blk_flush, the float adjoint) or as
// two rows of six consecutive floats, "runs" (env_runs_flush: the exact adjoint, and
// environments beyond the block limit).
// ------------------------------------------------------------------------------------------
constexpr int kBatch = 8;
constexpr int kBatchThreads = kBatch * 64;
constexpr int kMaxRes = 32;
constexpr int kVPT = kMaxRes * kMaxRes * 4 / kBatchThreads;   // values per thread (8)
constexpr int kMaxEntries = kBatch * 16;                      // (point, neighbour) pairs
constexpr int kEnvRuns = 64;                                  // staged runs per wavefront

struct EnvRun {
  int32_t b0, b1;     // float offsets of the run's two texels in g_env (-1: no run)
  float v[6];         // their three channel values each
};

// Stages the environment adjoint of the lanes [32h, 32h + 32) of the wavefront and adds it
// to g_env; every lane of the wavefront calls it (lanes without a sample pass valid=false).
template <bool DET = false>
__device__ __forceinline__ void env_runs_flush(const ShadeArgs& a, EnvRun* run, int lane,
                                               int h, bool valid, const Sample& s,
                                               const SampleAdj& r) {
  if ((lane >> 5) == h) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      EnvRun& e = run[(lane & 31) * 2 + q];
      if (valid) {
        e.b0 = s.et.off[2 * q] * 3;
        e.b1 = s.et.off[2 * q + 1] * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          e.v[c] = s.et.w[2 * q] * r.ge[c];
          e.v[3 + c] = s.et.w[2 * q + 1] * r.ge[c];
        }
      } else {
        e.b0 = -1;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int sub = lane / 6, comp = lane - 6 * sub;        // lanes 60..63 idle
  for (int q0 = 0; q0 < kEnvRuns; q0 += 10) {
    const int q = q0 + sub;
    if (lane < 60 && q < kEnvRuns) {
      const EnvRun& e = run[q];
      if (e.b0 >= 0)
        add_grad<DET>(a.g_env, a.det_env, a.det_ne, comp < 3 ? e.b0 + comp : e.b1 + comp - 3,
                      e.v[comp], a.det_flag);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Float environment adjoint in blocks: the lanes [32h, 32h + 32) stage their sample's
// footprint (4 texels x 3 channels, tap order (i0,j0) (i1,j0) (i0,j1) (i1,j1)) with the
// index of its 64-byte block record (see env_block_cols), then 12 consecutive lanes add
// one record, 5 records per instruction. Each sample costs one 64-byte atomic request at
// memory instead of the two 24-byte runs (2.6 requests on average) of env_runs_flush; the
// float atomics retire at the memory side, so the request count is their cost.
__device__ __forceinline__ void env_blk_flush(const ShadeArgs& a, float* stage, int lane,
                                              int h, bool valid, const Sample& s,
                                              const SampleAdj& r) {
  if ((lane >> 5) == h) {
    float* e = stage + (lane & 31) * kEnvBlkFloats;
    int32_t rec = -1;
    if (valid) {
      const int cls = (s.et.vj & 1) * 2 + (s.et.vi & 1);
      rec = (cls * a.env_bh + (s.et.vj >> 1)) * a.env_bw + (s.et.vi >> 1);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 3; ++c) e[3 * t + c] = s.et.w[t] * r.ge[c];
    }
    reinterpret_cast<int32_t*>(e)[12] = rec;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int sub = lane / 12, comp = lane - 12 * sub;      // lanes 60..63 idle
  for (int q0 = 0; q0 < 32; q0 += 5) {
    const int q = q0 + sub;
    if (lane < 60 && q < 32) {
      const float* e = stage + q * kEnvBlkFloats;
      const int32_t rec = reinterpret_cast<const int32_t*>(e)[12];
      if (rec >= 0) unsafeAtomicAdd(a.env_blk + (int64_t)rec * kEnvBlkFloats + comp, e[comp]);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Per-wavefront LDS scratch of the batched adjoint, in 32-bit words: the staged environment
// runs (kEnvRuns EnvRun records) and, after them, the sort of the texture splat (256 keys,
// 64 factors, 4 x 64 tap weights) share it.
constexpr int kScratchWords = 768;
static_assert(kEnvRuns * (int)sizeof(EnvRun) <= kScratchWords * 4, "env runs fit the scratch");
static_assert(32 * kEnvBlkFloats <= kScratchWords, "env blocks fit the scratch");

// Adds the texture adjoint of the wavefront's current samples (one per lane; valid = false
// lanes have none) to the point's LDS map H without atomics: the 256 (tap texel, entry)
// pairs are sorted by texel with a stable radix sort on wavefront ballots, and the first
// entry of every run of equal texels adds the run's values (tap weight x factor, in entry
// order) to H[texel] with a plain read-modify-write; runs hold distinct texels, so no two
// lanes write the same word. (LDS float atomics retire at ~0.3 lanes per clock per CU on
// this chip, an order of magnitude below plain LDS traffic.)
__device__ __forceinline__ void splat_sorted(float* H, uint32_t* scr, int lane, bool valid,
                                             const Sample& s, const SampleAdj& r,
                                             uint32_t nkey, int nbits) {
  uint32_t* buf = scr;                                            // [256] keys
  float4* fac = reinterpret_cast<float4*>(scr + 256);             // [64] factors
  float* wt = reinterpret_cast<float*>(scr + 512);                // [4][64] tap weights
  fac[lane] = make_float4(r.gl[0], r.gl[1], r.gl[2], r.go);
  uint32_t v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    wt[t * 64 + lane] = s.tt.w[t];
    const uint32_t key = valid ? (uint32_t)s.tt.off[t] : nkey;     // nkey sorts last
    v[t] = (key << 8) | ((uint32_t)t << 6) | (uint32_t)lane;
  }
  const uint64_t below = (1ull << lane) - 1ull;
  for (int bit = 8; bit < 8 + nbits; ++bit) {
    uint64_t bal[4];
    int zeros = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bal[i] = __ballot((v[i] >> bit) & 1u);
      zeros += 64 - __popcll(bal[i]);
    }
    int zb = 0, ob = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool one = (v[i] >> bit) & 1u;
      const int pos = one ? zeros + ob + __popcll(bal[i] & below) : zb + __popcll(~bal[i] & below);
      buf[pos] = v[i];
      const int ones = __popcll(bal[i]);
      ob += ones;
      zb += 64 - ones;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (bit + 1 < 8 + nbits) {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = buf[i * 64 + lane];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // lane takes sorted positions 4 lane .. 4 lane + 3
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = 4 * lane + i;
    uint32_t w = buf[p];
    const uint32_t key = w >> 8;
    if (key >= nkey) continue;
    if (p > 0 && (buf[p - 1] >> 8) == key) continue;     // not the first of its run
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int q = p;;) {
      const uint32_t e = w & 0xFFu;
      const float tw = wt[(e >> 6) * 64 + (e & 63u)];
      const float4 f = fac[e & 63u];
      acc.x += tw * f.x;
      acc.y += tw * f.y;
      acc.z += tw * f.z;
      acc.w += tw * f.w;
      if (++q >= 256) break;
      w = buf[q];
      if ((w >> 8) != key) break;
    }
    float4* h = reinterpret_cast<float4*>(H) + key;
    float4 hv = *h;
    hv.x += acc.x;
    hv.y += acc.y;
    hv.z += acc.z;
    hv.w += acc.w;
    *h = hv;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KT, typename TexT, bool EO = false, bool DET = false>
__global__ __launch_bounds__(kBatchThreads) void k_shade_bwd_batched(ShadeArgs a, int32_t k) {
  extern __shared__ float lds[];
  const int MV = a.R * a.R * 4;                         // values per map
  float* H = lds;                                       // [kBatch][MV]
  int32_t* eid = reinterpret_cast<int32_t*>(H + kBatch * MV);   // [kMaxEntries] probe ids
  float* ew = reinterpret_cast<float*>(eid + kMaxEntries);      // [kMaxEntries] weights
  int32_t* eslot = reinterpret_cast<int32_t*>(ew + kMaxEntries);  // [kMaxEntries] slot
  int32_t* uni = eslot + kMaxEntries;                   // [kMaxEntries] probe of slot
  int32_t* erank = uni + kMaxEntries;                   // [kMaxEntries] slot of a leader
  float* W = reinterpret_cast<float*>(erank + kMaxEntries);     // [kMaxEntries][kBatch]
  int32_t* misc = reinterpret_cast<int32_t*>(W + kMaxEntries * kBatch);  // [1]
  // [kBatch][kScratchWords], 16-byte aligned; indexed off the LDS array itself so that the
  // accesses stay LDS instructions (not generic ones that also wait on global memory)
  const int scr_off = (kBatch * MV + 5 * kMaxEntries + kMaxEntries * kBatch + 1 + 3) & ~3;

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int64_t g0 = die_block() * kBatch;
  const int bn = (int)min((int64_t)kBatch, a.n - g0);
  if (bn <= 0) return;
  const int ne = kBatch * k;

  for (int i = tid; i < kBatch * MV; i += kBatchThreads) H[i] = 0.0f;
  for (int i = tid; i < kMaxEntries * kBatch; i += kBatchThreads) W[i] = 0.0f;
  if (tid < ne) {
    const int b = tid / k, s2 = tid % k;
    int32_t id = -1;
    float w = 0.0f;
    if (b < bn) {
      const int32_t o = a.order ? a.order[g0 + b] : (int32_t)(g0 + b);
      if ((uint64_t)o < (uint64_t)a.n) {
        id = a.nb_idx[(int64_t)o * k + s2];
        w = a.nb_w[(int64_t)o * k + s2];
        if ((uint32_t)id >= (uint32_t)a.P) id = -1;
      }
    }
    eid[tid] = id;
    ew[tid] = w;
  }
  __syncthreads();
  // distinct probes of the batch: entry e leads if no earlier entry has its probe; slots are
  // the ranks of the leading entries (each thread scans at most kMaxEntries entries)
  int32_t lead = -1;
  if (tid < ne) {
    const int32_t id = eid[tid];
    if (id >= 0) {
      lead = tid;
      for (int e = 0; e < tid; ++e)
        if (eid[e] == id) { lead = e; break; }
    }
    eslot[tid] = lead;
  }
  __syncthreads();
  if (tid < ne && lead == tid) {
    int32_t rank = 0;
    for (int e = 0; e < tid; ++e) rank += (eslot[e] == e) ? 1 : 0;
    erank[tid] = rank;
    uni[rank] = eid[tid];
  }
  if (tid == 0) {
    int32_t n = 0;
    for (int e = 0; e < ne; ++e) n += (eslot[e] == e) ? 1 : 0;
    misc[0] = n;
  }
  __syncthreads();
  // added, not stored: a list that names one probe twice counts both entries, as the
  // forward does
  if (tid < ne && lead >= 0) atomicAdd(&W[erank[lead] * kBatch + tid / k], ew[tid]);
  __syncthreads();

  // --- splat: wavefront b takes point b, lanes take directions -----------------------------
  {
    const int b = wave;
    if (b < bn) {
      PointState ps;
      if (load_point(a, g0 + b, ps)) {
        Neighbors<KT> nb;
        nb.load(a, ps.p, k);
        const float g[3] = {a.grad[3 * ps.p], a.grad[3 * ps.p + 1], a.grad[3 * ps.p + 2]};
        float ga[3] = {0.0f, 0.0f, 0.0f}, gr = 0.0f, gm = 0.0f;
        float* Hb = H + b * MV;
        uint32_t* scr = reinterpret_cast<uint32_t*>(lds + scr_off + b * kScratchWords);
        EnvRun* rb = reinterpret_cast<EnvRun*>(lds + scr_off + b * kScratchWords);
        const uint32_t nkey = (uint32_t)(a.R * a.R);           // texels per map, <= 1024
        const int nbits = 32 - __clz((int)nkey);               // bits of keys 0 .. nkey
        for (int j0 = 0; j0 < a.S; j0 += 64) {     // uniform over the wavefront
          const int j = j0 + lane;
          Sample s;
          SampleAdj r;
          if (j < a.S) sample_adjoint<KT, TexT, EO>(a, ps, nb, k, j, g, ga, gr, gm, s, r);
          if (a.g_env) {
            if (!DET && a.env_blk) {
              float* eb = lds + scr_off + b * kScratchWords;
              env_blk_flush(a, eb, lane, 0, j < a.S, s, r);
              env_blk_flush(a, eb, lane, 1, j < a.S, s, r);
            } else {
              env_runs_flush<DET>(a, rb, lane, 0, j < a.S, s, r);
              env_runs_flush<DET>(a, rb, lane, 1, j < a.S, s, r);
            }
          }
          if (a.g_tex) splat_sorted(Hb, scr, lane, j < a.S, s, r, nkey, nbits);
        }
        const float v0 = wave_sum(ga[0]) * a.scale, v1 = wave_sum(ga[1]) * a.scale,
                    v2 = wave_sum(ga[2]) * a.scale;
        const float v3 = wave_sum(gr) * a.scale, v4 = wave_sum(gm) * a.scale;
        if (lane == 0) {
          if (a.g_albedo) {
            a.g_albedo[3 * ps.p] = v0;
            a.g_albedo[3 * ps.p + 1] = v1;
            a.g_albedo[3 * ps.p + 2] = v2;
          }
          if (a.g_rough) a.g_rough[ps.p] = v3;
          if (a.g_metal) a.g_metal[ps.p] = v4;
        }
      }
    }
  }
  __syncthreads();
  if (!a.g_tex) return;
  // --- per distinct probe: sum_b W[u][b] H_b, coalesced flush ------------------------------
  float h[kBatch][kVPT];
#pragma unroll
  for (int b = 0; b < kBatch; ++b)
#pragma unroll
    for (int i = 0; i < kVPT; ++i) {
      const int v = tid + kBatchThreads * i;
      h[b][i] = (b < bn && v < MV) ? H[b * MV + v] : 0.0f;
    }
  const int nu = misc[0];
  for (int u = 0; u < nu; ++u) {
    float acc[kVPT];
#pragma unroll
    for (int i = 0; i < kVPT; ++i) acc[i] = 0.0f;
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const float w = W[u * kBatch + b];
#pragma unroll
      for (int i = 0; i < kVPT; ++i) acc[i] = fmaf(w, h[b][i], acc[i]);
    }
    const int64_t base = (int64_t)uni[u] * MV;
#pragma unroll
    for (int i = 0; i < kVPT; ++i) {
      const int v = tid + kBatchThreads * i;
      // texels no sample reached stay untouched
      if (v < MV && acc[i] != 0.0f)
        add_grad<DET>(a.g_tex, a.det_tex, a.det_nt, base + v, acc[i], a.det_flag);
    }
  }
}

// Eq. 9 at caller-given world directions: one thread per (point, direction).
template <typename TexT>
__global__ __launch_bounds__(256) void k_query(ShadeArgs a, int32_t k, const float* dirs,
                                               int32_t D, float* Lin, float* O) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.n * (int64_t)D) return;
  const int64_t i = t / D;
  const double w[3] = {dirs[3 * t], dirs[3 * t + 1], dirs[3 * t + 2]};
  const Taps tt = oct_taps64(w, a.R);
  const TexT* tex = reinterpret_cast<const TexT*>(a.tex);
  const size_t RR = (size_t)a.R * a.R;
  float L0 = 0.0f, L1 = 0.0f, L2 = 0.0f, oc = 0.0f;
  for (int s = 0; s < k; ++s) {
    const int32_t id = a.nb_idx[i * k + s];
    if ((uint32_t)id >= (uint32_t)a.P) continue;
    const float wk = a.nb_w[i * k + s];
    const TexT* T = tex + (size_t)id * RR;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 x = load_texel(T, (size_t)tt.off[q]);
      const float c = wk * tt.w[q];
      L0 += c * x.x;
      L1 += c * x.y;
      L2 += c * x.z;
      oc += c * x.w;
    }
  }
  Lin[3 * t] = L0;
  Lin[3 * t + 1] = L1;
  Lin[3 * t + 2] = L2;
  O[t] = oc;
}

// lanes per point for S directions: 16, 32 or 64
static int lanes_for(int32_t S) { return S <= 16 ? 16 : (S <= 32 ? 32 : 64); }

static dim3 grid_for(int64_t n, int L) {
  const int64_t per_block = (int64_t)kWavesPerBlock * (64 / L);
  return dim3((unsigned)((n + per_block - 1) / per_block));
}

template <int KT, int L>
static void launch_prop_l(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  const dim3 grid = grid_for(a.n, L);
  if (format == SOP_TEXEL_F16)
    hipLaunchKernelGGL((k_shade_prop<KT, uint2, L>), grid, dim3(256), 0, s, a, k);
  else
    hipLaunchKernelGGL((k_shade_prop<KT, float4, L>), grid, dim3(256), 0, s, a, k);
}

template <int KT>
static void launch_prop_kt(int mode, const ShadeArgs& a, int32_t k, int32_t format, dim3 grid,
                           hipStream_t s) {
  if (mode == 0) {
    switch (lanes_for(a.S)) {
      case 16: launch_prop_l<KT, 16>(a, k, format, s); break;
      case 32: launch_prop_l<KT, 32>(a, k, format, s); break;
      default: launch_prop_l<KT, 64>(a, k, format, s); break;
    }
  } else {
    if (format == SOP_TEXEL_F16)
      hipLaunchKernelGGL((k_dump_integrand<KT, uint2>), grid, dim3(256), 0, s, a, k);
    else
      hipLaunchKernelGGL((k_dump_integrand<KT, float4>), grid, dim3(256), 0, s, a, k);
  }
}

static hipError_t dispatch_prop(int mode, const ShadeArgs& a, int32_t k, int32_t format,
                                hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const dim3 grid((unsigned)((a.n + kWavesPerBlock - 1) / kWavesPerBlock));
  switch (k) {
    case 4: launch_prop_kt<4>(mode, a, k, format, grid, s); break;
    case 8: launch_prop_kt<8>(mode, a, k, format, grid, s); break;
    default: launch_prop_kt<0>(mode, a, k, format, grid, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_shade_prop(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  return dispatch_prop(0, a, k, format, s);
}

template <int KT>
static void launch_prop_net_kt(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  const int64_t tiles = (a.n + 15) / 16;
  const dim3 grid((unsigned)((tiles + kWavesPerBlock - 1) / kWavesPerBlock));
  if (format == SOP_TEXEL_F16)
    hipLaunchKernelGGL((k_shade_prop_net<KT, uint2>), grid, dim3(256), 0, s, a, k);
  else
    hipLaunchKernelGGL((k_shade_prop_net<KT, float4>), grid, dim3(256), 0, s, a, k);
}

hipError_t launch_shade_prop_net(const ShadeArgs& a, int32_t k, int32_t format,
                                 hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (!a.mlp_params || !a.mlp_frags) return hipErrorInvalidValue;
  switch (k) {
    case 4: launch_prop_net_kt<4>(a, k, format, s); break;
    case 8: launch_prop_net_kt<8>(a, k, format, s); break;
    default: launch_prop_net_kt<0>(a, k, format, s); break;
  }
  return hipGetLastError();
}
hipError_t launch_dump_integrand(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  return dispatch_prop(1, a, k, format, s);
}

template <int KT, bool EO>
static void launch_fwd_e(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  constexpr int per_block = kWavesPerBlock * (64 / kFwdLanes);
  const dim3 grid((unsigned)((a.n + per_block - 1) / per_block));
  if (a.cosine) {
    if (format == SOP_TEXEL_F16)
      hipLaunchKernelGGL((k_shade_fwd_cl<KT, uint2, EO, true>), grid, dim3(256), 0, s, a, k);
    else
      hipLaunchKernelGGL((k_shade_fwd_cl<KT, float4, EO, true>), grid, dim3(256), 0, s, a, k);
    return;
  }
  if (format == SOP_TEXEL_F16)
    hipLaunchKernelGGL((k_shade_fwd_cl<KT, uint2, EO>), grid, dim3(256), 0, s, a, k);
  else
    hipLaunchKernelGGL((k_shade_fwd_cl<KT, float4, EO>), grid, dim3(256), 0, s, a, k);
}

template <int KT>
static void launch_kt(bool fwd, const ShadeArgs& a, int32_t k, int32_t format, dim3 grid,
                      hipStream_t s) {
  if (fwd) {
    if (a.env_oct)
      launch_fwd_e<KT, true>(a, k, format, s);
    else
      launch_fwd_e<KT, false>(a, k, format, s);
  } else if (a.env_oct) {
    if (format == SOP_TEXEL_F16)
      hipLaunchKernelGGL((k_shade_bwd<KT, uint2, true>), grid, dim3(256), 0, s, a, k);
    else
      hipLaunchKernelGGL((k_shade_bwd<KT, float4, true>), grid, dim3(256), 0, s, a, k);
  } else {
    if (format == SOP_TEXEL_F16)
      hipLaunchKernelGGL((k_shade_bwd<KT, uint2>), grid, dim3(256), 0, s, a, k);
    else
      hipLaunchKernelGGL((k_shade_bwd<KT, float4>), grid, dim3(256), 0, s, a, k);
  }
}

static hipError_t dispatch(bool fwd, const ShadeArgs& a, int32_t k, int32_t format,
                           hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const dim3 grid((unsigned)((a.n + kWavesPerBlock - 1) / kWavesPerBlock));
  switch (k) {
    case 4: launch_kt<4>(fwd, a, k, format, grid, s); break;
    case 8: launch_kt<8>(fwd, a, k, format, grid, s); break;
    default: launch_kt<0>(fwd, a, k, format, grid, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_shade_fwd(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  return dispatch(true, a, k, format, s);
}
template <int L>
static void launch_traced_l(const ShadeArgs& a, hipStream_t s) {
  if (a.env_oct)
    hipLaunchKernelGGL((k_shade_traced<L, true>), grid_for(a.n, L), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_shade_traced<L, false>), grid_for(a.n, L), dim3(256), 0, s, a);
}

hipError_t launch_shade_traced(const ShadeArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (!a.traced) return hipErrorInvalidValue;
  switch (lanes_for(a.S)) {
    case 16: launch_traced_l<16>(a, s); break;
    case 32: launch_traced_l<32>(a, s); break;
    default: launch_traced_l<64>(a, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_env_cdf(const float* env, int32_t T, uint32_t* mass, uint64_t* prefix,
                          uint64_t* tile_tmp, float* imax, int32_t* guide, hipStream_t s) {
  if (T < 1 || T > (1 << 20) || !env || !mass || !prefix || !tile_tmp || !imax || !guide)
    return hipErrorInvalidValue;
  const int ntiles = (T + kCdfTile - 1) / kCdfTile;
  hipLaunchKernelGGL(k_env_max, dim3(1), dim3(1024), 0, s, env, T, imax);
  hipLaunchKernelGGL(k_env_tiles, dim3(ntiles), dim3(1024), 0, s, env, T, imax, mass, prefix,
                     tile_tmp);
  hipLaunchKernelGGL(k_env_tile_scan, dim3(1), dim3(1024), 0, s, ntiles, tile_tmp, prefix, T);
  hipLaunchKernelGGL(k_env_add, dim3(ntiles), dim3(1024), 0, s, T, tile_tmp, prefix);
  hipLaunchKernelGGL(k_env_guide, dim3((kEnvGuide + 1 + 255) / 256), dim3(256), 0, s, prefix, T,
                     guide);
  return hipGetLastError();
}

template <int KT, int L>
static void launch_envis_l(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  const dim3 grid = grid_for(a.n, L);
  if (format == SOP_TEXEL_F16)
    hipLaunchKernelGGL((k_shade_envis<KT, uint2, L>), grid, dim3(256), 0, s, a, k);
  else
    hipLaunchKernelGGL((k_shade_envis<KT, float4, L>), grid, dim3(256), 0, s, a, k);
}

template <int KT>
static void launch_envis_kt(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  switch (lanes_for(a.S)) {
    case 16: launch_envis_l<KT, 16>(a, k, format, s); break;
    case 32: launch_envis_l<KT, 32>(a, k, format, s); break;
    default: launch_envis_l<KT, 64>(a, k, format, s); break;
  }
}

hipError_t launch_shade_envis(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (!a.env_mass || !a.env_prefix || !a.env_oct) return hipErrorInvalidValue;
  switch (k) {
    case 4: launch_envis_kt<4>(a, k, format, s); break;
    case 8: launch_envis_kt<8>(a, k, format, s); break;
    default: launch_envis_kt<0>(a, k, format, s); break;
  }
  return hipGetLastError();
}

template <int KT, int L>
static void launch_shadow_l(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  const dim3 grid = grid_for(a.n, L);
  if (format == SOP_TEXEL_F16)
    hipLaunchKernelGGL((k_shadow_ratio<KT, uint2, L>), grid, dim3(256), 0, s, a, k);
  else
    hipLaunchKernelGGL((k_shadow_ratio<KT, float4, L>), grid, dim3(256), 0, s, a, k);
}

template <int KT>
static void launch_shadow_kt(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  switch (lanes_for(a.S)) {
    case 16: launch_shadow_l<KT, 16>(a, k, format, s); break;
    case 32: launch_shadow_l<KT, 32>(a, k, format, s); break;
    default: launch_shadow_l<KT, 64>(a, k, format, s); break;
  }
}

hipError_t launch_shadow_ratio(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (a.shadow_sampler != 0 && (!a.env_mass || !a.env_prefix)) return hipErrorInvalidValue;
  if (a.shadow_sampler == 0 && !a.dir_tab) return hipErrorInvalidValue;
  switch (k) {
    case 4: launch_shadow_kt<4>(a, k, format, s); break;
    case 8: launch_shadow_kt<8>(a, k, format, s); break;
    default: launch_shadow_kt<0>(a, k, format, s); break;
  }
  return hipGetLastError();
}

size_t batched_lds_bytes(int32_t R) {
  return (size_t)kBatch * R * R * 4 * sizeof(float) + 5 * kMaxEntries * 4 +
         (size_t)kMaxEntries * kBatch * 4 + 4 + 15 + (size_t)kBatch * kScratchWords * 4;
}

template <int KT, bool EO, bool DET>
static void launch_batched_kte(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + kBatch - 1) / kBatch));
  const size_t lds = batched_lds_bytes(a.R);
  // dynamic LDS above 64 KB must be allowed per kernel (gfx950 has 160 KB per CU)
  (void)hipFuncSetAttribute(
      reinterpret_cast<const void*>(&k_shade_bwd_batched<KT, uint2, EO, DET>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute(
      reinterpret_cast<const void*>(&k_shade_bwd_batched<KT, float4, EO, DET>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (format == SOP_TEXEL_F16)
    hipLaunchKernelGGL((k_shade_bwd_batched<KT, uint2, EO, DET>), grid, dim3(kBatchThreads), lds,
                       s, a, k);
  else
    hipLaunchKernelGGL((k_shade_bwd_batched<KT, float4, EO, DET>), grid, dim3(kBatchThreads),
                       lds, s, a, k);
}

template <int KT, bool DET>
static void launch_batched_kt(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  if (a.env_oct)
    launch_batched_kte<KT, true, DET>(a, k, format, s);
  else
    launch_batched_kte<KT, false, DET>(a, k, format, s);
}

// general adjoint (res > 32 or K > 16) with exact accumulation
template <int KT>
static void launch_bwd_det_kt(const ShadeArgs& a, int32_t k, int32_t format, dim3 grid,
                              hipStream_t s) {
  if (a.env_oct) {
    if (format == SOP_TEXEL_F16)
      hipLaunchKernelGGL((k_shade_bwd<KT, uint2, true, true>), grid, dim3(256), 0, s, a, k);
    else
      hipLaunchKernelGGL((k_shade_bwd<KT, float4, true, true>), grid, dim3(256), 0, s, a, k);
  } else {
    if (format == SOP_TEXEL_F16)
      hipLaunchKernelGGL((k_shade_bwd<KT, uint2, false, true>), grid, dim3(256), 0, s, a, k);
    else
      hipLaunchKernelGGL((k_shade_bwd<KT, float4, false, true>), grid, dim3(256), 0, s, a, k);
  }
}

bool shade_bwd_batched(int32_t res, int32_t k) { return res <= kMaxRes && k <= 16; }

hipError_t launch_shade_bwd(const ShadeArgs& a, int32_t k, int32_t format, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const bool det = a.det_tex != nullptr || a.det_env != nullptr;
  if (det && (!a.det_flag || (a.g_tex && !a.det_tex) || (a.g_env && !a.det_env)))
    return hipErrorInvalidValue;
  if (!shade_bwd_batched(a.R, k)) {
    if (!det) return dispatch(false, a, k, format, s);
    const dim3 grid((unsigned)((a.n + kWavesPerBlock - 1) / kWavesPerBlock));
    switch (k) {
      case 4: launch_bwd_det_kt<4>(a, k, format, grid, s); break;
      case 8: launch_bwd_det_kt<8>(a, k, format, grid, s); break;
      default: launch_bwd_det_kt<0>(a, k, format, grid, s); break;
    }
    return hipGetLastError();
  }
  switch (k) {
    case 4:
      det ? launch_batched_kt<4, true>(a, k, format, s) : launch_batched_kt<4, false>(a, k, format, s);
      break;
    case 8:
      det ? launch_batched_kt<8, true>(a, k, format, s) : launch_batched_kt<8, false>(a, k, format, s);
      break;
    default:
      det ? launch_batched_kt<0, true>(a, k, format, s) : launch_batched_kt<0, false>(a, k, format, s);
      break;
  }
  return hipGetLastError();
}

// The exact sum held in the four words of value i: T = sum_k w_k 2^(32k) (signed words),
// carried into four 32-bit limbs and a signed top, its magnitude converted through FP64
// (a fixed sequence of operations: the same words always give the same float) and scaled
// by 2^-96.
__global__ __launch_bounds__(256) void k_det_finish(const unsigned long long* __restrict__ w,
                                                    int64_t n, const int32_t* __restrict__ flag,
                                                    float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (*flag) {
    out[i] = __int_as_float(0x7FC00000);
    return;
  }
  long long c = 0;
  unsigned __int128 lo = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long t = (long long)w[(size_t)k * n + i] + c;     // |w_k| < 2^63 - 2^32
    lo |= (unsigned __int128)(uint32_t)t << (32 * k);
    c = t >> 32;                                                    // floor
  }
  const bool neg = c < 0;
  unsigned long long top = (unsigned long long)c;
  if (neg) {                                                        // magnitude of c 2^128 + lo
    top = (unsigned long long)(-(c + 1)) + (lo == 0 ? 1ull : 0ull);
    lo = ~lo + 1;
  }
  const double mag = ((double)top * 0x1p64 + (double)(unsigned long long)(lo >> 64)) * 0x1p64 +
                     (double)(unsigned long long)lo;
  const double v = (neg ? -mag : mag) * 0x1p-96;
  out[i] += (float)v;
}

hipError_t launch_det_finish(const unsigned long long* words, int64_t n, const int32_t* flag,
                             float* out, hipStream_t s) {
  if (n == 0 || !out) return hipSuccess;
  if (!words || !flag) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_det_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, words, n,
                     flag, out);
  return hipGetLastError();
}

// g_env += the environment adjoint held in blocks: one thread per block value; the block's
// texel (corner + (dx, dy)) is wrapped and clamped (equirectangular) or mirrored
// (octahedral) exactly as the lookups wrap their taps. Untouched (zero) values add nothing.
__global__ __launch_bounds__(256) void k_env_blk_finish(const float* __restrict__ blk,
                                                        int32_t bw, int32_t bh, int32_t H,
                                                        int32_t W, int32_t oct,
                                                        float* __restrict__ g_env) {
  const int64_t per_cls = (int64_t)bh * bw * 12;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= 4 * per_cls) return;
  const int cls = (int)(i / per_cls);
  const int64_t rem = i - cls * per_cls;
  const int64_t rec = rem / 12;
  const int v = (int)(rem - rec * 12), t = v / 3, c = v - 3 * t;
  const float x = blk[((int64_t)cls * bh * bw + rec) * kEnvBlkFloats + v];
  if (x == 0.0f) return;
  const int br = (int)(rec / bw), bc = (int)(rec - (int64_t)br * bw);
  int ti = 2 * bc + (cls & 1) + (t & 1) - 2, tj = 2 * br + (cls >> 1) + (t >> 1) - 2;
  if (oct) {
    int oi, oj;
    oct_wrap(ti, tj, W, oi, oj);
    ti = oi;
    tj = oj;
  } else {
    ti = ti < 0 ? ti + W : (ti >= W ? ti - W : ti);
    ti = min(max(ti, 0), W - 1);
    tj = min(max(tj, 0), H - 1);
  }
  unsafeAtomicAdd(g_env + ((int64_t)tj * W + ti) * 3 + c, x);
}

hipError_t launch_env_blk_finish(const float* blk, int32_t bw, int32_t bh, int32_t H,
                                 int32_t W, bool octahedral, float* g_env, hipStream_t s) {
  if (!g_env) return hipSuccess;
  if (!blk) return hipErrorInvalidValue;
  const int64_t n = 4 * (int64_t)bw * bh * 12;
  hipLaunchKernelGGL(k_env_blk_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, blk,
                     bw, bh, H, W, octahedral ? 1 : 0, g_env);
  return hipGetLastError();
}

// per-call tables: directions, and reference directions of the environment's texel
// columns (phi_i = 2 pi (i + 0.5)/W - pi, i in [-1, W]) and rows (theta_j = pi (j + 0.5)/H,
// j in [-1, H]), all in FP64
__global__ __launch_bounds__(256) void k_dir_table(int32_t S, uint32_t rho, double4* tab,
                                                   int32_t H, int32_t W, double2* col_ref,
                                                   double2* row_ref) {
  const int32_t j = blockIdx.x * 256 + threadIdx.x;
  if (j < S) tab[j] = dir_entry(j, S, rho);
  if (col_ref && j < W + 2) {
    double sn, cs;
    sincospi(2.0 * ((double)(j - 1) + 0.5) / (double)W - 1.0, &sn, &cs);
    col_ref[j] = make_double2(cs, sn);
  }
  if (row_ref && j < H + 2) {
    double sn, cs;
    sincospi(((double)(j - 1) + 0.5) / (double)H, &sn, &cs);
    row_ref[j] = make_double2(cs, sn);
  }
}

// 20-bit Morton code of two 10-bit coordinates
__device__ __forceinline__ uint32_t morton2(uint32_t x, uint32_t y) {
  auto spread = [](uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
  };
  return spread(x) | (spread(y) << 1);
}

// The S directions of the call (dir_entry) ordered by the Z curve of their position on the
// hemispherical octahedral square (u, v) = (x + y, x - y) / (|x| + |y| + z) at 10 bits per
// axis, ties by index: a bitonic sort of (code << 12 | j) in one workgroup (S <= 4096).
__global__ __launch_bounds__(1024) void k_dir_sort(int32_t S, uint32_t rho, double4* sorted,
                                                  int32_t cosine) {
  __shared__ uint32_t key[SOP_MAX_DIRS];
  int n = 1;
  while (n < S) n <<= 1;
  for (int i = threadIdx.x; i < n; i += 1024) {
    uint32_t kv = 0xFFFFFFFFu;
    if (i < S) {
      const double4 e = dir_entry(i, S, rho, cosine != 0);
      const double l1 = fabs(e.x) + fabs(e.y) + e.z;
      const double u = (e.x + e.y) / l1, v = (e.x - e.y) / l1;
      const uint32_t qu = (uint32_t)fmin(fmax((u + 1.0) * 512.0, 0.0), 1023.0);
      const uint32_t qv = (uint32_t)fmin(fmax((v + 1.0) * 512.0, 0.0), 1023.0);
      kv = (morton2(qu, qv) << 12) | (uint32_t)i;
    }
    key[i] = kv;
  }
  __syncthreads();
  for (int size = 2; size <= n; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < n / 2; t += 1024) {
        const int i = 2 * stride * (t / stride) + (t % stride), j = i + stride;
        const uint32_t x = key[i], y = key[j];
        if ((x > y) == ((i & size) == 0)) {
          key[i] = y;
          key[j] = x;
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < S; i += 1024)
    sorted[i] = dir_entry((int)(key[i] & 0xFFFu), S, rho, cosine != 0);
}

hipError_t launch_dir_sort(int32_t S, uint32_t seed, int32_t per_point, double4* sorted,
                           hipStream_t s, int32_t cosine) {
  if (S < 1 || S > SOP_MAX_DIRS || !sorted) return hipErrorInvalidValue;
  const uint32_t rho = per_point ? 0u : rotation24(seed, false, 0u);
  hipLaunchKernelGGL(k_dir_sort, dim3(1), dim3(1024), 0, s, S, rho, sorted, cosine);
  return hipGetLastError();
}

hipError_t launch_dir_table(int32_t S, uint32_t seed, int32_t per_point, int32_t H, int32_t W,
                            double4* tab, double2* col_ref, double2* row_ref, hipStream_t s) {
  const uint32_t rho = per_point ? 0u : rotation24(seed, false, 0u);
  // the environment tables are optional (NULL: not formed)
  const int32_t n = max(S, max(col_ref ? W + 2 : 0, row_ref ? H + 2 : 0));
  hipLaunchKernelGGL(k_dir_table, dim3((n + 255) / 256), dim3(256), 0, s, S, rho, tab, H, W,
                     col_ref, row_ref);
  return hipGetLastError();
}

hipError_t launch_query(const ShadeArgs& a, int32_t k, int32_t format, const float* dirs,
                        int32_t D, float* Lin, float* O, hipStream_t s) {
  const int64_t total = a.n * (int64_t)D;
  if (total == 0) return hipSuccess;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (format == SOP_TEXEL_F16)
    hipLaunchKernelGGL(k_query<uint2>, grid, dim3(256), 0, s, a, k, dirs, D, Lin, O);
  else
    hipLaunchKernelGGL(k_query<float4>, grid, dim3(256), 0, s, a, k, dirs, D, Lin, O);
  return hipGetLastError();
}

}  // namespace sopk
