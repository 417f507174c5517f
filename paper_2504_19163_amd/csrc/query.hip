// Stage 3 on the GPU: bound-driven sampling of triangle tuples and Newton
// root-finding per shading point (Sec. 5.3-5.4, Alg. 1; Sec. 6.1 root-finding).
//
// Fused form (k_query_fused): one wave per shading point.  The wave reads the
// candidate list U of the point's grid cell (one entry per lane, chunks of
// 64), solves gamma of P_T = min(gamma E~_T, 1) by water-filling with wave
// reductions, draws each tuple's Bernoulli decision from Philox keyed by
// (seed, point index, tuple), runs Newton for the selected tuples lane-
// parallel (FP32 iterations, FP64 polish of every root) and reduces
// sum E(T) / P_T in a fixed lane order.
//
// Staged form: the same stages as separate launches with their intermediate
// results in HBM: gamma per point, selection count + scan + compaction into
// (point, tuple, P) pairs, Newton per pair, accumulation per point.
#include <atomic>
#include <utility>

#include "internal.hpp"
#include "path_dev.hpp"

namespace bbc {

struct QueryArgs {
  DevScene sc;
  int G;
  const float* rec;
  const float4* root;
  const uint32_t* toff;
  const uint32_t* lcode;
  const float4* luk;
  const float4* lgu;  // union of the bounds of each run of kLeafGroup leaves
  const uint32_t* coff;
  const uint32_t* gt;
  const float* ge;
  const float* pts;  // [3][pstride]: row r of point i at pts[r * pstride + i]
  int64_t n;
  int64_t pstride;
  float W;
  uint64_t seed;
  int64_t base;
  int mode;
  float* out;
  float* stats;
  unsigned long long* counters;  // nullable: pairs, starts, FP32 iterations, FP64 steps, roots
  // several requests in one launch (serving): point i belongs to request
  // preq[i]; nullable, then every point uses W, seed and base above
  const uint16_t* preq;
  const ReqDesc* reqs;
  int64_t ioff;  // index of point 0 of this launch inside the batch (a slice of a larger batch)
  // two reflections: the grid holds indices of constructed pairs; the random
  // stream is keyed by the pair number tid[T]
  const uint32_t* tid;
  int rec_floats;
};

__device__ __forceinline__ uint32_t tuple_key(const QueryArgs& a, uint32_t T) { return a.tid ? a.tid[T] : T; }

// A shading point's candidate list U (Sec. 6.1 bound storage): its cell's
// slice of the grid entries, then the cover-all slice (slice G^2).  Entry j of
// U is grid entry at(j).
struct CandList {
  uint32_t b0, n0, b1, n;
  __device__ __forceinline__ uint32_t at(uint32_t j) const { return j < n0 ? b0 + j : b1 + (j - n0); }
};
__device__ __forceinline__ CandList cand_list(const QueryArgs& a, uint32_t cell) {
  const uint32_t G2 = uint32_t(a.G) * uint32_t(a.G);
  CandList c;
  c.b0 = a.coff[cell];
  c.n0 = a.coff[cell + 1] - c.b0;
  c.b1 = a.coff[G2];
  c.n = c.n0 + (a.coff[G2 + 1] - c.b1);
  return c;
}

struct PointReq {
  float W;
  uint64_t seed, key;
};

// Sampling parameters of point i: expected sample count, seed, and the point's
// index inside its own request (the Philox counter), so a point draws the same
// numbers whether its request runs alone or batched with others.
__device__ __forceinline__ PointReq point_req(const QueryArgs& a, int64_t i) {
  if (!a.preq) return PointReq{a.W, a.seed, uint64_t(a.base + i)};
  const ReqDesc& r = a.reqs[a.preq[i]];
  return PointReq{r.W, r.seed, uint64_t(r.base + (i + a.ioff - r.start))};
}

// Per-lane work counters, summed per wave into the optional device counters.
struct WorkCount {
  uint32_t pairs = 0, starts = 0, it32 = 0, it64 = 0, roots = 0;
};

__device__ __forceinline__ void flush_counts(const QueryArgs& a, WorkCount w) {
  if (!a.counters) return;
  const unsigned long long v[5] = {wave_sum(w.pairs), wave_sum(w.starts), wave_sum(w.it32), wave_sum(w.it64),
                                   wave_sum(w.roots)};
  if ((threadIdx.x % BBC_WAVE) == 0)
    for (int k = 0; k < 5; ++k)
      if (v[k]) atomicAdd(&a.counters[k], v[k]);
}

struct Target {
  bool on;
  float u, v;
  double ud, vd;
  uint32_t cell;
  int64_t pt;  // shading point index (its sampling parameters and light points)
};

// Receiver texture coordinates of a shading point (least squares on the
// receiver parallelogram) and its grid cell (Sec. 6.1 bound storage).
__device__ __forceinline__ Target receiver_target(const QueryArgs& a, int64_t i) {
  Target t;
  const double x = a.pts[i], y = a.pts[a.pstride + i], z = a.pts[2 * a.pstride + i];
  const double rx = x - a.sc.q0[0], ry = y - a.sc.q0[1], rz = z - a.sc.q0[2];
  const double f1x = a.sc.f1[0], f1y = a.sc.f1[1], f1z = a.sc.f1[2];
  const double f2x = a.sc.f2[0], f2y = a.sc.f2[1], f2z = a.sc.f2[2];
  const double A = f1x * f1x + f1y * f1y + f1z * f1z, B = f1x * f2x + f1y * f2y + f1z * f2z;
  const double D = f2x * f2x + f2y * f2y + f2z * f2z;
  const double r1 = f1x * rx + f1y * ry + f1z * rz, r2 = f2x * rx + f2y * ry + f2z * rz;
  const double det = A * D - B * B;
  t.ud = (D * r1 - B * r2) / det;
  t.vd = (A * r2 - B * r1) / det;
  t.u = float(t.ud);
  t.v = float(t.vd);
  t.on = t.ud >= 0.0 && t.ud <= 1.0 && t.vd >= 0.0 && t.vd <= 1.0;
  const int cu = min(a.G - 1, max(0, int(floor(t.ud * a.G))));
  const int cv = min(a.G - 1, max(0, int(floor(t.vd * a.G))));
  t.cell = uint32_t(cu) * uint32_t(a.G) + uint32_t(cv);
  t.pt = i;
  return t;
}

// Water-filling solve of gamma (Sec. 5.4): W' = min(W, |U|); unbounded entries
// take P = 1, the finite positive entries share W_f = min(max(W' - n_inf, 1),
// n_fin) expected samples with P = min(gamma E~, 1).  Iterates the saturated
// set {gamma E~ >= 1}, which only grows, until it is stable.  Returns +inf when
// every finite entry is taken with P = 1.  One thread per shading point.
__device__ float solve_gamma(const float* ge, const CandList& cl, float W) {
  const uint32_t nU = cl.n;
  uint32_t n_inf = 0, n_fin = 0;
  float S = 0.f;
  // the loops over U are unrolled so that a thread's reads go out several at
  // a time (the sums keep list order)
#pragma unroll 8
  for (uint32_t j = 0; j < nU; ++j) {
    const float e = ge[cl.at(j)];
    n_inf += isinf(e) ? 1u : 0u;
    if (isfinite(e) && e > 0.f) {
      ++n_fin;
      S += e;
    }
  }
  const float Wp = fminf(W, float(nU));
  const float Wf = fminf(fmaxf(Wp - float(n_inf), 1.f), float(n_fin));
  if (n_fin == 0 || Wf >= float(n_fin)) return INFINITY;
  float gamma = Wf / S;
  uint32_t k = 0;
  for (uint32_t iter = 0; iter <= n_fin; ++iter) {
    uint32_t kn = 0;
    float Sn = 0.f;
#pragma unroll 8
    for (uint32_t j = 0; j < nU; ++j) {
      const float e = ge[cl.at(j)];
      if (isfinite(e) && e > 0.f) {
        if (gamma * e >= 1.f)
          ++kn;
        else
          Sn += e;
      }
    }
    if (kn == k || !(Sn > 0.f)) break;
    k = kn;
    gamma = (Wf - float(k)) / Sn;
  }
  return gamma;
}

// The same solve for a long list with the 64 lanes of a wave: lane l takes
// entries l, l + 64, ... of U and the counts and sums are combined by a
// butterfly (every lane ends with the same value, and the order of the FP32
// additions depends only on the list), so every lane returns the same gamma,
// whichever kernel or batch the point is in.  Lists longer than
// kLongList take this path in every query form.
constexpr uint32_t kLongList = 96;
__device__ float solve_gamma_wave(const float* ge, const CandList& cl, float W, int lane) {
  const uint32_t nU = cl.n;
  uint32_t n_inf = 0, n_fin = 0;
  float S = 0.f;
#pragma unroll 4
  for (uint32_t j = uint32_t(lane); j < nU; j += BBC_WAVE) {
    const float e = ge[cl.at(j)];
    n_inf += isinf(e) ? 1u : 0u;
    if (isfinite(e) && e > 0.f) {
      ++n_fin;
      S += e;
    }
  }
  n_inf = wave_sum(n_inf);
  n_fin = wave_sum(n_fin);
  S = wave_sum(S);
  const float Wp = fminf(W, float(nU));
  const float Wf = fminf(fmaxf(Wp - float(n_inf), 1.f), float(n_fin));
  if (n_fin == 0 || Wf >= float(n_fin)) return INFINITY;
  float gamma = Wf / S;
  uint32_t k = 0;
  for (uint32_t iter = 0; iter <= n_fin; ++iter) {
    uint32_t kn = 0;
    float Sn = 0.f;
#pragma unroll 4
    for (uint32_t j = uint32_t(lane); j < nU; j += BBC_WAVE) {
      const float e = ge[cl.at(j)];
      if (isfinite(e) && e > 0.f) {
        if (gamma * e >= 1.f)
          ++kn;
        else
          Sn += e;
      }
    }
    kn = wave_sum(kn);
    Sn = wave_sum(Sn);
    if (kn == k || !(Sn > 0.f)) break;
    k = kn;
    gamma = (Wf - float(k)) / Sn;
  }
  return gamma;
}

__device__ __forceinline__ float select_prob(float e, float gamma, bool exhaustive) {
  if (exhaustive) return 1.f;
  if (isinf(e)) return 1.f;
  if (!(e > 0.f)) return 0.f;
  return fminf(gamma * e, 1.f);
}

// One Newton start: the centre of a leaf of T whose position bound holds the
// target, and the box it may not leave (the leaf widened by one width on each
// side).  FP32 state carried between passes of the pooled form.
struct Start32 {
  float u, v, lu0, lu1, lv0, lv1, prev, t_last;
  int it;
};

__device__ __forceinline__ Start32 start_of(uint32_t code, float rx, float ry, float rz, float rw) {
  const int depth = int(code >> 28);
  const uint32_t iu = (code >> kCodeBits) & ((1u << kCodeBits) - 1), iv = code & ((1u << kCodeBits) - 1);
  const float sc = ldexpf(1.f, -depth);
  const float fu = (ry - rx) * sc, fv = (rw - rz) * sc;
  const float u0 = rx + float(iu) * fu, v0 = rz + float(iv) * fv;
  Start32 st;
  st.u = u0 + 0.5f * fu;
  st.v = v0 + 0.5f * fv;
  st.lu0 = u0 - fu;
  st.lu1 = u0 + 2.f * fu;
  st.lv0 = v0 - fv;
  st.lv1 = v0 + 2.f * fv;
  st.prev = INFINITY;
  st.t_last = -1.f;
  st.it = 0;
  return st;
}

// At most `steps` more FP32 Newton iterations of a start (20 in all).  The
// iteration stops when the step falls below 1e-5 or stagnates at FP32 noise
// level (below 1e-3 and no longer halving): for small triangles the FP32
// residual cannot resolve the root further, and the FP64 polish that follows
// runs to a receiver residual below 1e-9.  Returns 0 while the start is still
// running, 1 when it failed (singular Jacobian or the iterate left its box),
// 2 when it ended (converged or out of iterations).
template <int CH>
__device__ __forceinline__ int newton32(const TupleGeom<float>& Gf, float tu, float tv, Start32& st, int steps,
                                        WorkCount& wc) {
  for (int r = 0; r < steps; ++r) {
    if (st.it >= 20) return 2;
    ++st.it;
    ++wc.it32;  // FP32 path evaluations
    const PathT<float> p = eval_path<float>(Gf, CH, st.u, st.v);
    const float ru_ = p.uk - tu, rv_ = p.vk - tv;
    if (!(isfinite(p.det)) || p.det == 0.f) return 1;
    const float idet = recip(p.det);
    const float du = (p.J11 * ru_ - p.J01 * rv_) * idet;
    const float dv = (-p.J10 * ru_ + p.J00 * rv_) * idet;
    st.u -= du;
    st.v -= dv;
    st.t_last = p.t;
    if (!(st.u >= st.lu0 && st.u <= st.lu1 && st.v >= st.lv0 && st.v <= st.lv1)) return 1;
    const float step = fabsf(du) + fabsf(dv);
    if (step < 1e-5f || (step < 1e-3f && step > 0.5f * st.prev)) return 2;
    st.prev = step;
  }
  return st.it >= 20 ? 2 : 0;
}

// A start whose FP32 root lies clearly outside the triangle or behind the
// receiver cannot become admissible in the polish (margin 1e-3 >> FP32 error).
__device__ __forceinline__ bool worth_polish(const Start32& st) {
  return st.u >= -1e-3f && st.v >= -1e-3f && st.u + st.v <= 1.f + 1e-3f && st.t_last > 0.f;
}

// FP64 polish of an FP32 root (up to ten steps next to a fold, where
// convergence is only linear); the root is accepted when its FP64 residual on
// the receiver is below 1e-6 scene units and the path is admissible.  On
// acceptance writes the root and its irradiance.
template <int CH>
__device__ __forceinline__ bool polish64(const TupleGeom<double>& Gd, double tud, double tvd, float u, float v,
                                         double& ud, double& vd, double& E, WorkCount& wc) {
  ud = u;
  vd = v;
  ++wc.it64;  // FP64 path evaluations
  PathT<double> p = eval_path<double>(Gd, CH, ud, vd);
  double res = INFINITY;
  for (int it = 0; it < 10; ++it) {
    ++wc.it64;
    const double ru_ = p.uk - tud, rv_ = p.vk - tvd;
    if (!(p.det != 0.0) || !isfinite(p.det)) break;
    ud -= (p.J11 * ru_ - p.J01 * rv_) / p.det;
    vd -= (-p.J10 * ru_ + p.J00 * rv_) / p.det;
    p = eval_path<double>(Gd, CH, ud, vd);
    res = residual<double>(Gd, p, tud, tvd);
    if (res < 1e-9) break;
  }
  if (!(res < 1e-6) || !admissible<double>(Gd, CH, p, ud, vd)) return false;
  E = path_irradiance<double>(Gd, p);
  return true;
}

// The polish as a called function, for the two-reflection pooled kernel: its
// FP64 dual-number path evaluation otherwise sets that kernel's register
// count (256 VGPRs and 88 AGPRs inlined, one wave per SIMD); called, the
// kernel fits two waves per SIMD (FP32 kernels lose more to the call than
// they gain, and keep it inlined).
template <int CH>
__device__ __noinline__ bool polish64_called(const TupleGeom<double>& Gd, double tud, double tvd, float u, float v,
                                             double& ud, double& vd, double& E, WorkCount& wc) {
  return polish64<CH>(Gd, tud, tvd, u, v, ud, vd, E, wc);
}

// Roots of one tuple taken in start order: a root within 1e-7 (in u1) of one
// of the first four accepted roots is the same root found again.
struct RootSum {
  double ru0 = 0, rv0 = 0, ru1 = 0, rv1 = 0, ru2 = 0, rv2 = 0, ru3 = 0, rv3 = 0;
  int nr = 0;
  double ET = 0.0;

  __device__ __forceinline__ void add(double ud, double vd, double E, WorkCount& wc) {
    bool dup = false;
    if (nr > 0) dup = dup || (fabs(ru0 - ud) <= 1e-7 && fabs(rv0 - vd) <= 1e-7);
    if (nr > 1) dup = dup || (fabs(ru1 - ud) <= 1e-7 && fabs(rv1 - vd) <= 1e-7);
    if (nr > 2) dup = dup || (fabs(ru2 - ud) <= 1e-7 && fabs(rv2 - vd) <= 1e-7);
    if (nr > 3) dup = dup || (fabs(ru3 - ud) <= 1e-7 && fabs(rv3 - vd) <= 1e-7);
    if (dup) return;
    if (nr == 0) { ru0 = ud; rv0 = vd; }
    else if (nr == 1) { ru1 = ud; rv1 = vd; }
    else if (nr == 2) { ru2 = ud; rv2 = vd; }
    else if (nr == 3) { ru3 = ud; rv3 = vd; }
    ++nr;
    ET += E;
    ++wc.roots;
  }
};

// Sum of the irradiance of every admissible path of tuple T that Newton finds
// from the centres of T's leaves whose position bound contains the target
// (deterministic initialisation, Sec. 6.1): FP32 iterations that abandon a
// start leaving its box by more than one width, then the FP64 polish.  One
// thread does all of T's starts.
// The light point of a selected pair: for an area light x0 + z1 a + z2 b
// with (z1, z2) from Philox streams 3 and 4 of (seed, point, tuple), written
// over x0 in the pair's copy of the tuple record.  Area lights come with the
// single reflection only, whose tuple is emitter * n_tri + triangle.
// The light point of a selected pair of an area-light scene (Philox streams 3
// and 4 of (seed, point, tuple)): the FP64 point goes to the polish and the
// irradiance, its FP32 rounding into the pair's record copy for the FP32
// iterations.
__device__ __forceinline__ V3<double> pair_light_point(const QueryArgs& a, float* rec, int64_t i, uint32_t T) {
  const PointReq pr = point_req(a, i);
  const uint32_t tk = tuple_key(a, T);
  const double z1 = sample_stream(pr.seed, pr.key, tk, 3u), z2 = sample_stream(pr.seed, pr.key, tk, 4u);
  const int64_t e = int64_t(T) / a.sc.n_tri, ne = a.sc.n_emit;
  double x[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    x[c] = double(rec[18 + c]) + z1 * double(a.sc.eedge[c * ne + e]) + z2 * double(a.sc.eedge[(3 + c) * ne + e]);
    rec[18 + c] = float(x[c]);
  }
  return mk(x[0], x[1], x[2]);
}

template <int CH>
__device__ double tuple_irradiance(const QueryArgs& a, uint32_t T, const Target& tg, WorkCount& wc) {
  constexpr bool RR = CH == BBC_CHAIN_RR;
  constexpr int NF = RR ? kRecFloatsRR : kRecFloats, NL = RR ? 12 : 7;
  float rec[NF];
  const float4* r4 = reinterpret_cast<const float4*>(a.rec + size_t(T) * NF);
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const float4 q = r4[k];
    rec[4 * k] = q.x;
    rec[4 * k + 1] = q.y;
    rec[4 * k + 2] = q.z;
    rec[4 * k + 3] = q.w;
  }
  const uint32_t lb = __float_as_uint(rec[22]), le = __float_as_uint(rec[23]);
  if (lb == le) return 0.0;
  V3<double> xl = mk(0.0, 0.0, 0.0);
  if constexpr (!RR)
    if (a.sc.eedge) xl = pair_light_point(a, rec, tg.pt, T);
  const TupleGeom<float> Gf = tuple_geom_rec<float, RR>(rec, a.sc);
  RootSum rs;
  for (uint32_t k = lb; k < le; ++k) {
    const float4 uk = a.luk[k];
    if (!(tg.ud >= uk.x && tg.ud <= uk.y && tg.vd >= uk.z && tg.vd <= uk.w)) continue;
    Start32 st = start_of(a.lcode[k], rec[24], rec[25], rec[26], rec[27]);
    ++wc.starts;
    if (newton32<CH>(Gf, tg.u, tg.v, st, 20, wc) != 2 || !worth_polish(st)) continue;
    TupleGeom<double> Gd = tuple_geom_rec<double, RR>(rec, a.sc);
    if (!RR && a.sc.eedge) Gd.x0 = xl;
    double ud, vd, E;
    if (polish64<CH>(Gd, tg.ud, tg.vd, st.u, st.v, ud, vd, E, wc)) rs.add(ud, vd, E, wc);
  }
  return rs.ET;
}

// Inclusive prefix maximum over the 64 lanes: shifts within each row of 16
// lanes, then the last lane of row 0 (row 2) into rows 1 and 3 and the last
// lane of row 1 into rows 2 and 3 (DPP row_bcast); lanes without a source get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
  v = max(v, dpp_u32<0x111, 0xF>(v));  // row_shr:1
  v = max(v, dpp_u32<0x112, 0xF>(v));  // row_shr:2
  v = max(v, dpp_u32<0x114, 0xF>(v));  // row_shr:4
  v = max(v, dpp_u32<0x118, 0xF>(v));  // row_shr:8
  v = max(v, dpp_u32<0x142, 0xA>(v));  // row_bcast:15
  v = max(v, dpp_u32<0x143, 0xC>(v));  // row_bcast:31
  return v;
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, int lane) {
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < BBC_WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, BBC_WAVE);
    if (lane >= d) inc += o;
  }
  return inc - v;
}

// Fused form: one wave owns a tile of 64 consecutive shading points.  Lane =
// point for the gather, the gamma solve and the Bernoulli draws; the selected
// (point, tuple) pairs are compacted in LDS in point-then-entry order, Newton
// runs lane = pair, and each lane sums its own pairs' contributions in entry
// order, so the estimate is bit-identical to the staged form.
constexpr int kPairCap = 512;

template <int kWaves, int kTile, int CH>
__global__ void __launch_bounds__(64, kWaves) k_query_fused(QueryArgs a) {
  __shared__ uint32_t s_t[kPairCap];
  __shared__ float s_p[kPairCap];
  __shared__ uint8_t s_pt[kPairCap];
  __shared__ uint8_t s_nr[kPairCap];
  __shared__ double s_c[kPairCap];
  __shared__ double s_ud[kTile], s_vd[kTile];
  const int lane = threadIdx.x;
  const bool exhaustive = (a.mode & BBC_QUERY_EXHAUSTIVE) != 0;
  const int64_t n_tiles = (a.n + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t i = tile * kTile + lane;
    const bool valid = lane < kTile && i < a.n;
    Target tg{};
    CandList cl{0u, 0u, 0u, 0u};
    if (valid) {
      tg = receiver_target(a, i);
      if (tg.on) cl = cand_list(a, tg.cell);
    }
    const uint32_t nU = cl.n;
    if (lane < kTile) {
      s_ud[lane] = tg.ud;
      s_vd[lane] = tg.vd;
    }
    const PointReq pr = valid ? point_req(a, i) : PointReq{1.f, 0, 0};
    float gamma = (exhaustive || nU == 0 || nU > kLongList) ? INFINITY : solve_gamma(a.ge, cl, pr.W);
    if (!exhaustive) {  // long lists: the whole wave solves each in turn
      uint64_t longs = __ballot(nU > kLongList);
      while (longs) {
        const int q = __ffsll((unsigned long long)longs) - 1;
        longs &= longs - 1;
        const CandList cq{uint32_t(__shfl(int(cl.b0), q, BBC_WAVE)), uint32_t(__shfl(int(cl.n0), q, BBC_WAVE)),
                          uint32_t(__shfl(int(cl.b1), q, BBC_WAVE)), uint32_t(__shfl(int(cl.n), q, BBC_WAVE))};
        const float g = solve_gamma_wave(a.ge, cq, __shfl(pr.W, q, BBC_WAVE), lane);
        if (lane == q) gamma = g;
      }
    }
    const uint64_t key = pr.key;
    uint32_t cnt = 0;
    double mu2 = 0.0;
    for (uint32_t j = 0; j < nU; ++j) {
      const float e = a.ge[cl.at(j)];
      const float P = select_prob(e, gamma, exhaustive);
      if (P > 0.f && isfinite(e)) mu2 += double(e) * double(e) / double(P);
      cnt += selection_uniform(pr.seed, key, tuple_key(a, a.gt[cl.at(j)])) < P ? 1u : 0u;
    }
    const uint32_t off = wave_excl_scan(cnt, lane);
    const uint32_t total = __shfl(off + cnt, BBC_WAVE - 1, BBC_WAVE);
    double E = 0.0;
    uint32_t roots = 0, emitted = 0, cur = 0;
    WorkCount wc;
    for (uint32_t w0 = 0; w0 < total; w0 += kPairCap) {
      // this lane's pairs whose global index falls in [w0, w0 + cap)
      while (emitted < cnt && off + emitted < w0 + kPairCap) {
        const float e = a.ge[cl.at(cur)];
        const uint32_t T = a.gt[cl.at(cur)];
        const float P = select_prob(e, gamma, exhaustive);
        if (selection_uniform(pr.seed, key, tuple_key(a, T)) < P) {
          const uint32_t slot = off + emitted - w0;
          s_t[slot] = T;
          s_p[slot] = P;
          s_pt[slot] = uint8_t(lane);
          ++emitted;
        }
        ++cur;
      }
      __syncthreads();
      const uint32_t nslots = min(uint32_t(kPairCap), total - w0);
      for (uint32_t k = lane; k < nslots; k += BBC_WAVE) {
        const int pt = s_pt[k];
        Target t2;
        t2.on = true;
        t2.ud = s_ud[pt];
        t2.vd = s_vd[pt];
        t2.u = float(t2.ud);
        t2.v = float(t2.vd);
        t2.pt = tile * kTile + pt;
        const uint32_t r0 = wc.roots;
        ++wc.pairs;
        s_c[k] = tuple_irradiance<CH>(a, s_t[k], t2, wc) / double(s_p[k]);
        s_nr[k] = uint8_t(min(wc.roots - r0, 255u));
      }
      __syncthreads();
      const uint32_t lo = max(off, w0), hi = min(off + cnt, w0 + kPairCap);
      for (uint32_t k = lo; k < hi; ++k) {
        E += s_c[k - w0];
        roots += s_nr[k - w0];
      }
      __syncthreads();
    }
    flush_counts(a, wc);
    if (valid) {
      a.out[i] = float(E);
      if (a.stats) {
        a.stats[4 * i + 0] = float(nU);
        a.stats[4 * i + 1] = float(cnt);
        a.stats[4 * i + 2] = float(roots);
        a.stats[4 * i + 3] = float(mu2);
      }
    }
  }
}

static QueryArgs make_args(const Bounds* b, const float* pts, int64_t n, int32_t spp, uint64_t seed, int64_t base,
                           int32_t mode, float* out, float* stats, unsigned long long* counters) {
  QueryArgs a{};
  a.counters = counters;
  a.sc = b->scene;
  a.G = b->params.grid_res;
  a.rec = static_cast<const float*>(b->trec.p);
  a.root = static_cast<const float4*>(b->root.p);
  a.toff = static_cast<const uint32_t*>(b->toff.p);
  a.lcode = static_cast<const uint32_t*>(b->sc.p);
  a.luk = static_cast<const float4*>(b->su.p);
  a.lgu = static_cast<const float4*>(b->sug.p);
  a.coff = static_cast<const uint32_t*>(b->coff.p);
  a.gt = static_cast<const uint32_t*>(b->gt.p);
  a.ge = static_cast<const float*>(b->ge.p);
  a.tid = b->scene.chain == BBC_CHAIN_RR ? b->scene.tid : nullptr;
  a.rec_floats = b->rec_floats;
  a.pts = pts;
  a.n = n;
  a.pstride = n;
  a.W = float(spp);
  a.seed = seed;
  a.base = base;
  a.mode = mode;
  a.out = out;
  a.stats = stats;
  return a;
}

bbc_status launch_query(const Bounds* b, const float* pts, int64_t n, int32_t spp, uint64_t seed, int64_t base,
                        int32_t mode, float* out, float* stats, unsigned long long* counters, hipStream_t s) {
  if (n == 0) return BBC_OK;
  const QueryArgs a = make_args(b, pts, n, spp, seed, base, mode, out, stats, counters);
  const int tp = b->tune.query_tile;
  const int64_t tiles = (n + tp - 1) / tp;
  const unsigned grid = unsigned(std::min<int64_t>(tiles, int64_t(b->tune.query_grid)));
  const bool w4 = b->tune.query_waves >= 4;
  Bounds* mb = const_cast<Bounds*>(b);
  if (b->tune.timing) {
    mb->tev_used = 0;
    BBC_HIP(hipEventRecord(mb->tev[0], s));
  }
#define BBC_FUSED(W, TP)                                                                           \
  do {                                                                                             \
    if (a.sc.chain == BBC_CHAIN_RR)                                                                \
      hipLaunchKernelGGL((k_query_fused<W, TP, BBC_CHAIN_RR>), dim3(grid), dim3(64), 0, s, a);      \
    else if (a.sc.chain == BBC_CHAIN_T)                                                            \
      hipLaunchKernelGGL((k_query_fused<W, TP, BBC_CHAIN_T>), dim3(grid), dim3(64), 0, s, a);       \
    else                                                                                           \
      hipLaunchKernelGGL((k_query_fused<W, TP, BBC_CHAIN_R>), dim3(grid), dim3(64), 0, s, a);       \
  } while (0)
  if (tp == 16) {
    if (w4) BBC_FUSED(4, 16); else BBC_FUSED(2, 16);
  } else if (tp == 32) {
    if (w4) BBC_FUSED(4, 32); else BBC_FUSED(2, 32);
  } else {
    if (w4) BBC_FUSED(4, 64); else BBC_FUSED(2, 64);
  }
#undef BBC_FUSED
  if (b->tune.timing) {
    BBC_HIP(hipEventRecord(mb->tev[1], s));
    mb->tev_used = 1;
  }
  BBC_HIP(hipGetLastError());
  return BBC_OK;
}

// ---------------------------------------------------------------- staged form
struct StagedArgs {
  QueryArgs q;
  uint32_t* cell_b;   // [n] the point's grid cell (0 off the receiver, where |U| = 0)
  uint32_t* cnt;      // [n] |U|
  float* gamma;       // [n]
  uint32_t* off;      // [n + 1] exclusive scan of the selection counts
  double2* tgt;       // [n] receiver coordinates of the point
  uint32_t* redo;     // [kRedoCap] pairs the pooled Newton kernel could not finish
  uint32_t* pair_pt;  // [pairs]
  uint32_t* pair_t;
  float* pair_p;
  double* pair_c;
  uint8_t* pair_nr;   // [pairs] roots found per pair (written when stats are requested)
  uint32_t pair_cap;
  // the count pass's decisions, one bit per candidate, 16 per word, bit_stride
  // words per point; held in pair_c's space, which is free until Newton
  uint16_t* bits;
  uint32_t bit_stride;
};

__global__ void k_stage_gamma(StagedArgs s) {
  const QueryArgs& a = s.q;
  const bool exhaustive = (a.mode & BBC_QUERY_EXHAUSTIVE) != 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) s.off[a.n + 1] = 0u;  // redo count of the pooled Newton kernel
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * blockDim.x) {
    const Target tg = receiver_target(a, i);
    uint32_t nU = 0;
    float gamma = INFINITY;
    if (tg.on) {
      const CandList cl = cand_list(a, tg.cell);
      nU = cl.n;
      if (!exhaustive && nU > 0 && nU <= kLongList) gamma = solve_gamma(a.ge, cl, point_req(a, i).W);
    }
    s.cell_b[i] = tg.on ? tg.cell : 0u;
    s.gamma[i] = gamma;
    s.cnt[i] = nU;
    s.tgt[i] = make_double2(tg.ud, tg.vd);
  }
}

// Gamma of the points whose candidate lists are longer than kLongList: one
// wave per point (k_stage_gamma left them at +inf), after k_stage_gamma.
__global__ void __launch_bounds__(256) k_stage_gamma_long(StagedArgs s) {
  const QueryArgs& a = s.q;
  if (a.mode & BBC_QUERY_EXHAUSTIVE) return;
  const int lane = int(threadIdx.x % BBC_WAVE);
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x / BBC_WAVE);
  for (int64_t i = int64_t(blockIdx.x) * (blockDim.x / BBC_WAVE) + threadIdx.x / BBC_WAVE; i < a.n; i += waves) {
    const uint32_t nU = s.cnt[i];
    if (nU <= kLongList) continue;
    const float g = solve_gamma_wave(a.ge, cand_list(a, s.cell_b[i]), point_req(a, i).W, lane);
    if (lane == 0) s.gamma[i] = g;
  }
}

// The selections of shading point i in list order, one chunk of 64
// candidates at a time: chunk(take, T, P) runs on every lane of the wave for
// each chunk, lane l holding candidate j0 + l (take: selected; P: the
// probability its contribution is divided by).
//  * bound-optimal (Alg. 1) and uniform P = W'/|U|: independent decisions;
//  * one-sample (Sec. 5.2), W draws with P1 = E~ / sum E~: the running sum of
//    the finite bounds is formed in list order by every lane in lockstep
//    (FP32, the same order as a sequential loop), each candidate counts the
//    draws that fall in its interval, and a candidate drawn c times enters
//    once with P = W P1 / c; unbounded candidates enter with P = 1;
//  * bins (Sec. 5.3): the bound-optimal P packed next-fit in list order into
//    bins of total at most 1, one draw per bin; all lanes walk the packing in
//    lockstep and the candidate whose interval holds its bin's draw is taken.
//    A bin accepts a candidate while its running sum stays within 2^-20 of 1
//    (probabilities that sum to 1 exactly reach it only up to rounding); the
//    part of an interval above 1 is cut and the weight is the interval's
//    length, the candidate's selection probability.
constexpr float kBinSlack = 1.0f / 1048576.0f;
template <class F>
__device__ void point_selection(const QueryArgs& a, const StagedArgs& s, int64_t i, int lane, F&& chunk) {
  const uint32_t nU = s.cnt[i];
  const CandList cl = cand_list(a, s.cell_b[i]);
  const float gamma = s.gamma[i];
  const PointReq pr = point_req(a, i);
  const int sampler = a.mode & BBC_QUERY_SAMPLERS;
  const bool exhaustive = (a.mode & BBC_QUERY_EXHAUSTIVE) != 0;
  if (sampler == BBC_QUERY_ONE_SAMPLE) {
    float S = 0.f;
    int64_t last = -1;
    for (uint32_t j0 = 0; j0 < nU; j0 += BBC_WAVE) {
      const uint32_t j = j0 + lane;
      const float e = j < nU ? a.ge[cl.at(j)] : 0.f;
      const float ef = (isfinite(e) && e > 0.f) ? e : 0.f;
      const uint32_t cnt = min(uint32_t(BBC_WAVE), nU - j0);
      for (uint32_t q = 0; q < cnt; ++q) {
        const float eq = __shfl(ef, int(q), BBC_WAVE);
        if (eq > 0.f) {
          S = S + eq;
          last = int64_t(j0 + q);
        }
      }
    }
    const int W = int(pr.W);
    float C = 0.f;
    for (uint32_t j0 = 0; j0 < nU; j0 += BBC_WAVE) {
      const uint32_t j = j0 + lane;
      const float e = j < nU ? a.ge[cl.at(j)] : 0.f;
      const uint32_t T = j < nU ? a.gt[cl.at(j)] : 0u;
      const float ef = (isfinite(e) && e > 0.f) ? e : 0.f;
      const uint32_t cnt = min(uint32_t(BBC_WAVE), nU - j0);
      float lo = 0.f, hi = 0.f;
      for (uint32_t q = 0; q < cnt; ++q) {
        const float eq = __shfl(ef, int(q), BBC_WAVE);
        if (lane == int(q)) lo = C;
        if (eq > 0.f) C = C + eq;
        if (lane == int(q)) hi = C;
      }
      if (int64_t(j) == last) hi = INFINITY;  // a draw that rounds up to the total
      uint32_t c = 0;
      if (S > 0.f) {
        for (int d0 = 0; d0 < W; d0 += BBC_WAVE) {
          const float t = d0 + lane < W ? sample_stream(pr.seed, pr.key, uint32_t(d0 + lane), 1u) * S : -1.f;
          for (int q = 0; q < BBC_WAVE; ++q) {
            const float tq = __shfl(t, q, BBC_WAVE);
            c += (ef > 0.f && tq >= lo && tq < hi) ? 1u : 0u;
          }
        }
      }
      const bool inf = j < nU && isinf(e);
      const bool take = j < nU && (inf || c > 0u);
      const float P = inf ? 1.f : (c > 0u ? float(W) * (ef / S) / float(c) : 0.f);
      chunk(take, T, P);
    }
    return;
  }
  if (sampler == BBC_QUERY_BINS) {
    uint32_t bin = 0;
    float fill = 0.f;
    float r = sample_stream(pr.seed, pr.key, 0u, 2u);
    for (uint32_t j0 = 0; j0 < nU; j0 += BBC_WAVE) {
      const uint32_t j = j0 + lane;
      const uint32_t T = j < nU ? a.gt[cl.at(j)] : 0u;
      const float p = j < nU ? select_prob(a.ge[cl.at(j)], gamma, false) : 0.f;
      const uint32_t cnt = min(uint32_t(BBC_WAVE), nU - j0);
      bool take = false;
      float w = p;
      for (uint32_t q = 0; q < cnt; ++q) {
        const float pq = __shfl(p, int(q), BBC_WAVE);
        if (!(pq > 0.f)) continue;
        // a candidate that would overflow the bin, or whose interval would
        // be empty (a full bin, or pq below the rounding of the sum), opens
        // the next bin, so every candidate with pq > 0 can be selected
        if (!(fill + pq <= 1.f + kBinSlack && fminf(fill + pq, 1.f) > fill)) {
          ++bin;
          fill = 0.f;
          r = sample_stream(pr.seed, pr.key, bin, 2u);
        }
        const float lo = fill;
        fill = fill + pq;
        const float hi = fminf(fill, 1.f);
        if (lane == int(q)) {
          take = r >= lo && r < hi;
          w = hi - lo;
        }
      }
      chunk(take, T, w);
    }
    return;
  }
  const float Pu = fminf(pr.W, float(nU)) / float(nU);
  for (uint32_t j0 = 0; j0 < nU; j0 += BBC_WAVE) {
    const uint32_t j = j0 + lane;
    bool take = false;
    float P = 0.f;
    uint32_t T = 0;
    if (j < nU) {
      T = a.gt[cl.at(j)];
      P = sampler == BBC_QUERY_UNIFORM ? Pu : select_prob(a.ge[cl.at(j)], gamma, exhaustive);
      take = selection_uniform(pr.seed, pr.key, tuple_key(a, T)) < P;
    }
    chunk(take, T, P);
  }
}

__global__ void __launch_bounds__(64) k_stage_count(StagedArgs s, uint32_t* sel) {
  const QueryArgs& a = s.q;
  const int lane = threadIdx.x;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    uint32_t c = 0;
    point_selection(a, s, i, lane, [&](bool take, uint32_t, float) { c += take ? 1u : 0u; });
    c = wave_sum(c);
    if (lane == 0) sel[i] = c;
  }
}

__global__ void __launch_bounds__(64) k_stage_fill(StagedArgs s) {
  const QueryArgs& a = s.q;
  const int lane = threadIdx.x;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    uint32_t o = s.off[i];
    point_selection(a, s, i, lane, [&](bool take, uint32_t T, float P) {
      const uint64_t m = __ballot(take);
      const uint32_t rank = __popcll(m & ((1ull << lane) - 1ull));
      if (take && o + rank < s.pair_cap) {
        s.pair_pt[o + rank] = uint32_t(i);
        s.pair_t[o + rank] = T;
        s.pair_p[o + rank] = P;
      }
      o += __popcll(m);
    });
  }
}

// Count and fill for the samplers whose decisions are independent per
// candidate (bound-optimal, exhaustive, uniform): a group of GL = 16 lanes per
// point, four points per wave (a cell list holds ~16 candidates), the
// candidates of a point in list order in chunks of GL, so the pairs come out
// in the same order as from the one-wave-per-point kernels above.  The count
// pass draws the Bernoulli decisions (one Philox evaluation per candidate) and
// keeps them as bits; the fill pass reads the bits instead of drawing again.
constexpr int kSelLanes = 16, kSelAhead = 8;  // chunks whose reads go out together
template <bool FILL>
__global__ void __launch_bounds__(64) k_stage_select16(StagedArgs s, uint32_t* sel) {
  constexpr int GL = kSelLanes, NG = BBC_WAVE / GL;
  const QueryArgs& a = s.q;
  const int lane = threadIdx.x, g = lane / GL, gl = lane % GL;
  const bool exhaustive = (a.mode & BBC_QUERY_EXHAUSTIVE) != 0;
  const bool uniform = (a.mode & BBC_QUERY_SAMPLERS) == BBC_QUERY_UNIFORM;
  for (int64_t i0 = int64_t(blockIdx.x) * NG; i0 < a.n; i0 += int64_t(gridDim.x) * NG) {
    const int64_t i = i0 + g;
    const bool valid = i < a.n;
    const uint32_t nU = valid ? s.cnt[i] : 0u;
    const CandList cl = cand_list(a, valid ? s.cell_b[i] : 0u);
    const float gamma = valid ? s.gamma[i] : 0.f;
    const PointReq pr = point_req(a, valid ? i : i0);
    const float Pu = fminf(pr.W, float(nU)) / float(nU);
    uint16_t* bits = s.bits + size_t(valid ? i : 0) * s.bit_stride;
    uint32_t o = FILL && valid ? s.off[i] : 0u, c = 0;
    // the group's lanes run the same trip count
    if constexpr (FILL) {
      // kSelAhead chunks per trip: their decision words, then the taken
      // entries' tuples and bounds, are read together; the pairs are written
      // chunk by chunk in list order
      for (uint32_t j0 = 0; j0 < nU; j0 += GL * kSelAhead) {
        const uint32_t j = j0 + gl;
        uint32_t word[kSelAhead], Tq[kSelAhead];
        float Eq[kSelAhead];
        bool take[kSelAhead];
#pragma unroll
        for (int u = 0; u < kSelAhead; ++u) {
          const uint32_t j0u = j0 + uint32_t(u * GL);
          word[u] = j0u < nU ? bits[j0u / GL] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kSelAhead; ++u) {
          const uint32_t ju = j + uint32_t(u * GL);
          take[u] = ju < nU && ((word[u] >> gl) & 1u) != 0u;
          Tq[u] = 0u;
          Eq[u] = 0.f;
          if (take[u]) {
            const uint32_t x = cl.at(ju);
            Tq[u] = a.gt[x];
            if (!uniform) Eq[u] = a.ge[x];
          }
        }
#pragma unroll
        for (int u = 0; u < kSelAhead; ++u) {
          const float P = take[u] ? (uniform ? Pu : select_prob(Eq[u], gamma, exhaustive)) : 0.f;
          const uint32_t m = uint32_t(__ballot(take[u]) >> (GL * g)) & ((1u << GL) - 1u);
          const uint32_t rank = __popc(m & ((1u << gl) - 1u));
          if (take[u] && o + rank < s.pair_cap) {
            s.pair_pt[o + rank] = uint32_t(i);
            s.pair_t[o + rank] = Tq[u];
            s.pair_p[o + rank] = P;
          }
          o += __popc(m);
        }
      }
    } else {
      // kSelAhead chunks per trip: their grid entries (tuple and bound, then
      // the tuple's key) are read together before the draws, through indices
      // clamped to the list (reads past its end are not used)
      for (uint32_t j0 = 0; j0 < nU; j0 += GL * kSelAhead) {
        const uint32_t j = j0 + gl;
        uint32_t Tq[kSelAhead], Kq[kSelAhead];
        float Eq[kSelAhead];
#pragma unroll
        for (int u = 0; u < kSelAhead; ++u) {
          const uint32_t x = cl.at(min(j + uint32_t(u * GL), nU - 1u));
          Tq[u] = a.gt[x];
          Eq[u] = uniform ? 0.f : a.ge[x];
        }
#pragma unroll
        for (int u = 0; u < kSelAhead; ++u) Kq[u] = tuple_key(a, Tq[u]);
#pragma unroll
        for (int u = 0; u < kSelAhead; ++u) {
          const uint32_t ju = j + uint32_t(u * GL), j0u = j0 + uint32_t(u * GL);
          bool take = false;
          if (ju < nU) {
            const float P = uniform ? Pu : select_prob(Eq[u], gamma, exhaustive);
            take = P > 0.f && selection_uniform(pr.seed, pr.key, Kq[u]) < P;
          }
          const uint32_t m = uint32_t(__ballot(take) >> (GL * g)) & ((1u << GL) - 1u);
          if (gl == 0 && j0u < nU) bits[j0u / GL] = uint16_t(m);
          c += take ? 1u : 0u;
        }
      }
    }
    if constexpr (!FILL) {
#pragma unroll
      for (int m = GL / 2; m >= 1; m >>= 1) c += __shfl_xor(c, m, BBC_WAVE);
      if (valid && gl == 0) sel[i] = c;
    }
  }
}

// Newton over the selected pairs, one lane per pair for the whole of its
// starts.
template <int CH>
__global__ void __launch_bounds__(64) k_stage_newton(StagedArgs s, const uint32_t* total) {
  const QueryArgs& a = s.q;
  const uint32_t np = min(*total, s.pair_cap);
  WorkCount wc;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < np; k += gridDim.x * blockDim.x) {
    const int64_t i = s.pair_pt[k];
    const Target tg = receiver_target(a, i);
    ++wc.pairs;
    const uint32_t r0 = wc.roots;
    s.pair_c[k] = tuple_irradiance<CH>(a, s.pair_t[k], tg, wc) / double(s.pair_p[k]);
    if (a.stats) s.pair_nr[k] = uint8_t(min(wc.roots - r0, 255u));
  }
  flush_counts(a, wc);
}

// Pooled form of the same per-pair computation.  A wave takes 64 selected
// pairs at a time and spreads their Newton starts over its lanes instead of
// giving each lane one pair for all of its starts, which leaves most lanes
// idle while one lane iterates.  The starts (leaves of the pair's tuple whose
// position bound holds the target) are gathered into a pool in LDS; in each
// pass a lane advances one start by at most `steps` FP32 iterations and puts
// it back if it is still running; converged starts queue for the FP64 polish,
// which runs 64 at a time; accepted roots are summed per pair in leaf order
// with the same deduplication, so every pair's result is that of
// tuple_irradiance.  A pair whose roots do not fit the result buffer is redone
// by tuple_irradiance.
constexpr int kPool = 128;  // FP32 starts (ring); at most 127 are held
constexpr int kCand = 128;  // FP32 roots waiting for the polish; at most 127
constexpr int kRes = 96;    // accepted roots of the 64 pairs (about 7 on average)
constexpr uint32_t kRedoCap = 16384;  // listed pairs to redo per query
constexpr int kRunQ = 128;  // queued runs (ring); at most 71 are held
constexpr uint32_t kRunsPerTrip = BBC_WAVE / kLeafGroup;
// In the two-reflection kernel, a pair whose tuple has at least kRunMin
// leaves scans the unions of its leaves' runs of kLeafGroup first and tests
// only the leaves of runs whose union holds its target; smaller tuples test
// their leaves directly.  The other chains' tuples hold a few leaves each
// (about one on a refracting surface), and their kernels do without the
// run queue's LDS, which would cost them a resident workgroup per compute
// unit.
constexpr uint32_t kRunMin = 12;

template <int CH, bool AREA = false>
struct NewtonPool {
  static constexpr int NF = CH == BBC_CHAIN_RR ? 48 : 28;  // record floats Newton reads
  static constexpr int RS = NF + 1;                         // odd row stride: rows of different pairs do not share banks
  // the two-reflection kernel reads its pairs' records from global memory
  // (cache hits: 64 records of 192 bytes per batch) and keeps only their root
  // boxes and tuples here, which lets eight of its workgroups share a
  // compute unit's LDS instead of six
  static constexpr bool GREC = CH == BBC_CHAIN_RR;
  float rec[GREC ? 1 : BBC_WAVE * RS];
  float4 root[GREC ? BBC_WAVE : 1];
  uint32_t tT[GREC ? BBC_WAVE : 1];
  double lx[AREA ? BBC_WAVE : 1], ly[AREA ? BBC_WAVE : 1], lz[AREA ? BBC_WAVE : 1];  // FP64 light points
  float tu[BBC_WAVE], tv[BBC_WAVE];
  double tud[BBC_WAVE], tvd[BBC_WAVE];
  static constexpr bool RUNS = CH == BBC_CHAIN_RR;
  static constexpr int NQ = RUNS ? kRunQ : 1, NW = RUNS ? BBC_WAVE : 1;
  uint32_t lb[BBC_WAVE], lscan[BBC_WAVE + 1];
  uint32_t mark[BBC_WAVE];  // pair + 1 at the lane offset where its units start in a window
  uint32_t lend[NW], lg0[NW];  // leaf range end, first run (or none)
  uint32_t redo[BBC_WAVE];
  uint32_t gq[NQ];  // runs whose union holds their pair's target, leaves not tested yet
  uint8_t gp[NQ];
  float pu[kPool], pv[kPool], plu0[kPool], plu1[kPool], plv0[kPool], plv1[kPool], pprev[kPool], ptl[kPool];
  uint32_t pk[kPool], pmeta[kPool];  // leaf index; pair | iterations done << 8
  float cu[kCand], cv[kCand];
  uint32_t ck[kCand], cp[kCand];
  double rud[kRes], rvd[kRes], rE[kRes];
  uint32_t rk[kRes], rp[kRes];
};

// AREA: the scene's emitters are area lights, and each pair's record copy
// takes its own light point (a separate instantiation, so that the point-light
// kernel carries none of that code).
template <int CH, bool AREA = false>
// Two waves per SIMD at most 256 registers each (LDS allows six workgroups per
// compute unit): the register budget the compiler must meet.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_stage_newton_pool(StagedArgs s, const uint32_t* total, uint32_t* redo_n,
                                                          int steps, uint32_t res_cap) {
  constexpr bool RR = CH == BBC_CHAIN_RR;
  using Pool = NewtonPool<CH, AREA>;
  constexpr int NF = Pool::NF, RS = Pool::RS, NREC = RR ? kRecFloatsRR : kRecFloats;
  constexpr bool RUNS = Pool::RUNS, GREC = Pool::GREC;
  __shared__ Pool L;
  const QueryArgs& a = s.q;
  const int lane = int(threadIdx.x);
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t np = min(*total, s.pair_cap);
  WorkCount wc;
  // Batches of 64 pairs, strided over a grid that is resident as a whole (a
  // shared work counter measured slower: every batch paid a contended
  // atomic).  A batch's pair data is loaded ahead: its tuple and point while
  // the previous batch starts, the point's receiver coordinates and the
  // tuple's leaf range and root box once that batch's refill is done, so a
  // batch starts with only its tuple records and leaf bounds in flight.
  const uint32_t stride = gridDim.x;
  uint32_t nT = 0, nPt = 0, nLb = 0, nCnt = 0;
  double2 nTgt = make_double2(0.0, 0.0);
  float4 nRoot = make_float4(0.f, 0.f, 0.f, 0.f);
  auto fetch_pair = [&](uint32_t b) {
    const uint64_t kn = uint64_t(b) * BBC_WAVE + uint64_t(lane);
    if (kn < np) {
      nT = s.pair_t[kn];
      nPt = s.pair_pt[kn];
    }
  };
  auto fetch_rest = [&](uint32_t b) {
    const uint64_t kn = uint64_t(b) * BBC_WAVE + uint64_t(lane);
    if (kn < np) {
      nTgt = s.tgt[nPt];  // as receiver_target computed it for the gamma stage
      nLb = a.toff[nT];
      nCnt = a.toff[nT + 1] - nLb;
      nRoot = reinterpret_cast<const float4*>(a.rec + size_t(nT) * NREC)[6];
    }
  };
  fetch_pair(blockIdx.x);
  fetch_rest(blockIdx.x);
  for (uint32_t batch = blockIdx.x;; batch += stride) {
    if (uint64_t(batch) * BBC_WAVE >= np) break;
    const uint32_t k = batch * uint32_t(BBC_WAVE) + uint32_t(lane);
    const bool valid = k < np;
    const uint32_t T = nT, Pt = nPt, cnt = valid ? nCnt : 0u;
    // the pair's scan units: its leaves, or the runs of kLeafGroup leaves
    // that hold them when it has kRunMin leaves or more
    const bool runs = RUNS && cnt >= kRunMin;
    const uint32_t units = runs ? (nLb + cnt - 1u) / kLeafGroup - nLb / kLeafGroup + 1u : cnt;
    Target tg{};
    tg.ud = nTgt.x;
    tg.vd = nTgt.y;
    tg.u = float(nTgt.x);
    tg.v = float(nTgt.y);
    tg.on = true;
    tg.pt = Pt;
    L.redo[lane] = 0u;
    // the rest of the record (the root box is already here) stays in
    // registers until the first refill is under way
    float4 rq[GREC ? 1 : NF / 4];
    if (valid) {
      if constexpr (GREC) {
        L.root[lane] = nRoot;
        L.tT[lane] = T;
      } else {
        const float4* r4 = reinterpret_cast<const float4*>(a.rec + size_t(T) * NREC);
#pragma unroll
        for (int q = 0; q < NF / 4; ++q)
          if (q != 6) rq[q] = r4[q];
        float* R = &L.rec[lane * RS];
        R[24] = nRoot.x;
        R[25] = nRoot.y;
        R[26] = nRoot.z;
        R[27] = nRoot.w;
      }
      L.lb[lane] = nLb;
      if constexpr (RUNS) {
        L.lend[lane] = nLb + cnt;
        L.lg0[lane] = runs ? nLb / kLeafGroup : 0xffffffffu;
      }
      L.tu[lane] = tg.u;
      L.tv[lane] = tg.v;
      L.tud[lane] = tg.ud;
      L.tvd[lane] = tg.vd;
    }
    fetch_pair(batch + stride);
    const uint32_t ex = wave_excl_scan(units, lane);
    const uint32_t tot = __shfl(ex + units, BBC_WAVE - 1, BBC_WAVE);
    L.lscan[lane] = ex;
    if (lane == BBC_WAVE - 1) L.lscan[BBC_WAVE] = tot;
    __syncthreads();
    bool stored = false;
    // the tuple record of pair p (the root box at floats 24-27)
    auto recp = [&](uint32_t p) -> const float* {
      if constexpr (GREC)
        return a.rec + size_t(L.tT[p]) * NREC;
      else
        return &L.rec[p * RS];
    };
    auto store_rec = [&]() {
      if (!GREC && valid) {
        float* R = &L.rec[lane * RS];
#pragma unroll
        for (int q = 0; q < NF / 4; ++q) {
          if (q == 6) continue;
          R[4 * q] = rq[q].x;
          R[4 * q + 1] = rq[q].y;
          R[4 * q + 2] = rq[q].z;
          R[4 * q + 3] = rq[q].w;
        }
        if constexpr (AREA) {
          const V3<double> xl = pair_light_point(a, R, Pt, T);
          L.lx[lane] = xl.x;
          L.ly[lane] = xl.y;
          L.lz[lane] = xl.z;
        }
      }
      fetch_rest(batch + stride);
      stored = true;
    };

    // wave-uniform counters: unit slots scanned, pool ring head and size,
    // queued candidates, stored roots, queued runs' ring head and size
    uint32_t scan = 0, head = 0, pn = 0, cn = 0, rn = 0, ghead = 0, gn = 0;
    auto polish = [&](uint32_t n) {
      bool ok = false, keep = false;
      double ud = 0, vd = 0, E = 0;
      uint32_t p = 0, kk = 0;
      if (uint32_t(lane) < n) {
        p = L.cp[lane];
        kk = L.ck[lane];
        TupleGeom<double> Gd = tuple_geom_rec<double, RR>(recp(p), a.sc);
        if constexpr (AREA) Gd.x0 = mk(L.lx[p], L.ly[p], L.lz[p]);
        if constexpr (RR)
          ok = polish64_called<CH>(Gd, L.tud[p], L.tvd[p], L.cu[lane], L.cv[lane], ud, vd, E, wc);
        else
          ok = polish64<CH>(Gd, L.tud[p], L.tvd[p], L.cu[lane], L.cv[lane], ud, vd, E, wc);
      }
      const uint64_t m = __ballot(ok);
      if (ok) {
        const uint32_t r = rn + uint32_t(__popcll(m & below));
        if (r < res_cap) {
          L.rud[r] = ud;
          L.rvd[r] = vd;
          L.rE[r] = E;
          L.rk[r] = kk;
          L.rp[r] = p;
        } else if (atomicExch(&L.redo[p], 1u) == 0u) {  // first overflow of this pair: list it once
          const uint32_t slot = atomicAdd(redo_n, 1u);
          if (slot < kRedoCap) s.redo[slot] = batch * uint32_t(BBC_WAVE) + p;
        }
      }
      rn = min(rn + uint32_t(__popcll(m)), res_cap);
      // move the candidates not polished yet (fewer than 64) to the front
      float mu = 0.f, mv = 0.f;
      uint32_t mk = 0, mp = 0;
      const uint32_t rest = cn - n;
      keep = uint32_t(lane) < rest;
      if (keep) {
        mu = L.cu[n + lane];
        mv = L.cv[n + lane];
        mk = L.ck[n + lane];
        mp = L.cp[n + lane];
      }
      __syncthreads();
      if (keep) {
        L.cu[lane] = mu;
        L.cv[lane] = mv;
        L.ck[lane] = mk;
        L.cp[lane] = mp;
      }
      cn = rest;
      __syncthreads();
    };

    while (true) {
      // refill the pool until it holds a pass: each trip either scans the
      // next 64 unit slots (a leaf of a small tuple is tested at once, a run
      // whose union holds the target is queued) or tests the leaves of up to
      // kRunsPerTrip queued runs, kLeafGroup lanes per run.  Every leaf whose
      // bound holds the target becomes a start, as in a scan of all leaves;
      // the order of the starts in the pool does not change any result.
      while (pn < uint32_t(BBC_WAVE) && (scan < tot || gn > 0u)) {
        bool take = false;
        Start32 st{};
        uint32_t p = 0, kk = 0;
        auto test_leaf = [&]() {
          const float4 uk = a.luk[kk];
          const uint32_t code = a.lcode[kk];  // loaded with the bound (one round trip)
          const double ud = L.tud[p], vd = L.tvd[p];
          if (ud >= uk.x && ud <= uk.y && vd >= uk.z && vd <= uk.w) {
            take = true;
            if constexpr (GREC) {
              const float4 r = L.root[p];
              st = start_of(code, r.x, r.y, r.z, r.w);
            } else {
              const float* R = &L.rec[p * RS];
              st = start_of(code, R[24], R[25], R[26], R[27]);
            }
            ++wc.starts;
          }
        };
        if (RUNS && (gn >= kRunsPerTrip || (gn > 0u && scan >= tot))) {
          const uint32_t used = min(gn, kRunsPerTrip);
          const uint32_t slot = uint32_t(lane) / kLeafGroup;
          if (slot < used) {
            const uint32_t q = (ghead + slot) % uint32_t(kRunQ);
            p = L.gp[q];
            kk = L.gq[q] * kLeafGroup + uint32_t(lane) % kLeafGroup;
            if (kk >= L.lb[p] && kk < L.lend[p]) test_leaf();  // the run may hold other tuples' leaves
          }
          ghead = (ghead + used) % uint32_t(kRunQ);
          gn -= used;
        } else {
          const uint32_t j = scan + uint32_t(lane);
          bool hit = false;
          uint32_t g = 0;
          // the pair whose units hold j, the last with lscan[p] <= j (unit
          // starts are non-decreasing over the pairs): each pair with units
          // that start inside the window marks its offset, and the lanes take
          // the largest mark at or before them, or else the count of pairs
          // that start at or before the window's first slot
          L.mark[lane] = 0u;
          if (units > 0u && ex - scan < uint32_t(BBC_WAVE)) L.mark[ex - scan] = uint32_t(lane) + 1u;
          const uint32_t c0 = uint32_t(__popcll(__ballot(ex <= scan)));
          __syncthreads();
          const uint32_t pm = wave_incl_max(max(L.mark[lane], c0));
          if (j < tot) {
            p = pm - 1u;
            const uint32_t off = j - L.lscan[p];
            if constexpr (RUNS) {
              const uint32_t g0 = L.lg0[p];
              if (g0 != 0xffffffffu) {
                g = g0 + off;
                const float4 gu = a.lgu[g];
                const double ud = L.tud[p], vd = L.tvd[p];
                hit = ud >= gu.x && ud <= gu.y && vd >= gu.z && vd <= gu.w;
              } else {
                kk = L.lb[p] + off;
                test_leaf();
              }
            } else {
              kk = L.lb[p] + off;
              test_leaf();
            }
          }
          if constexpr (RUNS) {
            const uint64_t mg = __ballot(hit);
            if (hit) {
              const uint32_t q = (ghead + gn + uint32_t(__popcll(mg & below))) % uint32_t(kRunQ);
              L.gq[q] = g;
              L.gp[q] = uint8_t(p);
            }
            if (mg) __syncthreads();  // queued runs are read by other lanes in a later trip
            gn += uint32_t(__popcll(mg));
          }
          scan += uint32_t(BBC_WAVE);
        }
        const uint64_t m = __ballot(take);
        if (take) {
          const uint32_t q = (head + pn + uint32_t(__popcll(m & below))) % uint32_t(kPool);
          L.pu[q] = st.u;
          L.pv[q] = st.v;
          L.plu0[q] = st.lu0;
          L.plu1[q] = st.lu1;
          L.plv0[q] = st.lv0;
          L.plv1[q] = st.lv1;
          L.pprev[q] = st.prev;
          L.ptl[q] = st.t_last;
          L.pk[q] = kk;
          L.pmeta[q] = p;
        }
        pn += uint32_t(__popcll(m));
      }
      if (!stored) store_rec();
      if (pn == 0u) break;
      __syncthreads();
      // one pass of FP32 iterations over (up to) 64 starts
      const uint32_t tk = min(pn, uint32_t(BBC_WAVE));
      const bool act = uint32_t(lane) < tk;
      int status = 1;
      Start32 st{};
      uint32_t p = 0, kk = 0;
      if (act) {
        const uint32_t q = (head + uint32_t(lane)) % uint32_t(kPool);
        st.u = L.pu[q];
        st.v = L.pv[q];
        st.lu0 = L.plu0[q];
        st.lu1 = L.plu1[q];
        st.lv0 = L.plv0[q];
        st.lv1 = L.plv1[q];
        st.prev = L.pprev[q];
        st.t_last = L.ptl[q];
        kk = L.pk[q];
        const uint32_t meta = L.pmeta[q];
        p = meta & 0xffu;
        st.it = int(meta >> 8);
        const TupleGeom<float> Gf = tuple_geom_rec<float, RR>(recp(p), a.sc);
        status = newton32<CH>(Gf, L.tu[p], L.tv[p], st, steps, wc);
      }
      head = (head + tk) % uint32_t(kPool);
      pn -= tk;
      __syncthreads();
      const bool again = act && status == 0;
      const uint64_t mr = __ballot(again);
      if (again) {
        const uint32_t q = (head + pn + uint32_t(__popcll(mr & below))) % uint32_t(kPool);
        L.pu[q] = st.u;
        L.pv[q] = st.v;
        L.plu0[q] = st.lu0;
        L.plu1[q] = st.lu1;
        L.plv0[q] = st.lv0;
        L.plv1[q] = st.lv1;
        L.pprev[q] = st.prev;
        L.ptl[q] = st.t_last;
        L.pk[q] = kk;
        L.pmeta[q] = p | (uint32_t(st.it) << 8);
      }
      pn += uint32_t(__popcll(mr));
      const bool cand = act && status == 2 && worth_polish(st);
      const uint64_t mc = __ballot(cand);
      if (cand) {
        const uint32_t c = cn + uint32_t(__popcll(mc & below));
        L.cu[c] = st.u;
        L.cv[c] = st.v;
        L.ck[c] = kk;
        L.cp[c] = p;
      }
      cn += uint32_t(__popcll(mc));
      __syncthreads();
      if (cn >= uint32_t(BBC_WAVE)) polish(uint32_t(BBC_WAVE));
    }
    while (cn > 0u) polish(min(cn, uint32_t(BBC_WAVE)));
    __syncthreads();

    // each pair's roots in leaf order (the order of its starts)
    if (valid) {
      const uint32_t r0 = wc.roots;
      double ET;
      if (L.redo[lane]) {
        ET = NAN;  // redone by k_stage_redo
      } else {
        RootSum rs;
        uint32_t last = 0;
        bool first = true;
        while (true) {
          uint32_t best = 0xffffffffu;
          int bi = -1;
          for (uint32_t r = 0; r < rn; ++r) {
            if (L.rp[r] != uint32_t(lane)) continue;
            const uint32_t kr = L.rk[r];
            if ((first || kr > last) && kr < best) {
              best = kr;
              bi = int(r);
            }
          }
          if (bi < 0) break;
          rs.add(L.rud[bi], L.rvd[bi], L.rE[bi], wc);
          last = best;
          first = false;
        }
        ET = rs.ET;
      }
      ++wc.pairs;
      s.pair_c[k] = ET / double(s.pair_p[k]);
      if (a.stats) s.pair_nr[k] = uint8_t(min(wc.roots - r0, 255u));
    }
    __syncthreads();
  }
  flush_counts(a, wc);
}

// Pairs whose accepted roots did not fit the pooled kernel's result buffer
// (marked with a NaN contribution and listed) are redone one lane per pair;
// when the list itself overflowed, every pair is checked for the mark.
template <int CH>
__global__ void k_stage_redo(StagedArgs s, const uint32_t* total, const uint32_t* redo_n) {
  const uint32_t nr = *redo_n;
  if (nr == 0u) return;
  const bool listed = nr <= kRedoCap;
  const QueryArgs& a = s.q;
  const uint32_t np = min(*total, s.pair_cap);
  const uint32_t m = listed ? nr : np;
  WorkCount wc;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    const uint32_t k = listed ? s.redo[j] : j;
    if (!isnan(s.pair_c[k])) continue;
    const double2 t2 = s.tgt[s.pair_pt[k]];
    Target tg{};
    tg.ud = t2.x;
    tg.vd = t2.y;
    tg.u = float(t2.x);
    tg.v = float(t2.y);
    tg.on = true;
    tg.pt = s.pair_pt[k];
    WorkCount w2;
    s.pair_c[k] = tuple_irradiance<CH>(a, s.pair_t[k], tg, w2) / double(s.pair_p[k]);
    if (a.stats) s.pair_nr[k] = uint8_t(min(w2.roots, 255u));
    wc.roots += w2.roots;  // its starts and iterations were counted by the pooled pass
  }
  flush_counts(a, wc);
}

// Sum of each point's contributions in pair order (entry order of its cell),
// and the optional per-point statistics: |U|, |S|, roots, sum of E~^2 / P.
// A group of 16 lanes per point: the group loads 16 consecutive pairs at a
// time (coalesced) and adds them in list order through shuffles, so the sum is
// the sequential one, bit for bit (the fused query sums the same way); the
// trip count is the longest list of the wave's four points, the shorter lists
// padded with +0.0, which leaves a sum of non-negative terms unchanged.
// Lane J of each row of 16 lanes to the whole row (DPP row_newbcast, a VALU
// move: no LDS round trip as with a shuffle), for an FP64 value.
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(x), 0x150 + J, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(x >> 32), 0x150 + J, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
// E += the row's 16 values in lane order (every lane of the row gets the same sum).
template <int... J>
__device__ __forceinline__ void add_row(double& E, double v, std::integer_sequence<int, J...>) {
  ((E += row_bcast<J>(v)), ...);
}

__global__ void __launch_bounds__(256) k_stage_accum(StagedArgs s) {
  constexpr int GL = kSelLanes;
  const QueryArgs& a = s.q;
  const int lane = threadIdx.x % BBC_WAVE, gl = lane % GL;
  const bool exhaustive = (a.mode & BBC_QUERY_EXHAUSTIVE) != 0;
  // the moment bound sum E~^2 / P is reported for the bound-optimal P only
  const int sampler = a.mode & BBC_QUERY_SAMPLERS;
  const bool bound_p = sampler == 0 || sampler == BBC_QUERY_BINS;
  const int64_t groups = int64_t(gridDim.x) * (blockDim.x / GL);
  for (int64_t i0 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / GL - lane / GL; i0 < a.n;
       i0 += groups) {
    // i0: the wave's first point; this group's point
    const int64_t i = i0 + lane / GL;
    const bool valid = i < a.n;
    const uint32_t o0 = valid ? min(s.off[i], s.pair_cap) : 0u, o1 = valid ? min(s.off[i + 1], s.pair_cap) : 0u;
    const uint32_t len = o1 - o0;
    uint32_t most = len;
    most = max(most, uint32_t(__shfl_xor(int(most), 16, BBC_WAVE)));
    most = max(most, uint32_t(__shfl_xor(int(most), 32, BBC_WAVE)));
    double E = 0.0;
    uint32_t roots = 0;
    for (uint32_t b = 0; b < most; b += GL) {
      const bool in = b + gl < len;
      const double v = in ? s.pair_c[o0 + b + gl] : 0.0;
      if (a.stats && in) roots += s.pair_nr[o0 + b + gl];
      static_assert(GL == 16, "a group is a DPP row");
      add_row(E, v, std::make_integer_sequence<int, GL>{});
    }
    if (valid && gl == 0) a.out[i] = float(E);
    if (a.stats) {  // uniform across the launch
#pragma unroll
      for (int m = GL / 2; m >= 1; m >>= 1) roots += uint32_t(__shfl_xor(int(roots), m, BBC_WAVE));
      const uint32_t nU = valid ? s.cnt[i] : 0u;
      const CandList cl = cand_list(a, valid ? s.cell_b[i] : 0u);
      const float gamma = valid ? s.gamma[i] : 0.f;
      uint32_t mostU = nU;
      mostU = max(mostU, uint32_t(__shfl_xor(int(mostU), 16, BBC_WAVE)));
      mostU = max(mostU, uint32_t(__shfl_xor(int(mostU), 32, BBC_WAVE)));
      double mu2 = 0.0;
      for (uint32_t b = 0; b < mostU; b += GL) {
        double t = 0.0;
        if (b + gl < nU) {
          const float e = a.ge[cl.at(b + gl)];
          const float P = select_prob(e, gamma, exhaustive);
          if (bound_p && P > 0.f && isfinite(e)) t = double(e) * double(e) / double(P);
        }
        add_row(mu2, t, std::make_integer_sequence<int, GL>{});
      }
      if (valid && gl == 0) {
        a.stats[4 * i + 0] = float(nU);
        a.stats[4 * i + 1] = float(s.off[i + 1] - s.off[i]);
        a.stats[4 * i + 2] = float(roots);
        a.stats[4 * i + 3] = float(mu2);
      }
    }
  }
}

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t staged_pairs(const Bounds* b, int64_t n) { return size_t(n) * size_t(std::max<int64_t>(1, b->max_cell)); }

size_t staged_bytes(int64_t n, size_t pairs) {
  const size_t un = size_t(std::max<int64_t>(n, 1)), up = std::max<size_t>(pairs, 1);
  return 3 * align256(un * 4) + align256((un + 1) * 4 + 8) + align256(un * 16) + align256(size_t(kRedoCap) * 4) +
         align256(scan_tmp_bytes(int64_t(un)) + 64) +
         3 * align256(up * 4) + align256(up * 8) + align256(up);
}

void staged_carve(void* base, int64_t n, size_t pairs, StagedWork& w) {
  const size_t un = size_t(std::max<int64_t>(n, 1)), up = std::max<size_t>(pairs, 1);
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    void* r = p;
    p += align256(bytes);
    return r;
  };
  w.cell = static_cast<uint32_t*>(take(un * 4));
  w.gamma = static_cast<float*>(take(un * 4));
  w.cnt = static_cast<uint32_t*>(take(un * 4));
  w.off = static_cast<uint32_t*>(take((un + 1) * 4 + 8));
  w.tgt = static_cast<double2*>(take(un * 16));
  w.redo = static_cast<uint32_t*>(take(size_t(kRedoCap) * 4));
  w.scan = take(scan_tmp_bytes(int64_t(un)) + 64);
  w.pair_pt = static_cast<uint32_t*>(take(up * 4));
  w.pair_t = static_cast<uint32_t*>(take(up * 4));
  w.pair_p = static_cast<float*>(take(up * 4));
  w.pair_c = static_cast<double*>(take(up * 8));
  w.pair_nr = static_cast<uint8_t*>(take(up));
  w.pts = un;
  w.pairs = up;
}

// Workgroups of a pooled Newton kernel that fit on the device at once (its
// LDS and registers allow a few per compute unit), cached per device and chain.
template <typename K>
static bbc_status pool_grid(K kernel, int chain, int per_cu_tuned, int* out) {
  static std::atomic<int> cache[64][4];  // the three chains, then the area-light reflection
  static std::atomic<int> cus[64];
  int dev = 0;
  BBC_HIP(hipGetDevice(&dev));
  if (per_cu_tuned > 0) {
    int n_cu = dev < 64 ? cus[dev].load() : 0;
    if (n_cu <= 0) {
      BBC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
      if (dev < 64) cus[dev].store(n_cu);
    }
    *out = per_cu_tuned * std::max(1, n_cu);
    return BBC_OK;
  }
  if (dev < 64 && chain >= 0 && chain < 4 && cache[dev][chain].load() > 0) {
    *out = cache[dev][chain].load();
    return BBC_OK;
  }
  int per_cu = 0, n_cu = 0;
  BBC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), 64, 0));
  BBC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  *out = std::max(1, per_cu) * std::max(1, n_cu);
  if (dev < 64 && chain >= 0 && chain < 4) cache[dev][chain].store(*out);
  return BBC_OK;
}

// The five stage launches of one staged query; events (nullable) bracket the
// Newton kernel.
static bbc_status run_staged(const QueryArgs& q, const StagedWork& w, size_t pairs, int newton_steps,
                             int newton_results, int newton_grid_per_cu, hipEvent_t ev0, hipEvent_t ev1,
                             hipStream_t st) {
  const uint32_t res_cap = uint32_t(std::min(std::max(newton_results, 1), kRes));
  const int64_t n = q.n;
  StagedArgs s{};
  s.q = q;
  s.cell_b = w.cell;
  s.gamma = w.gamma;
  s.cnt = w.cnt;
  s.off = w.off;
  s.tgt = w.tgt;
  s.redo = w.redo;
  s.pair_pt = w.pair_pt;
  s.pair_t = w.pair_t;
  s.pair_p = w.pair_p;
  s.pair_c = w.pair_c;
  s.pair_nr = w.pair_nr;
  s.pair_cap = uint32_t(std::min<size_t>(pairs, 0xffffffffu));
  // pairs >= n * (the fullest cell's candidates), so n * bit_stride 16-bit
  // words fit pair_c's 8 * pairs bytes
  s.bits = reinterpret_cast<uint16_t*>(w.pair_c);
  s.bit_stride = uint32_t((pairs / size_t(std::max<int64_t>(n, 1)) + kSelLanes - 1) / kSelLanes);
  const unsigned grid = unsigned(std::min<int64_t>(n, 256 * 64));
  const unsigned gpt = unsigned(std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_stage_gamma, dim3(gpt), dim3(256), 0, st, s);
  const unsigned gl = unsigned(std::min<int64_t>((n + 3) / 4, 16384));
  hipLaunchKernelGGL(k_stage_gamma_long, dim3(gl), dim3(256), 0, st, s);
  // selection counts go to the head of the pair_pt buffer, are scanned into
  // off, and are overwritten by the fill kernel afterwards
  uint32_t* sel = w.pair_pt;
  const int sampler = q.mode & BBC_QUERY_SAMPLERS;
  const bool independent = sampler == 0 || sampler == BBC_QUERY_UNIFORM;
  const unsigned g16 = unsigned(std::min<int64_t>((n + 3) / 4, 256 * 64));
  if (independent)
    hipLaunchKernelGGL(k_stage_select16<false>, dim3(g16), dim3(64), 0, st, s, sel);
  else
    hipLaunchKernelGGL(k_stage_count, dim3(grid), dim3(64), 0, st, s, sel);
  bbc_status e = launch_scan_u32(sel, s.off, n, w.scan, st);
  if (e) return e;
  if (independent)
    hipLaunchKernelGGL(k_stage_select16<true>, dim3(g16), dim3(64), 0, st, s, sel);
  else
    hipLaunchKernelGGL(k_stage_fill, dim3(grid), dim3(64), 0, st, s);
  if (ev0) BBC_HIP(hipEventRecord(ev0, st));
  if (newton_steps > 0) {
    // as many workgroups as stay resident together, striding over the
    // batches of 64 pairs; then the rare pairs to redo (a list of at most
    // kRedoCap, or in its overflow a strided scan of every pair): a small
    // grid, since the launch mostly finds the list empty
    int nres = 0;
    const unsigned gr = unsigned(std::min<size_t>((pairs + 255) / 256, 128));
    if (q.sc.chain == BBC_CHAIN_RR) {
      if ((e = pool_grid(k_stage_newton_pool<BBC_CHAIN_RR>, BBC_CHAIN_RR, newton_grid_per_cu, &nres))) return e;
      const unsigned gq = unsigned(std::min<size_t>((pairs + 63) / 64, size_t(nres)));
      hipLaunchKernelGGL(k_stage_newton_pool<BBC_CHAIN_RR>, dim3(gq), dim3(64), 0, st, s, s.off + n, s.off + n + 1,
                         newton_steps, res_cap);
      if (ev1) BBC_HIP(hipEventRecord(ev1, st));
      hipLaunchKernelGGL(k_stage_redo<BBC_CHAIN_RR>, dim3(gr), dim3(256), 0, st, s, s.off + n, s.off + n + 1);
    } else if (q.sc.chain == BBC_CHAIN_T) {
      if ((e = pool_grid(k_stage_newton_pool<BBC_CHAIN_T>, BBC_CHAIN_T, newton_grid_per_cu, &nres))) return e;
      const unsigned gq = unsigned(std::min<size_t>((pairs + 63) / 64, size_t(nres)));
      hipLaunchKernelGGL(k_stage_newton_pool<BBC_CHAIN_T>, dim3(gq), dim3(64), 0, st, s, s.off + n, s.off + n + 1,
                         newton_steps, res_cap);
      if (ev1) BBC_HIP(hipEventRecord(ev1, st));
      hipLaunchKernelGGL(k_stage_redo<BBC_CHAIN_T>, dim3(gr), dim3(256), 0, st, s, s.off + n, s.off + n + 1);
    } else if (q.sc.eedge) {
      if ((e = pool_grid(k_stage_newton_pool<BBC_CHAIN_R, true>, 3, newton_grid_per_cu, &nres))) return e;
      const unsigned gq = unsigned(std::min<size_t>((pairs + 63) / 64, size_t(nres)));
      hipLaunchKernelGGL((k_stage_newton_pool<BBC_CHAIN_R, true>), dim3(gq), dim3(64), 0, st, s, s.off + n,
                         s.off + n + 1, newton_steps, res_cap);
      if (ev1) BBC_HIP(hipEventRecord(ev1, st));
      hipLaunchKernelGGL(k_stage_redo<BBC_CHAIN_R>, dim3(gr), dim3(256), 0, st, s, s.off + n, s.off + n + 1);
    } else {
      if ((e = pool_grid(k_stage_newton_pool<BBC_CHAIN_R>, BBC_CHAIN_R, newton_grid_per_cu, &nres))) return e;
      const unsigned gq = unsigned(std::min<size_t>((pairs + 63) / 64, size_t(nres)));
      hipLaunchKernelGGL(k_stage_newton_pool<BBC_CHAIN_R>, dim3(gq), dim3(64), 0, st, s, s.off + n, s.off + n + 1,
                         newton_steps, res_cap);
      if (ev1) BBC_HIP(hipEventRecord(ev1, st));
      hipLaunchKernelGGL(k_stage_redo<BBC_CHAIN_R>, dim3(gr), dim3(256), 0, st, s, s.off + n, s.off + n + 1);
    }
  } else {
    const unsigned gp = unsigned(std::min<size_t>((pairs + 63) / 64, 32768));
    if (q.sc.chain == BBC_CHAIN_RR)
      hipLaunchKernelGGL(k_stage_newton<BBC_CHAIN_RR>, dim3(gp), dim3(64), 0, st, s, s.off + n);
    else if (q.sc.chain == BBC_CHAIN_T)
      hipLaunchKernelGGL(k_stage_newton<BBC_CHAIN_T>, dim3(gp), dim3(64), 0, st, s, s.off + n);
    else
      hipLaunchKernelGGL(k_stage_newton<BBC_CHAIN_R>, dim3(gp), dim3(64), 0, st, s, s.off + n);
    if (ev1) BBC_HIP(hipEventRecord(ev1, st));
  }
  const unsigned ga = unsigned(std::min<int64_t>((n + 15) / 16, 65536));
  hipLaunchKernelGGL(k_stage_accum, dim3(ga), dim3(256), 0, st, s);
  BBC_HIP(hipGetLastError());
  return BBC_OK;
}

// Points per staged launch: the worst case of every launch (every candidate
// of the fullest cell selected) stays within kMaxStagedPairs pairs.
int64_t staged_slice(const Bounds* b, int64_t n) {
  const int64_t cap = std::min<int64_t>(b->tune.staged_pairs, int64_t(kMaxStagedPairs));
  const int64_t per = cap / std::max<int64_t>(1, b->max_cell);
  return std::max<int64_t>(1, std::min(n, per));
}

// One staged launch over points [i0, i0 + m) of a query of n points, in the
// carved work space w (sized for at least m points).
static bbc_status staged_slice_run(const Bounds* b, const float* pts, int64_t n, int64_t i0, int64_t m, int32_t spp,
                                   uint64_t seed, int64_t base, int32_t mode, float* out, float* stats,
                                   unsigned long long* counters, const StagedWork& w, hipEvent_t ev0, hipEvent_t ev1,
                                   hipStream_t st) {
  QueryArgs q = make_args(b, pts + i0, m, spp, seed, base + i0, mode, out + i0, stats ? stats + 4 * i0 : nullptr,
                          counters);
  q.pstride = n;
  return run_staged(q, w, w.pairs, b->tune.newton_steps, b->tune.newton_results, b->tune.newton_grid_per_cu, ev0,
                    ev1, st);
}

bbc_status launch_query_staged(Bounds* b, const float* pts, int64_t n, int32_t spp, uint64_t seed, int64_t base,
                               int32_t mode, float* out, float* stats, unsigned long long* counters, hipStream_t st) {
  if (n == 0) return BBC_OK;
  const int64_t slice = staged_slice(b, n);
  const size_t pairs = staged_pairs(b, slice);
  if (size_t(slice) > b->qw.pts || pairs > b->qw.pairs) {
    const int64_t np = std::max<int64_t>(slice, int64_t(b->qw.pts));
    const size_t pp = std::max(pairs, b->qw.pairs);
    bbc_status e = ensure(b->qw_buf, staged_bytes(np, pp), b);
    if (e) return e;
    staged_carve(b->qw_buf.p, np, pp, b->qw);
  }
  const bool timed = b->tune.timing != 0;
  if (b->tune.graph && !timed) {
    // every slice's launches in one graph, replayed on the handle's stream
    return run_as_graph(b->qgraph, st, [&](hipStream_t gs) -> bbc_status {
      for (int64_t i0 = 0; i0 < n; i0 += slice) {
        const int64_t m = std::min(slice, n - i0);
        bbc_status e = staged_slice_run(b, pts, n, i0, m, spp, seed, base, mode, out, stats, counters, b->qw, nullptr,
                                        nullptr, gs);
        if (e) return e;
      }
      return BBC_OK;
    });
  }
  if (timed) {
    // one pair of events around the Newton kernel of every slice
    const size_t want = size_t(2 * ((n + slice - 1) / slice));
    while (b->tev.size() < want) {
      hipEvent_t ev = nullptr;
      BBC_HIP(hipEventCreate(&ev));
      b->tev.push_back(ev);
    }
    b->tev_used = 0;
  }
  for (int64_t i0 = 0, k = 0; i0 < n; i0 += slice, ++k) {
    const int64_t m = std::min(slice, n - i0);
    bbc_status e = staged_slice_run(b, pts, n, i0, m, spp, seed, base, mode, out, stats, counters, b->qw,
                                    timed ? b->tev[2 * k] : nullptr, timed ? b->tev[2 * k + 1] : nullptr, st);
    if (e) return e;
    if (timed) b->tev_used = int(k + 1);
  }
  return BBC_OK;
}

bbc_status launch_query_staged_in(const Bounds* b, const float* pts, int64_t n, int32_t spp, uint64_t seed,
                                  int64_t base, int32_t mode, float* out, float* stats, void* work, size_t bytes,
                                  hipStream_t st) {
  if (n == 0) return BBC_OK;
  // the largest slice whose worst-case work space fits `bytes`
  int64_t lo = 0, hi = staged_slice(b, n);
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (staged_bytes(mid, staged_pairs(b, mid)) <= bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  if (lo == 0) {
    set_error("work space of " + std::to_string(bytes) + " bytes cannot hold one shading point's worst case (" +
              std::to_string(staged_bytes(1, staged_pairs(b, 1))) + " bytes for a cell of " +
              std::to_string(b->max_cell) + " candidates)");
    return BBC_EBUDGET;
  }
  StagedWork w;
  staged_carve(work, lo, staged_pairs(b, lo), w);
  for (int64_t i0 = 0; i0 < n; i0 += lo) {
    const int64_t m = std::min(lo, n - i0);
    bbc_status e = staged_slice_run(b, pts, n, i0, m, spp, seed, base, mode, out, stats, nullptr, w, nullptr, nullptr,
                                    st);
    if (e) return e;
  }
  return BBC_OK;
}

bbc_status launch_query_batch(const Bounds* b, const float* pts, int64_t n, const uint16_t* preq,
                              const ReqDesc* reqs, int32_t mode, float* out, const StagedWork& w, hipEvent_t ev0,
                              hipEvent_t ev1, hipStream_t st) {
  if (n == 0) return BBC_OK;
  const int64_t slice = staged_slice(b, n);
  if (size_t(slice) > w.pts || staged_pairs(b, slice) > w.pairs) {
    set_error("batch work space smaller than one slice of the batch");
    return BBC_EINVAL;
  }
  // consecutive slices of the batch over the same work space; each point
  // keeps its request's random stream through the slice offset
  for (int64_t i0 = 0; i0 < n; i0 += slice) {
    const int64_t m = std::min(slice, n - i0);
    QueryArgs q = make_args(b, pts + i0, m, 1, 0, 0, mode, out + i0, nullptr, nullptr);
    q.pstride = n;
    q.preq = preq + i0;
    q.reqs = reqs;
    q.ioff = i0;
    const bool ev = i0 == 0;
    bbc_status e = run_staged(q, w, w.pairs, b->tune.newton_steps, b->tune.newton_results,
                              b->tune.newton_grid_per_cu, ev ? ev0 : nullptr,
                              ev ? ev1 : nullptr, st);
    if (e) return e;
  }
  return BBC_OK;
}

}  // namespace bbc
