// Stage 1-2 on the GPU: tuple culling, domain initialisation and adaptive
// subdivision with Bernstein bounds (Sec. 4.1-4.4, Sec. 6.1).
//
// Work decomposition (one wave = one workgroup of 64 lanes per box, lanes
// over the Bernstein coefficients of the box's polynomials in LDS):
//   k_level0       every tuple's [0,1]^2 box, position bound only: culled /
//                  settled (root box [0,1]^2) / needs refinement
//   k_init         breadth-first domain initialisation of the unsettled tuples
//   k_subdiv<L>    one launch per depth L; persistent waves stride over the
//                  depth's queue: bound the box, emit a leaf or push its four
//                  children to the next depth's queue
//   *_fp64         the same decisions for boxes whose denominators could not
//                  be given a sign in FP32
//   k_*_t          the refraction chain: every box in FP64 (box_t.hpp)
//   k_pairs_*      two reflections: tuple construction over all triangle pairs
//   k_*_rr         two reflections: position and irradiance bounds in FP64 (box_rr.hpp)
// No host synchronisation happens between launches; every count lives in
// device memory and every buffer has a capacity checked on the device.
#include <atomic>

#include "box_r.hpp"
#include "box_ra.hpp"
#include "box_rr.hpp"
#include "box_t.hpp"
#include "internal.hpp"

namespace bbc {

struct BuildArgs {
  DevScene sc;
  int64_t n_tuples;
  int max_depth, init_levels, init_pieces, flags;
  float sigma, alpha;
  BuildCounters* C;
  float4* root;
  uint32_t* init_q;
  uint32_t* l0f_q;
  QItem* qin;
  QItem* qout;
  QItem* fq;
  uint32_t q_cap, fq_cap, leaf_cap;
  uint32_t* lt;
  uint32_t* lc;
  float4* lu;
  float2* le;
  const double* red;  // degree-reduction table (BBC_FLAG_DEGREE_REDUCTION), else null
  // single-reflection subdivision from split polynomials: the records of this
  // depth's items (null at depth 0) and of the next depth's, srec_cap each
  const double* srec_in;
  double* srec_out;
  uint32_t srec_cap;
};

// Outputs of a workgroup's boxes (queue items for the next depth, leaves,
// tuples for domain initialisation), staged in LDS by thread 0 and written
// with one atomic per counter per flush: boxes finish every few microseconds
// on every compute unit, and one global atomic per box on the same counter
// serialises the whole grid.
constexpr int kStageItems = 64, kStageLeaves = 32;
struct Stage {
  QItem item[kStageItems];
  uint32_t initq[kStageItems];
  uint32_t lt[kStageLeaves], lc[kStageLeaves];
  float4 lu[kStageLeaves];
  float2 le[kStageLeaves];
  uint32_t n_item, n_init, n_leaf, n_inf, max_depth, n_live, base_item, base_init, base_leaf;
};

__device__ __forceinline__ void stage_reset(Stage& S, int lane) {
  if (lane == 0) S.n_item = S.n_init = S.n_leaf = S.n_inf = S.max_depth = S.n_live = 0u;
}

// Room for four more items, leaves and tuples (one box's children, or one
// result from each of four lane groups).
__device__ __forceinline__ bool stage_full(const Stage& S) {
  return S.n_item > kStageItems - 4 || S.n_leaf > kStageLeaves - 4 || S.n_init > kStageItems - 4;
}

// Called by every thread of the workgroup; `items` go to queue qcount[depth].
template <int NT>
__device__ void stage_flush(const BuildArgs& a, int depth, Stage& S, int lane) {
  wave_sync();
  if (lane == 0) {
    S.base_item = S.n_item ? atomicAdd(&a.C->qcount[depth], S.n_item) : 0u;
    S.base_leaf = S.n_leaf ? atomicAdd(&a.C->n_leaves, S.n_leaf) : 0u;
    S.base_init = S.n_init ? atomicAdd(&a.C->n_init, S.n_init) : 0u;
    if (S.n_live) atomicAdd(&a.C->n_live, S.n_live);
    if (S.n_inf) atomicAdd(&a.C->n_inf, S.n_inf);
    if (S.n_leaf) atomicMax(&a.C->max_depth, S.max_depth);
    if (S.n_item && S.base_item + S.n_item > a.q_cap) atomicOr(&a.C->overflow, 1u);
    if (S.n_leaf && S.base_leaf + S.n_leaf > a.leaf_cap) atomicOr(&a.C->overflow, 2u);
  }
  wave_sync();
  const uint32_t ni = S.n_item, nl = S.n_leaf, nt = S.n_init;
  const uint32_t bi = S.base_item, bl = S.base_leaf, bt = S.base_init;
  for (uint32_t k = lane; k < ni; k += NT)
    if (bi + k < a.q_cap) a.qout[bi + k] = S.item[k];
  for (uint32_t k = lane; k < nt; k += NT) a.init_q[bt + k] = S.initq[k];  // capacity n_tuples: cannot overflow
  for (uint32_t k = lane; k < nl; k += NT)
    if (bl + k < a.leaf_cap) {
      a.lt[bl + k] = S.lt[k];
      a.lc[bl + k] = S.lc[k];
      a.lu[bl + k] = S.lu[k];
      a.le[bl + k] = S.le[k];
    }
  wave_sync();
  stage_reset(S, lane);
  wave_sync();
}

// A live tuple's root box: store it and stage the tuple's depth-0 queue item.
__device__ __forceinline__ void push_root(const BuildArgs& a, uint32_t t, float4 box, Stage& S) {
  a.root[t] = box;
  S.item[atomicAdd(&S.n_item, 1u)] = QItem{t, 0u};
  atomicAdd(&S.n_live, 1u);
}

// What a tuple's level-0 bound decides: culled, a root box [0,1]^2, or domain
// initialisation.  One thread per tuple.
__device__ __forceinline__ void level0_decide(const BuildArgs& a, uint32_t t, const BoxOut& o, Stage& S) {
  if (o.status == 2) {
    const uint32_t i = atomicAdd(&a.C->n_l0_fp64, 1u);
    a.l0f_q[i] = t;  // capacity n_tuples: cannot overflow
    return;
  }
  if (o.status == 0) return;
  if (o.settled || a.init_levels == 0)
    push_root(a, t, make_float4(0.f, 1.f, 0.f, 1.f), S);
  else
    S.initq[atomicAdd(&S.n_init, 1u)] = t;
}

// Level 0: the whole parameter square of every tuple, position bound only.
// ev(G, u0, u1, v0, v1) bounds one box.
template <class T, class Ev>
__device__ void level0_one(const BuildArgs& a, uint32_t t, Ev ev, int lane, Stage& S) {
  const TupleGeom<T> G = tuple_geom<T>(a.sc, t);
  if (!G.front) return;
  const BoxOut o = ev(G, T(0), T(1), T(0), T(1));
  if (lane != 0) return;
  level0_decide(a, t, o, S);
}

// The per-tuple loop of the level-0 kernels with staged outputs.
template <class T, int NT = BBC_WAVE, class Ev, class Tuples>
__device__ void level0_loop(const BuildArgs& a, Ev ev, int lane, Stage& S, uint32_t n, Tuples tuple_at) {
  stage_reset(S, lane);
  wave_sync();
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    level0_one<T>(a, tuple_at(i), ev, lane, S);
    wave_sync();
    if (stage_full(S)) stage_flush<NT>(a, 0, S, lane);
  }
  stage_flush<NT>(a, 0, S, lane);
}

// Position-only boxes of reflection tuples have at most 25 coefficients per
// polynomial: a wave bounds four of them at once, 16 lanes each.
constexpr int kGroup = 16, kGroups = BBC_WAVE / kGroup;

__global__ void __launch_bounds__(64) k_level0(BuildArgs a) {
  __shared__ LdsRPos<float> L[kGroups];
  __shared__ Stage S;
  const int g = threadIdx.x / kGroup, lane = threadIdx.x % kGroup;
  const uint32_t n = uint32_t(a.n_tuples);
  stage_reset(S, threadIdx.x);
  wave_sync();
  for (uint32_t i0 = blockIdx.x * kGroups; i0 < n; i0 += gridDim.x * kGroups) {
    const uint32_t t = i0 + g;
    const bool have = t < n;
    const TupleGeom<float> G = tuple_geom<float>(a.sc, have ? t : i0);
    const BoxOut o = eval_box_r<float, false, LdsRPos<float>, kGroup>(G, 0.f, 1.f, 0.f, 1.f, false, L[g], lane);
    if (have && lane == 0) level0_decide(a, t, o, S);
    wave_sync();
    if (stage_full(S)) stage_flush<BBC_WAVE>(a, 0, S, threadIdx.x);
  }
  stage_flush<BBC_WAVE>(a, 0, S, threadIdx.x);
}

__global__ void __launch_bounds__(64) k_level0_fp64(BuildArgs a) {
  __shared__ LdsRPos<double> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_r<double, false>(G, u0, u1, v0, v1, true, L, lane);
  };
  level0_loop<double>(a, ev, lane, S, a.C->n_l0_fp64, [&](uint32_t i) { return a.l0f_q[i]; });
}

__global__ void __launch_bounds__(64) k_level0_t(BuildArgs a) {
  __shared__ LdsT<double, false> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_t<double, false, BBC_WAVE>(G, u0, u1, v0, v1, true, a.flags, L, lane);
  };
  level0_loop<double>(a, ev, lane, S, uint32_t(a.n_tuples), [](uint32_t i) { return i; });
}

// Area lights (single reflection): every box over the whole light, in FP64.
__global__ void __launch_bounds__(64) k_level0_ra(BuildArgs a) {
  __shared__ LdsRA<double, false> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_ra<double, false, BBC_WAVE>(G, u0, u1, v0, v1, L, lane);
  };
  level0_loop<double>(a, ev, lane, S, uint32_t(a.n_tuples), [](uint32_t i) { return i; });
}

// Two-reflection position bounds (degree 16 per axis, FP64) take ~57 KB of
// LDS, so two workgroups fit a compute unit: four waves share each box, as in
// the subdivision, rather than one wave alone.
constexpr int kInitRRThreads = 256;
__global__ void __launch_bounds__(kInitRRThreads) k_level0_rr(BuildArgs a) {
  __shared__ LdsRR<double> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_rr<double, false, kInitRRThreads>(G, u0, u1, v0, v1, L, lane);
  };
  level0_loop<double, kInitRRThreads>(a, ev, lane, S, uint32_t(a.n_tuples), [](uint32_t i) { return i; });
}

// ---------------------------------------------------------------- tuple construction, two reflections
// A second-surface triangle joins a first-surface triangle's tuple when the
// interval bound of (x2 - x1) x d~1 covers zero in every component and
// (x2 - x1) . d~1 can be positive, with x1 and x2 over the triangles' bounding
// boxes and d~1 the reflected direction bounded by its Bernstein coefficients
// over [0,1]^2 (Sec. 6.1, tuple construction).  The light must be in front of
// the first triangle.  Plain FP64 interval arithmetic.
struct PairArgs {
  DevScene sc;
  const double* box2;  // [6][n_tri2]: lo xyz, hi xyz of every second-surface triangle
  uint32_t* rowcount;  // [n_emit * n_tri]
  const uint32_t* rowoff;
  uint32_t* tid;
};

__global__ void k_pair_boxes(DevScene sc, double* box2) {
  const int64_t n = sc.n_tri2;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    for (int k = 0; k < 3; ++k) {
      const double a = sc.pos2[k * n + t], b = sc.pos2[(3 + k) * n + t], c = sc.pos2[(6 + k) * n + t];
      box2[k * n + t] = fmin(a, fmin(b, c));
      box2[(3 + k) * n + t] = fmax(a, fmax(b, c));
    }
  }
}

struct PairRow {
  bool front;
  double alo[3], ahi[3], dlo[3], dhi[3];
};

// Bounding box of the first triangle and coefficient ranges of d~1 over
// [0,1]^2, in scaled Bernstein form (one thread).
__device__ PairRow pair_row(const DevScene& sc, int64_t row) {
  PairRow r;
  const int64_t n = sc.n_tri, t = row % n, e = row / n;
  const TupleGeom<double> G = tuple_geom_first<double>(sc, t, e);
  r.front = G.front;
  const V3<double> a0 = G.p0, a1 = G.p0 + G.e1, a2 = G.p0 + G.e2;
  for (int k = 0; k < 3; ++k) {
    r.alo[k] = fmin(comp(a0, k), fmin(comp(a1, k), comp(a2, k)));
    r.ahi[k] = fmax(comp(a0, k), fmax(comp(a1, k), comp(a2, k)));
  }
  // corner values (index 2 iu + iv) of n and d0; degree (1,1) scaled = plain
  double nc[3][4], dc[3][4];
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < 4; ++k) {
      const double u = (k & 2) ? 1.0 : 0.0, v = (k & 1) ? 1.0 : 0.0;
      nc[c][k] = comp(G.n0, c) + u * comp(G.dn1, c) + v * comp(G.dn2, c);
      dc[c][k] = comp(G.p0 - G.x0, c) + u * comp(G.e1, c) + v * comp(G.e2, c);
    }
  double nn[9] = {0}, dn[9] = {0};
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int i = (a >> 1) + (b >> 1), j = (a & 1) + (b & 1);
        nn[3 * i + j] += nc[c][a] * nc[c][b];
        dn[3 * i + j] += dc[c][a] * nc[c][b];
      }
  for (int c = 0; c < 3; ++c) {
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i <= 3; ++i)
      for (int j = 0; j <= 3; ++j) {
        double sv = 0.0;
        for (int a = 0; a <= 2; ++a)
          for (int b = 0; b <= 2; ++b) {
            const int di = i - a, dj = j - b;
            if (di < 0 || di > 1 || dj < 0 || dj > 1) continue;
            sv += nn[3 * a + b] * dc[c][2 * di + dj] - 2.0 * dn[3 * a + b] * nc[c][2 * di + dj];
          }
        const double bc = sv / double(binom_i(3, i) * binom_i(3, j));
        lo = fmin(lo, bc);
        hi = fmax(hi, bc);
      }
    r.dlo[c] = lo;
    r.dhi[c] = hi;
  }
  return r;
}

__device__ __forceinline__ void imul(double a, double b, double c, double d, double* lo, double* hi) {
  const double p0 = a * c, p1 = a * d, p2 = b * c, p3 = b * d;
  *lo = fmin(fmin(p0, p1), fmin(p2, p3));
  *hi = fmax(fmax(p0, p1), fmax(p2, p3));
}

__device__ __forceinline__ bool pair_test(const PairRow& r, const double* box2, int64_t n2, int64_t t2) {
  double xl[3], xh[3];
  for (int k = 0; k < 3; ++k) {
    xl[k] = box2[k * n2 + t2] - r.ahi[k];
    xh[k] = box2[(3 + k) * n2 + t2] - r.alo[k];
  }
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    double pl, ph, ql, qh;
    imul(xl[i], xh[i], r.dlo[j], r.dhi[j], &pl, &ph);
    imul(xl[j], xh[j], r.dlo[i], r.dhi[i], &ql, &qh);
    if (pl - qh > 0.0 || ph - ql < 0.0) return false;
  }
  double fh = 0.0;
  for (int k = 0; k < 3; ++k) {
    double pl, ph;
    imul(xl[k], xh[k], r.dlo[k], r.dhi[k], &pl, &ph);
    fh += ph;
  }
  return fh > 0.0;
}

constexpr int kPairThreads = 256;

// fill = false: count the candidates of every row; fill = true: write their
// tuple numbers in ascending order at the row's offset.
__global__ void __launch_bounds__(kPairThreads) k_pairs(PairArgs a, int fill) {
  __shared__ PairRow R;
  __shared__ uint32_t wsum[kPairThreads / BBC_WAVE];
  const int64_t rows = a.sc.n_emit * a.sc.n_tri, n2 = a.sc.n_tri2;
  const int lane = threadIdx.x % BBC_WAVE, w = threadIdx.x / BBC_WAVE;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    if (threadIdx.x == 0) R = pair_row(a.sc, row);
    __syncthreads();
    const PairRow r = R;
    uint32_t base = fill ? a.rowoff[row] : 0u, count = 0;
    for (int64_t c0 = 0; c0 < n2; c0 += kPairThreads) {
      const int64_t t2 = c0 + threadIdx.x;
      const bool pass = r.front && t2 < n2 && pair_test(r, a.box2, n2, t2);
      const uint64_t m = __ballot(pass);
      if (lane == 0) wsum[w] = uint32_t(__popcll(m));
      __syncthreads();
      uint32_t before = 0, total = 0;
      for (int k = 0; k < kPairThreads / BBC_WAVE; ++k) {
        if (k < w) before += wsum[k];
        total += wsum[k];
      }
      if (fill && pass) {
        const uint32_t rank = before + uint32_t(__popcll(m & ((1ull << lane) - 1ull)));
        a.tid[base + count + rank] = uint32_t(row * n2 + t2);
      }
      count += total;
      __syncthreads();
    }
    if (!fill && threadIdx.x == 0) a.rowcount[row] = count;
    __syncthreads();
  }
}

bbc_status launch_pairs(const DevScene& sc, double* box2, uint32_t* rowcount, const uint32_t* rowoff, uint32_t* tid,
                        bool fill, hipStream_t s) {
  const int64_t rows = sc.n_emit * sc.n_tri;
  if (!fill) {
    hipLaunchKernelGGL(k_pair_boxes, dim3(unsigned(std::min<int64_t>((sc.n_tri2 + 255) / 256, 1024))), dim3(256),
                       0, s, sc, box2);
    BBC_HIP(hipGetLastError());
  }
  PairArgs a{sc, box2, rowcount, rowoff, tid};
  hipLaunchKernelGGL(k_pairs, dim3(unsigned(std::min<int64_t>(rows, 8192))), dim3(kPairThreads), 0, s, a,
                     fill ? 1 : 0);
  BBC_HIP(hipGetLastError());
  return BBC_OK;
}

// Domain initialisation (Sec. 6.1): breadth-first refinement of [0,1]^2 that
// keeps boxes whose position bound meets the receiver; a box whose bound lies
// wholly inside [0,1]^2 with the receiver ahead is settled and kept as is.
// Stops when all kept boxes are settled, when more than init_pieces would be
// kept, or after init_levels levels; the root is the kept boxes' bounding box.
constexpr int kInitCap = 260;  // init_pieces <= 256, plus one parent's children
struct InitBox {
  uint32_t code;  // level << 28 | iu << 14 | iv
  uint32_t settled;
};

// One tuple's breadth-first initialisation; ev(cl, cu, cv) bounds the box
// (cu, cv) of level cl.
template <int NT = BBC_WAVE, class Ev>
__device__ void init_one(const BuildArgs& a, uint32_t t, Ev ev, InitBox* cur, InitBox* nxt, int lane, Stage& S) {
  int ncur = 1;
  if (lane == 0) cur[0] = InitBox{0u, 0u};
  wave_sync();
  bool dead = false;
  for (int level = 1; level <= a.init_levels; ++level) {
    bool all_settled = true;
    for (int j = 0; j < ncur; ++j) all_settled = all_settled && cur[j].settled;
    if (all_settled) break;
    int nn = 0;
    bool over = false;
    for (int j = 0; j < ncur && !over; ++j) {
      const InitBox b = cur[j];
      if (b.settled) {
        if (lane == 0) nxt[nn] = b;
        ++nn;
        over = nn > a.init_pieces;
        continue;
      }
      const int bl = int(b.code >> 28);
      const uint32_t iu = (b.code >> 14) & 0x3fffu, iv = b.code & 0x3fffu;
      for (int ch = 0; ch < 4 && !over; ++ch) {
        const uint32_t cu = 2 * iu + (ch >> 1), cv = 2 * iv + (ch & 1);
        const int cl = bl + 1;
        wave_sync();
        const BoxOut o = ev(cl, cu, cv);
        if (o.status == 1) {
          if (lane == 0) nxt[nn] = InitBox{uint32_t(cl) << 28 | cu << 14 | cv, o.settled ? 1u : 0u};
          ++nn;
          over = nn > a.init_pieces;
        }
      }
    }
    wave_sync();
    if (over) break;
    if (nn == 0) {
      dead = true;
      break;
    }
    for (int j = lane; j < nn; j += NT) cur[j] = nxt[j];
    ncur = nn;
    wave_sync();
  }
  if (!dead && lane == 0) {
    float u0 = 1.f, u1 = 0.f, v0 = 1.f, v1 = 0.f;
    for (int j = 0; j < ncur; ++j) {
      const int bl = int(cur[j].code >> 28);
      const float w = ldexpf(1.f, -bl);
      const uint32_t iu = (cur[j].code >> 14) & 0x3fffu, iv = cur[j].code & 0x3fffu;
      u0 = fminf(u0, iu * w);
      u1 = fmaxf(u1, (iu + 1) * w);
      v0 = fminf(v0, iv * w);
      v1 = fmaxf(v1, (iv + 1) * w);
    }
    push_root(a, t, make_float4(u0, u1, v0, v1), S);
  }
  wave_sync();
  if (stage_full(S)) stage_flush<NT>(a, 0, S, lane);
}

// Domain initialisation of reflection tuples: the four children of a box are
// bounded at once (16 lanes each, FP32); a child whose denominator sign is
// undecided is redone by the whole wave in FP64.  Children are kept in child
// order, so the result is that of the one-child-at-a-time loop.  The FP64
// redo starts after the FP32 results are read, so its tensors share the FP32
// tensors' LDS (15 KB per wave).
union InitLds {
  LdsRPos<float> f[kGroups];
  LdsRPos<double> d;
};
__global__ void __launch_bounds__(64) k_init(BuildArgs a) {
  __shared__ InitLds U;
  LdsRPos<float>* const Lf = U.f;
  LdsRPos<double>& Ld = U.d;
  __shared__ InitBox cur[kInitCap], nxt[kInitCap];
  __shared__ Stage S;
  __shared__ int res_status[kGroups], res_settled[kGroups];
  const int tid = threadIdx.x, g = tid / kGroup, lane = tid % kGroup;
  const uint32_t n = a.C->n_init;
  stage_reset(S, tid);
  wave_sync();
  for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
    const uint32_t t = a.init_q[it];
    const TupleGeom<float> Gf = tuple_geom<float>(a.sc, t);
    const TupleGeom<double> Gd = tuple_geom<double>(a.sc, t);
    int ncur = 1;
    if (tid == 0) cur[0] = InitBox{0u, 0u};
    wave_sync();
    bool dead = false;
    for (int level = 1; level <= a.init_levels; ++level) {
      bool all_settled = true;
      for (int j = 0; j < ncur; ++j) all_settled = all_settled && cur[j].settled;
      if (all_settled) break;
      int nn = 0;
      bool over = false;
      for (int j = 0; j < ncur && !over; ++j) {
        const InitBox b = cur[j];
        if (b.settled) {
          if (tid == 0) nxt[nn] = b;
          ++nn;
          over = nn > a.init_pieces;
          continue;
        }
        const int cl = int(b.code >> 28) + 1;
        const uint32_t iu = (b.code >> 14) & 0x3fffu, iv = b.code & 0x3fffu;
        const float w = ldexpf(1.f, -cl);
        const uint32_t cu = 2 * iu + (g >> 1), cv = 2 * iv + (g & 1);
        wave_sync();
        const BoxOut o = eval_box_r<float, false, LdsRPos<float>, kGroup>(Gf, cu * w, (cu + 1) * w, cv * w,
                                                                          (cv + 1) * w, false, Lf[g], lane);
        if (lane == 0) {
          res_status[g] = o.status;
          res_settled[g] = o.settled ? 1 : 0;
        }
        wave_sync();
        for (int ch = 0; ch < kGroups; ++ch) {
          if (res_status[ch] != 2) continue;
          const double wd = ldexp(1.0, -cl);
          const uint32_t du = 2 * iu + (ch >> 1), dv = 2 * iv + (ch & 1);
          wave_sync();
          const BoxOut od = eval_box_r<double, false>(Gd, du * wd, (du + 1) * wd, dv * wd, (dv + 1) * wd, true, Ld, tid);
          wave_sync();
          if (tid == 0) {
            res_status[ch] = od.status;
            res_settled[ch] = od.settled ? 1 : 0;
          }
          wave_sync();
        }
        for (int ch = 0; ch < kGroups && !over; ++ch) {
          if (res_status[ch] != 1) continue;
          if (tid == 0)
            nxt[nn] = InitBox{uint32_t(cl) << 28 | (2 * iu + (ch >> 1)) << 14 | (2 * iv + (ch & 1)),
                              uint32_t(res_settled[ch])};
          ++nn;
          over = nn > a.init_pieces;
        }
      }
      wave_sync();
      if (over) break;
      if (nn == 0) {
        dead = true;
        break;
      }
      for (int j = tid; j < nn; j += BBC_WAVE) cur[j] = nxt[j];
      ncur = nn;
      wave_sync();
    }
    if (!dead && tid == 0) {
      float u0 = 1.f, u1 = 0.f, v0 = 1.f, v1 = 0.f;
      for (int j = 0; j < ncur; ++j) {
        const int bl = int(cur[j].code >> 28);
        const float ww = ldexpf(1.f, -bl);
        const uint32_t iu = (cur[j].code >> 14) & 0x3fffu, iv = cur[j].code & 0x3fffu;
        u0 = fminf(u0, iu * ww);
        u1 = fmaxf(u1, (iu + 1) * ww);
        v0 = fminf(v0, iv * ww);
        v1 = fmaxf(v1, (iv + 1) * ww);
      }
      push_root(a, t, make_float4(u0, u1, v0, v1), S);
    }
    wave_sync();
    if (stage_full(S)) stage_flush<BBC_WAVE>(a, 0, S, tid);
  }
  stage_flush<BBC_WAVE>(a, 0, S, tid);
}

__global__ void __launch_bounds__(kInitRRThreads) k_init_rr(BuildArgs a) {
  __shared__ LdsRR<double> L;
  __shared__ InitBox cur[kInitCap], nxt[kInitCap];
  __shared__ Stage S;
  const int lane = threadIdx.x;
  const uint32_t n = a.C->n_init;
  stage_reset(S, lane);
  wave_sync();
  for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
    const uint32_t t = a.init_q[it];
    const TupleGeom<double> Gd = tuple_geom<double>(a.sc, t);
    auto ev = [&](int cl, uint32_t cu, uint32_t cv) {
      const double wd = ldexp(1.0, -cl);
      return eval_box_rr<double, false, kInitRRThreads>(Gd, cu * wd, (cu + 1) * wd, cv * wd, (cv + 1) * wd, L, lane);
    };
    init_one<kInitRRThreads>(a, t, ev, cur, nxt, lane, S);
  }
  stage_flush<kInitRRThreads>(a, 0, S, lane);
}

__global__ void __launch_bounds__(64) k_init_ra(BuildArgs a) {
  __shared__ LdsRA<double, false> L;
  __shared__ InitBox cur[kInitCap], nxt[kInitCap];
  __shared__ Stage S;
  const int lane = threadIdx.x;
  const uint32_t n = a.C->n_init;
  stage_reset(S, lane);
  wave_sync();
  for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
    const uint32_t t = a.init_q[it];
    const TupleGeom<double> Gd = tuple_geom<double>(a.sc, t);
    auto ev = [&](int cl, uint32_t cu, uint32_t cv) {
      const double wd = ldexp(1.0, -cl);
      return eval_box_ra<double, false, BBC_WAVE>(Gd, cu * wd, (cu + 1) * wd, cv * wd, (cv + 1) * wd, L, lane);
    };
    init_one(a, t, ev, cur, nxt, lane, S);
  }
  stage_flush<BBC_WAVE>(a, 0, S, lane);
}

__global__ void __launch_bounds__(64) k_init_t(BuildArgs a) {
  __shared__ LdsT<double, false> L;
  __shared__ InitBox cur[kInitCap], nxt[kInitCap];
  __shared__ Stage S;
  const int lane = threadIdx.x;
  const uint32_t n = a.C->n_init;
  stage_reset(S, lane);
  wave_sync();
  for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
    const uint32_t t = a.init_q[it];
    const TupleGeom<double> Gd = tuple_geom<double>(a.sc, t);
    auto ev = [&](int cl, uint32_t cu, uint32_t cv) {
      const double wd = ldexp(1.0, -cl);
      return eval_box_t<double, false, BBC_WAVE>(Gd, cu * wd, (cu + 1) * wd, cv * wd, (cv + 1) * wd, true, a.flags, L,
                                                 lane);
    };
    init_one(a, t, ev, cur, nxt, lane, S);
  }
  stage_flush<BBC_WAVE>(a, 0, S, lane);
}

// One box of the adaptive subdivision (Sec. 6.1): stop when the clipped
// position bound's area is below sigma, when E_hi / E_lo < alpha, or at the
// depth cap; otherwise split at the midpoint into four.
template <class T, class Ev>
__device__ void subdiv_one(const BuildArgs& a, QItem it, int depth, Ev ev, int lane, uint32_t* n_boxes, Stage& S) {
  const TupleGeom<T> G = tuple_geom<T>(a.sc, it.tuple);
  const float4 r = a.root[it.tuple];
  const uint32_t iu = it.code >> kCodeBits, iv = it.code & ((1u << kCodeBits) - 1);
  const T fu = (T(r.y) - T(r.x)) * T(ldexpf(1.f, -depth)), fv = (T(r.w) - T(r.z)) * T(ldexpf(1.f, -depth));
  const T u0 = T(r.x) + T(iu) * fu, u1 = T(r.x) + T(iu + 1) * fu;
  const T v0 = T(r.z) + T(iv) * fv, v1 = T(r.z) + T(iv + 1) * fv;
  const BoxOut o = ev(G, u0, u1, v0, v1);
  ++*n_boxes;
  if (lane != 0) return;
  if (o.status == 2) {
    const uint32_t i = atomicAdd(&a.C->fcount[depth], 1u);
    if (i < a.fq_cap)
      a.fq[i] = it;
    else
      atomicOr(&a.C->overflow, 8u);
    return;
  }
  if (o.status == 0) return;
  const float area = (o.uk[1] - o.uk[0]) * (o.uk[3] - o.uk[2]);
  bool stop = depth >= a.max_depth;
  if (!(a.flags & BBC_FLAG_FIXED_DEPTH)) {
    stop = stop || area < a.sigma;
    stop = stop || (o.E[0] > 0.f && isfinite(o.E[1]) && o.E[1] < a.alpha * o.E[0]);
  }
  if (stop) {
    const uint32_t k = S.n_leaf++;
    S.lt[k] = it.tuple;
    S.lc[k] = uint32_t(depth) << 28 | it.code;
    S.lu[k] = make_float4(o.uk[0], o.uk[1], o.uk[2], o.uk[3]);
    S.le[k] = make_float2(o.E[0], o.E[1]);
    if (isinf(o.E[1])) ++S.n_inf;
    S.max_depth = max(S.max_depth, uint32_t(depth));
    return;
  }
  for (uint32_t ch = 0; ch < 4; ++ch)
    S.item[S.n_item++] = QItem{it.tuple, (2 * iu + (ch >> 1)) << kCodeBits | (2 * iv + (ch & 1))};
}

// The per-box loop of the subdivision kernels: children go to depth + 1.
template <int NT, class Ev>
__device__ void subdiv_loop(const BuildArgs& a, int depth, Ev ev, int lane, Stage& S) {
  stage_reset(S, lane);
  wave_sync();
  const uint32_t n = min(a.C->qcount[depth], a.q_cap);
  uint32_t boxes = 0;
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    subdiv_one<double>(a, a.qin[i], depth, ev, lane, &boxes, S);
    wave_sync();
    if (stage_full(S)) stage_flush<NT>(a, depth + 1, S, lane);
  }
  stage_flush<NT>(a, depth + 1, S, lane);
  if (lane == 0 && boxes) atomicAdd(&a.C->n_boxes, boxes);
}

// The subdivision loop of the single-reflection chain with child records: a
// box at depth > 0 is bounded from the record its parent wrote (REC,
// eval_box_r_rec), a box at depth 0 from its corners;
// a box that is split reserves its children's four queue slots with one
// atomic and writes their records (split_box_r) next to them.  Decisions,
// leaves and children are those of subdiv_one.
template <bool REC, class Lds>
__device__ void subdiv_loop_split(const BuildArgs& a, int depth, Lds& L, Stage& S, int lane) {
  __shared__ uint32_t base;
  stage_reset(S, lane);
  wave_sync();
  const uint32_t nq = min(a.C->qcount[depth], a.q_cap);
  // REC: items past the record capacity have no record: the build is redone
  // with room for them
  if (REC && nq > a.srec_cap && blockIdx.x == 0 && lane == 0) atomicOr(&a.C->overflow, 32u);
  const uint32_t n = REC ? min(nq, a.srec_cap) : nq;
  uint32_t boxes = 0;
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const QItem it = a.qin[i];
    const float4 r = a.root[it.tuple];
    const uint32_t iu = it.code >> kCodeBits, iv = it.code & ((1u << kCodeBits) - 1);
    const double fu = (double(r.y) - double(r.x)) * double(ldexpf(1.f, -depth));
    const double fv = (double(r.w) - double(r.z)) * double(ldexpf(1.f, -depth));
    const double u0 = double(r.x) + double(iu) * fu, u1 = double(r.x) + double(iu + 1) * fu;
    const double v0 = double(r.z) + double(iv) * fv, v1 = double(r.z) + double(iv + 1) * fv;
    BoxTheta<double> th{};
    BoxOut o;
    if constexpr (REC)  // the record holds all the box needs from its tuple
      o = eval_box_r_rec<double>(a.srec_in + size_t(i) * kRecR, u0, v0, L, &th, lane);
    else
      o = eval_box_r<double, true>(tuple_geom<double>(a.sc, it.tuple), u0, u1, v0, v1, true, L, lane, &th);
    ++boxes;
    bool split = false;
    if (o.status == 2 && lane == 0) {  // not with final bounds; kept as in subdiv_one
      const uint32_t k = atomicAdd(&a.C->fcount[depth], 1u);
      if (k < a.fq_cap)
        a.fq[k] = it;
      else
        atomicOr(&a.C->overflow, 8u);
    }
    if (o.status == 1) {
      const float area = (o.uk[1] - o.uk[0]) * (o.uk[3] - o.uk[2]);
      bool stop = depth >= a.max_depth;
      if (!(a.flags & BBC_FLAG_FIXED_DEPTH)) {
        stop = stop || area < a.sigma;
        stop = stop || (o.E[0] > 0.f && isfinite(o.E[1]) && o.E[1] < a.alpha * o.E[0]);
      }
      if (stop) {
        if (lane == 0) {
          const uint32_t k = S.n_leaf++;
          S.lt[k] = it.tuple;
          S.lc[k] = uint32_t(depth) << 28 | it.code;
          S.lu[k] = make_float4(o.uk[0], o.uk[1], o.uk[2], o.uk[3]);
          S.le[k] = make_float2(o.E[0], o.E[1]);
          if (isinf(o.E[1])) ++S.n_inf;
          S.max_depth = max(S.max_depth, uint32_t(depth));
        }
      } else {
        split = true;
      }
    }
    if (split) {  // wave-uniform
      if (lane == 0) {
        base = atomicAdd(&a.C->qcount[depth + 1], 4u);
        if (base + 4u > a.q_cap) atomicOr(&a.C->overflow, 1u);
      }
      wave_sync();
      const uint32_t b0 = base;
      if (lane < 4 && b0 + uint32_t(lane) < a.q_cap)
        a.qout[b0 + lane] =
            QItem{it.tuple, (2 * iu + (uint32_t(lane) >> 1)) << kCodeBits | (2 * iv + (uint32_t(lane) & 1u))};
      if (a.srec_out && b0 + 4u <= a.srec_cap) split_box_r<double>(L, th, a.srec_out + size_t(b0) * kRecR, lane);
    }
    wave_sync();
    if (stage_full(S)) stage_flush<BBC_WAVE>(a, depth + 1, S, lane);
  }
  stage_flush<BBC_WAVE>(a, depth + 1, S, lane);
  if (lane == 0 && boxes) atomicAdd(&a.C->n_boxes, boxes);
}

// Subdivision boxes carry the irradiance bound, whose denominator det M has
// coefficients that cancel by two to five orders of magnitude; they are
// evaluated in FP64, which on this GPU issues at the rate of unpacked FP32.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_subdiv(BuildArgs a, int depth) {
  __shared__ LdsR<double> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_r<double, true>(G, u0, u1, v0, v1, true, L, lane);
  };
  subdiv_loop<BBC_WAVE>(a, depth, ev, lane, S);
}

// The same boxes bounded from their parents' split polynomials
// (BBC_TUNE_SUBDIV_SPLIT).
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_subdiv_split(BuildArgs a, int depth) {
  __shared__ LdsR<double> L;
  __shared__ Stage S;
  subdiv_loop_split<false>(a, depth, L, S, threadIdx.x);
}
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_subdiv_rec(BuildArgs a, int depth) {
  __shared__ LdsRRec<double> L;
  __shared__ Stage S;
  subdiv_loop_split<true>(a, depth, L, S, threadIdx.x);
}

// A two-reflection subdivision box also carries the irradiance bound, whose
// det M of degree (46, 46) takes ~90 KB of LDS: one box per compute unit,
// eight waves on it (two per SIMD hide more of each step's latency than one:
// the facing-walls build went from 0.90 to 0.78 s).
constexpr int kSubdivRRThreads = 512;
__global__ void __launch_bounds__(kSubdivRRThreads) k_subdiv_rr(BuildArgs a, int depth) {
  __shared__ LdsRR<double, true> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_rr<double, true, kSubdivRRThreads>(G, u0, u1, v0, v1, L, lane, a.red);
  };
  subdiv_loop<kSubdivRRThreads>(a, depth, ev, lane, S);
}

// The same box evaluation as a called function (BBC_TUNE_RR_OUTLINED): the
// workgroup's LDS block and the reduction buffers of the helpers it calls
// are then reached through the LDS lowering of non-kernel functions rather
// than fixed offsets; the builds must be identical.
__device__ __noinline__ BoxOut eval_box_rr_called(const TupleGeom<double>& G, double u0, double u1, double v0,
                                                  double v1, LdsRR<double, true>& L, int lane, const double* red) {
  return eval_box_rr<double, true, kSubdivRRThreads>(G, u0, u1, v0, v1, L, lane, red);
}
__global__ void __launch_bounds__(kSubdivRRThreads) k_subdiv_rr_called(BuildArgs a, int depth) {
  __shared__ LdsRR<double, true> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_rr_called(G, u0, u1, v0, v1, L, lane, a.red);
  };
  subdiv_loop<kSubdivRRThreads>(a, depth, ev, lane, S);
}

// An area-light reflection box (four axes, det M of degree (10,10,3,3)) takes
// ~70 KB of LDS: four waves share it.
constexpr int kSubdivRAThreads = 256;
__global__ void __launch_bounds__(kSubdivRAThreads) k_subdiv_ra(BuildArgs a, int depth) {
  __shared__ LdsRA<double, true> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_ra<double, true, kSubdivRAThreads>(G, u0, u1, v0, v1, L, lane);
  };
  subdiv_loop<kSubdivRAThreads>(a, depth, ev, lane, S);
}

// A refraction box takes ~1.5 Mflop of FP64 over ~90 KB of LDS, so one box
// fills a compute unit: four waves share it with the explicit irradiance
// bound, eight with the implicit one (its many small steps hide more latency
// with two waves per SIMD: 1.26 -> 0.97 s per water build, while the explicit
// bound's large convolutions gain nothing from the extra waves).
constexpr int kSubdivTThreads = 256, kSubdivTImplicitThreads = 512;
template <int NT>
__global__ void __launch_bounds__(NT) k_subdiv_t(BuildArgs a, int depth) {
  __shared__ LdsT<double, true> L;
  __shared__ Stage S;
  const int lane = threadIdx.x;
  auto ev = [&](const TupleGeom<double>& G, double u0, double u1, double v0, double v1) {
    return eval_box_t<double, true, NT>(G, u0, u1, v0, v1, true, a.flags, L, lane);
  };
  subdiv_loop<NT>(a, depth, ev, lane, S);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

bbc_status launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return BBC_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3(unsigned(blocks)), dim3(256), 0, s, p, v, n);
  BBC_HIP(hipGetLastError());
  return BBC_OK;
}

// Workgroups of `kernel` (64 threads) that stay resident together on the
// device: the persistent kernels stride statically over their items, so a
// grid of exactly one round has no tail of late-starting workgroups.
template <class K>
static bbc_status resident_grid(K kernel, int slot, int dev, int n_cu, unsigned* out) {
  static std::atomic<unsigned> cache[64][4];
  if (dev < 64 && cache[dev][slot].load() > 0u) {
    *out = cache[dev][slot].load();
    return BBC_OK;
  }
  int per_cu = 0;
  BBC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), 64, 0));
  *out = unsigned(std::max(1, per_cu)) * unsigned(std::max(1, n_cu));
  if (dev < 64) cache[dev][slot].store(*out);
  return BBC_OK;
}

// The degree-reduction table of eval_box_rr: P, the pseudo-inverse of the
// elevation matrix E from degree 16 to 46 (least squares through a
// Householder QR factorisation of E in long double: each column of P solves
// min |E x - e_t|), then E itself, then C(46, i).
static std::vector<double> make_reduction_table() {
  constexpr int n = kRedN, m = kRedM;
  auto C = [](int a, int b) {
    long double r = 1.0L;
    for (int k = 1; k <= b; ++k) r = r * (a - b + k) / k;
    return r;
  };
  std::vector<long double> R(size_t(n) * m, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j)
      if (i - j >= 0 && i - j <= kRedFrom - kRedTo)
        R[size_t(i) * m + j] = C(kRedFrom - kRedTo, i - j) * C(kRedTo, j) / C(kRedFrom, i);
  std::vector<double> out(static_cast<size_t>(kRedTable), 0.0);
  for (int i = 0; i < n * m; ++i) out[size_t(m) * n + i] = double(R[size_t(i)]);
  std::vector<std::vector<long double>> V(m);
  std::vector<long double> vn(m);
  for (int k = 0; k < m; ++k) {  // Householder reflector zeroing column k below the diagonal
    long double nr = 0.0L;
    for (int i = k; i < n; ++i) nr += R[size_t(i) * m + k] * R[size_t(i) * m + k];
    nr = sqrtl(nr);
    const long double alpha = R[size_t(k) * m + k] > 0 ? -nr : nr;
    V[k].assign(size_t(n - k), 0.0L);
    for (int i = k; i < n; ++i) V[k][size_t(i - k)] = R[size_t(i) * m + k];
    V[k][0] -= alpha;
    vn[k] = 0.0L;
    for (long double x : V[k]) vn[k] += x * x;
    for (int j = k; j < m; ++j) {
      long double d = 0.0L;
      for (int i = k; i < n; ++i) d += V[k][size_t(i - k)] * R[size_t(i) * m + j];
      for (int i = k; i < n; ++i) R[size_t(i) * m + j] -= 2.0L * d * V[k][size_t(i - k)] / vn[k];
    }
  }
  std::vector<long double> y(n), x(m);
  for (int t = 0; t < n; ++t) {
    std::fill(y.begin(), y.end(), 0.0L);
    y[size_t(t)] = 1.0L;
    for (int k = 0; k < m; ++k) {  // y = Q^T e_t
      long double d = 0.0L;
      for (int i = k; i < n; ++i) d += V[k][size_t(i - k)] * y[size_t(i)];
      for (int i = k; i < n; ++i) y[size_t(i)] -= 2.0L * d * V[k][size_t(i - k)] / vn[k];
    }
    for (int r = m - 1; r >= 0; --r) {  // R x = (Q^T e_t)[0, m)
      long double acc = y[size_t(r)];
      for (int c = r + 1; c < m; ++c) acc -= R[size_t(r) * m + c] * x[size_t(c)];
      x[size_t(r)] = acc / R[size_t(r) * m + r];
    }
    for (int r = 0; r < m; ++r) out[size_t(r) * n + t] = double(x[size_t(r)]);
  }
  for (int i = 0; i < n; ++i) out[size_t(2 * m * n + i)] = double(C(kRedFrom, i));
  return out;
}

bbc_status launch_build(Bounds* b, hipStream_t s) {
  BuildArgs a{};
  a.sc = b->scene;
  a.n_tuples = b->n_tuples;
  a.max_depth = b->params.max_depth;
  a.init_levels = b->params.init_levels;
  a.init_pieces = b->params.init_pieces;
  a.flags = b->params.flags;
  a.sigma = b->params.sigma;
  a.alpha = b->params.alpha;
  a.C = static_cast<BuildCounters*>(b->counters.p);
  a.root = static_cast<float4*>(b->root.p);
  a.init_q = static_cast<uint32_t*>(b->init_q.p);
  a.l0f_q = static_cast<uint32_t*>(b->l0f_q.p);
  a.fq = static_cast<QItem*>(b->fq.p);
  a.q_cap = uint32_t(b->q_cap);
  a.fq_cap = uint32_t(b->fq_cap);
  a.leaf_cap = uint32_t(b->leaf_cap);
  a.lt = static_cast<uint32_t*>(b->lt.p);
  a.lc = static_cast<uint32_t*>(b->lc.p);
  a.lu = static_cast<float4*>(b->lu.p);
  a.le = static_cast<float2*>(b->le.p);
  a.red = nullptr;
  a.srec_in = nullptr;
  a.srec_out = nullptr;
  a.srec_cap = 0;
  const bool split_rec = b->tune.subdiv_split && b->scene.chain == BBC_CHAIN_R && !b->scene.eedge;
  if (split_rec) {
    // a multiple of four: children come four at a time from qcount 0
    if (b->srec_cap == 0) {
      const size_t want = b->tune.subdiv_split > 1 ? size_t(b->tune.subdiv_split) : size_t(1) << 16;
      b->srec_cap = uint32_t(std::max<size_t>(std::min(b->q_cap, want), 4)) & ~3u;
    }
    const uint32_t cap = b->srec_cap;
    for (DevBuf& d : b->srec) {
      bbc_status e = ensure(d, size_t(cap) * kRecR * sizeof(double), b);
      if (e) return e;
    }
    b->srec_cap = cap;
    a.srec_cap = cap;
  }
  if ((a.flags & BBC_FLAG_DEGREE_REDUCTION) && b->scene.chain == BBC_CHAIN_RR) {
    if (!b->red_ready) {
      static const std::vector<double> table = make_reduction_table();
      bbc_status e = ensure(b->red_tab, table.size() * sizeof(double), b);
      if (e) return e;
      BBC_HIP(hipMemcpyAsync(b->red_tab.p, table.data(), table.size() * sizeof(double), hipMemcpyHostToDevice, s));
      b->red_ready = true;
    }
    a.red = static_cast<const double*>(b->red_tab.p);
  }
  int dev = 0;
  BBC_HIP(hipGetDevice(&dev));
  int n_cu = 256;
  BBC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  // persistent grids: a fixed number per compute unit when tuned, else one
  // resident round of each kernel
  const int per_cu = b->tune.build_grid_per_cu;
  unsigned g_fp64 = unsigned(n_cu) * 16u, g_init = g_fp64, g_sub = g_fp64;
  if (per_cu > 0) {
    g_fp64 = g_init = g_sub = unsigned(n_cu) * unsigned(per_cu);
  } else if (b->scene.chain == BBC_CHAIN_R && !b->scene.eedge) {
    bbc_status e = resident_grid(k_init, 0, dev, n_cu, &g_init);
    if (!e) e = resident_grid(k_subdiv, 1, dev, n_cu, &g_sub);
    if (!e) e = resident_grid(k_level0_fp64, 2, dev, n_cu, &g_fp64);
    if (e) return e;
  }
  const unsigned persistent = g_sub;
  // the record-path subdivision: one resident round (its own occupancy)
  unsigned g_rec = 0;
  if (b->tune.subdiv_split && b->scene.chain == BBC_CHAIN_R && !b->scene.eedge) {
    bbc_status e = resident_grid(k_subdiv_rec, 3, dev, n_cu, &g_rec);
    if (e) return e;
  }

  const bool timed = b->tune.timing && b->bev[0];
  b->subdiv_launches = a.max_depth + 1;
  // the whole launch sequence (counter reset, level 0, domain
  // initialisation, one subdivision launch per depth) on stream cs
  auto enqueue = [&](hipStream_t cs) -> bbc_status {
    bbc_status st = launch_fill_u32(static_cast<uint32_t*>(b->counters.p), 0u, sizeof(BuildCounters) / 4, cs);
    if (st) return st;
    a.qin = nullptr;
    a.qout = static_cast<QItem*>(b->q[0].p);
    const unsigned g0 = unsigned(std::max<int64_t>(1, std::min<int64_t>(b->n_tuples, int64_t(n_cu) * 64)));
    const bool refr = b->scene.chain == BBC_CHAIN_T, rr = b->scene.chain == BBC_CHAIN_RR;
    const bool area = b->scene.eedge != nullptr;
    if (area) {
      hipLaunchKernelGGL(k_level0_ra, dim3(g0), dim3(64), 0, cs, a);
    } else if (rr) {
      hipLaunchKernelGGL(k_level0_rr, dim3(g0), dim3(kInitRRThreads), 0, cs, a);
    } else if (refr) {
      hipLaunchKernelGGL(k_level0_t, dim3(g0), dim3(64), 0, cs, a);
    } else {
      hipLaunchKernelGGL(k_level0, dim3(g0), dim3(64), 0, cs, a);
      BBC_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_level0_fp64, dim3(g_fp64), dim3(64), 0, cs, a);
    }
    BBC_HIP(hipGetLastError());
    if (a.init_levels > 0) {
      if (area)
        hipLaunchKernelGGL(k_init_ra, dim3(persistent), dim3(64), 0, cs, a);
      else if (rr)
        hipLaunchKernelGGL(k_init_rr, dim3(persistent), dim3(kInitRRThreads), 0, cs, a);
      else if (refr)
        hipLaunchKernelGGL(k_init_t, dim3(persistent), dim3(64), 0, cs, a);
      else
        hipLaunchKernelGGL(k_init, dim3(g_init), dim3(64), 0, cs, a);
      BBC_HIP(hipGetLastError());
    }
    if (timed) BBC_HIP(hipEventRecord(b->bev[0], cs));
    for (int d = 0; d <= a.max_depth; ++d) {
      a.qin = static_cast<QItem*>(b->q[d & 1].p);
      a.qout = static_cast<QItem*>(b->q[(d + 1) & 1].p);
      if (split_rec) {  // records follow the queues' parity; none at depth 0
        a.srec_in = d > 0 ? static_cast<const double*>(b->srec[d & 1].p) : nullptr;
        a.srec_out = static_cast<double*>(b->srec[(d + 1) & 1].p);
      }
      if (area)
        hipLaunchKernelGGL(k_subdiv_ra, dim3(unsigned(n_cu) * 2u), dim3(kSubdivRAThreads), 0, cs, a, d);
      else if (rr && b->tune.rr_outlined)
        hipLaunchKernelGGL(k_subdiv_rr_called, dim3(unsigned(n_cu)), dim3(kSubdivRRThreads), 0, cs, a, d);
      else if (rr)
        hipLaunchKernelGGL(k_subdiv_rr, dim3(unsigned(n_cu)), dim3(kSubdivRRThreads), 0, cs, a, d);
      else if (refr && (a.flags & BBC_FLAG_IMPLICIT_IRR))
        hipLaunchKernelGGL(k_subdiv_t<kSubdivTImplicitThreads>, dim3(unsigned(n_cu) * 2u), dim3(kSubdivTImplicitThreads),
                           0, cs, a, d);
      else if (refr)
        hipLaunchKernelGGL(k_subdiv_t<kSubdivTThreads>, dim3(unsigned(n_cu) * 2u), dim3(kSubdivTThreads), 0, cs, a, d);
      else if (split_rec && d > 0)
        hipLaunchKernelGGL(k_subdiv_rec, dim3(g_rec), dim3(64), 0, cs, a, d);
      else if (split_rec)
        hipLaunchKernelGGL(k_subdiv_split, dim3(persistent), dim3(64), 0, cs, a, d);
      else
        hipLaunchKernelGGL(k_subdiv, dim3(persistent), dim3(64), 0, cs, a, d);
      BBC_HIP(hipGetLastError());
    }
    if (timed) {
      BBC_HIP(hipEventRecord(b->bev[1], cs));
      b->bev_recorded = true;
    }
    return BBC_OK;
  };
  // BBC_TUNE_BUILD_GRAPH: the sequence captured into the handle's build graph
  // and replayed (not with timing, whose events stay direct launches)
  if (b->tune.build_graph && !timed) return run_as_graph(b->bgraph, s, enqueue);
  return enqueue(s);
}

}  // namespace bbc
