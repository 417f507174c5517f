// Wave-cooperative Bernstein tensor arithmetic in LDS (gfx950, wave64).
//
// Representation.  A tensor-product polynomial of degree (D1, D2) on a box is
// held in *scaled* Bernstein form s_ij = C(D1,i) C(D2,j) b_ij, where b_ij are
// its Bernstein coefficients (Sec. 4.1, Eq. 1).  In this form the product of
// two polynomials is a plain 2-D convolution of their scaled coefficients, and
// raising the degree by one along an axis is the Pascal sum s'_i = s_{i-1} + s_i.
// Ratios b_i(p) / b_i(q) of two polynomials of equal degree are unchanged by
// the scaling, so the rational bound of Eq. eq_bbound reads directly off the
// scaled coefficients.
//
// Error control.  Every tensor carries, next to its values v, a magnitude
// companion m >= 0 (the same computation on absolute values) and a wave-uniform
// factor theta such that |computed - exact| <= theta * m holds coefficient-wise.
// Bounds built from (v +- theta m) intervals are therefore rounded outward.
//
// Layout: lanes stride over output coefficients; one workgroup is one wave, so
// callers put wave_sync() between dependent steps.
#pragma once
#include "dev_common.hpp"

namespace bbc {

template <class T, int N>
struct Ten {
  T v[N];
  T m[N];
};

// Conservative safety factor on magnitudes (they are themselves rounded).
template <class T>
__device__ __forceinline__ T safe_err(T theta, T m) {
  return theta * m * T(1.0009765625) + T(1e-30);
}

// C (=|+=) sgn * conv(A, B).  Degrees (A1,A2) x (B1,B2) -> (A1+B1, A2+B2).
// Each lane owns output coefficients and loops over the smaller operand.
template <int A1, int A2, int B1, int B2, bool ACC, class T, int NT = BBC_WAVE>
__device__ __forceinline__ void conv(const T* __restrict__ av, const T* __restrict__ am, const T* __restrict__ bv,
                                     const T* __restrict__ bm, T* __restrict__ cv, T* __restrict__ cm, T sgn,
                                     int lane) {
  if constexpr ((A1 + 1) * (A2 + 1) > (B1 + 1) * (B2 + 1)) {
    conv<B1, B2, A1, A2, ACC, T, NT>(bv, bm, av, am, cv, cm, sgn, lane);
  } else {
    constexpr int C2 = A2 + B2;
    constexpr int N = (A1 + B1 + 1) * (C2 + 1);
    for (int o = lane; o < N; o += NT) {
      const int k = o / (C2 + 1), l = o - k * (C2 + 1);
      T s = 0, sm = 0;
#pragma unroll
      for (int i = 0; i <= A1; ++i) {
#pragma unroll
        for (int j = 0; j <= A2; ++j) {
          const int kb = k - i, lb = l - j;
          if (kb >= 0 && kb <= B1 && lb >= 0 && lb <= B2) {
            s = fma(av[i * (A2 + 1) + j], bv[kb * (B2 + 1) + lb], s);
            sm = fma(am[i * (A2 + 1) + j], bm[kb * (B2 + 1) + lb], sm);
          }
        }
      }
      if (ACC) {
        cv[o] = fma(sgn, s, cv[o]);
        cm[o] = cm[o] + sm;
      } else {
        cv[o] = sgn * s;
        cm[o] = sm;
      }
    }
  }
}

// conv() with the LDS reads of each output batched: the terms go CH at a
// time (eight by default) through clamped, in-range indices (the loads issued
// together, a scheduling barrier, then the products), and a select leaves the
// partial sums unchanged for the terms outside the output's support.  The sums are
// those of conv(), valid terms in (i, j) order, bit for bit; conv() instead
// branches around each term and waits for each load, which leaves a box's
// chain of small steps bound by LDS latency.  The batched form takes more
// registers (up to 2 CH doubles of one chunk in flight): the reflection and
// refraction boxes gain from it (subdivision 14 % and 25 % faster), the
// two-reflection box, whose kernels then spill, keeps conv() (8 % slower
// batched).
template <int A1, int A2, int B1, int B2, bool ACC, class T, int NT = BBC_WAVE, int CH = 8>
__device__ __forceinline__ void conv_b(const T* __restrict__ av, const T* __restrict__ am, const T* __restrict__ bv,
                                       const T* __restrict__ bm, T* __restrict__ cv, T* __restrict__ cm, T sgn,
                                       int lane) {
  if constexpr ((A1 + 1) * (A2 + 1) > (B1 + 1) * (B2 + 1)) {
    conv_b<B1, B2, A1, A2, ACC, T, NT, CH>(bv, bm, av, am, cv, cm, sgn, lane);
  } else {
    constexpr int C2 = A2 + B2;
    constexpr int N = (A1 + B1 + 1) * (C2 + 1);
    constexpr int NA = (A1 + 1) * (A2 + 1);
    for (int o = lane; o < N; o += NT) {
      const int k = o / (C2 + 1), l = o - k * (C2 + 1);
      T s = 0, sm = 0;
#pragma unroll
      for (int t0 = 0; t0 < NA; t0 += CH) {
        T xb[CH], xm[CH];
        bool ok[CH];
#pragma unroll
        for (int u = 0; u < CH && t0 + u < NA; ++u) {
          const int i = (t0 + u) / (A2 + 1), j = (t0 + u) % (A2 + 1);
          const int kb = k - i, lb = l - j;
          const int b = min(max(kb, 0), B1) * (B2 + 1) + min(max(lb, 0), B2);
          ok[u] = kb >= 0 && kb <= B1 && lb >= 0 && lb <= B2;
          xb[u] = bv[b];
          xm[u] = bm[b];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < CH && t0 + u < NA; ++u) {
          const T ts = fma(av[t0 + u], xb[u], s);
          const T tm = fma(am[t0 + u], xm[u], sm);
          s = ok[u] ? ts : s;
          sm = ok[u] ? tm : sm;
        }
      }
      if (ACC) {
        cv[o] = fma(sgn, s, cv[o]);
        cm[o] = cm[o] + sm;
      } else {
        cv[o] = sgn * s;
        cm[o] = sm;
      }
    }
  }
}

// Relative error factor of a convolution result from its operands'.
template <int A1, int A2, int B1, int B2, class T>
__device__ __forceinline__ T conv_theta(T ta, T tb) {
  constexpr int n = ((A1 < B1 ? A1 : B1) + 1) * ((A2 < B2 ? A2 : B2) + 1);
  return ta + tb + ta * tb + T(n + 1) * Eps<T>::u;
}

// out (=|+=) sum_k alpha_k A_k over K tensors of N coefficients.
template <int N, int K, bool ACC, class T, int NT = BBC_WAVE>
__device__ __forceinline__ void combo(const T* const* av, const T* const* am, const T* alpha, T* __restrict__ ov,
                                      T* __restrict__ om, int lane) {
  for (int o = lane; o < N; o += NT) {
    T s = ACC ? ov[o] : T(0), sm = ACC ? om[o] : T(0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      s = fma(alpha[k], av[k][o], s);
      sm = fma(fabs(alpha[k]), am[k][o], sm);
    }
    ov[o] = s;
    om[o] = sm;
  }
}

// combo() with each output's K reads issued together before the sums (the
// same sums in k order), for the same chain as conv_b.
template <int N, int K, bool ACC, class T, int NT = BBC_WAVE>
__device__ __forceinline__ void combo_b(const T* const* av, const T* const* am, const T* alpha, T* __restrict__ ov,
                                        T* __restrict__ om, int lane) {
  for (int o = lane; o < N; o += NT) {
    T x[K], xm[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k] = av[k][o];
      xm[k] = am[k][o];
    }
    T s = ACC ? ov[o] : T(0), sm = ACC ? om[o] : T(0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      s = fma(alpha[k], x[k], s);
      sm = fma(fabs(alpha[k]), xm[k], sm);
    }
    ov[o] = s;
    om[o] = sm;
  }
}

// Degree elevation by one along both axes: (D1, D2) -> (D1+1, D2+1), scaled form.
template <int D1, int D2, class T, int NT = BBC_WAVE>
__device__ __forceinline__ void elev11(const T* __restrict__ iv, const T* __restrict__ im, T* __restrict__ ov,
                                       T* __restrict__ om, int lane) {
  constexpr int E2 = D2 + 1, N = (D1 + 2) * (D2 + 2);
  for (int o = lane; o < N; o += NT) {
    const int i = o / (E2 + 1), j = o - i * (E2 + 1);
    T a = 0, b = 0, c = 0, d = 0, ma = 0, mb = 0, mc = 0, md = 0;
    if (i <= D1 && j <= D2) { a = iv[i * (D2 + 1) + j]; ma = im[i * (D2 + 1) + j]; }
    if (i >= 1 && j <= D2) { b = iv[(i - 1) * (D2 + 1) + j]; mb = im[(i - 1) * (D2 + 1) + j]; }
    if (i <= D1 && j >= 1) { c = iv[i * (D2 + 1) + j - 1]; mc = im[i * (D2 + 1) + j - 1]; }
    if (i >= 1 && j >= 1) { d = iv[(i - 1) * (D2 + 1) + j - 1]; md = im[(i - 1) * (D2 + 1) + j - 1]; }
    ov[o] = (a + b) + (c + d);
    om[o] = (ma + mb) + (mc + md);
  }
}

// elev11() with its four reads unconditional (clamped indices; the terms
// outside the input taken as zero by a select), for the same chain as conv_b.
template <int D1, int D2, class T, int NT = BBC_WAVE>
__device__ __forceinline__ void elev11_b(const T* __restrict__ iv, const T* __restrict__ im, T* __restrict__ ov,
                                         T* __restrict__ om, int lane) {
  constexpr int E2 = D2 + 1, N = (D1 + 2) * (D2 + 2);
  for (int o = lane; o < N; o += NT) {
    const int i = o / (E2 + 1), j = o - i * (E2 + 1);
    const int i0 = min(i, D1), i1 = max(i - 1, 0), j0 = min(j, D2), j1 = max(j - 1, 0);
    const bool ka = i <= D1 && j <= D2, kb = i >= 1 && j <= D2, kc = i <= D1 && j >= 1, kd = i >= 1 && j >= 1;
    const T a = iv[i0 * (D2 + 1) + j0], b = iv[i1 * (D2 + 1) + j0];
    const T c = iv[i0 * (D2 + 1) + j1], d = iv[i1 * (D2 + 1) + j1];
    const T ma = im[i0 * (D2 + 1) + j0], mb = im[i1 * (D2 + 1) + j0];
    const T mc = im[i0 * (D2 + 1) + j1], md = im[i1 * (D2 + 1) + j1];
    ov[o] = ((ka ? a : T(0)) + (kb ? b : T(0))) + ((kc ? c : T(0)) + (kd ? d : T(0)));
    om[o] = ((ka ? ma : T(0)) + (kb ? mb : T(0))) + ((kc ? mc : T(0)) + (kd ? md : T(0)));
  }
}

// Degree elevation by (R1, R2): (D1, D2) -> (D1+R1, D2+R2), scaled form (the
// product with the constant 1 written at degree (R1, R2), whose scaled
// coefficients are C(R1,i) C(R2,j)).
template <int D1, int D2, int R1, int R2, class T, int NT = BBC_WAVE>
__device__ __forceinline__ void elev_by(const T* __restrict__ iv, const T* __restrict__ im, T* __restrict__ ov,
                                        T* __restrict__ om, int lane) {
  constexpr int E2 = D2 + R2, N = (D1 + R1 + 1) * (E2 + 1);
  for (int o = lane; o < N; o += NT) {
    const int k = o / (E2 + 1), l = o - k * (E2 + 1);
    T s = 0, sm = 0;
#pragma unroll
    for (int i = 0; i <= R1; ++i) {
#pragma unroll
      for (int j = 0; j <= R2; ++j) {
        const int a = k - i, b = l - j;
        if (a >= 0 && a <= D1 && b >= 0 && b <= D2) {
          const T w = T(binom_i(R1, i) * binom_i(R2, j));
          s = fma(w, iv[a * (D2 + 1) + b], s);
          sm = fma(w, im[a * (D2 + 1) + b], sm);
        }
      }
    }
    ov[o] = s;
    om[o] = sm;
  }
}

// Result of the rational range bound (Sec. 4.1, Eq. eq_bbound and its
// sign-failure rules).
enum : int { kDirect = 0, kSplit = 1, kUnbounded = 2 };
template <class T>
struct RB {
  int kind;
  T lo, hi;        // kDirect: [lo, hi]; kSplit: (-inf, lo] U [hi, +inf)
  bool uncertain;  // a coefficient's sign could not be decided at this precision
};

template <class T>
__device__ __forceinline__ T down(T x) {
  return x - fabs(x) * T(4) * Eps<T>::u - T(1e-38);
}
template <class T>
__device__ __forceinline__ T up(T x) {
  return x + fabs(x) * T(4) * Eps<T>::u + T(1e-38);
}

// Interval quotient [pl,ph] / [ql,qh] for a denominator interval free of zero.
template <class T>
__device__ __forceinline__ void iv_div(T pl, T ph, T ql, T qh, T* lo, T* hi) {
  const T a = pl / ql, b = pl / qh, c = ph / ql, d = ph / qh;
  *lo = down(min(min(a, b), min(c, d)));
  *hi = up(max(max(a, b), max(c, d)));
}

// Bound of p/q over N coefficient pairs of equal degree, produced on the fly
// by get(o, p, ep, q, eq) (value and absolute error bound of the o-th scaled
// coefficient of each).  With final = true a sign that cannot be decided
// counts as a sign failure; otherwise it is reported through `uncertain` so
// the caller can redo the box at higher precision.
template <class T, int NT = BBC_WAVE, class Get>
__device__ RB<T> ratio_bound_fn(int N, Get get, bool final, int lane) {
  bool q_pos = true, q_neg = true, q_anyp = false, q_anyn = false;
  bool p_pos = true, p_neg = true, p_anyp = false, p_anyn = false;
  for (int o = lane; o < N; o += NT) {
    T p, ep, q, eq;
    get(o, p, ep, q, eq);
    const bool qp = q - eq > T(0), qn = q + eq < T(0);
    const bool pp = p - ep > T(0), pn = p + ep < T(0);
    q_pos &= qp; q_neg &= qn; q_anyp |= qp; q_anyn |= qn;
    p_pos &= pp; p_neg &= pn; p_anyp |= pp; p_anyn |= pn;
  }
  q_pos = blk_all<NT>(q_pos);
  q_neg = blk_all<NT>(q_neg);
  const bool q_mixed = blk_any<NT>(q_anyp) && blk_any<NT>(q_anyn);
  p_pos = blk_all<NT>(p_pos);
  p_neg = blk_all<NT>(p_neg);
  const bool p_mixed = blk_any<NT>(p_anyp) && blk_any<NT>(p_anyn);
  RB<T> r;
  r.uncertain = false;
  const T inf = T(INFINITY);
  if (q_pos || q_neg) {
    T lo = inf, hi = -inf;
    for (int o = lane; o < N; o += NT) {
      T p, ep, q, eq;
      get(o, p, ep, q, eq);
      T a, b;
      iv_div(p - ep, p + ep, q - eq, q + eq, &a, &b);
      lo = min(lo, a);
      hi = max(hi, b);
    }
    r.kind = kDirect;
    r.lo = blk_min<NT>(lo);
    r.hi = blk_max<NT>(hi);
    return r;
  }
  if (!q_mixed && !final) {
    r.kind = kUnbounded;
    r.lo = r.hi = 0;
    r.uncertain = true;
    return r;
  }
  if (p_pos || p_neg) {
    // reciprocal rule: bound q/p in [a, b], then invert
    T lo = inf, hi = -inf;
    for (int o = lane; o < N; o += NT) {
      T p, ep, q, eq;
      get(o, p, ep, q, eq);
      T a, b;
      iv_div(q - eq, q + eq, p - ep, p + ep, &a, &b);
      lo = min(lo, a);
      hi = max(hi, b);
    }
    const T a = blk_min<NT>(lo), b = blk_max<NT>(hi);
    if (a > T(0) || b < T(0)) {
      r.kind = kDirect;
      r.lo = down(T(1) / b);
      r.hi = up(T(1) / a);
    } else if (a < T(0) && b > T(0)) {
      r.kind = kSplit;
      r.lo = up(T(1) / a);   // (-inf, 1/a]: widen toward +
      r.hi = down(T(1) / b); // [1/b, inf): widen toward -
    } else if (a == T(0) && b > T(0)) {
      r.kind = kDirect;
      r.lo = down(T(1) / b);
      r.hi = inf;
    } else if (b == T(0) && a < T(0)) {
      r.kind = kDirect;
      r.lo = -inf;
      r.hi = up(T(1) / a);
    } else {
      r.kind = kUnbounded;
      r.lo = r.hi = 0;
    }
    return r;
  }
  r.kind = kUnbounded;
  r.lo = r.hi = 0;
  r.uncertain = !p_mixed && !final;
  return r;
}

// Bound of p/q from N stored scaled coefficients of equal degree.
template <int N, class T, int NT = BBC_WAVE>
__device__ RB<T> ratio_bound(const T* pv, const T* pm, T tp, const T* qv, const T* qm, T tq, bool final, int lane) {
  return ratio_bound_fn<T, NT>(
      N,
      [&](int o, T& p, T& ep, T& q, T& eq) {
        q = qv[o];
        eq = safe_err(tq, qm[o]);
        p = pv[o];
        ep = safe_err(tp, pm[o]);
      },
      final, lane);
}

// Range [lo, hi] of a single polynomial from its scaled coefficients.
template <int D1, int D2, class T, int NT = BBC_WAVE>
__device__ void poly_range(const T* v, const T* m, T th, T* lo, T* hi, int lane) {
  constexpr int N = (D1 + 1) * (D2 + 1);
  T l = T(INFINITY), h = -T(INFINITY);
  for (int o = lane; o < N; o += NT) {
    const int i = o / (D2 + 1), j = o - i * (D2 + 1);
    const T w = T(binom_i(D1, i) * binom_i(D2, j));
    const T e = safe_err(th, m[o]);
    l = min(l, down((v[o] - e) / w));
    h = max(h, up((v[o] + e) / w));
  }
  *lo = blk_min<NT>(l);
  *hi = blk_max<NT>(h);
}

// Clip a ratio bound to [0, 1]; false when the intersection is empty.
template <class T>
__device__ __forceinline__ bool clip01(const RB<T>& rb, T* lo, T* hi) {
  if (rb.kind == kDirect) {
    *lo = max(rb.lo, T(0));
    *hi = min(rb.hi, T(1));
    return *lo <= *hi;
  }
  if (rb.kind == kSplit) {
    const bool left = rb.lo >= T(0), right = rb.hi <= T(1);
    if (!left && !right) return false;
    *lo = left ? T(0) : max(rb.hi, T(0));
    *hi = right ? T(1) : min(rb.lo, T(1));
    return true;
  }
  *lo = T(0);
  *hi = T(1);
  return true;
}

// Bound of |f| from a ratio bound of f.
template <class T>
__device__ __forceinline__ void abs_bound(const RB<T>& rb, T* lo, T* hi) {
  const T inf = T(INFINITY);
  if (rb.kind == kDirect) {
    const T a = fabs(rb.lo), b = fabs(rb.hi);
    *lo = (rb.lo <= T(0) && rb.hi >= T(0)) ? T(0) : min(a, b);
    *hi = max(a, b);
  } else if (rb.kind == kSplit) {
    *hi = inf;
    *lo = (rb.lo >= T(0) || rb.hi <= T(0)) ? T(0) : min(-rb.lo, rb.hi);
  } else {
    *lo = T(0);
    *hi = inf;
  }
}

}  // namespace bbc
