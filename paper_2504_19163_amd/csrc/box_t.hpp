// Position and irradiance bound of one box of a single-refraction tuple,
// evaluated by NT lanes (one or several waves) in FP64 with its polynomials in LDS (Sec. 4.2-4.4).
//
// Refraction (Eq. eq_refr_rational) writes the outgoing direction as
//   d~ = eta ((n.n) d0 - (d0.n) n) - sqrt(beta) n,
//   beta = (1 - eta^2)(n.n)(d0.d0) + eta^2 (d0.n)^2,
// which is rational only after sqrt(beta) is replaced by a linear function of
// beta plus a remainder (Sec. 4.3).  On a box with beta in [blo, bhi], blo > 0,
// the secant r(beta) = a beta + b through (blo, sqrt(blo)) and (bhi, sqrt(bhi))
// satisfies sqrt(beta) - r(beta) in [0, dhi], dhi = (sqrt(bhi) - sqrt(blo))^2 /
// (4 (sqrt(blo) + sqrt(bhi))), so sqrt(beta) = a beta + b + (1 - xi1) dlo +
// xi1 dhi for some remainder variable xi1 in [0, 1].  The derivative of
// sqrt(beta) along u is beta_u w with w = 1 / (2 sqrt(beta)) in
// [1 / (2 sqrt(bhi)), 1 / (2 sqrt(blo))]; a second remainder variable xi2
// carries w.  Every polynomial is therefore a tensor in (u, v, xi1, xi2),
// held here as slices over (xi1, xi2) of scaled (u, v) tensors; a product is a
// convolution over the slice indices of 2-D convolutions (scaled form in all
// four axes).
//
// det M uses the receiver-origin-free form of the reflection evaluator,
//   det M = -(Q^2 D0 + Q Tn D1 + Tn^2 D2),  D0 = det[e1, e2, d~],
//   D1 = det[d~_u, e2, d~] + det[e1, d~_v, d~],  D2 = det[d~_u, d~_v, d~],
// with d~_u = A_u - w beta_u n, A_u = (eta((n.n) d0 - (d0.n) n))_u - r n_u.
// Because det[n, n, .] = 0 the w^2 terms of D2 vanish identically, so det M
// has degree one in xi2 (three in xi1, fifteen in u and v).  It and Q^3 are
// raised to degree (16, 16, 3, 2) -- the degree of the cofactor expansion of M
// with the total derivatives written out -- on the fly inside the ratio bound.
#pragma once
#include "../../include/bbc.h"
#include "bern_dev.hpp"
#include "box_r.hpp"
#include "geom_dev.hpp"

namespace bbc {

// LDS layout (offsets in elements; a tensor of n coefficients takes 2n: its
// values, then their magnitudes).
struct TLay {
  // position part
  static constexpr int N = 0, D0v = 24, S = 48, SF1 = 72;               // (1,1) x 3 components
  static constexpr int NN = 96, DN = 114, DD = 132, BETA = 150;         // (2,2) x 3, (4,4)
  static constexpr int DT0 = 200;                                        // (3,3) x 3
  static constexpr int RT = 296;                                         // (4,4) x 2 xi1-slices
  static constexpr int DT = 396;                                         // (5,5,1) x 3
  static constexpr int Q = 828, TN = 972;                                // (5,5,1), (1,1)
  static constexpr int POS_END = 980;
  // irradiance part
  static constexpr int NNU = 980, NNV = 988, DDU = 996, DDV = 1004, DNU = 1012, DNV = 1020, G = 1028;
  static constexpr int BU = 1036, BV = 1068;                             // (3,3)
  static constexpr int DT0U = 1100, DT0V = 1154;                         // (2,2) x 3
  static constexpr int AU = 1208, AV = 1508;                             // (4,4,1) x 3
  static constexpr int DZ = 1808;                                        // D0 (5,5,1)
  static constexpr int Q2 = 1952, QT = 2678, T2 = 2874;                  // (10,10,2), (6,6,1), (2,2)
  static constexpr int D1 = 2892, D2 = 4092, Q3 = 2892;                  // (9,9,2,1), (13,13,3,1); Q3 reuses D1
  static constexpr int IRR_TMP = 7228;
  // scratch (offsets relative to the scratch base)
  static constexpr int CC = 0, PU = 432, PV = 628, QE = 824, TNE = 1020;  // position phase: 1164
  static constexpr int ND = 0, YP = 588, BNU = 2388;                      // irradiance: (6,6,1)x3, (9,9,2)x3, (4,4)x3
  static constexpr int X = 2538, E1ND = 2970, Z1 = 3166;                   // D1 phase
  static constexpr int BVAU = 2538, Z = 3306;                              // D2 phase: (7,7,1)x3, (13,13,2)
  static constexpr int DETM = 0;                                           // (15,15,3,1): 4096
  static constexpr int TMP_IRR = 4482, TMP_POS = 1164;
};


// A tensor of n coefficients (all slices) at offset off.
template <class T>
struct TP {
  T* v;
  T* m;
};
template <class T>
__device__ __forceinline__ TP<T> tpat(T* base, int off, int n) {
  return TP<T>{base + off, base + off + n};
}
template <class T>
__device__ __forceinline__ TP<T> slice(TP<T> t, int s, int n) {
  return TP<T>{t.v + s * n, t.m + s * n};
}
template <int NT, class T>
__device__ __forceinline__ void zero(TP<T> t, int n, int lane) {
  for (int o = lane; o < n; o += NT) {
    t.v[o] = T(0);
    t.m[o] = T(0);
  }
}
// c (=|+=) sgn a*b over 2-D slices of degrees (A1,A2), (B1,B2)
template <int A1, int A2, int B1, int B2, bool ACC, int NT, class T>
__device__ __forceinline__ void cv(TP<T> a, TP<T> b, TP<T> c, T sgn, int lane) {
  conv<A1, A2, B1, B2, ACC, T, NT>(a.v, a.m, b.v, b.m, c.v, c.m, sgn, lane);
}
// the same with the batched reads of conv_b (the refraction chain's box)
template <int A1, int A2, int B1, int B2, bool ACC, int NT, class T>
__device__ __forceinline__ void cvb(TP<T> a, TP<T> b, TP<T> c, T sgn, int lane) {
  conv_b<A1, A2, B1, B2, ACC, T, NT>(a.v, a.m, b.v, b.m, c.v, c.m, sgn, lane);
}
// error factor of a sum of `pairs` slice products
template <int A1, int A2, int B1, int B2, class T>
__device__ __forceinline__ T th_conv(T ta, T tb, int pairs) {
  constexpr int n = ((A1 < B1 ? A1 : B1) + 1) * ((A2 < B2 ? A2 : B2) + 1);
  return ta + tb + ta * tb + T(n * pairs + 2) * Eps<T>::u;
}

// ---- 4-D tensors of the implicit-differentiation bound: axes (u, v, u_k,
// v_k), values only in scaled Bernstein form, row-major with u slowest.
template <int D1, int D2, int D3, int D4>
struct N4 {
  static constexpr int n = (D1 + 1) * (D2 + 1) * (D3 + 1) * (D4 + 1);
};

// c (=|+=) sgn * a * b: a 4-D convolution, each output's valid index ranges in
// runtime loops.
template <int A1, int A2, int A3, int A4, int B1, int B2, int B3, int B4, bool ACC, int NT, class T>
__device__ __forceinline__ void cv4(const T* a, const T* b, T* c, T sgn, int lane) {
  constexpr int C2 = A2 + B2, C3 = A3 + B3, C4 = A4 + B4;
  constexpr int N = (A1 + B1 + 1) * (C2 + 1) * (C3 + 1) * (C4 + 1);
  for (int o = lane; o < N; o += NT) {
    int r = o;
    const int l = r % (C4 + 1);
    r /= C4 + 1;
    const int k = r % (C3 + 1);
    r /= C3 + 1;
    const int j = r % (C2 + 1), i = r / (C2 + 1);
    T s = T(0);
#pragma nounroll
    for (int i1 = max(0, i - B1); i1 <= min(i, A1); ++i1)
#pragma nounroll
      for (int j1 = max(0, j - B2); j1 <= min(j, A2); ++j1)
        for (int k1 = max(0, k - B3); k1 <= min(k, A3); ++k1)
          for (int l1 = max(0, l - B4); l1 <= min(l, A4); ++l1)
            s = fma(a[((i1 * (A2 + 1) + j1) * (A3 + 1) + k1) * (A4 + 1) + l1],
                    b[(((i - i1) * (B2 + 1) + (j - j1)) * (B3 + 1) + (k - k1)) * (B4 + 1) + (l - l1)], s);
    c[o] = ACC ? fma(sgn, s, c[o]) : sgn * s;
  }
}

// Local derivative along axis AX: s'_t = (t + 1) s_{t+1} - (D - t) s_t.
template <int D1, int D2, int D3, int D4, int AX, int NT, class T>
__device__ __forceinline__ void deriv4(const T* in, T* out, int lane) {
  constexpr int O1 = D1 - (AX == 0), O2 = D2 - (AX == 1), O3 = D3 - (AX == 2), O4 = D4 - (AX == 3);
  constexpr int DA = AX == 0 ? D1 : (AX == 1 ? D2 : (AX == 2 ? D3 : D4));
  for (int o = lane; o < (O1 + 1) * (O2 + 1) * (O3 + 1) * (O4 + 1); o += NT) {
    int r = o;
    const int l = r % (O4 + 1);
    r /= O4 + 1;
    const int k = r % (O3 + 1);
    r /= O3 + 1;
    const int j = r % (O2 + 1), i = r / (O2 + 1);
    const int t = AX == 0 ? i : (AX == 1 ? j : (AX == 2 ? k : l));
    auto at = [&](int ii, int jj, int kk, int ll) { return in[((ii * (D2 + 1) + jj) * (D3 + 1) + kk) * (D4 + 1) + ll]; };
    const T hi = at(i + (AX == 0), j + (AX == 1), k + (AX == 2), l + (AX == 3));
    out[o] = fma(T(t + 1), hi, -(T(DA - t) * at(i, j, k, l)));
  }
}

// Elevation by (R1, R2, R3, R4): the product with the constant 1 at that
// degree, whose scaled coefficients are C(R1,a) C(R2,b) C(R3,c) C(R4,d).
template <int D1, int D2, int D3, int D4, int R1, int R2, int R3, int R4, int NT, class T>
__device__ __forceinline__ void elev4(const T* in, T* out, int lane) {
  constexpr int E1 = D1 + R1, E2 = D2 + R2, E3 = D3 + R3, E4 = D4 + R4;
  for (int o = lane; o < (E1 + 1) * (E2 + 1) * (E3 + 1) * (E4 + 1); o += NT) {
    int r = o;
    const int l = r % (E4 + 1);
    r /= E4 + 1;
    const int k = r % (E3 + 1);
    r /= E3 + 1;
    const int j = r % (E2 + 1), i = r / (E2 + 1);
    T s = T(0);
    for (int a = 0; a <= R1; ++a)
      for (int b = 0; b <= R2; ++b)
        for (int c = 0; c <= R3; ++c)
          for (int d = 0; d <= R4; ++d) {
            const int ii = i - a, jj = j - b, kk = k - c, ll = l - d;
            if (ii >= 0 && ii <= D1 && jj >= 0 && jj <= D2 && kk >= 0 && kk <= D3 && ll >= 0 && ll <= D4)
              s = fma(T(binom_i(R1, a) * binom_i(R2, b) * binom_i(R3, c) * binom_i(R4, d)),
                      in[((ii * (D2 + 1) + jj) * (D3 + 1) + kk) * (D4 + 1) + ll], s);
          }
    out[o] = s;
  }
}

// ---- the same 4-D operations with magnitude companions (values at t.v,
// magnitudes at t.m; |computed - exact| <= theta * m coefficient-wise, as for
// the 2-D tensors of bern_dev.hpp), so the bounds built from them are rounded
// outward.
template <int A1, int A2, int A3, int A4, int B1, int B2, int B3, int B4, bool ACC, int NT, class T>
__device__ __forceinline__ void cv4m(TP<T> a, TP<T> b, TP<T> c, T sgn, int lane) {
  constexpr int C2 = A2 + B2, C3 = A3 + B3, C4 = A4 + B4;
  constexpr int N = (A1 + B1 + 1) * (C2 + 1) * (C3 + 1) * (C4 + 1);
  for (int o = lane; o < N; o += NT) {
    int r = o;
    const int l = r % (C4 + 1);
    r /= C4 + 1;
    const int k = r % (C3 + 1);
    r /= C3 + 1;
    const int j = r % (C2 + 1), i = r / (C2 + 1);
    T s = T(0), sm = T(0);
#pragma nounroll
    for (int i1 = max(0, i - B1); i1 <= min(i, A1); ++i1)
#pragma nounroll
      for (int j1 = max(0, j - B2); j1 <= min(j, A2); ++j1)
        for (int k1 = max(0, k - B3); k1 <= min(k, A3); ++k1)
          for (int l1 = max(0, l - B4); l1 <= min(l, A4); ++l1) {
            const int ia = ((i1 * (A2 + 1) + j1) * (A3 + 1) + k1) * (A4 + 1) + l1;
            const int ib = (((i - i1) * (B2 + 1) + (j - j1)) * (B3 + 1) + (k - k1)) * (B4 + 1) + (l - l1);
            s = fma(a.v[ia], b.v[ib], s);
            sm = fma(a.m[ia], b.m[ib], sm);
          }
    if (ACC) {
      c.v[o] = fma(sgn, s, c.v[o]);
      c.m[o] = fma(fabs(sgn), sm, c.m[o]);
    } else {
      c.v[o] = sgn * s;
      c.m[o] = fabs(sgn) * sm;
    }
  }
}
// cv4m() with the two inner axes unrolled: for each (i1, j1) the
// (A3 + 1)(A4 + 1) reads go out together through clamped indices, then the
// products, a select skipping the terms outside the output's support (the
// same sums in the same order, bit for bit).  Used by the implicit-
// differentiation and area-light boxes (their subdivision 4 % and 37 %
// faster than with cv4m).
template <int A1, int A2, int A3, int A4, int B1, int B2, int B3, int B4, bool ACC, int NT, class T>
__device__ __forceinline__ void cv4m_b(TP<T> a, TP<T> b, TP<T> c, T sgn, int lane) {
  constexpr int C2 = A2 + B2, C3 = A3 + B3, C4 = A4 + B4;
  constexpr int N = (A1 + B1 + 1) * (C2 + 1) * (C3 + 1) * (C4 + 1);
  constexpr int NI = (A3 + 1) * (A4 + 1);
  for (int o = lane; o < N; o += NT) {
    int r = o;
    const int l = r % (C4 + 1);
    r /= C4 + 1;
    const int k = r % (C3 + 1);
    r /= C3 + 1;
    const int j = r % (C2 + 1), i = r / (C2 + 1);
    T s = T(0), sm = T(0);
#pragma nounroll
    for (int i1 = max(0, i - B1); i1 <= min(i, A1); ++i1)
#pragma nounroll
      for (int j1 = max(0, j - B2); j1 <= min(j, A2); ++j1) {
        T xa[NI], xam[NI], xb[NI], xbm[NI];
        bool ok[NI];
#pragma unroll
        for (int t = 0; t < NI; ++t) {
          const int k1 = t / (A4 + 1), l1 = t % (A4 + 1);
          const int kb = k - k1, lb = l - l1;
          ok[t] = kb >= 0 && kb <= B3 && lb >= 0 && lb <= B4;
          const int ia = ((i1 * (A2 + 1) + j1) * (A3 + 1) + k1) * (A4 + 1) + l1;
          const int ib = (((i - i1) * (B2 + 1) + (j - j1)) * (B3 + 1) + min(max(kb, 0), B3)) * (B4 + 1) +
                         min(max(lb, 0), B4);
          xa[t] = a.v[ia];
          xam[t] = a.m[ia];
          xb[t] = b.v[ib];
          xbm[t] = b.m[ib];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < NI; ++t) {
          const T ts = fma(xa[t], xb[t], s), tm = fma(xam[t], xbm[t], sm);
          s = ok[t] ? ts : s;
          sm = ok[t] ? tm : sm;
        }
      }
    if (ACC) {
      c.v[o] = fma(sgn, s, c.v[o]);
      c.m[o] = fma(fabs(sgn), sm, c.m[o]);
    } else {
      c.v[o] = sgn * s;
      c.m[o] = fabs(sgn) * sm;
    }
  }
}
// Error factor of a 4-D product accumulated into a sum of `terms` products.
template <int A1, int A2, int A3, int A4, int B1, int B2, int B3, int B4, class T>
__device__ __forceinline__ T th_cv4(T ta, T tb, int terms) {
  constexpr int n = ((A1 < B1 ? A1 : B1) + 1) * ((A2 < B2 ? A2 : B2) + 1) * ((A3 < B3 ? A3 : B3) + 1) *
                    ((A4 < B4 ? A4 : B4) + 1);
  return ta + tb + ta * tb + T(n + terms + 2) * Eps<T>::u;
}

template <int D1, int D2, int D3, int D4, int AX, int NT, class T>
__device__ __forceinline__ void deriv4m(TP<T> in, TP<T> out, int lane) {
  constexpr int O1 = D1 - (AX == 0), O2 = D2 - (AX == 1), O3 = D3 - (AX == 2), O4 = D4 - (AX == 3);
  constexpr int DA = AX == 0 ? D1 : (AX == 1 ? D2 : (AX == 2 ? D3 : D4));
  for (int o = lane; o < (O1 + 1) * (O2 + 1) * (O3 + 1) * (O4 + 1); o += NT) {
    int r = o;
    const int l = r % (O4 + 1);
    r /= O4 + 1;
    const int k = r % (O3 + 1);
    r /= O3 + 1;
    const int j = r % (O2 + 1), i = r / (O2 + 1);
    const int t = AX == 0 ? i : (AX == 1 ? j : (AX == 2 ? k : l));
    auto at = [&](int ii, int jj, int kk, int ll) { return ((ii * (D2 + 1) + jj) * (D3 + 1) + kk) * (D4 + 1) + ll; };
    const int ih = at(i + (AX == 0), j + (AX == 1), k + (AX == 2), l + (AX == 3)), il = at(i, j, k, l);
    out.v[o] = fma(T(t + 1), in.v[ih], -(T(DA - t) * in.v[il]));
    out.m[o] = fma(T(t + 1), in.m[ih], T(DA - t) * in.m[il]);
  }
}

template <int D1, int D2, int D3, int D4, int R1, int R2, int R3, int R4, int NT, class T>
__device__ __forceinline__ void elev4m(TP<T> in, TP<T> out, int lane) {
  constexpr int E1 = D1 + R1, E2 = D2 + R2, E3 = D3 + R3, E4 = D4 + R4;
  for (int o = lane; o < (E1 + 1) * (E2 + 1) * (E3 + 1) * (E4 + 1); o += NT) {
    int r = o;
    const int l = r % (E4 + 1);
    r /= E4 + 1;
    const int k = r % (E3 + 1);
    r /= E3 + 1;
    const int j = r % (E2 + 1), i = r / (E2 + 1);
    T s = T(0), sm = T(0);
    for (int a = 0; a <= R1; ++a)
      for (int b = 0; b <= R2; ++b)
        for (int c = 0; c <= R3; ++c)
          for (int d = 0; d <= R4; ++d) {
            const int ii = i - a, jj = j - b, kk = k - c, ll = l - d;
            if (ii >= 0 && ii <= D1 && jj >= 0 && jj <= D2 && kk >= 0 && kk <= D3 && ll >= 0 && ll <= D4) {
              const T w = T(binom_i(R1, a) * binom_i(R2, b) * binom_i(R3, c) * binom_i(R4, d));
              const int ix = ((ii * (D2 + 1) + jj) * (D3 + 1) + kk) * (D4 + 1) + ll;
              s = fma(w, in.v[ix], s);
              sm = fma(w, in.m[ix], sm);
            }
          }
    out.v[o] = s;
    out.m[o] = sm;
  }
}
// elev4m() with its reads eight terms at a time through clamped indices
// (the loads together, then the products; a select skips the terms outside
// the input: the same sums in the same order, bit for bit).  The area-light
// box uses it; the implicit-differentiation bound keeps elev4m(), whose
// elevation by (2, 2, 2, 2) (81 terms per output) runs slower unrolled.
template <int D1, int D2, int D3, int D4, int R1, int R2, int R3, int R4, int NT, class T>
__device__ __forceinline__ void elev4m_b(TP<T> in, TP<T> out, int lane) {
  constexpr int E1 = D1 + R1, E2 = D2 + R2, E3 = D3 + R3, E4 = D4 + R4;
  constexpr int NR = (R1 + 1) * (R2 + 1) * (R3 + 1) * (R4 + 1), CH = 8;
  for (int o = lane; o < (E1 + 1) * (E2 + 1) * (E3 + 1) * (E4 + 1); o += NT) {
    int r = o;
    const int l = r % (E4 + 1);
    r /= E4 + 1;
    const int k = r % (E3 + 1);
    r /= E3 + 1;
    const int j = r % (E2 + 1), i = r / (E2 + 1);
    T s = T(0), sm = T(0);
#pragma unroll
    for (int t0 = 0; t0 < NR; t0 += CH) {
      T x[CH], xm[CH];
      bool ok[CH];
#pragma unroll
      for (int u = 0; u < CH && t0 + u < NR; ++u) {
        const int t = t0 + u;
        const int d = t % (R4 + 1), c = (t / (R4 + 1)) % (R3 + 1), b = (t / ((R4 + 1) * (R3 + 1))) % (R2 + 1),
                  a = t / ((R4 + 1) * (R3 + 1) * (R2 + 1));
        const int ii = i - a, jj = j - b, kk = k - c, ll = l - d;
        ok[u] = ii >= 0 && ii <= D1 && jj >= 0 && jj <= D2 && kk >= 0 && kk <= D3 && ll >= 0 && ll <= D4;
        const int ix = ((min(max(ii, 0), D1) * (D2 + 1) + min(max(jj, 0), D2)) * (D3 + 1) + min(max(kk, 0), D3)) *
                           (D4 + 1) +
                       min(max(ll, 0), D4);
        x[u] = in.v[ix];
        xm[u] = in.m[ix];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < CH && t0 + u < NR; ++u) {
        const int t = t0 + u;
        const int d = t % (R4 + 1), c = (t / (R4 + 1)) % (R3 + 1), b = (t / ((R4 + 1) * (R3 + 1))) % (R2 + 1),
                  a = t / ((R4 + 1) * (R3 + 1) * (R2 + 1));
        const T w = T(binom_i(R1, a) * binom_i(R2, b) * binom_i(R3, c) * binom_i(R4, d));
        const T ts = fma(w, x[u], s), tm = fma(w, xm[u], sm);
        s = ok[u] ? ts : s;
        sm = ok[u] ? tm : sm;
      }
    }
    out.v[o] = s;
    out.m[o] = sm;
  }
}
template <int R1, int R2, int R3, int R4, class T>
__device__ __forceinline__ T th_elev4(T t) {
  return t + T((R1 + 1) * (R2 + 1) * (R3 + 1) * (R4 + 1) + 1) * Eps<T>::u;
}

// Range of a 4-D polynomial from its scaled coefficients and their error
// bounds, rounded outward.
template <int D1, int D2, int D3, int D4, class T, int NT>
__device__ __forceinline__ void range4m(TP<T> t, T th, T* lo, T* hi, int lane) {
  T l = T(INFINITY), h = -T(INFINITY);
  for (int o = lane; o < N4<D1, D2, D3, D4>::n; o += NT) {
    int r = o;
    const int d = r % (D4 + 1);
    r /= D4 + 1;
    const int c = r % (D3 + 1);
    r /= D3 + 1;
    const int b = r % (D2 + 1), a = r / (D2 + 1);
    const T w = T(binom_i(D1, a) * binom_i(D2, b) * binom_i(D3, c) * binom_i(D4, d));
    const T e = safe_err(th, t.m[o]);
    l = min(l, down((t.v[o] - e) / w));
    h = max(h, up((t.v[o] + e) / w));
  }
  *lo = blk_min<NT>(l);
  *hi = blk_max<NT>(h);
}

// Ratio bound of p/q over n coefficient pairs of equal degree with their
// error bounds (Eq. eq_bbound, rounded outward).
template <class T, int NT>
__device__ __forceinline__ RB<T> ratio4m(int n, TP<T> p, T tp, TP<T> q, T tq, bool final, int lane) {
  return ratio_bound_fn<T, NT>(
      n,
      [&](int o, T& pv, T& ep, T& qv, T& eq) {
        pv = p.v[o];
        ep = safe_err(tp, p.m[o]);
        qv = q.v[o];
        eq = safe_err(tq, q.m[o]);
      },
      final, lane);
}

// LDS offsets of the implicit-differentiation tensors, after the position
// part's live linear forms, d0.d0 and n_g.d0 (TLay::G); a tensor of n
// coefficients takes 2n (values, then magnitudes).
struct ILay {
  static constexpr int D1 = TLay::G + 8, C0 = D1 + 96, C1 = C0 + 54, D1D1 = C1 + 216;  // (1,1,1,1)x3, (2,2,0,0)x3, (2,2,1,1)x3, (2,2,2,2)
  static constexpr int C0U = D1D1 + 162, C0V = C0U + 24, C1U = C0V + 24, C1V = C1U + 96;  // (1,1,0,0)x3, (1,1,1,1)x3
  static constexpr int C1K = C1V + 96, C1L = C1K + 24, DE = C1L + 24, D1E = DE + 16;    // (1,1,0,0)x3, (1,1)x2, (1,1,1,1)x4
  static constexpr int GU = D1E + 128, GV = GU + 72, GK = GV + 72, GL = GK + 18;        // (2,2,1,1), (2,2,0,0)
  static constexpr int A0SQ = GL + 18, A0SQE = A0SQ + 50, A1SQ = A0SQE + 200;           // (4,4,0,0), (4,4,1,1), (4,4,2,2)
  static constexpr int SU = A1SQ + 450, SV = SU + 32, TU = SV + 32, TV = TU + 288;       // (3,3,0,0), (3,3,2,2)
  static constexpr int TK = TV + 288, TL = TK + 128, FU = TL + 128, FV = FU + 648;       // (3,3,1,1), (5,5,2,2)
  static constexpr int FK = FV + 648, FL = FK + 288, J1 = FL + 288, JK = J1 + 2048;      // (5,5,1,1), (7,7,3,3)
  static constexpr int J1E = JK + 512, JKE = J1E + 3200, END = JKE + 3200;              // (7,7,1,1), (9,9,3,3) x 2
};

template <class T, bool IRR>
struct LdsT {
  static constexpr int kIrr = TLay::IRR_TMP + TLay::TMP_IRR > ILay::END ? TLay::IRR_TMP + TLay::TMP_IRR : ILay::END;
  T buf[IRR ? kIrr : TLay::POS_END + TLay::TMP_POS];
};

template <class T, bool IRR, int NT>
__device__ BoxOut eval_box_t(const TupleGeom<T>& G, T u0, T u1, T v0, T v1, bool final, int flags, LdsT<T, IRR>& L,
                             int lane) {
  const T eps = Eps<T>::u;
  T* B = L.buf;
  T* Tm = B + (IRR ? TLay::IRR_TMP : TLay::POS_END);  // scratch
  BoxOut out;
  out.status = 0;
  out.settled = false;
  out.uk[0] = 0.f;
  out.uk[1] = 1.f;
  out.uk[2] = 0.f;
  out.uk[3] = 1.f;
  out.E[0] = 0.f;
  out.E[1] = INFINITY;
  if (!G.front || u0 + v0 >= T(1)) return out;
  const T eta = G.eta, e2 = eta * eta, om = T(1) - e2;

  // ---- linear forms n, d0, s at the box corners (scaled = plain at degree 1)
  const V3<T> pmx = G.p0 - G.x0, pmq = G.p0 - G.q0;
  for (int task = lane; task < 36; task += NT) {
    const int which = task / 12, c = (task / 4) % 3, k = task % 4;
    const T u = (k & 2) ? u1 : u0, v = (k & 1) ? v1 : v0;
    T a, b, d;
    if (which == 0) {
      a = comp(G.n0, c); b = comp(G.dn1, c); d = comp(G.dn2, c);
    } else if (which == 1) {
      a = comp(pmx, c); b = comp(G.e1, c); d = comp(G.e2, c);
    } else {
      a = comp(pmq, c); b = comp(G.e1, c); d = comp(G.e2, c);
    }
    const int base = which == 0 ? TLay::N : (which == 1 ? TLay::D0v : TLay::S);
    TP<T> dst = tpat(B, base + 8 * c, 4);
    dst.v[k] = fma(d, v, fma(b, u, a));
    dst.m[k] = fabs(a) + fabs(b) * fabs(u) + fabs(d) * fabs(v);
  }
  const T th_lin = T(4) * eps;
  auto nC = [&](int c) { return tpat(B, TLay::N + 8 * c, 4); };
  auto dC = [&](int c) { return tpat(B, TLay::D0v + 8 * c, 4); };
  auto sC = [&](int c) { return tpat(B, TLay::S + 8 * c, 4); };
  auto sfC = [&](int c) { return tpat(B, TLay::SF1 + 8 * c, 4); };
  auto dtC = [&](int c) { return tpat(B, TLay::DT + 144 * c, 72); };  // both xi1-slices of one component
  wave_sync();

  // ---- s x f1 and the degree-(2,2) products n.n, d0.n, d0.d0
  {
    const T* sv[3] = {sC(0).v, sC(1).v, sC(2).v};
    const T* sm[3] = {sC(0).m, sC(1).m, sC(2).m};
    const V3<T> f1 = G.f1;
    const T ax[3] = {T(0), f1.z, -f1.y}, ay[3] = {-f1.z, T(0), f1.x}, az[3] = {f1.y, -f1.x, T(0)};
    combo_b<4, 3, false, T, NT>(sv, sm, ax, sfC(0).v, sfC(0).m, lane);
    combo_b<4, 3, false, T, NT>(sv, sm, ay, sfC(1).v, sfC(1).m, lane);
    combo_b<4, 3, false, T, NT>(sv, sm, az, sfC(2).v, sfC(2).m, lane);
    const TP<T> nn = tpat(B, TLay::NN, 9), dn = tpat(B, TLay::DN, 9), dd = tpat(B, TLay::DD, 9);
    cvb<1, 1, 1, 1, false, NT>(nC(0), nC(0), nn, T(1), lane);
    cvb<1, 1, 1, 1, false, NT>(dC(0), nC(0), dn, T(1), lane);
    cvb<1, 1, 1, 1, false, NT>(dC(0), dC(0), dd, T(1), lane);
    for (int c = 1; c < 3; ++c) {
      cvb<1, 1, 1, 1, true, NT>(nC(c), nC(c), nn, T(1), lane);
      cvb<1, 1, 1, 1, true, NT>(dC(c), nC(c), dn, T(1), lane);
      cvb<1, 1, 1, 1, true, NT>(dC(c), dC(c), dd, T(1), lane);
    }
  }
  const T th_sf1 = th_lin + T(4) * eps;
  const T th_nn = th_conv<1, 1, 1, 1>(th_lin, th_lin, 3) + T(3) * eps;
  wave_sync();
  const TP<T> nn = tpat(B, TLay::NN, 9), dn = tpat(B, TLay::DN, 9), dd = tpat(B, TLay::DD, 9);
  {
    T lo, hi;
    poly_range<2, 2, T, NT>(dn.v, dn.m, th_nn, &lo, &hi, lane);
    if (lo >= T(0)) return out;  // the light reaches the back of the shading normal everywhere
  }
  // ---- beta and the secant of its square root
  const TP<T> beta = tpat(B, TLay::BETA, 25);
  cvb<2, 2, 2, 2, false, NT>(nn, dd, beta, om, lane);
  cvb<2, 2, 2, 2, true, NT>(dn, dn, beta, e2, lane);
  const T th_beta = th_conv<2, 2, 2, 2>(th_nn, th_nn, 2) + T(4) * eps;
  wave_sync();
  T blo, bhi;
  poly_range<4, 4, T, NT>(beta.v, beta.m, th_beta, &blo, &bhi, lane);
  if (bhi <= T(0)) return out;  // total internal reflection everywhere
  if (blo <= T(0)) {            // the square root cannot be bounded here: universal bound
    out.status = 1;
    return out;
  }
  const bool remainder = !(flags & BBC_FLAG_NO_REMAINDER);
  const T sa = sqrt(blo), sb = sqrt(bhi);
  const T ra = T(1) / (sa + sb), rb = sa * sb / (sa + sb);
  // remainder interval of the computed secant, widened by its rounding
  const T slack = T(16) * eps * sb;
  const T dlo = remainder ? -slack : T(0);
  const T dhi = remainder ? up((sb - sa) * (sb - sa) / (T(4) * (sa + sb))) + slack : T(0);
  const T wlo = remainder ? down(T(0.5) / up(sb)) : ra, whi = remainder ? up(T(0.5) / down(sa)) : ra;
  // rt_k = a beta + b + d_k (xi1-slices k = 0, 1)
  const TP<T> rt = tpat(B, TLay::RT, 50);
  for (int o = lane; o < 50; o += NT) {
    const int k = o / 25, r = o - 25 * k, i = r / 5, j = r - 5 * i;
    const T w = T(binom_i(4, i) * binom_i(4, j));
    const T c = rb + (k ? dhi : dlo);
    rt.v[o] = fma(ra, beta.v[r], c * w);
    rt.m[o] = fma(fabs(ra), beta.m[r], fabs(c) * w);
  }
  const T th_rt = th_beta + T(4) * eps;
  // ---- dt0 = eta ((n.n) d0 - (d0.n) n)
  for (int c = 0; c < 3; ++c) {
    const TP<T> d = tpat(B, TLay::DT0 + 32 * c, 16);
    cvb<2, 2, 1, 1, false, NT>(nn, dC(c), d, eta, lane);
    cvb<2, 2, 1, 1, true, NT>(dn, nC(c), d, -eta, lane);
  }
  const T th_dt0 = th_conv<2, 2, 1, 1>(th_nn, th_lin, 2) + T(3) * eps;
  wave_sync();
  // ---- d~_k = dt0 (raised to (5,5)) - rt_k n
  for (int c = 0; c < 3; ++c) {
    const TP<T> d = tpat(B, TLay::DT0 + 32 * c, 16);
    for (int k = 0; k < 2; ++k) {
      const TP<T> o = slice(dtC(c), k, 36);
      elev_by<3, 3, 2, 2, T, NT>(d.v, d.m, o.v, o.m, lane);
      cvb<4, 4, 1, 1, true, NT>(slice(rt, k, 25), nC(c), o, T(-1), lane);
    }
  }
  const T th_dt = max(th_dt0 + T(10) * eps, th_conv<4, 4, 1, 1>(th_rt, th_lin, 1)) + T(2) * eps;
  wave_sync();

  // ---- cc = d~ x f2, Tn = (s x f1).f2
  const TP<T> Tn = tpat(B, TLay::TN, 4);
  {
    const V3<T> f2 = G.f2;
    const T ax[3] = {T(0), f2.z, -f2.y}, ay[3] = {-f2.z, T(0), f2.x}, az[3] = {f2.y, -f2.x, T(0)};
    const T* al[3] = {ax, ay, az};
    const T* dv[3] = {dtC(0).v, dtC(1).v, dtC(2).v};
    const T* dm[3] = {dtC(0).m, dtC(1).m, dtC(2).m};
    for (int c = 0; c < 3; ++c) {
      const TP<T> cc = tpat(Tm, TLay::CC + 144 * c, 72);
      combo_b<72, 3, false, T, NT>(dv, dm, al[c], cc.v, cc.m, lane);
    }
    const T* sv[3] = {sfC(0).v, sfC(1).v, sfC(2).v};
    const T* sm[3] = {sfC(0).m, sfC(1).m, sfC(2).m};
    const T af2[3] = {f2.x, f2.y, f2.z};
    combo_b<4, 3, false, T, NT>(sv, sm, af2, Tn.v, Tn.m, lane);
  }
  const T th_cc = th_dt + T(3) * eps;
  const T th_Tn = th_sf1 + T(3) * eps;
  wave_sync();
  // ---- Pu = cc.s, Pv = (s x f1).d~, Q = cc.f1 (per xi1-slice)
  const TP<T> Pu = tpat(Tm, TLay::PU, 98), Pv = tpat(Tm, TLay::PV, 98), Q = tpat(B, TLay::Q, 72);
  const TP<T> Qe = tpat(Tm, TLay::QE, 98), Tne = tpat(Tm, TLay::TNE, 72);
  for (int k = 0; k < 2; ++k) {
    for (int c = 0; c < 3; ++c) {
      const TP<T> cc = slice(tpat(Tm, TLay::CC + 144 * c, 72), k, 36);
      if (c == 0) {
        cvb<5, 5, 1, 1, false, NT>(cc, sC(c), slice(Pu, k, 49), T(1), lane);
        cvb<5, 5, 1, 1, false, NT>(slice(dtC(c), k, 36), sfC(c), slice(Pv, k, 49), T(1), lane);
      } else {
        cvb<5, 5, 1, 1, true, NT>(cc, sC(c), slice(Pu, k, 49), T(1), lane);
        cvb<5, 5, 1, 1, true, NT>(slice(dtC(c), k, 36), sfC(c), slice(Pv, k, 49), T(1), lane);
      }
    }
  }
  {
    const T* cvp[3], *cmp[3];
    for (int c = 0; c < 3; ++c) {
      const TP<T> cc = tpat(Tm, TLay::CC + 144 * c, 72);
      cvp[c] = cc.v;
      cmp[c] = cc.m;
    }
    const T af1[3] = {G.f1.x, G.f1.y, G.f1.z};
    combo_b<72, 3, false, T, NT>(cvp, cmp, af1, Q.v, Q.m, lane);
    for (int k = 0; k < 2; ++k) {
      const TP<T> o = slice(Tne, k, 36);
      elev_by<1, 1, 4, 4, T, NT>(Tn.v, Tn.m, o.v, o.m, lane);
    }
  }
  const T th_P = th_conv<5, 5, 1, 1>(th_cc, th_lin, 3) + T(3) * eps;
  const T th_Q = th_cc + T(3) * eps;
  const T th_Tne = th_Tn + T(26) * eps;
  wave_sync();
  for (int k = 0; k < 2; ++k) {
    const TP<T> qi = slice(Q, k, 36), qo = slice(Qe, k, 49);
    elev11_b<5, 5, T, NT>(qi.v, qi.m, qo.v, qo.m, lane);
  }
  const T th_Qe = th_Q + T(4) * eps;
  wave_sync();

  // ---- position bound (Sec. 4.2) and the sign of the ray parameter
  const RB<T> tb = ratio_bound<72, T, NT>(Tne.v, Tne.m, th_Tne, Q.v, Q.m, th_Q, final, lane);
  const RB<T> ub = ratio_bound<98, T, NT>(Pu.v, Pu.m, th_P, Qe.v, Qe.m, th_Qe, final, lane);
  const RB<T> vb = ratio_bound<98, T, NT>(Pv.v, Pv.m, th_P, Qe.v, Qe.m, th_Qe, final, lane);
  if (tb.uncertain || ub.uncertain || vb.uncertain) {
    out.status = 2;
    return out;
  }
  if (tb.kind == kDirect && tb.hi <= T(0)) return out;  // every ray points away from the receiver
  T ulo, uhi, vlo, vhi;
  if (!clip01(ub, &ulo, &uhi) || !clip01(vb, &vlo, &vhi)) return out;
  out.uk[0] = out_lo(ulo);
  out.uk[1] = out_hi(uhi);
  out.uk[2] = out_lo(vlo);
  out.uk[3] = out_hi(vhi);
  out.settled = ub.kind == kDirect && vb.kind == kDirect && ub.lo >= T(0) && ub.hi <= T(1) && vb.lo >= T(0) &&
                vb.hi <= T(1) && tb.kind == kDirect && tb.lo > T(0);
  out.status = 1;
  if constexpr (!IRR) {
    return out;
  } else {
    if (flags & BBC_FLAG_IMPLICIT_IRR) {
      // ---- irradiance by implicit differentiation (Sec. 4.4): F (Snell's law
      // along b) and G (coplanarity) over the box times U_k, |du1/du_k| =
      // |det J_k / det J_1|; b = (1,0,0), (0,1,0), intervals intersected.
      // The partial derivatives of F and G are formed by the product rule from
      // the exact derivatives of the linear forms (d0_u = e1, n_u = dn1,
      // d1_u = -e1, d1_uk = f1, ...), not by differencing F's coefficients: a
      // difference of neighbouring coefficients cancels to O(w) of its terms,
      // and the rounding bound of det J_1 would grow by (degree / w)^2.  det J_1
      // has degree (7,7,3,3) and det J_k (7,7,1,1); both are elevated to
      // (9,9,3,3), the degree at which differencing F would give them, so the
      // coefficient ratios are those of the same polynomials at that degree.
      // Every tensor carries magnitudes; the bound is rounded outward.
      const T wk = uhi - ulo, wl = vhi - vlo;
      if (!(wk > T(0) && wl > T(0))) return out;
      const TP<T> d1 = tpat(B, ILay::D1, 48), c0 = tpat(B, ILay::C0, 27), c1 = tpat(B, ILay::C1, 108);
      const TP<T> d1d1 = tpat(B, ILay::D1D1, 81), g = tpat(B, TLay::G, 4);
      const TP<T> c0u = tpat(B, ILay::C0U, 12), c0v = tpat(B, ILay::C0V, 12);  // (1,1,0,0) x 3
      const TP<T> c1u = tpat(B, ILay::C1U, 48), c1v = tpat(B, ILay::C1V, 48);  // (1,1,1,1) x 3
      const TP<T> c1k = tpat(B, ILay::C1K, 12), c1l = tpat(B, ILay::C1L, 12);  // (1,1,0,0) x 3
      const TP<T> de = tpat(B, ILay::DE, 8);     // d0.e1, d0.e2 (1,1,0,0)
      const TP<T> d1e = tpat(B, ILay::D1E, 64);  // d1.e1, d1.e2, d1.f1, d1.f2 (1,1,1,1)
      const V3<T> e1 = G.e1, e2 = G.e2, dn1 = G.dn1, dn2 = G.dn2, f1 = G.f1, f2 = G.f2;
      {
        const T* dv[3] = {dC(0).v, dC(1).v, dC(2).v};
        const T* dm[3] = {dC(0).m, dC(1).m, dC(2).m};
        const T ag[3] = {G.ng.x, G.ng.y, G.ng.z};
        combo_b<4, 3, false, T, NT>(dv, dm, ag, g.v, g.m, lane);
        const T ae1[3] = {e1.x, e1.y, e1.z}, ae2[3] = {e2.x, e2.y, e2.z};
        combo_b<4, 3, false, T, NT>(dv, dm, ae1, slice(de, 0, 4).v, slice(de, 0, 4).m, lane);
        combo_b<4, 3, false, T, NT>(dv, dm, ae2, slice(de, 1, 4).v, slice(de, 1, 4).m, lane);
        // d1 = x_k - x1 = -(x1 - q0) + u_k f1 + v_k f2 at the 16 corners
        for (int o = lane; o < 48; o += NT) {
          const int c = o / 16, r = o - 16 * c, ij = r / 4, k = (r / 2) & 1, l = r & 1;
          const T uk = k ? uhi : ulo, vk = l ? vhi : vlo;
          d1.v[o] = fma(vk, comp(f2, c), fma(uk, comp(f1, c), -sC(c).v[ij]));
          d1.m[o] = fabs(vk) * fabs(comp(f2, c)) + fabs(uk) * fabs(comp(f1, c)) + sC(c).m[ij];
        }
        // component c of a x n + d0 x m at the four (u, v) corners, for constant a, m
        auto cross_lin = [&](V3<T> a, V3<T> mv, TP<T> dst, int o) {
          const int c = o / 4, ij = o - 4 * c, p = (c + 1) % 3, q = (c + 2) % 3;
          const TP<T> np = nC(p), nq = nC(q), dp = dC(p), dq = dC(q);
          // (a x n)_c = a_p n_q - a_q n_p,  (d0 x m)_c = d0_p m_q - d0_q m_p
          dst.v[o] = fma(comp(a, p), nq.v[ij], -(comp(a, q) * np.v[ij])) +
                     fma(dp.v[ij], comp(mv, q), -(dq.v[ij] * comp(mv, p)));
          dst.m[o] = fabs(comp(a, p)) * nq.m[ij] + fabs(comp(a, q)) * np.m[ij] + dp.m[ij] * fabs(comp(mv, q)) +
                     dq.m[ij] * fabs(comp(mv, p));
        };
        const V3<T> zero{T(0), T(0), T(0)};
        for (int o = lane; o < 12; o += NT) {
          cross_lin(e1, dn1, c0u, o);  // (d0 x n)_u = e1 x n + d0 x dn1
          cross_lin(e2, dn2, c0v, o);
          cross_lin(f1, zero, c1k, o);  // (d1 x n)_uk = f1 x n
          cross_lin(f2, zero, c1l, o);
        }
      }
      const T th_d1 = th_lin + T(3) * eps;
      const T th_g = th_lin + T(8) * eps;
      const T th_de = th_lin + T(5) * eps;
      const T th_c0u = th_lin + T(6) * eps;  // also c1k, c1l
      wave_sync();
      for (int c = 0; c < 3; ++c) {  // c0 = d0 x n, c1 = d1 x n
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        cv4m_b<1, 1, 0, 0, 1, 1, 0, 0, false, NT>(dC(a), nC(b), slice(c0, c, 9), T(1), lane);
        cv4m_b<1, 1, 0, 0, 1, 1, 0, 0, true, NT>(dC(b), nC(a), slice(c0, c, 9), T(-1), lane);
        cv4m_b<1, 1, 1, 1, 1, 1, 0, 0, false, NT>(slice(d1, a, 16), nC(b), slice(c1, c, 36), T(1), lane);
        cv4m_b<1, 1, 1, 1, 1, 1, 0, 0, true, NT>(slice(d1, b, 16), nC(a), slice(c1, c, 36), T(-1), lane);
        if (c == 0)
          cv4m_b<1, 1, 1, 1, 1, 1, 1, 1, false, NT>(slice(d1, c, 16), slice(d1, c, 16), d1d1, T(1), lane);
        else
          cv4m_b<1, 1, 1, 1, 1, 1, 1, 1, true, NT>(slice(d1, c, 16), slice(d1, c, 16), d1d1, T(1), lane);
      }
      // (d1 x n)_u = -e1 x n + d1 x dn1 (the first term constant along u_k, v_k)
      for (int o = lane; o < 48; o += NT) {
        const int c = o / 16, r = o - 16 * c, ij = r / 4, p = (c + 1) % 3, q = (c + 2) % 3;
        const TP<T> np = nC(p), nq = nC(q), dp = slice(d1, p, 16), dq = slice(d1, q, 16);
        c1u.v[o] = fma(comp(e1, q), np.v[ij], -(comp(e1, p) * nq.v[ij])) +
                   fma(dp.v[r], comp(dn1, q), -(dq.v[r] * comp(dn1, p)));
        c1u.m[o] = fabs(comp(e1, q)) * np.m[ij] + fabs(comp(e1, p)) * nq.m[ij] + dp.m[r] * fabs(comp(dn1, q)) +
                   dq.m[r] * fabs(comp(dn1, p));
        c1v.v[o] = fma(comp(e2, q), np.v[ij], -(comp(e2, p) * nq.v[ij])) +
                   fma(dp.v[r], comp(dn2, q), -(dq.v[r] * comp(dn2, p)));
        c1v.m[o] = fabs(comp(e2, q)) * np.m[ij] + fabs(comp(e2, p)) * nq.m[ij] + dp.m[r] * fabs(comp(dn2, q)) +
                   dq.m[r] * fabs(comp(dn2, p));
      }
      {
        const T* dv[3] = {slice(d1, 0, 16).v, slice(d1, 1, 16).v, slice(d1, 2, 16).v};
        const T* dm[3] = {slice(d1, 0, 16).m, slice(d1, 1, 16).m, slice(d1, 2, 16).m};
        const T a0[3] = {e1.x, e1.y, e1.z}, a1[3] = {e2.x, e2.y, e2.z}, a2[3] = {f1.x, f1.y, f1.z},
                a3[3] = {f2.x, f2.y, f2.z};
        combo_b<16, 3, false, T, NT>(dv, dm, a0, slice(d1e, 0, 16).v, slice(d1e, 0, 16).m, lane);
        combo_b<16, 3, false, T, NT>(dv, dm, a1, slice(d1e, 1, 16).v, slice(d1e, 1, 16).m, lane);
        combo_b<16, 3, false, T, NT>(dv, dm, a2, slice(d1e, 2, 16).v, slice(d1e, 2, 16).m, lane);
        combo_b<16, 3, false, T, NT>(dv, dm, a3, slice(d1e, 3, 16).v, slice(d1e, 3, 16).m, lane);
      }
      const T th_c0 = th_cv4<1, 1, 0, 0, 1, 1, 0, 0>(th_lin, th_lin, 2);
      const T th_c1 = th_cv4<1, 1, 1, 1, 1, 1, 0, 0>(th_d1, th_lin, 2);
      const T th_d1d1 = th_cv4<1, 1, 1, 1, 1, 1, 1, 1>(th_d1, th_d1, 3);
      const T th_c1u = th_d1 + T(6) * eps;
      const T th_d1e = th_d1 + T(5) * eps;
      wave_sync();
      // ---- G_u = c0_u . d1 - c0 . e1 (2,2,1,1), G_v likewise, G_uk = c0 . f1,
      // G_vk = c0 . f2 (2,2,0,0)
      const TP<T> gu = tpat(B, ILay::GU, 36), gv = tpat(B, ILay::GV, 36), gk = tpat(B, ILay::GK, 9),
                  gl = tpat(B, ILay::GL, 9);
      for (int c = 0; c < 3; ++c) {
        if (c == 0) {
          cv4m_b<1, 1, 0, 0, 1, 1, 1, 1, false, NT>(slice(c0u, c, 4), slice(d1, c, 16), gu, T(1), lane);
          cv4m_b<1, 1, 0, 0, 1, 1, 1, 1, false, NT>(slice(c0v, c, 4), slice(d1, c, 16), gv, T(1), lane);
        } else {
          cv4m_b<1, 1, 0, 0, 1, 1, 1, 1, true, NT>(slice(c0u, c, 4), slice(d1, c, 16), gu, T(1), lane);
          cv4m_b<1, 1, 0, 0, 1, 1, 1, 1, true, NT>(slice(c0v, c, 4), slice(d1, c, 16), gv, T(1), lane);
        }
      }
      // the same lane owns each coefficient of gu, gv in the loops above and here
      for (int o = lane; o < 36; o += NT) {
        const int ij = o / 4;  // (2,2) index; constant along u_k, v_k (degree 1 in scaled form: replicated)
        T su = gu.v[o], sum = gu.m[o], sv = gv.v[o], svm = gv.m[o];
        for (int c = 0; c < 3; ++c) {
          const TP<T> cc = slice(c0, c, 9);
          su = fma(-comp(e1, c), cc.v[ij], su);
          sum = fma(fabs(comp(e1, c)), cc.m[ij], sum);
          sv = fma(-comp(e2, c), cc.v[ij], sv);
          svm = fma(fabs(comp(e2, c)), cc.m[ij], svm);
        }
        gu.v[o] = su;
        gu.m[o] = sum;
        gv.v[o] = sv;
        gv.m[o] = svm;
      }
      {
        const T* cv0[3] = {slice(c0, 0, 9).v, slice(c0, 1, 9).v, slice(c0, 2, 9).v};
        const T* cm0[3] = {slice(c0, 0, 9).m, slice(c0, 1, 9).m, slice(c0, 2, 9).m};
        const T af1[3] = {f1.x, f1.y, f1.z}, af2[3] = {f2.x, f2.y, f2.z};
        combo_b<9, 3, false, T, NT>(cv0, cm0, af1, gk.v, gk.m, lane);
        combo_b<9, 3, false, T, NT>(cv0, cm0, af2, gl.v, gl.m, lane);
      }
      const T th_gu = max(th_cv4<1, 1, 0, 0, 1, 1, 1, 1>(th_c0u, th_d1, 6), th_c0 + T(8) * eps) + T(2) * eps;
      const T th_gk = th_c0 + T(5) * eps;
      wave_sync();
      T glo, ghi, hlo, hhi;
      poly_range<1, 1, T, NT>(g.v, g.m, th_g, &glo, &ghi, lane);
      poly_range<2, 2, T, NT>(dd.v, dd.m, th_nn, &hlo, &hhi, lane);
      const T aglo = (glo <= T(0) && ghi >= T(0)) ? T(0) : min(fabs(glo), fabs(ghi));
      const T aghi = max(fabs(glo), fabs(ghi));
      const T Glo = down(aglo / (hhi * sqrt(hhi)));
      const T Ghi = hlo > T(0) ? up(aghi / (hlo * sqrt(hlo))) : T(INFINITY);
      const T k = G.I0 * G.a1 / G.ak;
      const T klo = k * (T(1) - T(16) * eps), khi = k * (T(1) + T(16) * eps);
      const TP<T> a0sq = tpat(B, ILay::A0SQ, 25), a0sqe = tpat(B, ILay::A0SQE, 100), a1sq = tpat(B, ILay::A1SQ, 225);
      const TP<T> su = tpat(B, ILay::SU, 16), sv = tpat(B, ILay::SV, 16), tu = tpat(B, ILay::TU, 144),
                  tv = tpat(B, ILay::TV, 144), tk = tpat(B, ILay::TK, 64), tl = tpat(B, ILay::TL, 64);
      const TP<T> fu = tpat(B, ILay::FU, 324), fv = tpat(B, ILay::FV, 324), fk = tpat(B, ILay::FK, 144),
                  fl = tpat(B, ILay::FL, 144);
      const TP<T> j1 = tpat(B, ILay::J1, 1024), jk = tpat(B, ILay::JK, 256), j1e = tpat(B, ILay::J1E, 1600),
                  jke = tpat(B, ILay::JKE, 1600);
      const T th_a0sq = th_cv4<2, 2, 0, 0, 2, 2, 0, 0>(th_c0, th_c0, 1);
      const T th_a1sq = th_cv4<2, 2, 1, 1, 2, 2, 1, 1>(th_c1, th_c1, 1);
      const T th_su = th_cv4<2, 2, 0, 0, 1, 1, 0, 0>(th_c0, th_c0u, 1);
      const T th_tu = th_cv4<2, 2, 1, 1, 1, 1, 1, 1>(th_c1, th_c1u, 1);
      const T th_tk = th_cv4<2, 2, 1, 1, 1, 1, 0, 0>(th_c1, th_c0u, 1);
      // F_u / 2 = (d0.e1) a1^2 + |d0|^2 a1 a1_u + eta^2 (d1.e1) a0^2 - eta^2 |d1|^2 a0 a0_u
      // F_uk / 2 = |d0|^2 a1 a1_uk - eta^2 (d1.f1) a0^2  (d0, n, a0 do not depend on u_k);
      // eta is an FP32 input, so eta^2 is exact in FP64
      const T th_fu = max(max(th_cv4<1, 1, 0, 0, 4, 4, 2, 2>(th_de, th_a1sq, 4), th_cv4<2, 2, 0, 0, 3, 3, 2, 2>(th_nn, th_tu, 4)),
                          max(th_cv4<1, 1, 1, 1, 4, 4, 1, 1>(th_d1e, th_a0sq, 4), th_cv4<2, 2, 2, 2, 3, 3, 0, 0>(th_d1d1, th_su, 4))) +
                      T(2) * eps;
      const T th_fk = max(th_cv4<2, 2, 0, 0, 3, 3, 1, 1>(th_nn, th_tk, 2), th_cv4<1, 1, 1, 1, 4, 4, 0, 0>(th_d1e, th_a0sq, 2)) +
                      T(2) * eps;
      const T th_j1 = th_cv4<5, 5, 2, 2, 2, 2, 1, 1>(th_fu, th_gu, 2);
      const T th_jk = th_cv4<5, 5, 1, 1, 2, 2, 0, 0>(th_fk, th_gk, 2);
      const T th_j1e = th_elev4<2, 2, 0, 0>(th_j1), th_jke = th_elev4<2, 2, 2, 2>(th_jk);
      const T ee = eta * eta;
      T Elo = T(0), Ehi = T(INFINITY);
      for (int bax = 0; bax < 2; ++bax) {  // b = (1,0,0), then (0,1,0)
        wave_sync();
        const TP<T> a0 = slice(c0, bax, 9), a1 = slice(c1, bax, 36);
        cv4m_b<2, 2, 0, 0, 2, 2, 0, 0, false, NT>(a0, a0, a0sq, T(1), lane);
        cv4m_b<2, 2, 1, 1, 2, 2, 1, 1, false, NT>(a1, a1, a1sq, T(1), lane);
        cv4m_b<2, 2, 0, 0, 1, 1, 0, 0, false, NT>(a0, slice(c0u, bax, 4), su, T(1), lane);
        cv4m_b<2, 2, 0, 0, 1, 1, 0, 0, false, NT>(a0, slice(c0v, bax, 4), sv, T(1), lane);
        cv4m_b<2, 2, 1, 1, 1, 1, 1, 1, false, NT>(a1, slice(c1u, bax, 16), tu, T(1), lane);
        cv4m_b<2, 2, 1, 1, 1, 1, 1, 1, false, NT>(a1, slice(c1v, bax, 16), tv, T(1), lane);
        cv4m_b<2, 2, 1, 1, 1, 1, 0, 0, false, NT>(a1, slice(c1k, bax, 4), tk, T(1), lane);
        cv4m_b<2, 2, 1, 1, 1, 1, 0, 0, false, NT>(a1, slice(c1l, bax, 4), tl, T(1), lane);
        wave_sync();
        elev4m<4, 4, 0, 0, 0, 0, 1, 1, NT>(a0sq, a0sqe, lane);  // replication: exact
        cv4m_b<1, 1, 0, 0, 4, 4, 2, 2, false, NT>(slice(de, 0, 4), a1sq, fu, T(1), lane);
        cv4m_b<2, 2, 0, 0, 3, 3, 2, 2, true, NT>(dd, tu, fu, T(1), lane);
        cv4m_b<2, 2, 2, 2, 3, 3, 0, 0, true, NT>(d1d1, su, fu, -ee, lane);
        cv4m_b<1, 1, 0, 0, 4, 4, 2, 2, false, NT>(slice(de, 1, 4), a1sq, fv, T(1), lane);
        cv4m_b<2, 2, 0, 0, 3, 3, 2, 2, true, NT>(dd, tv, fv, T(1), lane);
        cv4m_b<2, 2, 2, 2, 3, 3, 0, 0, true, NT>(d1d1, sv, fv, -ee, lane);
        cv4m_b<2, 2, 0, 0, 3, 3, 1, 1, false, NT>(dd, tk, fk, T(1), lane);
        cv4m_b<1, 1, 1, 1, 4, 4, 0, 0, true, NT>(slice(d1e, 2, 16), a0sq, fk, -ee, lane);
        cv4m_b<2, 2, 0, 0, 3, 3, 1, 1, false, NT>(dd, tl, fl, T(1), lane);
        cv4m_b<1, 1, 1, 1, 4, 4, 0, 0, true, NT>(slice(d1e, 3, 16), a0sq, fl, -ee, lane);
        wave_sync();
        cv4m_b<1, 1, 1, 1, 4, 4, 1, 1, true, NT>(slice(d1e, 0, 16), a0sqe, fu, ee, lane);
        cv4m_b<1, 1, 1, 1, 4, 4, 1, 1, true, NT>(slice(d1e, 1, 16), a0sqe, fv, ee, lane);
        wave_sync();
        // det J_1 = F_u G_v - F_v G_u (7,7,3,3), det J_k = F_uk G_vk - F_vk G_uk (7,7,1,1)
        cv4m_b<5, 5, 2, 2, 2, 2, 1, 1, false, NT>(fu, gv, j1, T(1), lane);
        cv4m_b<5, 5, 2, 2, 2, 2, 1, 1, true, NT>(fv, gu, j1, T(-1), lane);
        cv4m_b<5, 5, 1, 1, 2, 2, 0, 0, false, NT>(fk, gl, jk, T(1), lane);
        cv4m_b<5, 5, 1, 1, 2, 2, 0, 0, true, NT>(fl, gk, jk, T(-1), lane);
        wave_sync();
        elev4m<7, 7, 3, 3, 2, 2, 0, 0, NT>(j1, j1e, lane);
        elev4m<7, 7, 1, 1, 2, 2, 2, 2, NT>(jk, jke, lane);
        wave_sync();
        const RB<T> rb = ratio4m<T, NT>(N4<9, 9, 3, 3>::n, jke, th_jke, j1e, th_j1e, true, lane);
        T rlo, rhi;
        abs_bound(rb, &rlo, &rhi);
        const T elo = (Glo <= T(0) || rlo <= T(0)) ? T(0) : down(klo * down(Glo * rlo));
        const T ehi = (isinf(Ghi) || isinf(rhi)) ? T(INFINITY) : up(khi * up(Ghi * rhi));
        Elo = max(Elo, elo);
        Ehi = min(Ehi, ehi);
      }
      out.E[0] = out_lo(Elo);
      out.E[1] = out_hi(Ehi);
      return out;
    }
    // ---- derivative linear forms, n_g.d0, and beta_u, beta_v
    const TP<T> nnu = tpat(B, TLay::NNU, 4), nnv = tpat(B, TLay::NNV, 4), ddu = tpat(B, TLay::DDU, 4),
                ddv = tpat(B, TLay::DDV, 4), dnu = tpat(B, TLay::DNU, 4), dnv = tpat(B, TLay::DNV, 4),
                g = tpat(B, TLay::G, 4);
    {
      const T* nv[3] = {nC(0).v, nC(1).v, nC(2).v};
      const T* nm[3] = {nC(0).m, nC(1).m, nC(2).m};
      const T* dv[3] = {dC(0).v, dC(1).v, dC(2).v};
      const T* dm[3] = {dC(0).m, dC(1).m, dC(2).m};
      const T a_nnu[3] = {T(2) * G.dn1.x, T(2) * G.dn1.y, T(2) * G.dn1.z};
      const T a_nnv[3] = {T(2) * G.dn2.x, T(2) * G.dn2.y, T(2) * G.dn2.z};
      const T a_ddu[3] = {T(2) * G.e1.x, T(2) * G.e1.y, T(2) * G.e1.z};
      const T a_ddv[3] = {T(2) * G.e2.x, T(2) * G.e2.y, T(2) * G.e2.z};
      const T ag[3] = {G.ng.x, G.ng.y, G.ng.z};
      combo_b<4, 3, false, T, NT>(nv, nm, a_nnu, nnu.v, nnu.m, lane);
      combo_b<4, 3, false, T, NT>(nv, nm, a_nnv, nnv.v, nnv.m, lane);
      combo_b<4, 3, false, T, NT>(dv, dm, a_ddu, ddu.v, ddu.m, lane);
      combo_b<4, 3, false, T, NT>(dv, dm, a_ddv, ddv.v, ddv.m, lane);
      combo_b<4, 3, false, T, NT>(dv, dm, ag, g.v, g.m, lane);
      const T* xv[6] = {nv[0], nv[1], nv[2], dv[0], dv[1], dv[2]};
      const T* xm[6] = {nm[0], nm[1], nm[2], dm[0], dm[1], dm[2]};
      const T a_dnu[6] = {G.e1.x, G.e1.y, G.e1.z, G.dn1.x, G.dn1.y, G.dn1.z};
      const T a_dnv[6] = {G.e2.x, G.e2.y, G.e2.z, G.dn2.x, G.dn2.y, G.dn2.z};
      combo_b<4, 6, false, T, NT>(xv, xm, a_dnu, dnu.v, dnu.m, lane);
      combo_b<4, 6, false, T, NT>(xv, xm, a_dnv, dnv.v, dnv.m, lane);
    }
    const T th_l2 = th_lin + T(8) * eps;
    const T th_g = th_lin + T(8) * eps;
    wave_sync();
    const TP<T> bu = tpat(B, TLay::BU, 16), bv = tpat(B, TLay::BV, 16);
    cvb<1, 1, 2, 2, false, NT>(nnu, dd, bu, om, lane);
    cvb<2, 2, 1, 1, true, NT>(nn, ddu, bu, om, lane);
    cvb<2, 2, 1, 1, true, NT>(dn, dnu, bu, T(2) * e2, lane);
    cvb<1, 1, 2, 2, false, NT>(nnv, dd, bv, om, lane);
    cvb<2, 2, 1, 1, true, NT>(nn, ddv, bv, om, lane);
    cvb<2, 2, 1, 1, true, NT>(dn, dnv, bv, T(2) * e2, lane);
    const T th_bu = th_conv<2, 2, 1, 1>(th_nn, th_l2, 3) + T(4) * eps;
    // dt0_u = eta (nnu d0 + nn e1 - dnu n - dn dn1), and the same in v
    for (int c = 0; c < 3; ++c) {
      const TP<T> du = tpat(B, TLay::DT0U + 18 * c, 9), dv = tpat(B, TLay::DT0V + 18 * c, 9);
      cvb<1, 1, 1, 1, false, NT>(nnu, dC(c), du, eta, lane);
      cvb<1, 1, 1, 1, true, NT>(dnu, nC(c), du, -eta, lane);
      cvb<1, 1, 1, 1, false, NT>(nnv, dC(c), dv, eta, lane);
      cvb<1, 1, 1, 1, true, NT>(dnv, nC(c), dv, -eta, lane);
      const T* xv[2] = {nn.v, dn.v};
      const T* xm[2] = {nn.m, dn.m};
      const T au[2] = {eta * comp(G.e1, c), -eta * comp(G.dn1, c)};
      const T av[2] = {eta * comp(G.e2, c), -eta * comp(G.dn2, c)};
      combo_b<9, 2, true, T, NT>(xv, xm, au, du.v, du.m, lane);
      combo_b<9, 2, true, T, NT>(xv, xm, av, dv.v, dv.m, lane);
    }
    const T th_dt0u = max(th_conv<1, 1, 1, 1>(th_l2, th_lin, 2), th_nn + T(2) * eps) + T(8) * eps;
    wave_sync();
    // A_u = dt0_u (raised to (4,4)) - rt dn1, A_v likewise; D0 = (e1 x e2).d~; X = e2 x d~;
    // nd = n x d~; bnu = beta_u n
    auto auC = [&](int c) { return tpat(B, TLay::AU + 100 * c, 50); };
    auto avC = [&](int c) { return tpat(B, TLay::AV + 100 * c, 50); };
    auto ndC = [&](int c) { return tpat(Tm, TLay::ND + 196 * c, 98); };
    auto ypC = [&](int c) { return tpat(Tm, TLay::YP + 600 * c, 300); };
    auto bnuC = [&](int c) { return tpat(Tm, TLay::BNU + 50 * c, 25); };
    auto xC = [&](int c) { return tpat(Tm, TLay::X + 144 * c, 72); };
    const TP<T> D0 = tpat(B, TLay::DZ, 72);
    for (int c = 0; c < 3; ++c) {
      const TP<T> du = tpat(B, TLay::DT0U + 18 * c, 9), dv = tpat(B, TLay::DT0V + 18 * c, 9);
      const T* rv[1] = {nullptr};
      const T* rm[1] = {nullptr};
      for (int k = 0; k < 2; ++k) {
        const TP<T> a = slice(auC(c), k, 25), b = slice(avC(c), k, 25), r = slice(rt, k, 25);
        elev_by<2, 2, 2, 2, T, NT>(du.v, du.m, a.v, a.m, lane);
        elev_by<2, 2, 2, 2, T, NT>(dv.v, dv.m, b.v, b.m, lane);
        rv[0] = r.v;
        rm[0] = r.m;
        const T cu[1] = {-comp(G.dn1, c)}, cvv[1] = {-comp(G.dn2, c)};
        combo_b<25, 1, true, T, NT>(rv, rm, cu, a.v, a.m, lane);
        combo_b<25, 1, true, T, NT>(rv, rm, cvv, b.v, b.m, lane);
      }
      cvb<3, 3, 1, 1, false, NT>(bu, nC(c), bnuC(c), T(1), lane);
    }
    {
      const V3<T> n12 = cross(G.e1, G.e2), ee2 = G.e2;
      const T* dv[3] = {dtC(0).v, dtC(1).v, dtC(2).v};
      const T* dm[3] = {dtC(0).m, dtC(1).m, dtC(2).m};
      const T a12[3] = {n12.x, n12.y, n12.z};
      combo_b<72, 3, false, T, NT>(dv, dm, a12, D0.v, D0.m, lane);
      const T xx[3] = {T(0), -ee2.z, ee2.y}, xy[3] = {ee2.z, T(0), -ee2.x}, xz[3] = {-ee2.y, ee2.x, T(0)};
      combo_b<72, 3, false, T, NT>(dv, dm, xx, xC(0).v, xC(0).m, lane);
      combo_b<72, 3, false, T, NT>(dv, dm, xy, xC(1).v, xC(1).m, lane);
      combo_b<72, 3, false, T, NT>(dv, dm, xz, xC(2).v, xC(2).m, lane);
      for (int c = 0; c < 3; ++c) {
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        for (int k = 0; k < 2; ++k) {
          cvb<1, 1, 5, 5, false, NT>(nC(a), slice(dtC(b), k, 36), slice(ndC(c), k, 49), T(1), lane);
          cvb<1, 1, 5, 5, true, NT>(nC(b), slice(dtC(a), k, 36), slice(ndC(c), k, 49), T(-1), lane);
        }
      }
    }
    const T th_A = max(th_dt0u + T(10) * eps, th_rt + T(2) * eps) + T(2) * eps;
    const T th_D0 = th_dt + T(4) * eps;
    const T th_X = th_dt + T(3) * eps;
    const T th_nd = th_conv<1, 1, 5, 5>(th_lin, th_dt, 2);
    const T th_bnu = th_conv<3, 3, 1, 1>(th_bu, th_lin, 1);
    wave_sync();
    // ---- Yp = A_v x d~ (xi1 degree 2), e1.nd
    for (int c = 0; c < 3; ++c) zero<NT>(ypC(c), 300, lane);
    wave_sync();
    for (int c = 0; c < 3; ++c) {
      const int a = (c + 1) % 3, b = (c + 2) % 3;
      for (int k1 = 0; k1 < 2; ++k1)
        for (int k2 = 0; k2 < 2; ++k2) {
          const TP<T> o = slice(ypC(c), k1 + k2, 100);
          cvb<4, 4, 5, 5, true, NT>(slice(avC(a), k1, 25), slice(dtC(b), k2, 36), o, T(1), lane);
          cvb<4, 4, 5, 5, true, NT>(slice(avC(b), k1, 25), slice(dtC(a), k2, 36), o, T(-1), lane);
        }
    }
    const TP<T> e1nd = tpat(Tm, TLay::E1ND, 98);
    {
      const T* xv[3] = {ndC(0).v, ndC(1).v, ndC(2).v};
      const T* xm[3] = {ndC(0).m, ndC(1).m, ndC(2).m};
      const T ae1[3] = {G.e1.x, G.e1.y, G.e1.z};
      combo_b<98, 3, false, T, NT>(xv, xm, ae1, e1nd.v, e1nd.m, lane);
    }
    const T th_Yp = th_conv<4, 4, 5, 5>(th_A, th_dt, 4) + T(2) * eps;
    const T th_e1nd = th_nd + T(3) * eps;
    wave_sync();
    // ---- D1 = A_u.X + e1.Yp - w (beta_u n.X + beta_v e1.nd)
    const TP<T> D1 = tpat(B, TLay::D1, 600), Z1 = tpat(Tm, TLay::Z1, 200);
    zero<NT>(D1, 600, lane);
    zero<NT>(Z1, 200, lane);
    wave_sync();
    for (int c = 0; c < 3; ++c) {
      for (int k1 = 0; k1 < 2; ++k1)
        for (int k2 = 0; k2 < 2; ++k2)
          cvb<4, 4, 5, 5, true, NT>(slice(auC(c), k1, 25), slice(xC(c), k2, 36), slice(D1, 2 * (k1 + k2), 100), T(1),
                               lane);
      for (int j = 0; j < 2; ++j)
        cvb<4, 4, 5, 5, true, NT>(bnuC(c), slice(xC(c), j, 36), slice(Z1, j, 100), T(1), lane);
    }
    for (int j = 0; j < 2; ++j) cvb<3, 3, 6, 6, true, NT>(bv, slice(e1nd, j, 49), slice(Z1, j, 100), T(1), lane);
    {
      const T ae1[3] = {G.e1.x, G.e1.y, G.e1.z};
      for (int m = 0; m < 3; ++m) {
        const TP<T> o = slice(D1, 2 * m, 100);
        for (int idx = lane; idx < 100; idx += NT) {
          T s = o.v[idx], sm = o.m[idx];
          for (int c = 0; c < 3; ++c) {
            const TP<T> y = slice(ypC(c), m, 100);
            s = fma(ae1[c], y.v[idx], s);
            sm = fma(fabs(ae1[c]), y.m[idx], sm);
          }
          o.v[idx] = s;
          o.m[idx] = sm;
        }
      }
    }
    const T th_Z1 = max(th_conv<4, 4, 5, 5>(th_bnu, th_X, 3), th_conv<3, 3, 6, 6>(th_bu, th_e1nd, 1)) + T(2) * eps;
    const T th_D10 = max(th_conv<4, 4, 5, 5>(th_A, th_X, 12), th_Yp + T(4) * eps) + T(4) * eps;
    wave_sync();
    // D1(m, l) = D1_0(m) - w_l (Z1(m-1) + Z1(m))
    for (int o = lane; o < 300; o += NT) {
      const int m = o / 100, idx = o - 100 * m;
      T z = T(0), zm = T(0);
      if (m >= 1) { z += Z1.v[(m - 1) * 100 + idx]; zm += Z1.m[(m - 1) * 100 + idx]; }
      if (m <= 1) { z += Z1.v[m * 100 + idx]; zm += Z1.m[m * 100 + idx]; }
      const T b0 = D1.v[2 * m * 100 + idx], bm = D1.m[2 * m * 100 + idx];
      D1.v[2 * m * 100 + idx] = fma(-wlo, z, b0);
      D1.m[2 * m * 100 + idx] = fma(wlo, zm, bm);
      D1.v[(2 * m + 1) * 100 + idx] = fma(-whi, z, b0);
      D1.m[(2 * m + 1) * 100 + idx] = fma(whi, zm, bm);
    }
    const T th_D1 = max(th_D10, th_Z1 + T(2) * eps) + T(3) * eps;
    wave_sync();
    // ---- D2 = A_u.Yp - w (beta_u n.Yp + beta_v A_u.nd)
    auto bvauC = [&](int c) { return tpat(Tm, TLay::BVAU + 256 * c, 128); };
    const TP<T> D2 = tpat(B, TLay::D2, 1568), Z = tpat(Tm, TLay::Z, 588);
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < 2; ++k) cvb<3, 3, 4, 4, false, NT>(bv, slice(auC(c), k, 25), slice(bvauC(c), k, 64), T(1), lane);
    zero<NT>(D2, 1568, lane);
    zero<NT>(Z, 588, lane);
    wave_sync();
    for (int c = 0; c < 3; ++c) {
      for (int k1 = 0; k1 < 2; ++k1)
        for (int k2 = 0; k2 < 3; ++k2)
          cvb<4, 4, 9, 9, true, NT>(slice(auC(c), k1, 25), slice(ypC(c), k2, 100), slice(D2, 2 * (k1 + k2), 196), T(1),
                               lane);
      for (int j = 0; j < 3; ++j)
        cvb<4, 4, 9, 9, true, NT>(bnuC(c), slice(ypC(c), j, 100), slice(Z, j, 196), T(1), lane);
      for (int k1 = 0; k1 < 2; ++k1)
        for (int k2 = 0; k2 < 2; ++k2)
          cvb<7, 7, 6, 6, true, NT>(slice(bvauC(c), k1, 64), slice(ndC(c), k2, 49), slice(Z, k1 + k2, 196), T(1), lane);
    }
    const T th_bvau = th_conv<3, 3, 4, 4>(th_bu, th_A, 1);
    const T th_Z = max(th_conv<4, 4, 9, 9>(th_bnu, th_Yp, 3), th_conv<7, 7, 6, 6>(th_bvau, th_nd, 6)) + T(2) * eps;
    const T th_D20 = th_conv<4, 4, 9, 9>(th_A, th_Yp, 6) + T(2) * eps;
    wave_sync();
    for (int o = lane; o < 4 * 196; o += NT) {
      const int m = o / 196, idx = o - 196 * m;
      T z = T(0), zm = T(0);
      if (m >= 1) { z += Z.v[(m - 1) * 196 + idx]; zm += Z.m[(m - 1) * 196 + idx]; }
      if (m <= 2) { z += Z.v[m * 196 + idx]; zm += Z.m[m * 196 + idx]; }
      const T b0 = D2.v[2 * m * 196 + idx], bm = D2.m[2 * m * 196 + idx];
      D2.v[2 * m * 196 + idx] = fma(-wlo, z, b0);
      D2.m[2 * m * 196 + idx] = fma(wlo, zm, bm);
      D2.v[(2 * m + 1) * 196 + idx] = fma(-whi, z, b0);
      D2.m[(2 * m + 1) * 196 + idx] = fma(whi, zm, bm);
    }
    const T th_D2 = max(th_D20, th_Z + T(2) * eps) + T(3) * eps;
    // ---- Q^2, Q Tn, Tn^2
    const TP<T> Q2 = tpat(B, TLay::Q2, 363), QT = tpat(B, TLay::QT, 98), T2 = tpat(B, TLay::T2, 9);
    zero<NT>(Q2, 363, lane);
    wave_sync();
    for (int k1 = 0; k1 < 2; ++k1)
      for (int k2 = 0; k2 < 2; ++k2)
        cvb<5, 5, 5, 5, true, NT>(slice(Q, k1, 36), slice(Q, k2, 36), slice(Q2, k1 + k2, 121), T(1), lane);
    for (int k = 0; k < 2; ++k) cvb<5, 5, 1, 1, false, NT>(slice(Q, k, 36), Tn, slice(QT, k, 49), T(1), lane);
    cvb<1, 1, 1, 1, false, NT>(Tn, Tn, T2, T(1), lane);
    const T th_Q2 = th_conv<5, 5, 5, 5>(th_Q, th_Q, 2);
    const T th_QT = th_conv<5, 5, 1, 1>(th_Q, th_Tn, 1);
    const T th_T2 = th_conv<1, 1, 1, 1>(th_Tn, th_Tn, 1);
    wave_sync();
    // ---- det M = -(Q^2 D0 + Q Tn D1 + Tn^2 D2), slices (m, l) with m <= 3, l <= 1
    const TP<T> detM = tpat(Tm, TLay::DETM, 2048);
    zero<NT>(detM, 2048, lane);
    wave_sync();
    for (int k1 = 0; k1 < 3; ++k1)
      for (int k2 = 0; k2 < 2; ++k2)
        cvb<10, 10, 5, 5, true, NT>(slice(Q2, k1, 121), slice(D0, k2, 36), slice(detM, 2 * (k1 + k2), 256), T(-1), lane);
    wave_sync();
    for (int o = lane; o < 4 * 256; o += NT) {
      const int m = o / 256, idx = o - 256 * m;
      detM.v[(2 * m + 1) * 256 + idx] = detM.v[2 * m * 256 + idx];
      detM.m[(2 * m + 1) * 256 + idx] = detM.m[2 * m * 256 + idx];
    }
    wave_sync();
    for (int l = 0; l < 2; ++l) {
      for (int k1 = 0; k1 < 2; ++k1)
        for (int k2 = 0; k2 < 3; ++k2)
          cvb<6, 6, 9, 9, true, NT>(slice(QT, k1, 49), slice(D1, 2 * k2 + l, 100), slice(detM, 2 * (k1 + k2) + l, 256),
                               T(-1), lane);
      for (int m = 0; m < 4; ++m)
        cvb<2, 2, 13, 13, true, NT>(T2, slice(D2, 2 * m + l, 196), slice(detM, 2 * m + l, 256), T(-1), lane);
    }
    const T th_detM = max(max(th_conv<10, 10, 5, 5>(th_Q2, th_D0, 6), th_conv<6, 6, 9, 9>(th_QT, th_D1, 6)),
                          th_conv<2, 2, 13, 13>(th_T2, th_D2, 1)) +
                      T(6) * eps;
    wave_sync();
    // ---- Q^3 (xi1 degree 3) in the space of D1, D2
    const TP<T> Q3 = tpat(B, TLay::Q3, 1024);
    zero<NT>(Q3, 1024, lane);
    wave_sync();
    for (int k1 = 0; k1 < 3; ++k1)
      for (int k2 = 0; k2 < 2; ++k2)
        cvb<10, 10, 5, 5, true, NT>(slice(Q2, k1, 121), slice(Q, k2, 36), slice(Q3, k1 + k2, 256), T(1), lane);
    const T th_Q3 = th_conv<10, 10, 5, 5>(th_Q2, th_Q, 6) + T(2) * eps;
    wave_sync();
    // ---- |Q^3 / det M| from the coefficients at degree (16, 16, 3, 2), raised on the fly
    const T tq3 = th_Q3 + T(8) * eps, tdm = th_detM + T(8) * eps;
    const RB<T> rbm = ratio_bound_fn<T, NT>(
        4 * 3 * 289,
        [&](int o, T& p, T& ep, T& q, T& eq) {
          const int m = o / 867, r1 = o - 867 * m, l = r1 / 289, r = r1 - 289 * l, i = r / 17, j = r - 17 * i;
          T pv = T(0), pm = T(0), qv = T(0), qm = T(0);
          for (int a = i - 1; a <= i; ++a) {
            if (a < 0 || a > 15) continue;
            for (int b = j - 1; b <= j; ++b) {
              if (b < 0 || b > 15) continue;
              const int id = a * 16 + b;
              pv += Q3.v[m * 256 + id];
              pm += Q3.m[m * 256 + id];
              if (l <= 1) {
                qv += detM.v[(2 * m) * 256 + id];
                qm += detM.m[(2 * m) * 256 + id];
              }
              if (l >= 1) {
                qv += detM.v[(2 * m + 1) * 256 + id];
                qm += detM.m[(2 * m + 1) * 256 + id];
              }
            }
          }
          const T cl = l == 1 ? T(2) : T(1);
          p = cl * pv;
          ep = safe_err(tq3, cl * pm);
          q = qv;
          eq = safe_err(tdm, qm);
        },
        final, lane);
    if (rbm.uncertain) {
      out.status = 2;
      return out;
    }
    T rlo, rhi;
    abs_bound(rbm, &rlo, &rhi);
    // dOmega0/dA1 = |g| / h^(3/2) with g = n_g . d0 and h = d0 . d0, bounded factor-wise
    T glo, ghi, hlo, hhi;
    poly_range<1, 1, T, NT>(g.v, g.m, th_g, &glo, &ghi, lane);
    poly_range<2, 2, T, NT>(dd.v, dd.m, th_nn, &hlo, &hhi, lane);
    const T aglo = (glo <= T(0) && ghi >= T(0)) ? T(0) : min(fabs(glo), fabs(ghi));
    const T aghi = max(fabs(glo), fabs(ghi));
    const T Glo = down(aglo / (hhi * sqrt(hhi)));
    const T Ghi = hlo > T(0) ? up(aghi / (hlo * sqrt(hlo))) : T(INFINITY);
    const T k = G.I0 * G.a1 / G.ak;
    const T klo = k * (T(1) - T(16) * eps), khi = k * (T(1) + T(16) * eps);
    const T Elo = (Glo <= T(0) || rlo <= T(0)) ? T(0) : down(klo * down(Glo * rlo));
    const T Ehi = (isinf(Ghi) || isinf(rhi)) ? T(INFINITY) : up(khi * up(Ghi * rhi));
    out.E[0] = out_lo(Elo);
    out.E[1] = out_hi(Ehi);
    return out;
  }
}

}  // namespace bbc
