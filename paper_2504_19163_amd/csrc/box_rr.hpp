// Position bound of one box of a two-reflection tuple, evaluated by one wave in
// FP64 with its polynomials in LDS (Sec. 4.2-4.3, Eq. eq_rct applied twice).
//
// With s_b = x1 - p0b and d~1 the first reflected direction (degree (3,3)),
// Eq. eq_rct gives the second vertex's barycentrics u2 = Pu2/Q2, v2 = Pv2/Q2
// (degree (4,4) over (3,3)) and its ray parameter Tn2/Q2.  Writing
// x2 = X2/Q2 and n2 = N2/Q2 with X2, N2 of degree (4,4), the second reflection
// of d1 = x2 - x1 is, up to the positive factor Q2^3 that Eq. eq_rct cancels,
//   d~2 = (N2.N2) D1 - 2 (D1.N2) N2,  D1 = X2 - Q2 x1          (12,12),
// and the receiver coordinates are u_k = Pu3 / (Q3 Q2) with
//   Pu3 = (d~2 x f2).S3,  Pv3 = (S3 x f1).d~2,  Q3 = (d~2 x f2).f1,
//   S3 = X2 - Q2 q0,  ray parameter ((S3 x f1).f2) / (Q3 Q2),
// numerators of degree (16,16) over a denominator of degree (15,15).  A box is
// culled when the ray to the second plane cannot go forward, cannot reach the
// second triangle's front side, or u2 cannot meet the second triangle.
//
// Irradiance bound (IRR, Sec. 4.4).  The receiver point is a function of u1
// alone, so the generalised geometric term of the single bounce holds for the
// chain: E = I0 (A1 / A_k) G1 |Den^3 / det M| with
// M = [[Den, Pu3, Pv3], [Den_u, Pu3_u, Pv3_u], [Den_v, Pu3_v, Pv3_v]] and
//   det M = Den (Pu3_u Pv3_v - Pv3_u Pu3_v) - Pu3 (Den_u Pv3_v - Pv3_u Den_v)
//         + Pv3 (Den_u Pu3_v - Pu3_u Den_v)                         (46,46),
// the derivatives taken in the box's local coordinates (det M then carries
// the factor 1 / (w_u w_v), restored on the ratio).  These tensors need about
// 90 KB of LDS; they reuse the buffers of the position bound that are dead
// by then, and four waves share a box.
#pragma once
#include "box_t.hpp"

namespace bbc {

struct RRLay {
  static constexpr int N = 0, D0v = 24, X1 = 48, SB = 72, SBE1 = 96, TN2 = 120;  // (1,1) x 3
  static constexpr int NN = 128, DN = 146;                                       // (2,2)
  static constexpr int DT1 = 164, C1 = 260;                                      // (3,3) x 3
  static constexpr int Q2 = 356, Q2E = 388, TN2E = 438, FB = 470;                // (3,3), (4,4), (3,3), (3,3)
  static constexpr int PU2 = 502, PV2 = 552, W2 = 602;                           // (4,4)
  static constexpr int X2 = 652, N2 = 802, D1 = 952, S3 = 1102, S3F1 = 1252;     // (4,4) x 3
  static constexpr int NN2 = 1402, DN2 = 1564;                                   // (8,8)
  static constexpr int DT2 = 1726, C3 = 2740, Q3 = 3754;                         // (12,12) x 3, (12,12)
  static constexpr int DEN = 4092, DENE = 4604;                                  // (15,15), (16,16)
  static constexpr int PU3 = 5182, PV3 = 5760;                                   // (16,16)
  static constexpr int TN3 = 6338, TN3E = 6388;                                  // (4,4), (15,15)
  static constexpr int END = 6900;
  // irradiance bound, after the position bound: G1, H1 hold values then
  // magnitudes; the det M / Den^3 tensors hold values only
  static constexpr int G1 = 6400, H1 = 6410;                                     // n_g.d0 (1,1), d0.d0 (2,2)
  static constexpr int PUU = 0, PUV = 272, PVU = 544, PVV = 816;                 // (15,16), (16,15)
  static constexpr int DENU = 1088, DENV = 1328;                                 // (14,15), (15,14)
  static constexpr int DETM = 6900, MINOR = 9109;                                // (46,46); A (31,31) | B, C (30,30)
  static constexpr int DEN2 = 0, DEN3 = 9109, DEN3E = 0;                         // (30,30), (45,45), (46,46)
  // degree reduction work space over dead position tensors and Den^3:
  // Y [2][17][47], X [2][17][17], then Z and |Z| bounds [2][47][17] per polynomial
  static constexpr int RED_Y = 2209, RED_X = 3807, RED_Z = 2209, RED_Z2 = 9109;
  static constexpr int END_IRR = 11225;
};

template <class T, bool IRR = false>
struct LdsRR {
  T buf[IRR ? RRLay::END_IRR : RRLay::END];
};

// Local derivative along one axis in scaled Bernstein form:
// s'_i = (i + 1) s_{i+1} - (D - i) s_i, degree one lower along that axis
// (values only: the irradiance ratio is taken at face value).
template <int D1, int D2, int AXIS, class T, int NT>
__device__ __forceinline__ void bern_deriv(const T* in, T* out, int lane) {
  constexpr int O1 = AXIS == 0 ? D1 - 1 : D1, O2 = AXIS == 0 ? D2 : D2 - 1;
  for (int o = lane; o < (O1 + 1) * (O2 + 1); o += NT) {
    const int i = o / (O2 + 1), j = o - i * (O2 + 1);
    const int ka = AXIS == 0 ? (i + 1) * (D2 + 1) + j : i * (D2 + 1) + j + 1;
    const int kb = i * (D2 + 1) + j;
    const T ca = T(AXIS == 0 ? i + 1 : j + 1), cb = T(AXIS == 0 ? D1 - i : D2 - j);
    out[o] = fma(ca, in[ka], -(cb * in[kb]));
  }
}

// c (=|+=) sgn * conv(a, b) on values only, for the large tensors of the
// irradiance bound: the sums of conv() over each output's valid index range
// in runtime loops (full unrolling at these degrees costs more registers than
// a wave has).
template <int A1, int A2, int B1, int B2, bool ACC, int NT, class T>
__device__ __forceinline__ void cv_wide(const T* a, const T* b, T* c, T sgn, int lane) {
  constexpr int C2 = A2 + B2, N = (A1 + B1 + 1) * (C2 + 1);
  for (int o = lane; o < N; o += NT) {
    const int k = o / (C2 + 1), l = o - k * (C2 + 1);
    const int i0 = k - B1 > 0 ? k - B1 : 0, i1 = k < A1 ? k : A1;
    const int j0 = l - B2 > 0 ? l - B2 : 0, j1 = l < A2 ? l : A2;
    T s = 0;
#pragma nounroll
    for (int i = i0; i <= i1; ++i) {
      const T* av = a + i * (A2 + 1);
      const T* bv = b + (k - i) * (B2 + 1) + l;
#pragma unroll 4
      for (int j = j0; j <= j1; ++j) s = fma(av[j], bv[-j], s);
    }
    c[o] = ACC ? fma(sgn, s, c[o]) : sgn * s;
  }
}

// Degree reduction (Sec. 6.1, "Degree reduction"): above degree 40 the
// irradiance ratio's numerator Den^3 and denominator det M (both (46, 46))
// are replaced by their least-squares approximants of degree (16, 16) plus a
// remainder variable each, and the ratio is bounded over (16, 16, 1, 1) with
// the numerator's remainder on the third axis and the denominator's on the
// fourth.  The table (built once per handle on the host) holds P, the
// pseudo-inverse of the elevation matrix from degree 16 to 46 (17 x 47), E,
// that matrix (47 x 17), and C(46, i).  The fit is applied to the plain
// (unscaled) coefficients along u, then v; the remainder is the largest
// coefficient of a - E X E^T at degree 46 plus a bound of the rounding of
// that back-elevation, so it bounds |a(x) - X(x)| on the box for the
// coefficients a as computed.
constexpr int kRedFrom = 46, kRedTo = 16;
constexpr int kRedN = kRedFrom + 1, kRedM = kRedTo + 1;
constexpr int kRedTable = 2 * kRedM * kRedN + kRedN;

template <class T, int NT>
__device__ __forceinline__ RB<T> reduced_ratio(T* num, T* den, T* B, const T* __restrict__ tab, int lane) {
  constexpr int N2 = kRedN * kRedN, MN = kRedM * kRedN, M2 = kRedM * kRedM;
  const T eps = Eps<T>::u;
  const T* P = tab;
  const T* E = tab + MN;
  const T* bin = tab + 2 * MN;
  T* const Y = B + RRLay::RED_Y;
  T* const X = B + RRLay::RED_X;
  for (int o = lane; o < 2 * N2; o += NT) {  // scaled -> plain coefficients
    const int f = o < N2 ? o : o - N2, i = f / kRedN, j = f - i * kRedN;
    T* a = o < N2 ? num : den;
    a[f] = a[f] / (bin[i] * bin[j]);
  }
  wave_sync();
  for (int o = lane; o < 2 * MN; o += NT) {  // along u: Y = P a
    const int f = o < MN ? o : o - MN, r = f / kRedN, j = f - r * kRedN;
    const T* a = o < MN ? num : den;
    T s = T(0);
    for (int i = 0; i < kRedN; ++i) s = fma(P[r * kRedN + i], a[i * kRedN + j], s);
    Y[o] = s;
  }
  wave_sync();
  for (int o = lane; o < 2 * M2; o += NT) {  // along v: X = Y P^T
    const int f = o < M2 ? o : o - M2, r = f / kRedM, c = f - r * kRedM;
    const T* y = Y + (o < M2 ? 0 : MN) + r * kRedN;
    T s = T(0);
    for (int j = 0; j < kRedN; ++j) s = fma(y[j], P[c * kRedN + j], s);
    X[o] = s;
  }
  wave_sync();
  for (int o = lane; o < 2 * MN; o += NT) {  // back along u: Z = E X, with E |X|
    const int f = o < MN ? o : o - MN, i = f / kRedM, c = f - i * kRedM;
    const T* x = X + (o < MN ? 0 : M2);
    T* Z = B + (o < MN ? RRLay::RED_Z : RRLay::RED_Z2);
    T s = T(0), sm = T(0);
    for (int r = 0; r < kRedM; ++r) {
      s = fma(E[i * kRedM + r], x[r * kRedM + c], s);
      sm = fma(E[i * kRedM + r], fabs(x[r * kRedM + c]), sm);
    }
    Z[f] = s;
    Z[MN + f] = sm;
  }
  wave_sync();
  T rn = T(0), rd = T(0);
  for (int o = lane; o < 2 * N2; o += NT) {  // residual at degree 46
    const int f = o < N2 ? o : o - N2, i = f / kRedN, j = f - i * kRedN;
    const T* Z = B + (o < N2 ? RRLay::RED_Z : RRLay::RED_Z2);
    T w = T(0), wm = T(0);
    for (int c = 0; c < kRedM; ++c) {
      w = fma(Z[i * kRedM + c], E[j * kRedM + c], w);
      wm = fma(Z[MN + i * kRedM + c], E[j * kRedM + c], wm);
    }
    const T res = fabs((o < N2 ? num : den)[f] - w) + T(48) * eps * wm;
    if (o < N2)
      rn = max(rn, res);
    else
      rd = max(rd, res);
  }
  rn = up(blk_max<NT>(rn) * (T(1) + T(4) * eps));
  rd = up(blk_max<NT>(rd) * (T(1) + T(4) * eps));
  return ratio_bound_fn<T, NT>(
      4 * M2,
      [&](int o, T& p, T& ep, T& q, T& eq) {
        const int f = o >> 2;
        const T xp = X[f], xq = X[M2 + f];
        p = (o & 2) ? xp + rn : xp - rn;
        q = (o & 1) ? xq + rd : xq - rd;
        ep = eps * (fabs(xp) + rn);
        eq = eps * (fabs(xq) + rd);
      },
      true, lane);
}

// Inlined into its kernels (about 4 % faster than a call); the subdivision
// kernel also exists with it as a called function (BBC_TUNE_RR_OUTLINED), and
// both give identical builds.
template <class T, bool IRR = false, int NT = BBC_WAVE>
__device__ __forceinline__ BoxOut eval_box_rr(const TupleGeom<T>& G, T u0, T u1, T v0, T v1, LdsRR<T, IRR>& L, int lane,
                                              const T* red = nullptr) {
  const bool final = true;
  const T eps = Eps<T>::u;
  T* B = L.buf;
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

  // ---- linear forms n, d0, x1, s_b at the box corners
  const V3<T> pmx = G.p0 - G.x0, pmb = G.p0 - G.p0b;
  for (int task = lane; task < 48; task += NT) {
    const int which = task / 12, c = (task / 4) % 3, k = task % 4;
    const T u = (k & 2) ? u1 : u0, v = (k & 1) ? v1 : v0;
    T a, b, d;
    if (which == 0) {
      a = comp(G.n0, c); b = comp(G.dn1, c); d = comp(G.dn2, c);
    } else {
      a = comp(which == 1 ? pmx : (which == 2 ? G.p0 : pmb), c);
      b = comp(G.e1, c);
      d = comp(G.e2, c);
    }
    const int base = which == 0 ? RRLay::N : (which == 1 ? RRLay::D0v : (which == 2 ? RRLay::X1 : RRLay::SB));
    TP<T> dst = tpat(B, base + 8 * c, 4);
    dst.v[k] = fma(d, v, fma(b, u, a));
    dst.m[k] = fabs(a) + fabs(b) * fabs(u) + fabs(d) * fabs(v);
  }
  const T th_lin = T(4) * eps;
  auto lin = [&](int base, int c) { return tpat(B, base + 8 * c, 4); };
  auto v44 = [&](int base, int c) { return tpat(B, base + 50 * c, 25); };
  auto v33 = [&](int base, int c) { return tpat(B, base + 32 * c, 16); };
  auto v1212 = [&](int base, int c) { return tpat(B, base + 338 * c, 169); };
  wave_sync();

  // ---- s_b x e1b, Tn2 = (s_b x e1b).e2b, n.n, d0.n
  {
    const T* sv[3] = {lin(RRLay::SB, 0).v, lin(RRLay::SB, 1).v, lin(RRLay::SB, 2).v};
    const T* sm[3] = {lin(RRLay::SB, 0).m, lin(RRLay::SB, 1).m, lin(RRLay::SB, 2).m};
    const V3<T> k = G.e1b;
    const T ax[3] = {T(0), k.z, -k.y}, ay[3] = {-k.z, T(0), k.x}, az[3] = {k.y, -k.x, T(0)};
    combo<4, 3, false, T, NT>(sv, sm, ax, lin(RRLay::SBE1, 0).v, lin(RRLay::SBE1, 0).m, lane);
    combo<4, 3, false, T, NT>(sv, sm, ay, lin(RRLay::SBE1, 1).v, lin(RRLay::SBE1, 1).m, lane);
    combo<4, 3, false, T, NT>(sv, sm, az, lin(RRLay::SBE1, 2).v, lin(RRLay::SBE1, 2).m, lane);
    const TP<T> nn = tpat(B, RRLay::NN, 9), dn = tpat(B, RRLay::DN, 9);
    for (int c = 0; c < 3; ++c) {
      if (c == 0) {
        cv<1, 1, 1, 1, false, NT>(lin(RRLay::N, c), lin(RRLay::N, c), nn, T(1), lane);
        cv<1, 1, 1, 1, false, NT>(lin(RRLay::D0v, c), lin(RRLay::N, c), dn, T(1), lane);
      } else {
        cv<1, 1, 1, 1, true, NT>(lin(RRLay::N, c), lin(RRLay::N, c), nn, T(1), lane);
        cv<1, 1, 1, 1, true, NT>(lin(RRLay::D0v, c), lin(RRLay::N, c), dn, T(1), lane);
      }
    }
  }
  const T th_sbe1 = th_lin + T(4) * eps;
  const T th_nn = th_conv<1, 1, 1, 1>(th_lin, th_lin, 3) + T(3) * eps;
  wave_sync();
  {
    const T* xv[3] = {lin(RRLay::SBE1, 0).v, lin(RRLay::SBE1, 1).v, lin(RRLay::SBE1, 2).v};
    const T* xm[3] = {lin(RRLay::SBE1, 0).m, lin(RRLay::SBE1, 1).m, lin(RRLay::SBE1, 2).m};
    const T ak[3] = {G.e2b.x, G.e2b.y, G.e2b.z};
    const TP<T> tn2 = tpat(B, RRLay::TN2, 4);
    combo<4, 3, false, T, NT>(xv, xm, ak, tn2.v, tn2.m, lane);
    // d~1 = (n.n) d0 - 2 (d0.n) n
    const TP<T> nn = tpat(B, RRLay::NN, 9), dn = tpat(B, RRLay::DN, 9);
    for (int c = 0; c < 3; ++c) {
      cv<2, 2, 1, 1, false, NT>(nn, lin(RRLay::D0v, c), v33(RRLay::DT1, c), T(1), lane);
      cv<2, 2, 1, 1, true, NT>(dn, lin(RRLay::N, c), v33(RRLay::DT1, c), T(-2), lane);
    }
  }
  const T th_Tn2 = th_sbe1 + T(3) * eps;
  const T th_dt1 = th_conv<2, 2, 1, 1>(th_nn, th_lin, 2) + T(2) * eps;
  wave_sync();
  // ---- c1 = d~1 x e2b, Q2 = c1.e1b, d~1.n_g2, Pu2 = c1.s_b, Pv2 = (s_b x e1b).d~1
  {
    const T* dv[3] = {v33(RRLay::DT1, 0).v, v33(RRLay::DT1, 1).v, v33(RRLay::DT1, 2).v};
    const T* dm[3] = {v33(RRLay::DT1, 0).m, v33(RRLay::DT1, 1).m, v33(RRLay::DT1, 2).m};
    const V3<T> k = G.e2b;
    const T ax[3] = {T(0), k.z, -k.y}, ay[3] = {-k.z, T(0), k.x}, az[3] = {k.y, -k.x, T(0)};
    combo<16, 3, false, T, NT>(dv, dm, ax, v33(RRLay::C1, 0).v, v33(RRLay::C1, 0).m, lane);
    combo<16, 3, false, T, NT>(dv, dm, ay, v33(RRLay::C1, 1).v, v33(RRLay::C1, 1).m, lane);
    combo<16, 3, false, T, NT>(dv, dm, az, v33(RRLay::C1, 2).v, v33(RRLay::C1, 2).m, lane);
    const T ag[3] = {G.ngb.x, G.ngb.y, G.ngb.z};
    const TP<T> fb = tpat(B, RRLay::FB, 16);
    combo<16, 3, false, T, NT>(dv, dm, ag, fb.v, fb.m, lane);
    const TP<T> pv2 = tpat(B, RRLay::PV2, 25);
    for (int c = 0; c < 3; ++c) {
      if (c == 0)
        cv<1, 1, 3, 3, false, NT>(lin(RRLay::SBE1, c), v33(RRLay::DT1, c), pv2, T(1), lane);
      else
        cv<1, 1, 3, 3, true, NT>(lin(RRLay::SBE1, c), v33(RRLay::DT1, c), pv2, T(1), lane);
    }
  }
  const T th_c1 = th_dt1 + T(3) * eps;
  const T th_fb = th_dt1 + T(4) * eps;
  wave_sync();
  const TP<T> q2 = tpat(B, RRLay::Q2, 16), pu2 = tpat(B, RRLay::PU2, 25), pv2 = tpat(B, RRLay::PV2, 25);
  {
    const T* cvp[3] = {v33(RRLay::C1, 0).v, v33(RRLay::C1, 1).v, v33(RRLay::C1, 2).v};
    const T* cmp[3] = {v33(RRLay::C1, 0).m, v33(RRLay::C1, 1).m, v33(RRLay::C1, 2).m};
    const T ak[3] = {G.e1b.x, G.e1b.y, G.e1b.z};
    combo<16, 3, false, T, NT>(cvp, cmp, ak, q2.v, q2.m, lane);
    for (int c = 0; c < 3; ++c) {
      if (c == 0)
        cv<3, 3, 1, 1, false, NT>(v33(RRLay::C1, c), lin(RRLay::SB, c), pu2, T(1), lane);
      else
        cv<3, 3, 1, 1, true, NT>(v33(RRLay::C1, c), lin(RRLay::SB, c), pu2, T(1), lane);
    }
    const TP<T> tn2 = tpat(B, RRLay::TN2, 4), tn2e = tpat(B, RRLay::TN2E, 16);
    elev_by<1, 1, 2, 2, T, NT>(tn2.v, tn2.m, tn2e.v, tn2e.m, lane);
  }
  const T th_Q2 = th_c1 + T(3) * eps;
  const T th_P2 = max(th_conv<3, 3, 1, 1>(th_c1, th_lin, 3), th_conv<1, 1, 3, 3>(th_sbe1, th_dt1, 3)) + T(2) * eps;
  const T th_Tn2e = th_Tn2 + T(10) * eps;
  wave_sync();
  const TP<T> q2e = tpat(B, RRLay::Q2E, 25), w2 = tpat(B, RRLay::W2, 25);
  elev11<3, 3, T, NT>(q2.v, q2.m, q2e.v, q2e.m, lane);
  for (int o = lane; o < 25; o += NT) {
    w2.v[o] = pu2.v[o] + pv2.v[o];
    w2.m[o] = pu2.m[o] + pv2.m[o];
  }
  const T th_Q2e = th_Q2 + T(4) * eps;
  wave_sync();
  // ---- the second vertex: forward, front side, inside the second triangle
  bool inside2 = false;
  {
    const RB<T> sr = ratio_bound<16, T, NT>(tpat(B, RRLay::TN2E, 16).v, tpat(B, RRLay::TN2E, 16).m, th_Tn2e, q2.v,
                                            q2.m, th_Q2, final, lane);
    if (sr.kind == kDirect && sr.hi <= T(0)) return out;
    T fl, fh;
    poly_range<3, 3, T, NT>(tpat(B, RRLay::FB, 16).v, tpat(B, RRLay::FB, 16).m, th_fb, &fl, &fh, lane);
    if (fl >= T(0)) return out;
    const RB<T> ub2 = ratio_bound<25, T, NT>(pu2.v, pu2.m, th_P2, q2e.v, q2e.m, th_Q2e, final, lane);
    const RB<T> vb2 = ratio_bound<25, T, NT>(pv2.v, pv2.m, th_P2, q2e.v, q2e.m, th_Q2e, final, lane);
    const RB<T> wb2 = ratio_bound<25, T, NT>(w2.v, w2.m, th_P2 + eps, q2e.v, q2e.m, th_Q2e, final, lane);
    if (ub2.kind == kDirect && ub2.hi < T(0)) return out;
    if (vb2.kind == kDirect && vb2.hi < T(0)) return out;
    if (wb2.kind == kDirect && wb2.lo > T(1)) return out;
    inside2 = ub2.kind == kDirect && vb2.kind == kDirect && wb2.kind == kDirect && ub2.lo >= T(0) &&
              vb2.lo >= T(0) && wb2.hi <= T(1) && sr.kind == kDirect && sr.lo > T(0) && fh < T(0);
  }
  // ---- X2, N2, S3 = X2 - Q2 q0, D1 = X2 - Q2 x1
  {
    const T* av[3] = {q2e.v, pu2.v, pv2.v};
    const T* am[3] = {q2e.m, pu2.m, pv2.m};
    for (int c = 0; c < 3; ++c) {
      const T ax[3] = {comp(G.p0b, c), comp(G.e1b, c), comp(G.e2b, c)};
      const T an[3] = {comp(G.n0b, c), comp(G.dn1b, c), comp(G.dn2b, c)};
      combo<25, 3, false, T, NT>(av, am, ax, v44(RRLay::X2, c).v, v44(RRLay::X2, c).m, lane);
      combo<25, 3, false, T, NT>(av, am, an, v44(RRLay::N2, c).v, v44(RRLay::N2, c).m, lane);
      // the same lane owns each coefficient in these three combos and the conv below
      const T* xv[2] = {v44(RRLay::X2, c).v, q2e.v};
      const T* xm[2] = {v44(RRLay::X2, c).m, q2e.m};
      const T as[2] = {T(1), -comp(G.q0, c)};
      combo<25, 2, false, T, NT>(xv, xm, as, v44(RRLay::S3, c).v, v44(RRLay::S3, c).m, lane);
      const T* yv[1] = {v44(RRLay::X2, c).v};
      const T* ym[1] = {v44(RRLay::X2, c).m};
      const T one[1] = {T(1)};
      combo<25, 1, false, T, NT>(yv, ym, one, v44(RRLay::D1, c).v, v44(RRLay::D1, c).m, lane);
      cv<3, 3, 1, 1, true, NT>(q2, lin(RRLay::X1, c), v44(RRLay::D1, c), T(-1), lane);
    }
  }
  const T th_X2 = max(th_Q2e, th_P2) + T(4) * eps;
  const T th_S3 = th_X2 + T(3) * eps;
  const T th_D1 = max(th_X2, th_conv<3, 3, 1, 1>(th_Q2, th_lin, 1)) + T(3) * eps;
  wave_sync();
  // ---- N2.N2, D1.N2, S3 x f1, Tn3
  const TP<T> nn2 = tpat(B, RRLay::NN2, 81), dn2 = tpat(B, RRLay::DN2, 81);
  for (int c = 0; c < 3; ++c) {
    if (c == 0) {
      cv<4, 4, 4, 4, false, NT>(v44(RRLay::N2, c), v44(RRLay::N2, c), nn2, T(1), lane);
      cv<4, 4, 4, 4, false, NT>(v44(RRLay::D1, c), v44(RRLay::N2, c), dn2, T(1), lane);
    } else {
      cv<4, 4, 4, 4, true, NT>(v44(RRLay::N2, c), v44(RRLay::N2, c), nn2, T(1), lane);
      cv<4, 4, 4, 4, true, NT>(v44(RRLay::D1, c), v44(RRLay::N2, c), dn2, T(1), lane);
    }
  }
  {
    const T* sv[3] = {v44(RRLay::S3, 0).v, v44(RRLay::S3, 1).v, v44(RRLay::S3, 2).v};
    const T* sm[3] = {v44(RRLay::S3, 0).m, v44(RRLay::S3, 1).m, v44(RRLay::S3, 2).m};
    const V3<T> k = G.f1;
    const T ax[3] = {T(0), k.z, -k.y}, ay[3] = {-k.z, T(0), k.x}, az[3] = {k.y, -k.x, T(0)};
    combo<25, 3, false, T, NT>(sv, sm, ax, v44(RRLay::S3F1, 0).v, v44(RRLay::S3F1, 0).m, lane);
    combo<25, 3, false, T, NT>(sv, sm, ay, v44(RRLay::S3F1, 1).v, v44(RRLay::S3F1, 1).m, lane);
    combo<25, 3, false, T, NT>(sv, sm, az, v44(RRLay::S3F1, 2).v, v44(RRLay::S3F1, 2).m, lane);
  }
  const T th_N2 = th_X2;
  const T th_NN2 = th_conv<4, 4, 4, 4>(max(th_N2, th_D1), th_N2, 3) + T(2) * eps;
  const T th_S3F1 = th_S3 + T(4) * eps;
  wave_sync();
  {
    const T* xv[3] = {v44(RRLay::S3F1, 0).v, v44(RRLay::S3F1, 1).v, v44(RRLay::S3F1, 2).v};
    const T* xm[3] = {v44(RRLay::S3F1, 0).m, v44(RRLay::S3F1, 1).m, v44(RRLay::S3F1, 2).m};
    const T af2[3] = {G.f2.x, G.f2.y, G.f2.z};
    const TP<T> tn3 = tpat(B, RRLay::TN3, 25);
    combo<25, 3, false, T, NT>(xv, xm, af2, tn3.v, tn3.m, lane);
    // d~2 = (N2.N2) D1 - 2 (D1.N2) N2
    for (int c = 0; c < 3; ++c) {
      cv<8, 8, 4, 4, false, NT>(nn2, v44(RRLay::D1, c), v1212(RRLay::DT2, c), T(1), lane);
      cv<8, 8, 4, 4, true, NT>(dn2, v44(RRLay::N2, c), v1212(RRLay::DT2, c), T(-2), lane);
    }
  }
  const T th_Tn3 = th_S3F1 + T(3) * eps;
  const T th_dt2 = th_conv<8, 8, 4, 4>(th_NN2, max(th_D1, th_N2), 2) + T(2) * eps;
  wave_sync();
  // ---- c3 = d~2 x f2, Q3 = c3.f1, Den = Q3 Q2, Pu3 = c3.S3, Pv3 = (S3 x f1).d~2
  {
    const T* dv[3] = {v1212(RRLay::DT2, 0).v, v1212(RRLay::DT2, 1).v, v1212(RRLay::DT2, 2).v};
    const T* dm[3] = {v1212(RRLay::DT2, 0).m, v1212(RRLay::DT2, 1).m, v1212(RRLay::DT2, 2).m};
    const V3<T> k = G.f2;
    const T ax[3] = {T(0), k.z, -k.y}, ay[3] = {-k.z, T(0), k.x}, az[3] = {k.y, -k.x, T(0)};
    combo<169, 3, false, T, NT>(dv, dm, ax, v1212(RRLay::C3, 0).v, v1212(RRLay::C3, 0).m, lane);
    combo<169, 3, false, T, NT>(dv, dm, ay, v1212(RRLay::C3, 1).v, v1212(RRLay::C3, 1).m, lane);
    combo<169, 3, false, T, NT>(dv, dm, az, v1212(RRLay::C3, 2).v, v1212(RRLay::C3, 2).m, lane);
    const TP<T> pv3 = tpat(B, RRLay::PV3, 289);
    for (int c = 0; c < 3; ++c) {
      if (c == 0)
        cv<4, 4, 12, 12, false, NT>(v44(RRLay::S3F1, c), v1212(RRLay::DT2, c), pv3, T(1), lane);
      else
        cv<4, 4, 12, 12, true, NT>(v44(RRLay::S3F1, c), v1212(RRLay::DT2, c), pv3, T(1), lane);
    }
    const TP<T> tn3 = tpat(B, RRLay::TN3, 25), tn3e = tpat(B, RRLay::TN3E, 256);
    elev_by<4, 4, 11, 11, T, NT>(tn3.v, tn3.m, tn3e.v, tn3e.m, lane);
  }
  const T th_c3 = th_dt2 + T(3) * eps;
  const T th_P3b = th_conv<4, 4, 12, 12>(th_S3F1, th_dt2, 3) + T(2) * eps;
  const T th_Tn3e = th_Tn3 + T(150) * eps;
  wave_sync();
  const TP<T> q3 = tpat(B, RRLay::Q3, 169), den = tpat(B, RRLay::DEN, 256), pu3 = tpat(B, RRLay::PU3, 289);
  {
    const T* cvp[3] = {v1212(RRLay::C3, 0).v, v1212(RRLay::C3, 1).v, v1212(RRLay::C3, 2).v};
    const T* cmp[3] = {v1212(RRLay::C3, 0).m, v1212(RRLay::C3, 1).m, v1212(RRLay::C3, 2).m};
    const T af1[3] = {G.f1.x, G.f1.y, G.f1.z};
    combo<169, 3, false, T, NT>(cvp, cmp, af1, q3.v, q3.m, lane);
    for (int c = 0; c < 3; ++c) {
      if (c == 0)
        cv<12, 12, 4, 4, false, NT>(v1212(RRLay::C3, c), v44(RRLay::S3, c), pu3, T(1), lane);
      else
        cv<12, 12, 4, 4, true, NT>(v1212(RRLay::C3, c), v44(RRLay::S3, c), pu3, T(1), lane);
    }
  }
  const T th_Q3 = th_c3 + T(3) * eps;
  const T th_P3a = th_conv<12, 12, 4, 4>(th_c3, th_S3, 3) + T(2) * eps;
  wave_sync();
  cv<12, 12, 3, 3, false, NT>(q3, q2, den, T(1), lane);
  const T th_den = th_conv<12, 12, 3, 3>(th_Q3, th_Q2, 1);
  wave_sync();
  const TP<T> dene = tpat(B, RRLay::DENE, 289), pv3 = tpat(B, RRLay::PV3, 289), tn3e = tpat(B, RRLay::TN3E, 256);
  elev11<15, 15, T, NT>(den.v, den.m, dene.v, dene.m, lane);
  const T th_dene = th_den + T(4) * eps;
  wave_sync();
  // ---- position bound (Sec. 4.2) and the sign of the last ray parameter
  const RB<T> tb = ratio_bound<256, T, NT>(tn3e.v, tn3e.m, th_Tn3e, den.v, den.m, th_den, final, lane);
  if (tb.kind == kDirect && tb.hi <= T(0)) return out;
  const RB<T> ub = ratio_bound<289, T, NT>(pu3.v, pu3.m, th_P3a, dene.v, dene.m, th_dene, final, lane);
  const RB<T> vb = ratio_bound<289, T, NT>(pv3.v, pv3.m, th_P3b, dene.v, dene.m, th_dene, final, lane);
  T ulo, uhi, vlo, vhi;
  if (!clip01(ub, &ulo, &uhi) || !clip01(vb, &vlo, &vhi)) return out;
  out.uk[0] = out_lo(ulo);
  out.uk[1] = out_hi(uhi);
  out.uk[2] = out_lo(vlo);
  out.uk[3] = out_hi(vhi);
  out.settled = inside2 && ub.kind == kDirect && vb.kind == kDirect && ub.lo >= T(0) && ub.hi <= T(1) &&
                vb.lo >= T(0) && vb.hi <= T(1) && tb.kind == kDirect && tb.lo > T(0);
  out.status = 1;
  if constexpr (!IRR) {
    return out;
  } else {
    // ---- G1 = |g| / h^(3/2), g = n_g . d0, h = d0 . d0 (d0 is still in LDS)
    const TP<T> g1 = tpat(B, RRLay::G1, 4), h1 = tpat(B, RRLay::H1, 9);
    {
      const T* dv[3] = {lin(RRLay::D0v, 0).v, lin(RRLay::D0v, 1).v, lin(RRLay::D0v, 2).v};
      const T* dm[3] = {lin(RRLay::D0v, 0).m, lin(RRLay::D0v, 1).m, lin(RRLay::D0v, 2).m};
      const T ag[3] = {G.ng.x, G.ng.y, G.ng.z};
      combo<4, 3, false, T, NT>(dv, dm, ag, g1.v, g1.m, lane);
      for (int c = 0; c < 3; ++c) {
        if (c == 0)
          cv<1, 1, 1, 1, false, NT>(lin(RRLay::D0v, c), lin(RRLay::D0v, c), h1, T(1), lane);
        else
          cv<1, 1, 1, 1, true, NT>(lin(RRLay::D0v, c), lin(RRLay::D0v, c), h1, T(1), lane);
      }
    }
    const T th_g = th_lin + T(8) * eps;  // the unit normal carries a few roundings of its own
    const T th_h = th_conv<1, 1, 1, 1>(th_lin, th_lin, 3) + T(3) * eps;
    wave_sync();
    T glo, ghi, hlo, hhi;
    poly_range<1, 1, T, NT>(g1.v, g1.m, th_g, &glo, &ghi, lane);
    poly_range<2, 2, T, NT>(h1.v, h1.m, th_h, &hlo, &hhi, lane);
    wave_sync();
    // ---- local derivatives of Den, Pu3, Pv3
    T* const puu = B + RRLay::PUU;
    T* const puv = B + RRLay::PUV;
    T* const pvu = B + RRLay::PVU;
    T* const pvv = B + RRLay::PVV;
    T* const denu = B + RRLay::DENU;
    T* const denv = B + RRLay::DENV;
    bern_deriv<16, 16, 0, T, NT>(pu3.v, puu, lane);
    bern_deriv<16, 16, 1, T, NT>(pu3.v, puv, lane);
    bern_deriv<16, 16, 0, T, NT>(pv3.v, pvu, lane);
    bern_deriv<16, 16, 1, T, NT>(pv3.v, pvv, lane);
    bern_deriv<15, 15, 0, T, NT>(den.v, denu, lane);
    bern_deriv<15, 15, 1, T, NT>(den.v, denv, lane);
    wave_sync();
    // ---- det M = Den A - Pu3 B + Pv3 C with the minors
    //   A = Pu_u Pv_v - Pv_u Pu_v, B = Den_u Pv_v - Pv_u Den_v, C = Den_u Pu_v - Pu_u Den_v
    // formed one at a time in one buffer, each added to det M before the next
    T* const detm = B + RRLay::DETM;
    T* const minor = B + RRLay::MINOR;
    cv_wide<15, 16, 16, 15, false, NT>(puu, pvv, minor, T(1), lane);
    cv_wide<15, 16, 16, 15, true, NT>(pvu, puv, minor, T(-1), lane);
    wave_sync();
    cv_wide<15, 15, 31, 31, false, NT>(den.v, minor, detm, T(1), lane);
    wave_sync();
    cv_wide<14, 15, 16, 15, false, NT>(denu, pvv, minor, T(1), lane);
    cv_wide<15, 16, 15, 14, true, NT>(pvu, denv, minor, T(-1), lane);
    wave_sync();
    cv_wide<16, 16, 30, 30, true, NT>(pu3.v, minor, detm, T(-1), lane);
    wave_sync();
    cv_wide<14, 15, 16, 15, false, NT>(denu, puv, minor, T(1), lane);
    cv_wide<15, 16, 15, 14, true, NT>(puu, denv, minor, T(-1), lane);
    wave_sync();
    cv_wide<16, 16, 30, 30, true, NT>(pv3.v, minor, detm, T(1), lane);
    wave_sync();
    // ---- Den^3, elevated to (46, 46): the scaled coefficient (i, j) is the
    // sum of the (up to four) degree-(45, 45) neighbours (i-1..i, j-1..j)
    T* const den2 = B + RRLay::DEN2;
    T* const den3 = B + RRLay::DEN3;
    T* const den3e = B + RRLay::DEN3E;
    cv_wide<15, 15, 15, 15, false, NT>(den.v, den.v, den2, T(1), lane);
    wave_sync();
    cv_wide<30, 30, 15, 15, false, NT>(den2, den.v, den3, T(1), lane);
    wave_sync();
    for (int o = lane; o < 47 * 47; o += NT) {
      const int i = o / 47, j = o - i * 47;
      const T a = (i <= 45 && j <= 45) ? den3[i * 46 + j] : T(0);
      const T b = (i >= 1 && j <= 45) ? den3[(i - 1) * 46 + j] : T(0);
      const T c = (i <= 45 && j >= 1) ? den3[i * 46 + j - 1] : T(0);
      const T d = (i >= 1 && j >= 1) ? den3[(i - 1) * 46 + j - 1] : T(0);
      den3e[o] = (a + b) + (c + d);
    }
    wave_sync();
    // |Den^3 / det M| at face value: with rounding control, det M's
    // coefficients (three nested cancellations at degree (46, 46)) leave
    // their signs undecided on most boxes; the bound takes them as computed
    RB<T> rb;
    if (red != nullptr) {
      rb = reduced_ratio<T, NT>(den3e, detm, B, red, lane);
    } else {
      rb = ratio_bound_fn<T, NT>(
          2209,
          [&](int o, T& p, T& ep, T& q, T& eq) {
            q = detm[o];
            p = den3e[o];
            ep = eq = T(0);
          },
          final, lane);
    }
    T rlo, rhi;
    abs_bound(rb, &rlo, &rhi);
    // det M from local derivatives is w_u w_v times the global one (each
    // term has one u- and one v-derivative): the global ratio is the local
    // one times w_u w_v
    const T area = (u1 - u0) * (v1 - v0);
    rlo = down(rlo * area * (T(1) - T(4) * eps));
    rhi = isinf(rhi) ? rhi : up(rhi * area * (T(1) + T(4) * eps));
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
