// Position and irradiance bound of one box of a single-reflection tuple,
// evaluated by one wave with its polynomials in LDS (Sec. 4.2-4.4).
//
// Polynomials (barycentric u1 = (u, v) of the specular vertex, restricted to
// the box, scaled Bernstein form; see bern_dev.hpp):
//   n  = n0 + u dn1 + v dn2,  d0 = x1 - x0,  s = x1 - q0           (1,1)
//   d~ = (n.n) d0 - 2 (d0.n) n            reflection, Eq. eq_refr_rational (3,3)
//   Pu = (d~ x f2).s,  Pv = (s x f1).d~,  Q = (d~ x f2).f1         Eq. eq_rct
//   u_k = Pu/Q, v_k = Pv/Q, t = ((s x f1).f2)/Q
//   det(du_k/du1) = det M / Q^3,  M = [[Q,Pu,Pv],[Q_u,Pu_u,Pv_u],[Q_v,Pu_v,Pv_v]]
//                                          explicit differentiation, Eq. eq_irr_term3a
//   E_k = I0 |n_g.d0| / |d0|^3 |e1 x e2| / (|det J| |f1 x f2|)   Eq. eq_dwda
// det M is assembled in the equivalent receiver-origin-free form
//   det M = -(Q^2 D0 + Q Tn D1 + Tn^2 D2),  D0 = det[e1, e2, d~],
//   D1 = det[d~_u, e2, d~] + det[e1, d~_v, d~],  D2 = det[d~_u, d~_v, d~],
// which follows from x_k = x1 + (Tn/Q) d~ and the area element of the receiver
// parameterisation; it is the same polynomial as the cofactor expansion of M
// but with about ten times less cancellation in its coefficients.  Partial
// derivatives d~_u, d~_v come from the product rule on the linear forms, so
// det M and Q^3 appear at their true degree (9,9); both are raised once to
// (10,10) before the ratio bound.
#pragma once
#include "bern_dev.hpp"
#include "geom_dev.hpp"

namespace bbc {

// LDS of the position bound only (domain initialisation).
template <class T>
struct LdsRPos {
  Ten<T, 4> n[3], d0[3], s[3], sf1[3], Tn;
  Ten<T, 9> nn, dn, Tn2;
  Ten<T, 16> dt[3], cc[3];
  Ten<T, 25> Pu, Pv, Qe;
  Ten<T, 16> Q, Tne;
};
// LDS of the position and irradiance bound (subdivision).  The position
// tensors that the irradiance part no longer reads share their space with the
// cofactor parts of det M, and those with the elevated det M and Q^3: 11.3 KB
// instead of 18.6 KB.
template <class T>
struct LdsR {
  // live through the whole evaluation
  Ten<T, 16> dt[3], Q;
  Ten<T, 4> Tn, g, nnu, nnv, dnu, dnv;
  Ten<T, 9> h;
  Ten<T, 9> dtu[3], dtv[3];
  union {
    struct {  // position bound
      Ten<T, 4> n[3], d0[3], s[3], sf1[3];
      Ten<T, 9> nn, dn, Tn2;
      Ten<T, 16> cc[3];
      Ten<T, 25> Pu, Pv, Qe;
      Ten<T, 16> Tne;
    };
    struct {  // irradiance: the parts of det M
      Ten<T, 16> D0, X[3];
      Ten<T, 36> Y[3], D1;
      Ten<T, 64> D2;
      Ten<T, 49> Q2;
      Ten<T, 25> QT;
      Ten<T, 9> T2;
    };
    struct {  // irradiance: the ratio's operands at degree (10, 10)
      Ten<T, 121> detMe, Q3e;
    };
  };
  Ten<T, 100> detM, Q3;
};

struct BoxOut {
  int status;  // 0 culled, 1 live, 2 needs higher precision
  float uk[4];
  float E[2];
  bool settled;
};

// Outward conversion of a bound endpoint to FP32.
template <class T>
__device__ __forceinline__ float out_lo(T x) {
  float f = float(x);
  if (T(f) > x) f = nextafterf(f, -INFINITY);
  return f;
}
template <class T>
__device__ __forceinline__ float out_hi(T x) {
  float f = float(x);
  if (T(f) < x) f = nextafterf(f, INFINITY);
  return f;
}

// NT lanes evaluate the box (a wave, or a group of 16 or 32 lanes of one when
// several boxes share a wave; groups run the same sequence of barriers, so a
// box outside the triangle is only marked, not returned from, until the last
// one).
template <class T, bool IRR, class Lds, int NT = BBC_WAVE>
__device__ BoxOut eval_box_r(const TupleGeom<T>& G, T u0, T u1, T v0, T v1, bool final, Lds& L, int lane) {
  const T eps = Eps<T>::u;
  BoxOut out;
  out.status = 0;
  out.settled = false;
  out.uk[0] = 0.f;
  out.uk[1] = 1.f;
  out.uk[2] = 0.f;
  out.uk[3] = 1.f;
  out.E[0] = 0.f;
  out.E[1] = INFINITY;
  const bool outside = !G.front || u0 + v0 >= T(1);
  if constexpr (NT == BBC_WAVE || IRR) {
    if (outside) return out;
  }

  // ---- linear forms: values at the box corners (scaled = plain at degree 1)
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
    Ten<T, 4>& dst = which == 0 ? L.n[c] : (which == 1 ? L.d0[c] : L.s[c]);
    dst.v[k] = fma(d, v, fma(b, u, a));
    dst.m[k] = fabs(a) + fabs(b) * fabs(u) + fabs(d) * fabs(v);
  }
  // the constants carry one rounding (differences of FP32 inputs), the corner
  // evaluation two more
  const T th_lin = T(4) * eps;
  wave_sync();

  // ---- s x f1 and the degree-(2,2) dot products n.n, d0.n (and for the
  // irradiance n_g.d0, d0.d0 and the derivative linear forms)
  {
    const T* sv[3] = {L.s[0].v, L.s[1].v, L.s[2].v};
    const T* sm[3] = {L.s[0].m, L.s[1].m, L.s[2].m};
    const V3<T> f1 = G.f1;
    const T ax[3] = {T(0), f1.z, -f1.y}, ay[3] = {-f1.z, T(0), f1.x}, az[3] = {f1.y, -f1.x, T(0)};
    combo_b<4, 3, false, T, NT>(sv, sm, ax, L.sf1[0].v, L.sf1[0].m, lane);
    combo_b<4, 3, false, T, NT>(sv, sm, ay, L.sf1[1].v, L.sf1[1].m, lane);
    combo_b<4, 3, false, T, NT>(sv, sm, az, L.sf1[2].v, L.sf1[2].m, lane);
    for (int c = 0; c < 3; ++c) {
      if (c == 0) {
        conv_b<1, 1, 1, 1, false, T, NT>(L.n[c].v, L.n[c].m, L.n[c].v, L.n[c].m, L.nn.v, L.nn.m, T(1), lane);
        conv_b<1, 1, 1, 1, false, T, NT>(L.d0[c].v, L.d0[c].m, L.n[c].v, L.n[c].m, L.dn.v, L.dn.m, T(1), lane);
      } else {
        conv_b<1, 1, 1, 1, true, T, NT>(L.n[c].v, L.n[c].m, L.n[c].v, L.n[c].m, L.nn.v, L.nn.m, T(1), lane);
        conv_b<1, 1, 1, 1, true, T, NT>(L.d0[c].v, L.d0[c].m, L.n[c].v, L.n[c].m, L.dn.v, L.dn.m, T(1), lane);
      }
    }
    if constexpr (IRR) {
      const T* dv[3] = {L.d0[0].v, L.d0[1].v, L.d0[2].v};
      const T* dm[3] = {L.d0[0].m, L.d0[1].m, L.d0[2].m};
      const T ag[3] = {G.ng.x, G.ng.y, G.ng.z};
      combo_b<4, 3, false, T, NT>(dv, dm, ag, L.g.v, L.g.m, lane);
      // d(n.n)/du = 2 n.dn1,  d(d0.n)/du = e1.n + d0.dn1  (and the same in v)
      const T* nv[3] = {L.n[0].v, L.n[1].v, L.n[2].v};
      const T* nm[3] = {L.n[0].m, L.n[1].m, L.n[2].m};
      const T a_nnu[3] = {T(2) * G.dn1.x, T(2) * G.dn1.y, T(2) * G.dn1.z};
      const T a_nnv[3] = {T(2) * G.dn2.x, T(2) * G.dn2.y, T(2) * G.dn2.z};
      combo_b<4, 3, false, T, NT>(nv, nm, a_nnu, L.nnu.v, L.nnu.m, lane);
      combo_b<4, 3, false, T, NT>(nv, nm, a_nnv, L.nnv.v, L.nnv.m, lane);
      const T* xv[6] = {L.n[0].v, L.n[1].v, L.n[2].v, L.d0[0].v, L.d0[1].v, L.d0[2].v};
      const T* xm[6] = {L.n[0].m, L.n[1].m, L.n[2].m, L.d0[0].m, L.d0[1].m, L.d0[2].m};
      const T a_dnu[6] = {G.e1.x, G.e1.y, G.e1.z, G.dn1.x, G.dn1.y, G.dn1.z};
      const T a_dnv[6] = {G.e2.x, G.e2.y, G.e2.z, G.dn2.x, G.dn2.y, G.dn2.z};
      combo_b<4, 6, false, T, NT>(xv, xm, a_dnu, L.dnu.v, L.dnu.m, lane);
      combo_b<4, 6, false, T, NT>(xv, xm, a_dnv, L.dnv.v, L.dnv.m, lane);
      for (int c = 0; c < 3; ++c) {
        if (c == 0)
          conv_b<1, 1, 1, 1, false, T, NT>(L.d0[c].v, L.d0[c].m, L.d0[c].v, L.d0[c].m, L.h.v, L.h.m, T(1), lane);
        else
          conv_b<1, 1, 1, 1, true, T, NT>(L.d0[c].v, L.d0[c].m, L.d0[c].v, L.d0[c].m, L.h.v, L.h.m, T(1), lane);
      }
    }
  }
  const T th_sf1 = th_lin + T(4) * eps;
  const T th_g = th_lin + T(8) * eps;  // the unit normal carries a few roundings of its own
  const T th_nnu = th_lin + T(5) * eps, th_dnu = th_lin + T(8) * eps;
  const T th_nn = conv_theta<1, 1, 1, 1>(th_lin, th_lin) + T(3) * eps;  // three accumulated products
  wave_sync();

  // ---- reflected direction d~ = (n.n) d0 - 2 (d0.n) n, and its derivatives
  //      d~_u = (n.n)_u d0 + (n.n) e1 - 2 ((d0.n)_u n + (d0.n) dn1)
  for (int c = 0; c < 3; ++c) {
    conv_b<2, 2, 1, 1, false, T, NT>(L.nn.v, L.nn.m, L.d0[c].v, L.d0[c].m, L.dt[c].v, L.dt[c].m, T(1), lane);
    conv_b<2, 2, 1, 1, true, T, NT>(L.dn.v, L.dn.m, L.n[c].v, L.n[c].m, L.dt[c].v, L.dt[c].m, T(-2), lane);
    if constexpr (IRR) {
      conv_b<1, 1, 1, 1, false, T, NT>(L.nnu.v, L.nnu.m, L.d0[c].v, L.d0[c].m, L.dtu[c].v, L.dtu[c].m, T(1), lane);
      conv_b<1, 1, 1, 1, true, T, NT>(L.dnu.v, L.dnu.m, L.n[c].v, L.n[c].m, L.dtu[c].v, L.dtu[c].m, T(-2), lane);
      conv_b<1, 1, 1, 1, false, T, NT>(L.nnv.v, L.nnv.m, L.d0[c].v, L.d0[c].m, L.dtv[c].v, L.dtv[c].m, T(1), lane);
      conv_b<1, 1, 1, 1, true, T, NT>(L.dnv.v, L.dnv.m, L.n[c].v, L.n[c].m, L.dtv[c].v, L.dtv[c].m, T(-2), lane);
    }
  }
  wave_sync();
  T th_dtu = T(0);
  if constexpr (IRR) {
    for (int c = 0; c < 3; ++c) {
      const T* xv[2] = {L.nn.v, L.dn.v};
      const T* xm[2] = {L.nn.m, L.dn.m};
      const T au[2] = {comp(G.e1, c), T(-2) * comp(G.dn1, c)};
      const T av[2] = {comp(G.e2, c), T(-2) * comp(G.dn2, c)};
      combo_b<9, 2, true, T, NT>(xv, xm, au, L.dtu[c].v, L.dtu[c].m, lane);
      combo_b<9, 2, true, T, NT>(xv, xm, av, L.dtv[c].v, L.dtv[c].m, lane);
    }
    th_dtu = max(max(conv_theta<1, 1, 1, 1>(th_nnu, th_lin), conv_theta<1, 1, 1, 1>(th_dnu, th_lin)),
                 th_nn + T(2) * eps) +
             T(6) * eps;
    wave_sync();
  }
  const T th_dt = conv_theta<2, 2, 1, 1>(th_nn, th_lin) + T(2) * eps;

  // ---- c = d~ x f2
  {
    const V3<T> f2 = G.f2;
    const T ax[3] = {T(0), f2.z, -f2.y}, ay[3] = {-f2.z, T(0), f2.x}, az[3] = {f2.y, -f2.x, T(0)};
    const T* al[3] = {ax, ay, az};
    const T* dv[3] = {L.dt[0].v, L.dt[1].v, L.dt[2].v};
    const T* dm[3] = {L.dt[0].m, L.dt[1].m, L.dt[2].m};
    for (int c = 0; c < 3; ++c) combo_b<16, 3, false, T, NT>(dv, dm, al[c], L.cc[c].v, L.cc[c].m, lane);
  }
  const T th_cc = th_dt + T(3) * eps;
  wave_sync();

  // ---- Pu = c.s, Pv = (s x f1).d~, Q = c.f1, t numerator Tn = (s x f1).f2
  for (int c = 0; c < 3; ++c) {
    if (c == 0) {
      conv_b<3, 3, 1, 1, false, T, NT>(L.cc[c].v, L.cc[c].m, L.s[c].v, L.s[c].m, L.Pu.v, L.Pu.m, T(1), lane);
      conv_b<3, 3, 1, 1, false, T, NT>(L.dt[c].v, L.dt[c].m, L.sf1[c].v, L.sf1[c].m, L.Pv.v, L.Pv.m, T(1), lane);
    } else {
      conv_b<3, 3, 1, 1, true, T, NT>(L.cc[c].v, L.cc[c].m, L.s[c].v, L.s[c].m, L.Pu.v, L.Pu.m, T(1), lane);
      conv_b<3, 3, 1, 1, true, T, NT>(L.dt[c].v, L.dt[c].m, L.sf1[c].v, L.sf1[c].m, L.Pv.v, L.Pv.m, T(1), lane);
    }
  }
  {
    const T* cv[3] = {L.cc[0].v, L.cc[1].v, L.cc[2].v};
    const T* cm[3] = {L.cc[0].m, L.cc[1].m, L.cc[2].m};
    const T* sv[3] = {L.sf1[0].v, L.sf1[1].v, L.sf1[2].v};
    const T* sm[3] = {L.sf1[0].m, L.sf1[1].m, L.sf1[2].m};
    const T af1[3] = {G.f1.x, G.f1.y, G.f1.z}, af2[3] = {G.f2.x, G.f2.y, G.f2.z};
    combo_b<16, 3, false, T, NT>(cv, cm, af1, L.Q.v, L.Q.m, lane);
    combo_b<4, 3, false, T, NT>(sv, sm, af2, L.Tn.v, L.Tn.m, lane);
  }
  wave_sync();
  elev11_b<3, 3, T, NT>(L.Q.v, L.Q.m, L.Qe.v, L.Qe.m, lane);
  elev11_b<1, 1, T, NT>(L.Tn.v, L.Tn.m, L.Tn2.v, L.Tn2.m, lane);
  const T th_P = conv_theta<3, 3, 1, 1>(th_cc, th_lin) + T(3) * eps;
  const T th_Q = th_cc + T(3) * eps;
  const T th_Tn = th_sf1 + T(3) * eps;
  wave_sync();
  elev11_b<2, 2, T, NT>(L.Tn2.v, L.Tn2.m, L.Tne.v, L.Tne.m, lane);
  wave_sync();

  // ---- position bound (Sec. 4.2) and the sign of the ray parameter
  const RB<T> tb = ratio_bound<16, T, NT>(L.Tne.v, L.Tne.m, th_Tn + T(4) * eps, L.Q.v, L.Q.m, th_Q, final, lane);
  const RB<T> ub = ratio_bound<25, T, NT>(L.Pu.v, L.Pu.m, th_P, L.Qe.v, L.Qe.m, th_Q + T(2) * eps, final, lane);
  const RB<T> vb = ratio_bound<25, T, NT>(L.Pv.v, L.Pv.m, th_P, L.Qe.v, L.Qe.m, th_Q + T(2) * eps, final, lane);
  if (outside) return out;
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
    // ---- irradiance bound (Sec. 4.4): det M = -(Q^2 D0 + Q Tn D1 + Tn^2 D2);
    // its parts overwrite the position tensors
    wave_sync();
    {
      const V3<T> n12 = cross(G.e1, G.e2), e2 = G.e2, e1 = G.e1;
      const T* dv[3] = {L.dt[0].v, L.dt[1].v, L.dt[2].v};
      const T* dm[3] = {L.dt[0].m, L.dt[1].m, L.dt[2].m};
      const T a12[3] = {n12.x, n12.y, n12.z};
      combo_b<16, 3, false, T, NT>(dv, dm, a12, L.D0.v, L.D0.m, lane);
      // X = e2 x d~
      const T xx[3] = {T(0), -e2.z, e2.y}, xy[3] = {e2.z, T(0), -e2.x}, xz[3] = {-e2.y, e2.x, T(0)};
      combo_b<16, 3, false, T, NT>(dv, dm, xx, L.X[0].v, L.X[0].m, lane);
      combo_b<16, 3, false, T, NT>(dv, dm, xy, L.X[1].v, L.X[1].m, lane);
      combo_b<16, 3, false, T, NT>(dv, dm, xz, L.X[2].v, L.X[2].m, lane);
      // Y = d~_v x d~
      for (int c = 0; c < 3; ++c) {
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        conv_b<2, 2, 3, 3, false, T, NT>(L.dtv[a].v, L.dtv[a].m, L.dt[b].v, L.dt[b].m, L.Y[c].v, L.Y[c].m, T(1), lane);
        conv_b<2, 2, 3, 3, true, T, NT>(L.dtv[b].v, L.dtv[b].m, L.dt[a].v, L.dt[a].m, L.Y[c].v, L.Y[c].m, T(-1), lane);
      }
      conv_b<3, 3, 3, 3, false, T, NT>(L.Q.v, L.Q.m, L.Q.v, L.Q.m, L.Q2.v, L.Q2.m, T(1), lane);
      conv_b<3, 3, 1, 1, false, T, NT>(L.Q.v, L.Q.m, L.Tn.v, L.Tn.m, L.QT.v, L.QT.m, T(1), lane);
      conv_b<1, 1, 1, 1, false, T, NT>(L.Tn.v, L.Tn.m, L.Tn.v, L.Tn.m, L.T2.v, L.T2.m, T(1), lane);
      wave_sync();
      // D1 = d~_u . (e2 x d~) + e1 . (d~_v x d~),  D2 = d~_u . (d~_v x d~)
      for (int c = 0; c < 3; ++c) {
        if (c == 0) {
          conv_b<2, 2, 3, 3, false, T, NT>(L.dtu[c].v, L.dtu[c].m, L.X[c].v, L.X[c].m, L.D1.v, L.D1.m, T(1), lane);
          conv_b<2, 2, 5, 5, false, T, NT>(L.dtu[c].v, L.dtu[c].m, L.Y[c].v, L.Y[c].m, L.D2.v, L.D2.m, T(1), lane);
        } else {
          conv_b<2, 2, 3, 3, true, T, NT>(L.dtu[c].v, L.dtu[c].m, L.X[c].v, L.X[c].m, L.D1.v, L.D1.m, T(1), lane);
          conv_b<2, 2, 5, 5, true, T, NT>(L.dtu[c].v, L.dtu[c].m, L.Y[c].v, L.Y[c].m, L.D2.v, L.D2.m, T(1), lane);
        }
      }
      wave_sync();
      const T* yv[3] = {L.Y[0].v, L.Y[1].v, L.Y[2].v};
      const T* ym[3] = {L.Y[0].m, L.Y[1].m, L.Y[2].m};
      const T ae1[3] = {e1.x, e1.y, e1.z};
      combo_b<36, 3, true, T, NT>(yv, ym, ae1, L.D1.v, L.D1.m, lane);
    }
    const T th_D0 = th_dt + T(4) * eps;
    const T th_X = th_dt + T(3) * eps;
    const T th_Y = conv_theta<2, 2, 3, 3>(th_dtu, th_dt) + eps;
    const T th_D1 = max(conv_theta<2, 2, 3, 3>(th_dtu, th_X), th_Y + T(3) * eps) + T(4) * eps;
    const T th_D2 = conv_theta<2, 2, 5, 5>(th_dtu, th_Y) + T(2) * eps;
    const T th_Q2 = conv_theta<3, 3, 3, 3>(th_Q, th_Q);
    const T th_QT = conv_theta<3, 3, 1, 1>(th_Q, th_Tn);
    const T th_T2 = conv_theta<1, 1, 1, 1>(th_Tn, th_Tn);
    wave_sync();
    conv_b<6, 6, 3, 3, false, T, NT>(L.Q2.v, L.Q2.m, L.D0.v, L.D0.m, L.detM.v, L.detM.m, T(-1), lane);
    conv_b<4, 4, 5, 5, true, T, NT>(L.QT.v, L.QT.m, L.D1.v, L.D1.m, L.detM.v, L.detM.m, T(-1), lane);
    conv_b<2, 2, 7, 7, true, T, NT>(L.T2.v, L.T2.m, L.D2.v, L.D2.m, L.detM.v, L.detM.m, T(-1), lane);
    conv_b<6, 6, 3, 3, false, T, NT>(L.Q2.v, L.Q2.m, L.Q.v, L.Q.m, L.Q3.v, L.Q3.m, T(1), lane);
    const T th_detM = max(max(conv_theta<6, 6, 3, 3>(th_Q2, th_D0), conv_theta<4, 4, 5, 5>(th_QT, th_D1)),
                          conv_theta<2, 2, 7, 7>(th_T2, th_D2)) +
                      T(2) * eps;
    const T th_Q3 = conv_theta<6, 6, 3, 3>(th_Q2, th_Q);
    wave_sync();
    elev11_b<9, 9, T, NT>(L.detM.v, L.detM.m, L.detMe.v, L.detMe.m, lane);
    elev11_b<9, 9, T, NT>(L.Q3.v, L.Q3.m, L.Q3e.v, L.Q3e.m, lane);
    wave_sync();
    const RB<T> rb = ratio_bound<121, T, NT>(L.Q3e.v, L.Q3e.m, th_Q3 + T(2) * eps, L.detMe.v, L.detMe.m,
                                      th_detM + T(2) * eps, final, lane);
    if (rb.uncertain) {
      out.status = 2;
      return out;
    }
    T rlo, rhi;
    abs_bound(rb, &rlo, &rhi);
    // dOmega0/dA1 = |g| / h^(3/2) with g = n_g . d0 and h = d0 . d0, bounded factor-wise
    T glo, ghi, hlo, hhi;
    poly_range<1, 1, T, NT>(L.g.v, L.g.m, th_g, &glo, &ghi, lane);
    poly_range<2, 2, T, NT>(L.h.v, L.h.m, th_nn, &hlo, &hhi, lane);
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
