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
// LDS of the position and irradiance bound (subdivision).  The polynomials a
// box's bounds are read from (Pu, Pv, Q, Tn, det M, Q^3, g, h) come first, in
// the order of a child record in HBM (see split_box_r); the position tensors
// that the irradiance part no longer reads share their space with the
// cofactor parts of det M, and those with the elevated det M and Q^3 and with
// the children's half-split tensors.
template <class T>
struct LdsR {
  struct {  // the box's record
    Ten<T, 25> Pu, Pv;
    Ten<T, 16> Q;
    Ten<T, 4> Tn;
    Ten<T, 100> detM, Q3;
    Ten<T, 4> g;
    Ten<T, 9> h;
  };
  // live through the whole evaluation
  Ten<T, 16> dt[3];
  Ten<T, 4> nnu, nnv, dnu, dnv;
  Ten<T, 9> dtu[3], dtv[3];
  union {
    struct {  // position bound
      Ten<T, 4> n[3], d0[3], s[3], sf1[3];
      Ten<T, 9> nn, dn, Tn2;
      Ten<T, 16> cc[3];
      Ten<T, 25> Qe;
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
    T half[1132];  // the children's tensors split along u (split_box_r)
  };
};

// LDS of a box bounded from its record (eval_box_r_rec, split_box_r): the
// record block as in LdsR, then the elevated operands, or the children's
// half-split tensors.
template <class T>
struct LdsRRec {
  struct {
    Ten<T, 25> Pu, Pv;
    Ten<T, 16> Q;
    Ten<T, 4> Tn;
    Ten<T, 100> detM, Q3;
    Ten<T, 4> g;
    Ten<T, 9> h;
  };
  union {
    struct {
      Ten<T, 25> Qe;
      Ten<T, 9> Tn2;
      Ten<T, 16> Tne;
    };
    struct {
      Ten<T, 121> detMe, Q3e;
    };
    T half[1132];
  };
};

// A box's record: the scaled Bernstein coefficients and magnitudes of Pu, Pv,
// Q, Tn, det M, Q^3, g and h in the order of LdsR's first block, then their
// error factors and the tuple's constant factor; kRecR doubles per box.
constexpr int kRecCoef = 2 * (25 + 25 + 16 + 4 + 100 + 100 + 4 + 9), kRecR = 576;
template <class T>
struct BoxTheta {
  T P, Q, Tn, detM, Q3, g, h;  // error factors
  T k;                          // the tuple's constant factor I0 a1 / ak
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

// Position bound of a box from Tn, Q, Pu and Pv in L with error factors
// th_Tn, th_Q, th_P (Sec. 4.2): Q and Tn raised to the degrees of Pu and Q, the
// ratio bounds of t = Tn/Q, u_k = Pu/Q and v_k = Pv/Q, the clip to the
// receiver.  False when the box is done (outside its triangle, culled, or to be
// redone at higher precision: out.status says which).
template <class T, class Lds, int NT>
__device__ bool pos_bound_r(Lds& L, T th_P, T th_Q, T th_Tn, bool final, bool outside, BoxOut& out, int lane) {
  const T eps = Eps<T>::u;
  elev11_b<3, 3, T, NT>(L.Q.v, L.Q.m, L.Qe.v, L.Qe.m, lane);
  elev11_b<1, 1, T, NT>(L.Tn.v, L.Tn.m, L.Tn2.v, L.Tn2.m, lane);
  wave_sync();
  elev11_b<2, 2, T, NT>(L.Tn2.v, L.Tn2.m, L.Tne.v, L.Tne.m, lane);
  wave_sync();

  // ---- position bound (Sec. 4.2) and the sign of the ray parameter
  const RB<T> tb = ratio_bound<16, T, NT>(L.Tne.v, L.Tne.m, th_Tn + T(4) * eps, L.Q.v, L.Q.m, th_Q, final, lane);
  const RB<T> ub = ratio_bound<25, T, NT>(L.Pu.v, L.Pu.m, th_P, L.Qe.v, L.Qe.m, th_Q + T(2) * eps, final, lane);
  const RB<T> vb = ratio_bound<25, T, NT>(L.Pv.v, L.Pv.m, th_P, L.Qe.v, L.Qe.m, th_Q + T(2) * eps, final, lane);
  if (outside) return false;
  if (tb.uncertain || ub.uncertain || vb.uncertain) {
    out.status = 2;
    return false;
  }
  if (tb.kind == kDirect && tb.hi <= T(0)) return false;  // every ray points away from the receiver
  T ulo, uhi, vlo, vhi;
  if (!clip01(ub, &ulo, &uhi) || !clip01(vb, &vlo, &vhi)) return false;
  out.uk[0] = out_lo(ulo);
  out.uk[1] = out_hi(uhi);
  out.uk[2] = out_lo(vlo);
  out.uk[3] = out_hi(vhi);
  out.settled = ub.kind == kDirect && vb.kind == kDirect && ub.lo >= T(0) && ub.hi <= T(1) && vb.lo >= T(0) &&
                vb.hi <= T(1) && tb.kind == kDirect && tb.lo > T(0);
  out.status = 1;
  return true;
}

// Irradiance bound of a live box from det M, Q^3, g and h in L with their
// error factors (Sec. 4.4, Eq. eq_dwda): det M and Q^3 raised to (10, 10),
// the ratio bound of Q^3 / det M, the solid-angle factor |g| / h^(3/2)
// bounded factor-wise, times the tuple's constant factor k = I0 a1 / ak.
template <class T, int NT, class Lds>
__device__ void irr_bound_r(T k, Lds& L, T th_detM, T th_Q3, T th_g, T th_h, bool final, BoxOut& out, int lane) {
  const T eps = Eps<T>::u;
  elev11_b<9, 9, T, NT>(L.detM.v, L.detM.m, L.detMe.v, L.detMe.m, lane);
  elev11_b<9, 9, T, NT>(L.Q3.v, L.Q3.m, L.Q3e.v, L.Q3e.m, lane);
  wave_sync();
  const RB<T> rb = ratio_bound<121, T, NT>(L.Q3e.v, L.Q3e.m, th_Q3 + T(2) * eps, L.detMe.v, L.detMe.m,
                                    th_detM + T(2) * eps, final, lane);
  if (rb.uncertain) {
    out.status = 2;
    return;
  }
  T rlo, rhi;
  abs_bound(rb, &rlo, &rhi);
  // dOmega0/dA1 = |g| / h^(3/2) with g = n_g . d0 and h = d0 . d0, bounded factor-wise
  T glo, ghi, hlo, hhi;
  poly_range<1, 1, T, NT>(L.g.v, L.g.m, th_g, &glo, &ghi, lane);
  poly_range<2, 2, T, NT>(L.h.v, L.h.m, th_h, &hlo, &hhi, lane);
  const T aglo = (glo <= T(0) && ghi >= T(0)) ? T(0) : min(fabs(glo), fabs(ghi));
  const T aghi = max(fabs(glo), fabs(ghi));
  const T Glo = down(aglo / (hhi * sqrt(hhi)));
  const T Ghi = hlo > T(0) ? up(aghi / (hlo * sqrt(hlo))) : T(INFINITY);
  const T klo = k * (T(1) - T(16) * eps), khi = k * (T(1) + T(16) * eps);
  const T Elo = (Glo <= T(0) || rlo <= T(0)) ? T(0) : down(klo * down(Glo * rlo));
  const T Ehi = (isinf(Ghi) || isinf(rhi)) ? T(INFINITY) : up(khi * up(Ghi * rhi));
  out.E[0] = out_lo(Elo);
  out.E[1] = out_hi(Ehi);
}

// NT lanes evaluate the box (a wave, or a group of 16 or 32 lanes of one when
// several boxes share a wave; groups run the same sequence of barriers, so a
// box outside the triangle is only marked, not returned from, until the last
// one).
template <class T, bool IRR, class Lds, int NT = BBC_WAVE>
__device__ BoxOut eval_box_r(const TupleGeom<T>& G, T u0, T u1, T v0, T v1, bool final, Lds& L, int lane,
                             BoxTheta<T>* th = nullptr) {
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
  const T th_P = conv_theta<3, 3, 1, 1>(th_cc, th_lin) + T(3) * eps;
  const T th_Q = th_cc + T(3) * eps;
  const T th_Tn = th_sf1 + T(3) * eps;
  if (!pos_bound_r<T, Lds, NT>(L, th_P, th_Q, th_Tn, final, outside, out, lane)) return out;
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
    const T k = G.I0 * G.a1 / G.ak;
    if (th) *th = BoxTheta<T>{th_P, th_Q, th_Tn, th_detM, th_Q3, th_g, th_nn, k};
    irr_bound_r<T, NT>(k, L, th_detM, th_Q3, th_g, th_nn, final, out, lane);
    return out;
  }
}

// ---- Subdivision from the parent's polynomials (Sec. 4.1: the Bernstein
// coefficients of a polynomial on half of its box follow from those on the
// whole box).  Record layout (doubles): Pu 0, Pv 50, Q 100, Tn 132, det M 140,
// Q^3 340, g 540, h 548 (each tensor's values, then its magnitudes), the error
// factors (P, Q, Tn, det M, Q^3, g, h) and the tuple's constant at kRecCoef.
constexpr int kRecPu = 0, kRecPv = 50, kRecQ = 100, kRecTn = 132, kRecDM = 140, kRecQ3 = 340, kRecG = 540,
              kRecH = 548;
static_assert(kRecH + 18 == kRecCoef && kRecCoef + 8 <= kRecR, "record layout");

// Bounds of a box whose polynomials its parent wrote to `rec` (a record of
// kRecR doubles); the same steps as eval_box_r after its products, so the box
// ends with its record in L for split_box_r.  `th` receives the error factors
// and the tuple's constant.  The tuple faces its light (its parent was live).
template <class T, class Lds, int NT = BBC_WAVE>
__device__ BoxOut eval_box_r_rec(const T* __restrict__ rec, T u0, T v0, Lds& L, BoxTheta<T>* th, int lane) {
  static_assert(sizeof(Ten<T, 25>) == 50 * sizeof(T), "tensors are packed");
  BoxOut out;
  out.status = 0;
  out.settled = false;
  out.uk[0] = 0.f;
  out.uk[1] = 1.f;
  out.uk[2] = 0.f;
  out.uk[3] = 1.f;
  out.E[0] = 0.f;
  out.E[1] = INFINITY;
  if (u0 + v0 >= T(1)) return out;
  T* dst = L.Pu.v;
  for (int o = lane; o < kRecCoef; o += NT) dst[o] = rec[o];
  const BoxTheta<T> t{rec[kRecCoef],     rec[kRecCoef + 1], rec[kRecCoef + 2], rec[kRecCoef + 3],
                      rec[kRecCoef + 4], rec[kRecCoef + 5], rec[kRecCoef + 6], rec[kRecCoef + 7]};
  *th = t;
  wave_sync();
  if (!pos_bound_r<T, Lds, NT>(L, t.P, t.Q, t.Tn, true, false, out, lane)) return out;
  wave_sync();
  irr_bound_r<T, NT>(t.k, L, t.detM, t.Q3, t.g, t.h, true, out, lane);
  return out;
}

// One row of a tensor of degree (D1, D2) split along its first axis at the
// midpoint, in scaled form: left half s'_i = 2^-i sum_{j<=i} C(D1-j, i-j) s_j,
// right half s'_i = 2^-(D1-i) sum_{j>=i} C(j, i) s_j, along the row of stride
// `st` and length D1 + 1 starting at `in`; the halves go to out0 and out1 with
// the same stride.  Magnitudes take the same non-negative weights.
template <int D1, class T>
__device__ __forceinline__ void split_row(const T* in, const T* inm, int st, T* o0, T* o0m, T* o1, T* o1m) {
  T x[D1 + 1], xm[D1 + 1];
#pragma unroll
  for (int j = 0; j <= D1; ++j) {
    x[j] = in[j * st];
    xm[j] = inm[j * st];
  }
#pragma unroll
  for (int i = 0; i <= D1; ++i) {
    T a = 0, am = 0, b = 0, bm = 0;
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const T w = T(binom_i(D1 - j, i - j));
      a = fma(w, x[j], a);
      am = fma(w, xm[j], am);
    }
#pragma unroll
    for (int j = i; j <= D1; ++j) {
      const T w = T(binom_i(j, i));
      b = fma(w, x[j], b);
      bm = fma(w, xm[j], bm);
    }
    const T sa = T(1) / T(1 << i), sb = T(1) / T(1 << (D1 - i));  // powers of two: exact
    o0[i * st] = a * sa;
    o0m[i * st] = am * sa;
    o1[i * st] = b * sb;
    o1m[i * st] = bm * sb;
    __builtin_amdgcn_sched_barrier(0);  // one output pair at a time: bounded registers
  }
}

// Tensor (D1, D2) at (v, m): along u into the halves h (values [2][D1+1][D2+1],
// then magnitudes), one row per lane.
template <int D1, int D2, class T>
__device__ __forceinline__ void split_u_rows(const T* v, const T* m, T* h, int r) {
  constexpr int N2 = D2 + 1, NN = (D1 + 1) * N2;
  if (r < N2) split_row<D1>(v + r, m + r, N2, h + r, h + 2 * NN + r, h + NN + r, h + 3 * NN + r);
}
// Halves h along v into the four children's records at `rec` (child cu << 1 |
// cv at rec + child * kRecR, tensor at offset `off`: values, then magnitudes);
// row r = (cu, i) per lane.
template <int D1, int D2, class T>
__device__ __forceinline__ void split_v_rows(const T* h, T* rec, int off, int r) {
  constexpr int N2 = D2 + 1, NN = (D1 + 1) * N2;
  if (r < 2 * (D1 + 1)) {
    const int cu = r / (D1 + 1), i = r - cu * (D1 + 1);
    const T* in = h + cu * NN + i * N2;
    const T* inm = h + 2 * NN + cu * NN + i * N2;
    T* c0 = rec + (cu << 1) * kRecR + off + i * N2;        // v half 0
    T* c1 = rec + ((cu << 1) | 1) * kRecR + off + i * N2;  // v half 1
    split_row<D2>(in, inm, 1, c0, c0 + NN, c1, c1 + NN);
  }
}

// Splits the box whose record is in L (with error factors th) into the
// records of its four children at rec (kRecR doubles each, child cu << 1 | cv:
// u half cu, v half cv, as the subdivision codes its children).  Each axis adds
// (D + 2) eps to a tensor's error factor: D + 1 rounded terms of exact integer
// weights, times a power of two, and the magnitudes' own rounding.  The
// tuple's constant is copied.
template <class T, class Lds, int NT = BBC_WAVE>
__device__ void split_box_r(Lds& L, const BoxTheta<T>& th, T* __restrict__ rec, int lane) {
  const T eps = Eps<T>::u;
  // halves along u, one row per lane; tensors of one degree share a branch
  // (det M and Q^3: lanes 0-19, Pu and Pv: 20-29, Q: 30-33, Tn and g: 34-37,
  // h: 38-40)
  T* H = L.half;
  constexpr int hDM = 0, hQ3 = 400, hPu = 800, hPv = 900, hQ = 1000, hTn = 1064, hG = 1080, hH = 1096;
  static_assert(hH + 36 <= int(sizeof(L.half) / sizeof(T)), "half-split buffer");
  wave_sync();
  if (lane < 20) {
    const bool q3 = lane >= 10;
    split_u_rows<9, 9>(q3 ? L.Q3.v : L.detM.v, q3 ? L.Q3.m : L.detM.m, H + (q3 ? hQ3 : hDM), lane - (q3 ? 10 : 0));
  } else if (lane < 30) {
    const bool pv = lane >= 25;
    split_u_rows<4, 4>(pv ? L.Pv.v : L.Pu.v, pv ? L.Pv.m : L.Pu.m, H + (pv ? hPv : hPu), lane - (pv ? 25 : 20));
  } else if (lane < 34) {
    split_u_rows<3, 3>(L.Q.v, L.Q.m, H + hQ, lane - 30);
  } else if (lane < 38) {
    const bool g = lane >= 36;
    split_u_rows<1, 1>(g ? L.g.v : L.Tn.v, g ? L.g.m : L.Tn.m, H + (g ? hG : hTn), lane - (g ? 36 : 34));
  } else if (lane < 41) {
    split_u_rows<2, 2>(L.h.v, L.h.m, H + hH, lane - 38);
  }
  wave_sync();
  // halves along v into the records, one row (u half, index) per lane: det M
  // and Q^3 (lanes 0-39), Pu and Pv (40-59), Tn (60-63); then Q (0-7), g
  // (8-11), h (12-17)
  if (lane < 40) {
    const bool q3 = lane >= 20;
    split_v_rows<9, 9>(H + (q3 ? hQ3 : hDM), rec, q3 ? kRecQ3 : kRecDM, lane - (q3 ? 20 : 0));
  } else if (lane < 60) {
    const bool pv = lane >= 50;
    split_v_rows<4, 4>(H + (pv ? hPv : hPu), rec, pv ? kRecPv : kRecPu, lane - (pv ? 50 : 40));
  } else {
    split_v_rows<1, 1>(H + hTn, rec, kRecTn, lane - 60);
  }
  if (lane < 8) {
    split_v_rows<3, 3>(H + hQ, rec, kRecQ, lane);
  } else if (lane < 12) {
    split_v_rows<1, 1>(H + hG, rec, kRecG, lane - 8);
  } else if (lane < 18) {
    split_v_rows<2, 2>(H + hH, rec, kRecH, lane - 12);
  }
  // error factors
  if (lane < 32) {
    const int c = lane / 8, k = lane - 8 * (lane / 8);
    const T f[8] = {th.P + T(4 + 4 + 4) * eps, th.Q + T(3 + 3 + 4) * eps, th.Tn + T(1 + 1 + 4) * eps,
                    th.detM + T(9 + 9 + 4) * eps, th.Q3 + T(9 + 9 + 4) * eps, th.g + T(1 + 1 + 4) * eps,
                    th.h + T(2 + 2 + 4) * eps, th.k};
    rec[c * kRecR + kRecCoef + k] = f[k];
  }
  wave_sync();
}

}  // namespace bbc
