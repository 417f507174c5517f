// Position and irradiance bound of one box of a single-reflection tuple lit
// by an area light x0 + z1 a + z2 b, (z1, z2) in [0,1]^2 (the emitter
// variable of the implementation section's area-light remark).  The light's
// two parameters are two more axes of every polynomial, never subdivided, so
// the bounds hold for every point of the light:
//   d0 = x1 - x0 - z1 a - z2 b          degree (1,1,1,1) in (u, v, z1, z2),
//   d~ = (n.n) d0 - 2 (d0.n) n          (3,3,1,1),
//   u_k = Pu/Q, v_k = Pv/Q (Eq. eq_rct)   Pu, Pv (4,4,1,1), Q (3,3,1,1),
//   E = I0 (A1/A_k) G1 |Q^3 / det M|   (Sec. 4.4), M = [[Q, Pu, Pv],
//   [Q_u, Pu_u, Pv_u], [Q_v, Pu_v, Pv_v]] with u-, v-derivatives only:
//   det M (9,9,3,3) and Q^3 both raised to (10,10,3,3).
// FP64 in scaled Bernstein form; every tensor carries magnitudes and an error
// factor theta (|computed - exact| <= theta * m), so the position and
// irradiance bounds are rounded outward (Eq. eq_bbound).
#pragma once
#include "box_t.hpp"

namespace bbc {

// LDS offsets (doubles) of the values; the magnitudes follow at the same
// offsets plus the size of the value block (RALay::mo).  Corner tensors
// (1,1,1,1) are indexed ((i * 2 + j) * 2 + k) * 2 + l over (u, v, z1, z2).
struct RALay {
  static constexpr int D0 = 0, N = 48, S = 60, NN = 72, DN = 81;          // 3x16, 3x4, 3x4, 9, 36
  static constexpr int DT = 117, CC = 309, SF1 = 501, PU = 513, PV = 613;  // 3x64, 3x64, 3x4, 100, 100
  static constexpr int Q = 713, TN = 777, TNE = 781, QE = 845;             // 64, 4, 64, 100
  static constexpr int POS_END = 945;
  static constexpr int GG = 945, HH = 961, NNU = 1042, NNV = 1046;        // 16, 81, 4, 4
  static constexpr int DNU = 1050, DNV = 1066, DTU = 1082, DTV = 1190;     // 16, 16, 3x36, 3x36
  static constexpr int CCU = 1298, CCV = 1406, QU = 1514, QV = 1550;       // 3x36, 3x36, 36, 36
  static constexpr int PUU = 1586, PUV = 1650, PVU = 1714, PVV = 1778;     // 64 each
  static constexpr int AM = 1842, BM = 2283, CM = 2607, Q2 = 2931;         // 441, 324, 324, 441
  static constexpr int DETM = 3372, Q3 = 4972, Q3E = 6572, END = 8508;     // 1600, 1600, 1936
  static constexpr int DETME = GG;                                         // 1936, over the dead GG .. CM
  static constexpr int mo(bool irr) { return irr ? END : POS_END; }
};

template <class T, bool IRR>
struct LdsRA {
  T buf[2 * RALay::mo(IRR)];
};

template <class T, bool IRR, int NT>
__device__ __forceinline__ BoxOut eval_box_ra(const TupleGeom<T>& G, T u0, T u1, T v0, T v1, LdsRA<T, IRR>& L,
                                              int lane) {
  T* B = L.buf;
  constexpr int MO = RALay::mo(IRR);
  auto at = [&](int off) { return TP<T>{B + off, B + MO + off}; };
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
  if (!G.front || u0 + v0 >= T(1)) return out;
  const TP<T> d0 = at(RALay::D0), nv = at(RALay::N), sv = at(RALay::S);
  // ---- corner values: d0 over (u, v, z1, z2), n and s = x1 - q0 over (u, v)
  // (the constants carry one rounding, the corner evaluation up to four more)
  const V3<T> pmx = G.p0 - G.x0, pmq = G.p0 - G.q0;
  for (int o = lane; o < 72; o += NT) {
    if (o < 48) {
      const int c = o / 16, r = o - 16 * c, i = r >> 3, j = (r >> 2) & 1, k = (r >> 1) & 1, l = r & 1;
      const T u = i ? u1 : u0, v = j ? v1 : v0;
      d0.v[o] = comp(pmx, c) + u * comp(G.e1, c) + v * comp(G.e2, c) - (T(k) * comp(G.ea, c) + T(l) * comp(G.eb, c));
      d0.m[o] = fabs(comp(pmx, c)) + fabs(u) * fabs(comp(G.e1, c)) + fabs(v) * fabs(comp(G.e2, c)) +
                T(k) * fabs(comp(G.ea, c)) + T(l) * fabs(comp(G.eb, c));
    } else {
      const int w = (o - 48) / 12, c = ((o - 48) / 4) % 3, r = (o - 48) & 3;
      const T u = (r >> 1) ? u1 : u0, v = (r & 1) ? v1 : v0;
      const V3<T> base = w == 0 ? G.n0 : pmq, du = w == 0 ? G.dn1 : G.e1, dv = w == 0 ? G.dn2 : G.e2;
      const TP<T> dst = w == 0 ? nv : sv;
      dst.v[4 * c + r] = comp(base, c) + u * comp(du, c) + v * comp(dv, c);
      dst.m[4 * c + r] = fabs(comp(base, c)) + fabs(u) * fabs(comp(du, c)) + fabs(v) * fabs(comp(dv, c));
    }
  }
  const T th_lin = T(8) * eps;
  wave_sync();
  const TP<T> nn = at(RALay::NN), dn = at(RALay::DN), sf1 = at(RALay::SF1), tn = at(RALay::TN);
  for (int c = 0; c < 3; ++c) {
    if (c == 0) {
      cv4m_b<1, 1, 0, 0, 1, 1, 0, 0, false, NT>(slice(nv, c, 4), slice(nv, c, 4), nn, T(1), lane);
      cv4m_b<1, 1, 1, 1, 1, 1, 0, 0, false, NT>(slice(d0, c, 16), slice(nv, c, 4), dn, T(1), lane);
    } else {
      cv4m_b<1, 1, 0, 0, 1, 1, 0, 0, true, NT>(slice(nv, c, 4), slice(nv, c, 4), nn, T(1), lane);
      cv4m_b<1, 1, 1, 1, 1, 1, 0, 0, true, NT>(slice(d0, c, 16), slice(nv, c, 4), dn, T(1), lane);
    }
  }
  for (int o = lane; o < 4; o += NT) {  // s x f1 and (s x f1).f2
    const V3<T> sc = mk(sv.v[o], sv.v[4 + o], sv.v[8 + o]);
    const V3<T> sm = mk(sv.m[o], sv.m[4 + o], sv.m[8 + o]);
    const V3<T> af1 = mk(fabs(G.f1.x), fabs(G.f1.y), fabs(G.f1.z));
    const V3<T> x = cross(sc, G.f1);
    const V3<T> xm = mk(sm.y * af1.z + sm.z * af1.y, sm.z * af1.x + sm.x * af1.z, sm.x * af1.y + sm.y * af1.x);
    sf1.v[o] = x.x;
    sf1.v[4 + o] = x.y;
    sf1.v[8 + o] = x.z;
    sf1.m[o] = xm.x;
    sf1.m[4 + o] = xm.y;
    sf1.m[8 + o] = xm.z;
    tn.v[o] = dot(x, G.f2);
    tn.m[o] = xm.x * fabs(G.f2.x) + xm.y * fabs(G.f2.y) + xm.z * fabs(G.f2.z);
  }
  const T th_nn = th_cv4<1, 1, 0, 0, 1, 1, 0, 0>(th_lin, th_lin, 3);
  const T th_sf1 = th_lin + T(3) * eps, th_tn = th_sf1 + T(4) * eps;
  wave_sync();
  // ---- d~ = (n.n) d0 - 2 (d0.n) n, c = d~ x f2, and Tn raised to Q's degree
  const TP<T> dt = at(RALay::DT), cc = at(RALay::CC), tne = at(RALay::TNE);
  for (int c = 0; c < 3; ++c) {
    cv4m_b<2, 2, 0, 0, 1, 1, 1, 1, false, NT>(nn, slice(d0, c, 16), slice(dt, c, 64), T(1), lane);
    cv4m_b<2, 2, 1, 1, 1, 1, 0, 0, true, NT>(dn, slice(nv, c, 4), slice(dt, c, 64), T(-2), lane);
  }
  elev4m_b<1, 1, 0, 0, 2, 2, 1, 1, NT>(tn, tne, lane);
  const T th_dt = th_cv4<2, 2, 1, 1, 1, 1, 0, 0>(th_nn, th_lin, 2);
  const T th_tne = th_elev4<2, 2, 1, 1>(th_tn);
  wave_sync();
  for (int o = lane; o < 64; o += NT) {
    const V3<T> x = cross(mk(dt.v[o], dt.v[64 + o], dt.v[128 + o]), G.f2);
    const V3<T> m = mk(dt.m[o], dt.m[64 + o], dt.m[128 + o]);
    const V3<T> af = mk(fabs(G.f2.x), fabs(G.f2.y), fabs(G.f2.z));
    cc.v[o] = x.x;
    cc.v[64 + o] = x.y;
    cc.v[128 + o] = x.z;
    cc.m[o] = m.y * af.z + m.z * af.y;
    cc.m[64 + o] = m.z * af.x + m.x * af.z;
    cc.m[128 + o] = m.x * af.y + m.y * af.x;
  }
  const T th_cc = th_dt + T(3) * eps;
  wave_sync();
  // ---- Pu = c.s, Pv = (s x f1).d~, Q = c.f1
  const TP<T> pu = at(RALay::PU), pv = at(RALay::PV), q = at(RALay::Q);
  for (int c = 0; c < 3; ++c) {
    if (c == 0) {
      cv4m_b<3, 3, 1, 1, 1, 1, 0, 0, false, NT>(slice(cc, c, 64), slice(sv, c, 4), pu, T(1), lane);
      cv4m_b<1, 1, 0, 0, 3, 3, 1, 1, false, NT>(slice(sf1, c, 4), slice(dt, c, 64), pv, T(1), lane);
    } else {
      cv4m_b<3, 3, 1, 1, 1, 1, 0, 0, true, NT>(slice(cc, c, 64), slice(sv, c, 4), pu, T(1), lane);
      cv4m_b<1, 1, 0, 0, 3, 3, 1, 1, true, NT>(slice(sf1, c, 4), slice(dt, c, 64), pv, T(1), lane);
    }
  }
  for (int o = lane; o < 64; o += NT) {
    q.v[o] = dot(mk(cc.v[o], cc.v[64 + o], cc.v[128 + o]), G.f1);
    q.m[o] = cc.m[o] * fabs(G.f1.x) + cc.m[64 + o] * fabs(G.f1.y) + cc.m[128 + o] * fabs(G.f1.z);
  }
  const T th_p = max(th_cv4<3, 3, 1, 1, 1, 1, 0, 0>(th_cc, th_lin, 3), th_cv4<1, 1, 0, 0, 3, 3, 1, 1>(th_sf1, th_dt, 3));
  const T th_q = th_cc + T(4) * eps;
  wave_sync();
  const TP<T> qe = at(RALay::QE);
  elev4m_b<3, 3, 1, 1, 1, 1, 0, 0, NT>(q, qe, lane);
  const T th_qe = th_elev4<1, 1, 0, 0>(th_q);
  wave_sync();
  // ---- position bound (Sec. 4.2) over the box and the whole light
  const RB<T> tb = ratio4m<T, NT>(64, tne, th_tne, q, th_q, true, lane);
  const RB<T> ub = ratio4m<T, NT>(100, pu, th_p, qe, th_qe, true, lane);
  const RB<T> vb = ratio4m<T, NT>(100, pv, th_p, qe, th_qe, true, lane);
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
    // ---- irradiance bound (Sec. 4.4) over the box and the whole light.  The
    // u-, v-derivatives of Q, Pu, Pv are formed by the product rule from the
    // exact derivatives of the linear forms (d0_u = s_u = e1, n_u = dn1), not
    // by differencing their coefficients (which cancels to O(w) of the terms
    // and would inflate det M's rounding bound by (degree / w)^2); det M then
    // has degree (9,9,3,3) and is elevated, with Q^3, to (10,10,3,3), the
    // degree at which differencing would give it.
    const TP<T> gg = at(RALay::GG), hh = at(RALay::HH), nnu = at(RALay::NNU), nnv = at(RALay::NNV);
    const TP<T> dnu = at(RALay::DNU), dnv = at(RALay::DNV), dtu = at(RALay::DTU), dtv = at(RALay::DTV);
    const TP<T> ccu = at(RALay::CCU), ccv = at(RALay::CCV), qu = at(RALay::QU), qv = at(RALay::QV);
    const TP<T> puu = at(RALay::PUU), puv = at(RALay::PUV), pvu = at(RALay::PVU), pvv = at(RALay::PVV);
    const V3<T> e1 = G.e1, e2 = G.e2, dn1 = G.dn1, dn2 = G.dn2;
    for (int o = lane; o < 16; o += NT) {
      gg.v[o] = dot(mk(d0.v[o], d0.v[16 + o], d0.v[32 + o]), G.ng);
      gg.m[o] = d0.m[o] * fabs(G.ng.x) + d0.m[16 + o] * fabs(G.ng.y) + d0.m[32 + o] * fabs(G.ng.z);
      // (d0.n)_u = e1.n + d0.dn1 over (u, v, z1, z2)
      const int ij = o >> 2;
      T su = T(0), sum = T(0), sv2 = T(0), svm = T(0);
      for (int c = 0; c < 3; ++c) {
        const T nc = nv.v[4 * c + ij], ncm = nv.m[4 * c + ij], dc = d0.v[16 * c + o], dcm = d0.m[16 * c + o];
        su = fma(comp(e1, c), nc, fma(dc, comp(dn1, c), su));
        sum += fabs(comp(e1, c)) * ncm + dcm * fabs(comp(dn1, c));
        sv2 = fma(comp(e2, c), nc, fma(dc, comp(dn2, c), sv2));
        svm += fabs(comp(e2, c)) * ncm + dcm * fabs(comp(dn2, c));
      }
      dnu.v[o] = su;
      dnu.m[o] = sum;
      dnv.v[o] = sv2;
      dnv.m[o] = svm;
    }
    for (int o = lane; o < 4; o += NT) {  // (n.n)_u = 2 n.dn1
      T su = T(0), sum = T(0), sv2 = T(0), svm = T(0);
      for (int c = 0; c < 3; ++c) {
        const T nc = nv.v[4 * c + o], ncm = nv.m[4 * c + o];
        su = fma(T(2) * comp(dn1, c), nc, su);
        sum += T(2) * fabs(comp(dn1, c)) * ncm;
        sv2 = fma(T(2) * comp(dn2, c), nc, sv2);
        svm += T(2) * fabs(comp(dn2, c)) * ncm;
      }
      nnu.v[o] = su;
      nnu.m[o] = sum;
      nnv.v[o] = sv2;
      nnv.m[o] = svm;
    }
    for (int c = 0; c < 3; ++c) {
      if (c == 0)
        cv4m_b<1, 1, 1, 1, 1, 1, 1, 1, false, NT>(slice(d0, c, 16), slice(d0, c, 16), hh, T(1), lane);
      else
        cv4m_b<1, 1, 1, 1, 1, 1, 1, 1, true, NT>(slice(d0, c, 16), slice(d0, c, 16), hh, T(1), lane);
    }
    const T th_g = th_lin + T(8) * eps;  // the unit normal carries a few roundings of its own
    const T th_h = th_cv4<1, 1, 1, 1, 1, 1, 1, 1>(th_lin, th_lin, 3);
    const T th_nnu = th_lin + T(5) * eps, th_dnu = th_lin + T(8) * eps;
    wave_sync();
    T glo, ghi, hlo, hhi;
    range4m<1, 1, 1, 1, T, NT>(gg, th_g, &glo, &ghi, lane);
    range4m<2, 2, 2, 2, T, NT>(hh, th_h, &hlo, &hhi, lane);
    // d~_u = (n.n)_u d0 + (n.n) e1 - 2 (d0.n)_u n - 2 (d0.n) dn1   (2,2,1,1)
    for (int c = 0; c < 3; ++c) {
      cv4m_b<1, 1, 0, 0, 1, 1, 1, 1, false, NT>(nnu, slice(d0, c, 16), slice(dtu, c, 36), T(1), lane);
      cv4m_b<1, 1, 1, 1, 1, 1, 0, 0, true, NT>(dnu, slice(nv, c, 4), slice(dtu, c, 36), T(-2), lane);
      cv4m_b<1, 1, 0, 0, 1, 1, 1, 1, false, NT>(nnv, slice(d0, c, 16), slice(dtv, c, 36), T(1), lane);
      cv4m_b<1, 1, 1, 1, 1, 1, 0, 0, true, NT>(dnv, slice(nv, c, 4), slice(dtv, c, 36), T(-2), lane);
      // the same lane owns each coefficient in the products above and here
      for (int o = lane; o < 36; o += NT) {
        const int ij = o >> 2;  // (n.n) is constant along z1, z2 (replicated in scaled form)
        const TP<T> tu = slice(dtu, c, 36), tv = slice(dtv, c, 36);
        tu.v[o] = fma(-T(2) * comp(dn1, c), dn.v[o], fma(comp(e1, c), nn.v[ij], tu.v[o]));
        tu.m[o] += T(2) * fabs(comp(dn1, c)) * dn.m[o] + fabs(comp(e1, c)) * nn.m[ij];
        tv.v[o] = fma(-T(2) * comp(dn2, c), dn.v[o], fma(comp(e2, c), nn.v[ij], tv.v[o]));
        tv.m[o] += T(2) * fabs(comp(dn2, c)) * dn.m[o] + fabs(comp(e2, c)) * nn.m[ij];
      }
    }
    const T th_dtu = max(max(th_cv4<1, 1, 0, 0, 1, 1, 1, 1>(th_nnu, th_lin, 4), th_cv4<1, 1, 1, 1, 1, 1, 0, 0>(th_dnu, th_lin, 4)),
                         th_nn + T(2) * eps) +
                     T(4) * eps;
    wave_sync();
    for (int o = lane; o < 36; o += NT) {  // (d~ x f2)_u = d~_u x f2
      const V3<T> af = mk(fabs(G.f2.x), fabs(G.f2.y), fabs(G.f2.z));
      for (int w = 0; w < 2; ++w) {
        const TP<T> t = w ? dtv : dtu, r = w ? ccv : ccu;
        const V3<T> x = cross(mk(t.v[o], t.v[36 + o], t.v[72 + o]), G.f2);
        const V3<T> m = mk(t.m[o], t.m[36 + o], t.m[72 + o]);
        r.v[o] = x.x;
        r.v[36 + o] = x.y;
        r.v[72 + o] = x.z;
        r.m[o] = m.y * af.z + m.z * af.y;
        r.m[36 + o] = m.z * af.x + m.x * af.z;
        r.m[72 + o] = m.x * af.y + m.y * af.x;
      }
    }
    const T th_ccu = th_dtu + T(3) * eps;
    wave_sync();
    // Q_u = c_u.f1 (2,2,1,1); Pu_u = c_u.s + c.e1, Pv_u = (e1 x f1).d~ + (s x f1).d~_u (3,3,1,1)
    {
      const T* cuv[3] = {slice(ccu, 0, 36).v, slice(ccu, 1, 36).v, slice(ccu, 2, 36).v};
      const T* cum[3] = {slice(ccu, 0, 36).m, slice(ccu, 1, 36).m, slice(ccu, 2, 36).m};
      const T* cvv[3] = {slice(ccv, 0, 36).v, slice(ccv, 1, 36).v, slice(ccv, 2, 36).v};
      const T* cvm[3] = {slice(ccv, 0, 36).m, slice(ccv, 1, 36).m, slice(ccv, 2, 36).m};
      const T af1[3] = {G.f1.x, G.f1.y, G.f1.z};
      combo<36, 3, false, T, NT>(cuv, cum, af1, qu.v, qu.m, lane);
      combo<36, 3, false, T, NT>(cvv, cvm, af1, qv.v, qv.m, lane);
    }
    for (int c = 0; c < 3; ++c) {
      if (c == 0) {
        cv4m_b<2, 2, 1, 1, 1, 1, 0, 0, false, NT>(slice(ccu, c, 36), slice(sv, c, 4), puu, T(1), lane);
        cv4m_b<2, 2, 1, 1, 1, 1, 0, 0, false, NT>(slice(ccv, c, 36), slice(sv, c, 4), puv, T(1), lane);
        cv4m_b<1, 1, 0, 0, 2, 2, 1, 1, false, NT>(slice(sf1, c, 4), slice(dtu, c, 36), pvu, T(1), lane);
        cv4m_b<1, 1, 0, 0, 2, 2, 1, 1, false, NT>(slice(sf1, c, 4), slice(dtv, c, 36), pvv, T(1), lane);
      } else {
        cv4m_b<2, 2, 1, 1, 1, 1, 0, 0, true, NT>(slice(ccu, c, 36), slice(sv, c, 4), puu, T(1), lane);
        cv4m_b<2, 2, 1, 1, 1, 1, 0, 0, true, NT>(slice(ccv, c, 36), slice(sv, c, 4), puv, T(1), lane);
        cv4m_b<1, 1, 0, 0, 2, 2, 1, 1, true, NT>(slice(sf1, c, 4), slice(dtu, c, 36), pvu, T(1), lane);
        cv4m_b<1, 1, 0, 0, 2, 2, 1, 1, true, NT>(slice(sf1, c, 4), slice(dtv, c, 36), pvv, T(1), lane);
      }
    }
    {
      // e1 x f1 and e2 x f2 with the magnitudes of their products
      const V3<T> g1 = cross(e1, G.f1), g2 = cross(e2, G.f1);
      const V3<T> ae1 = mk(fabs(e1.x), fabs(e1.y), fabs(e1.z)), ae2 = mk(fabs(e2.x), fabs(e2.y), fabs(e2.z));
      const V3<T> af1 = mk(fabs(G.f1.x), fabs(G.f1.y), fabs(G.f1.z));
      const V3<T> g1m = mk(ae1.y * af1.z + ae1.z * af1.y, ae1.z * af1.x + ae1.x * af1.z, ae1.x * af1.y + ae1.y * af1.x);
      const V3<T> g2m = mk(ae2.y * af1.z + ae2.z * af1.y, ae2.z * af1.x + ae2.x * af1.z, ae2.x * af1.y + ae2.y * af1.x);
      // the same lane owns each coefficient in the products above and here
      for (int o = lane; o < 64; o += NT) {
        T a = puu.v[o], am2 = puu.m[o], b = puv.v[o], bm2 = puv.m[o];
        T c2 = pvu.v[o], cm2 = pvu.m[o], d2 = pvv.v[o], dm2 = pvv.m[o];
        for (int c = 0; c < 3; ++c) {
          const T ccv2 = cc.v[64 * c + o], ccm2 = cc.m[64 * c + o], dtv2 = dt.v[64 * c + o], dtm2 = dt.m[64 * c + o];
          a = fma(comp(e1, c), ccv2, a);
          am2 += fabs(comp(e1, c)) * ccm2;
          b = fma(comp(e2, c), ccv2, b);
          bm2 += fabs(comp(e2, c)) * ccm2;
          c2 = fma(comp(g1, c), dtv2, c2);
          cm2 += comp(g1m, c) * dtm2;
          d2 = fma(comp(g2, c), dtv2, d2);
          dm2 += comp(g2m, c) * dtm2;
        }
        puu.v[o] = a;
        puu.m[o] = am2;
        puv.v[o] = b;
        puv.m[o] = bm2;
        pvu.v[o] = c2;
        pvu.m[o] = cm2;
        pvv.v[o] = d2;
        pvv.m[o] = dm2;
      }
    }
    const T th_qd = th_ccu + T(4) * eps;
    const T th_pd = max(max(th_cv4<2, 2, 1, 1, 1, 1, 0, 0>(th_ccu, th_lin, 6), th_cv4<1, 1, 0, 0, 2, 2, 1, 1>(th_sf1, th_dtu, 6)),
                        max(th_cc, th_dt) + T(4) * eps) +
                    T(2) * eps;
    wave_sync();
    // A = Pu_u Pv_v - Pv_u Pu_v, Bm = Q_u Pv_v - Pv_u Q_v, Cm = Q_u Pu_v - Pu_u Q_v, Q^2
    const TP<T> am = at(RALay::AM), bm = at(RALay::BM), cm = at(RALay::CM), q2 = at(RALay::Q2);
    cv4m_b<3, 3, 1, 1, 3, 3, 1, 1, false, NT>(puu, pvv, am, T(1), lane);
    cv4m_b<3, 3, 1, 1, 3, 3, 1, 1, true, NT>(pvu, puv, am, T(-1), lane);
    cv4m_b<2, 2, 1, 1, 3, 3, 1, 1, false, NT>(qu, pvv, bm, T(1), lane);
    cv4m_b<3, 3, 1, 1, 2, 2, 1, 1, true, NT>(pvu, qv, bm, T(-1), lane);
    cv4m_b<2, 2, 1, 1, 3, 3, 1, 1, false, NT>(qu, puv, cm, T(1), lane);
    cv4m_b<3, 3, 1, 1, 2, 2, 1, 1, true, NT>(puu, qv, cm, T(-1), lane);
    cv4m_b<3, 3, 1, 1, 3, 3, 1, 1, false, NT>(q, q, q2, T(1), lane);
    const T th_a = th_cv4<3, 3, 1, 1, 3, 3, 1, 1>(th_pd, th_pd, 2);
    const T th_bc = max(th_cv4<2, 2, 1, 1, 3, 3, 1, 1>(th_qd, th_pd, 2), th_cv4<3, 3, 1, 1, 2, 2, 1, 1>(th_pd, th_qd, 2));
    const T th_q2 = th_cv4<3, 3, 1, 1, 3, 3, 1, 1>(th_q, th_q, 1);
    wave_sync();
    // det M = Q A - Pu Bm + Pv Cm (9,9,3,3); Q^3 (9,9,3,3)
    const TP<T> detm = at(RALay::DETM), q3 = at(RALay::Q3), q3e = at(RALay::Q3E), detme = at(RALay::DETME);
    cv4m_b<3, 3, 1, 1, 6, 6, 2, 2, false, NT>(q, am, detm, T(1), lane);
    cv4m_b<4, 4, 1, 1, 5, 5, 2, 2, true, NT>(pu, bm, detm, T(-1), lane);
    cv4m_b<4, 4, 1, 1, 5, 5, 2, 2, true, NT>(pv, cm, detm, T(1), lane);
    cv4m_b<6, 6, 2, 2, 3, 3, 1, 1, false, NT>(q2, q, q3, T(1), lane);
    const T th_detm = max(th_cv4<3, 3, 1, 1, 6, 6, 2, 2>(th_q, th_a, 3), th_cv4<4, 4, 1, 1, 5, 5, 2, 2>(th_p, th_bc, 3));
    const T th_q3 = th_cv4<6, 6, 2, 2, 3, 3, 1, 1>(th_q2, th_q, 1);
    wave_sync();
    // det M's elevation overwrites the dead factors (GG .. CM)
    elev4m_b<9, 9, 3, 3, 1, 1, 0, 0, NT>(detm, detme, lane);
    elev4m_b<9, 9, 3, 3, 1, 1, 0, 0, NT>(q3, q3e, lane);
    const T th_detme = th_elev4<1, 1, 0, 0>(th_detm);
    const T th_q3e = th_elev4<1, 1, 0, 0>(th_q3);
    wave_sync();
    const RB<T> rb = ratio4m<T, NT>(N4<10, 10, 3, 3>::n, q3e, th_q3e, detme, th_detme, true, lane);
    T rlo, rhi;
    abs_bound(rb, &rlo, &rhi);
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
