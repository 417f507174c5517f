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
//   det M (10,10,3,3) over Q^3 raised to the same degree.
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
  static constexpr int GG = 945, HH = 961, QU = 1042, QV = 1090;           // 16, 81, 48, 48
  static constexpr int PUU = 1138, PUV = 1218, PVU = 1298, PVV = 1378;     // 80 each
  static constexpr int AM = 1458, BM = 2034, CM = 2475, DETM = 2916;       // 576, 441, 441, 1936
  static constexpr int Q2 = 4852, Q3 = 5293, Q3E = 6893, END = 8829;       // 441, 1600, 1936
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
      cv4m<1, 1, 0, 0, 1, 1, 0, 0, false, NT>(slice(nv, c, 4), slice(nv, c, 4), nn, T(1), lane);
      cv4m<1, 1, 1, 1, 1, 1, 0, 0, false, NT>(slice(d0, c, 16), slice(nv, c, 4), dn, T(1), lane);
    } else {
      cv4m<1, 1, 0, 0, 1, 1, 0, 0, true, NT>(slice(nv, c, 4), slice(nv, c, 4), nn, T(1), lane);
      cv4m<1, 1, 1, 1, 1, 1, 0, 0, true, NT>(slice(d0, c, 16), slice(nv, c, 4), dn, T(1), lane);
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
    cv4m<2, 2, 0, 0, 1, 1, 1, 1, false, NT>(nn, slice(d0, c, 16), slice(dt, c, 64), T(1), lane);
    cv4m<2, 2, 1, 1, 1, 1, 0, 0, true, NT>(dn, slice(nv, c, 4), slice(dt, c, 64), T(-2), lane);
  }
  elev4m<1, 1, 0, 0, 2, 2, 1, 1, NT>(tn, tne, lane);
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
      cv4m<3, 3, 1, 1, 1, 1, 0, 0, false, NT>(slice(cc, c, 64), slice(sv, c, 4), pu, T(1), lane);
      cv4m<1, 1, 0, 0, 3, 3, 1, 1, false, NT>(slice(sf1, c, 4), slice(dt, c, 64), pv, T(1), lane);
    } else {
      cv4m<3, 3, 1, 1, 1, 1, 0, 0, true, NT>(slice(cc, c, 64), slice(sv, c, 4), pu, T(1), lane);
      cv4m<1, 1, 0, 0, 3, 3, 1, 1, true, NT>(slice(sf1, c, 4), slice(dt, c, 64), pv, T(1), lane);
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
  elev4m<3, 3, 1, 1, 1, 1, 0, 0, NT>(q, qe, lane);
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
    // ---- irradiance bound (Sec. 4.4) over the box and the whole light
    const TP<T> gg = at(RALay::GG), hh = at(RALay::HH), qu = at(RALay::QU), qv = at(RALay::QV);
    const TP<T> puu = at(RALay::PUU), puv = at(RALay::PUV), pvu = at(RALay::PVU), pvv = at(RALay::PVV);
    for (int o = lane; o < 16; o += NT) {
      gg.v[o] = dot(mk(d0.v[o], d0.v[16 + o], d0.v[32 + o]), G.ng);
      gg.m[o] = d0.m[o] * fabs(G.ng.x) + d0.m[16 + o] * fabs(G.ng.y) + d0.m[32 + o] * fabs(G.ng.z);
    }
    for (int c = 0; c < 3; ++c) {
      if (c == 0)
        cv4m<1, 1, 1, 1, 1, 1, 1, 1, false, NT>(slice(d0, c, 16), slice(d0, c, 16), hh, T(1), lane);
      else
        cv4m<1, 1, 1, 1, 1, 1, 1, 1, true, NT>(slice(d0, c, 16), slice(d0, c, 16), hh, T(1), lane);
    }
    deriv4m<3, 3, 1, 1, 0, NT>(q, qu, lane);
    deriv4m<3, 3, 1, 1, 1, NT>(q, qv, lane);
    deriv4m<4, 4, 1, 1, 0, NT>(pu, puu, lane);
    deriv4m<4, 4, 1, 1, 1, NT>(pu, puv, lane);
    deriv4m<4, 4, 1, 1, 0, NT>(pv, pvu, lane);
    deriv4m<4, 4, 1, 1, 1, NT>(pv, pvv, lane);
    const T th_g = th_lin + T(8) * eps;  // the unit normal carries a few roundings of its own
    const T th_h = th_cv4<1, 1, 1, 1, 1, 1, 1, 1>(th_lin, th_lin, 3);
    const T th_qd = th_q + T(3) * eps, th_pd = th_p + T(3) * eps;
    wave_sync();
    // A = Pu_u Pv_v - Pv_u Pu_v, Bm = Q_u Pv_v - Pv_u Q_v, Cm = Q_u Pu_v - Pu_u Q_v, Q^2
    const TP<T> am = at(RALay::AM), bm = at(RALay::BM), cm = at(RALay::CM), q2 = at(RALay::Q2);
    cv4m<3, 4, 1, 1, 4, 3, 1, 1, false, NT>(puu, pvv, am, T(1), lane);
    cv4m<3, 4, 1, 1, 4, 3, 1, 1, true, NT>(pvu, puv, am, T(-1), lane);
    cv4m<2, 3, 1, 1, 4, 3, 1, 1, false, NT>(qu, pvv, bm, T(1), lane);
    cv4m<3, 4, 1, 1, 3, 2, 1, 1, true, NT>(pvu, qv, bm, T(-1), lane);
    cv4m<2, 3, 1, 1, 4, 3, 1, 1, false, NT>(qu, puv, cm, T(1), lane);
    cv4m<3, 4, 1, 1, 3, 2, 1, 1, true, NT>(puu, qv, cm, T(-1), lane);
    cv4m<3, 3, 1, 1, 3, 3, 1, 1, false, NT>(q, q, q2, T(1), lane);
    const T th_a = th_cv4<3, 4, 1, 1, 4, 3, 1, 1>(th_pd, th_pd, 2);
    const T th_bc = max(th_cv4<2, 3, 1, 1, 4, 3, 1, 1>(th_qd, th_pd, 2), th_cv4<3, 4, 1, 1, 3, 2, 1, 1>(th_pd, th_qd, 2));
    const T th_q2 = th_cv4<3, 3, 1, 1, 3, 3, 1, 1>(th_q, th_q, 1);
    T glo, ghi, hlo, hhi;
    range4m<1, 1, 1, 1, T, NT>(gg, th_g, &glo, &ghi, lane);
    range4m<2, 2, 2, 2, T, NT>(hh, th_h, &hlo, &hhi, lane);
    wave_sync();
    // det M = Q A - Pu Bm + Pv Cm (10,10,3,3); Q^3 (9,9,3,3)
    const TP<T> detm = at(RALay::DETM), q3 = at(RALay::Q3), q3e = at(RALay::Q3E);
    cv4m<3, 3, 1, 1, 7, 7, 2, 2, false, NT>(q, am, detm, T(1), lane);
    cv4m<4, 4, 1, 1, 6, 6, 2, 2, true, NT>(pu, bm, detm, T(-1), lane);
    cv4m<4, 4, 1, 1, 6, 6, 2, 2, true, NT>(pv, cm, detm, T(1), lane);
    cv4m<6, 6, 2, 2, 3, 3, 1, 1, false, NT>(q2, q, q3, T(1), lane);
    const T th_detm = max(th_cv4<3, 3, 1, 1, 7, 7, 2, 2>(th_q, th_a, 3),
                          max(th_cv4<4, 4, 1, 1, 6, 6, 2, 2>(th_p, th_bc, 3), th_cv4<4, 4, 1, 1, 6, 6, 2, 2>(th_p, th_bc, 3)));
    const T th_q3 = th_cv4<6, 6, 2, 2, 3, 3, 1, 1>(th_q2, th_q, 1);
    wave_sync();
    elev4m<9, 9, 3, 3, 1, 1, 0, 0, NT>(q3, q3e, lane);
    const T th_q3e = th_elev4<1, 1, 0, 0>(th_q3);
    wave_sync();
    const RB<T> rb = ratio4m<T, NT>(N4<10, 10, 3, 3>::n, q3e, th_q3e, detm, th_detm, true, lane);
    T rlo, rhi;
    abs_bound(rb, &rlo, &rhi);
    // local u-, v-derivatives: the global ratio is the local one times w_u w_v
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
