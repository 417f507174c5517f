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
// Values only in scaled Bernstein form, FP64, coefficients taken at face
// value (the 4-D tensors reach 1936 coefficients).
#pragma once
#include "box_t.hpp"

namespace bbc {

// LDS offsets (doubles).  Corner tensors (1,1,1,1) are indexed
// ((i * 2 + j) * 2 + k) * 2 + l over (u, v, z1, z2).
struct RALay {
  static constexpr int D0 = 0, N = 48, S = 60, NN = 72, DN = 81;          // 3x16, 3x4, 3x4, 9, 36
  static constexpr int DT = 117, CC = 309, SF1 = 501, PU = 513, PV = 613;  // 3x64, 3x64, 3x4, 100, 100
  static constexpr int Q = 713, TN = 777, TNE = 781, QE = 845;             // 64, 4, 64, 100
  static constexpr int POS_END = 945;
  static constexpr int GG = 945, HH = 961, QU = 1042, QV = 1090;           // 16, 81, 48, 48
  static constexpr int PUU = 1138, PUV = 1218, PVU = 1298, PVV = 1378;     // 80 each
  static constexpr int AM = 1458, BM = 2034, CM = 2475, DETM = 2916;       // 576, 441, 441, 1936
  static constexpr int Q2 = 4852, Q3 = 5293, Q3E = 6893, END = 8829;       // 441, 1600, 1936
};

template <class T, bool IRR>
struct LdsRA {
  T buf[IRR ? RALay::END : RALay::POS_END];
};

// Range of a 4-D polynomial from its scaled coefficients (values only).
template <int D1, int D2, int D3, int D4, class T, int NT>
__device__ __forceinline__ void range4(const T* v, T* lo, T* hi, int lane) {
  T l = T(INFINITY), h = -T(INFINITY);
  for (int o = lane; o < N4<D1, D2, D3, D4>::n; o += NT) {
    int r = o;
    const int d = r % (D4 + 1);
    r /= D4 + 1;
    const int c = r % (D3 + 1);
    r /= D3 + 1;
    const int b = r % (D2 + 1), a = r / (D2 + 1);
    const T x = v[o] / T(binom_i(D1, a) * binom_i(D2, b) * binom_i(D3, c) * binom_i(D4, d));
    l = min(l, x);
    h = max(h, x);
  }
  *lo = blk_min<NT>(l);
  *hi = blk_max<NT>(h);
}

template <class T, int NT>
__device__ __forceinline__ RB<T> ratio_face(int n, const T* p, const T* q, int lane) {
  return ratio_bound_fn<T, NT>(
      n,
      [&](int o, T& pv, T& ep, T& qv, T& eq) {
        pv = p[o];
        qv = q[o];
        ep = eq = T(0);
      },
      true, lane);
}

template <class T, bool IRR, int NT>
__device__ __forceinline__ BoxOut eval_box_ra(const TupleGeom<T>& G, T u0, T u1, T v0, T v1, LdsRA<T, IRR>& L,
                                              int lane) {
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
  T* const d0 = B + RALay::D0;
  T* const nv = B + RALay::N;
  T* const sv = B + RALay::S;
  // ---- corner values: d0 over (u, v, z1, z2), n and s = x1 - q0 over (u, v)
  const V3<T> pmx = G.p0 - G.x0, pmq = G.p0 - G.q0;
  for (int o = lane; o < 72; o += NT) {
    if (o < 48) {
      const int c = o / 16, r = o - 16 * c, i = r >> 3, j = (r >> 2) & 1, k = (r >> 1) & 1, l = r & 1;
      const T u = i ? u1 : u0, v = j ? v1 : v0;
      d0[o] = comp(pmx, c) + u * comp(G.e1, c) + v * comp(G.e2, c) - (T(k) * comp(G.ea, c) + T(l) * comp(G.eb, c));
    } else {
      const int w = (o - 48) / 12, c = ((o - 48) / 4) % 3, r = (o - 48) & 3;
      const T u = (r >> 1) ? u1 : u0, v = (r & 1) ? v1 : v0;
      if (w == 0)
        nv[4 * c + r] = comp(G.n0, c) + u * comp(G.dn1, c) + v * comp(G.dn2, c);
      else
        sv[4 * c + r] = comp(pmq, c) + u * comp(G.e1, c) + v * comp(G.e2, c);
    }
  }
  wave_sync();
  T* const nn = B + RALay::NN;
  T* const dn = B + RALay::DN;
  T* const sf1 = B + RALay::SF1;
  T* const tn = B + RALay::TN;
  for (int c = 0; c < 3; ++c) {
    if (c == 0) {
      cv4<1, 1, 0, 0, 1, 1, 0, 0, false, NT>(nv, nv, nn, T(1), lane);
      cv4<1, 1, 1, 1, 1, 1, 0, 0, false, NT>(d0, nv, dn, T(1), lane);
    } else {
      cv4<1, 1, 0, 0, 1, 1, 0, 0, true, NT>(nv + 4 * c, nv + 4 * c, nn, T(1), lane);
      cv4<1, 1, 1, 1, 1, 1, 0, 0, true, NT>(d0 + 16 * c, nv + 4 * c, dn, T(1), lane);
    }
  }
  for (int o = lane; o < 4; o += NT) {  // s x f1 and (s x f1).f2
    const V3<T> sc = mk(sv[o], sv[4 + o], sv[8 + o]);
    const V3<T> x = cross(sc, G.f1);
    sf1[o] = x.x;
    sf1[4 + o] = x.y;
    sf1[8 + o] = x.z;
    tn[o] = dot(x, G.f2);
  }
  wave_sync();
  // ---- d~ = (n.n) d0 - 2 (d0.n) n, c = d~ x f2, and Tn raised to Q's degree
  T* const dt = B + RALay::DT;
  T* const cc = B + RALay::CC;
  T* const tne = B + RALay::TNE;
  for (int c = 0; c < 3; ++c) {
    cv4<2, 2, 0, 0, 1, 1, 1, 1, false, NT>(nn, d0 + 16 * c, dt + 64 * c, T(1), lane);
    cv4<2, 2, 1, 1, 1, 1, 0, 0, true, NT>(dn, nv + 4 * c, dt + 64 * c, T(-2), lane);
  }
  elev4<1, 1, 0, 0, 2, 2, 1, 1, NT>(tn, tne, lane);
  wave_sync();
  for (int o = lane; o < 64; o += NT) {
    const V3<T> x = cross(mk(dt[o], dt[64 + o], dt[128 + o]), G.f2);
    cc[o] = x.x;
    cc[64 + o] = x.y;
    cc[128 + o] = x.z;
  }
  wave_sync();
  // ---- Pu = c.s, Pv = (s x f1).d~, Q = c.f1
  T* const pu = B + RALay::PU;
  T* const pv = B + RALay::PV;
  T* const q = B + RALay::Q;
  for (int c = 0; c < 3; ++c) {
    if (c == 0) {
      cv4<3, 3, 1, 1, 1, 1, 0, 0, false, NT>(cc, sv, pu, T(1), lane);
      cv4<1, 1, 0, 0, 3, 3, 1, 1, false, NT>(sf1, dt, pv, T(1), lane);
    } else {
      cv4<3, 3, 1, 1, 1, 1, 0, 0, true, NT>(cc + 64 * c, sv + 4 * c, pu, T(1), lane);
      cv4<1, 1, 0, 0, 3, 3, 1, 1, true, NT>(sf1 + 4 * c, dt + 64 * c, pv, T(1), lane);
    }
  }
  for (int o = lane; o < 64; o += NT) q[o] = dot(mk(cc[o], cc[64 + o], cc[128 + o]), G.f1);
  wave_sync();
  T* const qe = B + RALay::QE;
  elev4<3, 3, 1, 1, 1, 1, 0, 0, NT>(q, qe, lane);
  wave_sync();
  // ---- position bound (Sec. 4.2) over the box and the whole light
  const RB<T> tb = ratio_face<T, NT>(64, tne, q, lane);
  const RB<T> ub = ratio_face<T, NT>(100, pu, qe, lane);
  const RB<T> vb = ratio_face<T, NT>(100, pv, qe, lane);
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
    T* const gg = B + RALay::GG;
    T* const hh = B + RALay::HH;
    T* const qu = B + RALay::QU;
    T* const qv = B + RALay::QV;
    T* const puu = B + RALay::PUU;
    T* const puv = B + RALay::PUV;
    T* const pvu = B + RALay::PVU;
    T* const pvv = B + RALay::PVV;
    for (int o = lane; o < 16; o += NT) gg[o] = dot(mk(d0[o], d0[16 + o], d0[32 + o]), G.ng);
    for (int c = 0; c < 3; ++c) {
      if (c == 0)
        cv4<1, 1, 1, 1, 1, 1, 1, 1, false, NT>(d0, d0, hh, T(1), lane);
      else
        cv4<1, 1, 1, 1, 1, 1, 1, 1, true, NT>(d0 + 16 * c, d0 + 16 * c, hh, T(1), lane);
    }
    deriv4<3, 3, 1, 1, 0, NT>(q, qu, lane);
    deriv4<3, 3, 1, 1, 1, NT>(q, qv, lane);
    deriv4<4, 4, 1, 1, 0, NT>(pu, puu, lane);
    deriv4<4, 4, 1, 1, 1, NT>(pu, puv, lane);
    deriv4<4, 4, 1, 1, 0, NT>(pv, pvu, lane);
    deriv4<4, 4, 1, 1, 1, NT>(pv, pvv, lane);
    wave_sync();
    // A = Pu_u Pv_v - Pv_u Pu_v, Bm = Q_u Pv_v - Pv_u Q_v, Cm = Q_u Pu_v - Pu_u Q_v, Q^2
    T* const am = B + RALay::AM;
    T* const bm = B + RALay::BM;
    T* const cm = B + RALay::CM;
    T* const q2 = B + RALay::Q2;
    cv4<3, 4, 1, 1, 4, 3, 1, 1, false, NT>(puu, pvv, am, T(1), lane);
    cv4<3, 4, 1, 1, 4, 3, 1, 1, true, NT>(pvu, puv, am, T(-1), lane);
    cv4<2, 3, 1, 1, 4, 3, 1, 1, false, NT>(qu, pvv, bm, T(1), lane);
    cv4<3, 4, 1, 1, 3, 2, 1, 1, true, NT>(pvu, qv, bm, T(-1), lane);
    cv4<2, 3, 1, 1, 4, 3, 1, 1, false, NT>(qu, puv, cm, T(1), lane);
    cv4<3, 4, 1, 1, 3, 2, 1, 1, true, NT>(puu, qv, cm, T(-1), lane);
    cv4<3, 3, 1, 1, 3, 3, 1, 1, false, NT>(q, q, q2, T(1), lane);
    T glo, ghi, hlo, hhi;
    range4<1, 1, 1, 1, T, NT>(gg, &glo, &ghi, lane);
    range4<2, 2, 2, 2, T, NT>(hh, &hlo, &hhi, lane);
    wave_sync();
    // det M = Q A - Pu Bm + Pv Cm (10,10,3,3); Q^3 (9,9,3,3)
    T* const detm = B + RALay::DETM;
    T* const q3 = B + RALay::Q3;
    T* const q3e = B + RALay::Q3E;
    cv4<3, 3, 1, 1, 7, 7, 2, 2, false, NT>(q, am, detm, T(1), lane);
    cv4<4, 4, 1, 1, 6, 6, 2, 2, true, NT>(pu, bm, detm, T(-1), lane);
    cv4<4, 4, 1, 1, 6, 6, 2, 2, true, NT>(pv, cm, detm, T(1), lane);
    cv4<6, 6, 2, 2, 3, 3, 1, 1, false, NT>(q2, q, q3, T(1), lane);
    wave_sync();
    elev4<9, 9, 3, 3, 1, 1, 0, 0, NT>(q3, q3e, lane);
    wave_sync();
    const RB<T> rb = ratio_face<T, NT>(N4<10, 10, 3, 3>::n, q3e, detm, lane);
    T rlo, rhi;
    abs_bound(rb, &rlo, &rhi);
    // local u-, v-derivatives: the global ratio is the local one times w_u w_v
    const T eps = Eps<T>::u;
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
