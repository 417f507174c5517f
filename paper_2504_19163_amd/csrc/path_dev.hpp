// Exact path evaluation and Newton root-finding in the triangle domain
// (Sec. 4.3-4.4 for the map and its irradiance, Sec. 6.1 for root-finding),
// plus the Philox4x32-10 stream used by the selection step of Alg. 1.
#pragma once
#include "geom_dev.hpp"

namespace bbc {

template <class T>
struct PathT {
  T uk, vk, t;
  T J00, J01, J10, J11, det;  // d(u_k, v_k) / d(u, v)
  T dn, beta;
  V3<T> x1;
};

// Receiver coordinates of the path through barycentric (u, v) and their
// Jacobian, by forward differentiation of the rational map of Eq. eq_rct with
// the outgoing direction of Eq. eq_refr_rational (chain 0: reflection,
// chain 1: refraction).
template <class T>
__device__ __forceinline__ PathT<T> eval_path(const TupleGeom<T>& G, int chain, T u, T v) {
  PathT<T> r;
  const V3<T> x1 = G.p0 + u * G.e1 + v * G.e2;
  const V3<T> n = G.n0 + u * G.dn1 + v * G.dn2;
  const V3<T> d = x1 - G.x0;
  const T nn = dot(n, n), nn_u = T(2) * dot(n, G.dn1), nn_v = T(2) * dot(n, G.dn2);
  const T dn = dot(d, n), dn_u = dot(G.e1, n) + dot(d, G.dn1), dn_v = dot(G.e2, n) + dot(d, G.dn2);
  V3<T> dt, dt_u, dt_v;
  r.beta = T(1);
  if (chain == 0) {
    dt = nn * d - (T(2) * dn) * n;
    dt_u = nn_u * d + nn * G.e1 - T(2) * (dn_u * n + dn * G.dn1);
    dt_v = nn_v * d + nn * G.e2 - T(2) * (dn_v * n + dn * G.dn2);
  } else {
    const T eta = G.eta, e2 = eta * eta;
    const T dd = dot(d, d), dd_u = T(2) * dot(d, G.e1), dd_v = T(2) * dot(d, G.e2);
    const T beta = (T(1) - e2) * nn * dd + e2 * dn * dn;
    const T beta_u = (T(1) - e2) * (nn_u * dd + nn * dd_u) + e2 * T(2) * dn * dn_u;
    const T beta_v = (T(1) - e2) * (nn_v * dd + nn * dd_v) + e2 * T(2) * dn * dn_v;
    r.beta = beta;
    const T sb = sqrt(max(beta, T(0)));
    const T sb_u = beta_u / (T(2) * sb), sb_v = beta_v / (T(2) * sb);
    dt = eta * (nn * d - dn * n) - sb * n;
    dt_u = eta * (nn_u * d + nn * G.e1 - dn_u * n - dn * G.dn1) - sb_u * n - sb * G.dn1;
    dt_v = eta * (nn_v * d + nn * G.e2 - dn_v * n - dn * G.dn2) - sb_v * n - sb * G.dn2;
  }
  const V3<T> s = x1 - G.q0;
  const V3<T> c = cross(dt, G.f2), c_u = cross(dt_u, G.f2), c_v = cross(dt_v, G.f2);
  const T Q = dot(c, G.f1), Q_u = dot(c_u, G.f1), Q_v = dot(c_v, G.f1);
  const T Pu = dot(c, s), Pu_u = dot(c_u, s) + dot(c, G.e1), Pu_v = dot(c_v, s) + dot(c, G.e2);
  const V3<T> sf1 = cross(s, G.f1), sf1_u = cross(G.e1, G.f1), sf1_v = cross(G.e2, G.f1);
  const T Pv = dot(sf1, dt), Pv_u = dot(sf1_u, dt) + dot(sf1, dt_u), Pv_v = dot(sf1_v, dt) + dot(sf1, dt_v);
  const T iq = T(1) / Q;
  r.uk = Pu * iq;
  r.vk = Pv * iq;
  r.t = dot(sf1, G.f2) * iq;
  r.J00 = (Pu_u - r.uk * Q_u) * iq;
  r.J01 = (Pu_v - r.uk * Q_v) * iq;
  r.J10 = (Pv_u - r.vk * Q_u) * iq;
  r.J11 = (Pv_v - r.vk * Q_v) * iq;
  r.det = r.J00 * r.J11 - r.J01 * r.J10;
  r.dn = dn;
  r.x1 = x1;
  return r;
}

// Admissible specular path: inside the closed triangle, the receiver ahead of
// the specular vertex, and for refraction no total internal reflection with
// light arriving on the front of the shading normal.
template <class T>
__device__ __forceinline__ bool admissible(const TupleGeom<T>& G, int chain, const PathT<T>& p, T u, T v) {
  bool ok = G.front && u >= T(0) && v >= T(0) && u + v <= T(1) && p.t > T(0) && isfinite(p.uk) && isfinite(p.vk);
  if (chain == 1) ok = ok && p.beta > T(0) && p.dn < T(0);
  return ok;
}

// Irradiance of the path, E_k = I0 dOmega0/dA1 |dx1/du1| |du1/du_k| |du_k/dx_k|
// (Eq. eq_dwda), visibility and Fresnel factors dropped.
template <class T>
__device__ __forceinline__ T path_irradiance(const TupleGeom<T>& G, const PathT<T>& p) {
  const V3<T> d = p.x1 - G.x0;
  const T l2 = dot(d, d);
  return G.I0 * fabs(dot(G.ng, d)) / (l2 * sqrt(l2)) * G.a1 / (fabs(p.det) * G.ak);
}

template <class T>
__device__ __forceinline__ T residual(const TupleGeom<T>& G, const PathT<T>& p, T us, T vs) {
  const V3<T> r = (p.uk - us) * G.f1 + (p.vk - vs) * G.f2;
  return sqrt(dot(r, r));
}

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC 2011): ten rounds of two 32x32 -> 64-bit products and a Weyl key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// The rng() of Alg. 1 for (seed, point index, tuple): top 24 bits of word 0.
__device__ __forceinline__ float selection_uniform(uint64_t seed, uint64_t point, uint32_t tuple) {
  const uint4 o = philox4x32_10(make_uint4(uint32_t(point), uint32_t(point >> 32), tuple, 0u),
                                make_uint2(uint32_t(seed), uint32_t(seed >> 32)));
  return float(o.x >> 8) * (1.0f / 16777216.0f);
}

}  // namespace bbc
