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
  T s2, u2, v2, f2;  // two reflections: ray parameter and barycentrics of x2, d~1 . n_g2
};

// Value and partial derivatives in (u, v) (forward differentiation).
template <class T>
struct Dl {
  T v, a, b;
};
template <class T>
__device__ __forceinline__ Dl<T> operator+(Dl<T> x, Dl<T> y) { return Dl<T>{x.v + y.v, x.a + y.a, x.b + y.b}; }
template <class T>
__device__ __forceinline__ Dl<T> operator-(Dl<T> x, Dl<T> y) { return Dl<T>{x.v - y.v, x.a - y.a, x.b - y.b}; }
template <class T>
__device__ __forceinline__ Dl<T> operator*(Dl<T> x, Dl<T> y) {
  return Dl<T>{x.v * y.v, x.a * y.v + x.v * y.a, x.b * y.v + x.v * y.b};
}
template <class T>
__device__ __forceinline__ Dl<T> operator*(T s, Dl<T> x) { return Dl<T>{s * x.v, s * x.a, s * x.b}; }
// Reciprocal: FP64 correctly rounded (the polish); FP32 by the hardware's
// approximate reciprocal (1 ulp), enough for the FP32 iterations, which only
// bring a start to the FP64 polish that decides the root.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
template <class T>
__device__ __forceinline__ Dl<T> operator/(Dl<T> x, Dl<T> y) {
  const T iy = recip(y.v), q = x.v * iy;
  return Dl<T>{q, (x.a - q * y.a) * iy, (x.b - q * y.b) * iy};
}
template <class T>
struct DV {
  Dl<T> x, y, z;
};
template <class T>
__device__ __forceinline__ DV<T> dlin(V3<T> base, V3<T> du, V3<T> dv, T u, T v) {
  return DV<T>{Dl<T>{base.x + u * du.x + v * dv.x, du.x, dv.x}, Dl<T>{base.y + u * du.y + v * dv.y, du.y, dv.y},
               Dl<T>{base.z + u * du.z + v * dv.z, du.z, dv.z}};
}
template <class T>
__device__ __forceinline__ DV<T> dconst(V3<T> a) {
  return DV<T>{Dl<T>{a.x, T(0), T(0)}, Dl<T>{a.y, T(0), T(0)}, Dl<T>{a.z, T(0), T(0)}};
}
template <class T>
__device__ __forceinline__ DV<T> operator+(DV<T> a, DV<T> b) { return DV<T>{a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T>
__device__ __forceinline__ DV<T> operator-(DV<T> a, DV<T> b) { return DV<T>{a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T>
__device__ __forceinline__ DV<T> operator*(Dl<T> s, DV<T> a) { return DV<T>{s * a.x, s * a.y, s * a.z}; }
template <class T>
__device__ __forceinline__ Dl<T> ddot(DV<T> a, DV<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T>
__device__ __forceinline__ Dl<T> ddotc(DV<T> a, V3<T> k) { return k.x * a.x + k.y * a.y + k.z * a.z; }
template <class T>
__device__ __forceinline__ DV<T> dcrossc(DV<T> a, V3<T> k) {  // a x k, k constant
  return DV<T>{k.z * a.y - k.y * a.z, k.x * a.z - k.z * a.x, k.y * a.x - k.x * a.y};
}
template <class T>
__device__ __forceinline__ DV<T> dscale(DV<T> a, Dl<T> s) { return s * a; }

// Two reflections: Eq. eq_rct maps x1 and the reflected direction d~1 to the
// barycentrics u2 of the second vertex, whose interpolated normal reflects
// d1 = x2 - x1 into d~2, and Eq. eq_rct again maps (x2, d~2) to the receiver.
template <class T>
__device__ PathT<T> eval_path_rr(const TupleGeom<T>& G, T u, T v) {
  PathT<T> r;
  const DV<T> x1 = dlin(G.p0, G.e1, G.e2, u, v);
  const DV<T> n1 = dlin(G.n0, G.dn1, G.dn2, u, v);
  const DV<T> d0 = x1 - dconst(G.x0);
  const Dl<T> two{T(2), T(0), T(0)};
  const DV<T> dt1 = ddot(n1, n1) * d0 - (two * ddot(d0, n1)) * n1;
  const DV<T> sb = x1 - dconst(G.p0b);
  const DV<T> c1 = dcrossc(dt1, G.e2b);
  const DV<T> sbe1 = dcrossc(sb, G.e1b);
  const Dl<T> Q2 = ddotc(c1, G.e1b);
  const Dl<T> u2 = ddot(c1, sb) / Q2, v2 = ddot(sbe1, dt1) / Q2, s2 = ddotc(sbe1, G.e2b) / Q2;
  const DV<T> x2 = dconst(G.p0b) + u2 * dconst(G.e1b) + v2 * dconst(G.e2b);
  const DV<T> n2 = dconst(G.n0b) + u2 * dconst(G.dn1b) + v2 * dconst(G.dn2b);
  const DV<T> d1 = x2 - x1;
  const DV<T> dt2 = ddot(n2, n2) * d1 - (two * ddot(d1, n2)) * n2;
  const DV<T> s3 = x2 - dconst(G.q0);
  const DV<T> c3 = dcrossc(dt2, G.f2);
  const DV<T> s3f1 = dcrossc(s3, G.f1);
  const Dl<T> Q3 = ddotc(c3, G.f1);
  const Dl<T> uk = ddot(c3, s3) / Q3, vk = ddot(s3f1, dt2) / Q3, t3 = ddotc(s3f1, G.f2) / Q3;
  r.uk = uk.v;
  r.vk = vk.v;
  r.t = t3.v;
  r.J00 = uk.a;
  r.J01 = uk.b;
  r.J10 = vk.a;
  r.J11 = vk.b;
  r.det = r.J00 * r.J11 - r.J01 * r.J10;
  r.dn = T(0);
  r.beta = T(1);
  r.x1 = mk(x1.x.v, x1.y.v, x1.z.v);
  r.s2 = s2.v;
  r.u2 = u2.v;
  r.v2 = v2.v;
  r.f2 = dt1.x.v * G.ngb.x + dt1.y.v * G.ngb.y + dt1.z.v * G.ngb.z;
  return r;
}

// Receiver coordinates of the path through barycentric (u, v) and their
// Jacobian, by forward differentiation of the rational map of Eq. eq_rct with
// the outgoing direction of Eq. eq_refr_rational (chain 0: reflection,
// chain 1: refraction).
template <class T>
__device__ __forceinline__ PathT<T> eval_path(const TupleGeom<T>& G, int chain, T u, T v) {
  if (chain == 2) return eval_path_rr<T>(G, u, v);
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
  const T iq = recip(Q);
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
// the specular vertex, for refraction no total internal reflection with light
// arriving on the front of the shading normal, and for two reflections the
// second vertex inside its closed triangle, ahead of the first and reached on
// its front side.
template <class T>
__device__ __forceinline__ bool admissible(const TupleGeom<T>& G, int chain, const PathT<T>& p, T u, T v) {
  bool ok = G.front && u >= T(0) && v >= T(0) && u + v <= T(1) && p.t > T(0) && isfinite(p.uk) && isfinite(p.vk);
  if (chain == 1) ok = ok && p.beta > T(0) && p.dn < T(0);
  if (chain == 2)
    ok = ok && p.s2 > T(0) && p.u2 >= T(0) && p.v2 >= T(0) && p.u2 + p.v2 <= T(1) && p.f2 < T(0);
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
    // one 32 x 32 -> 64-bit product per word (v_mad_u64_u32) gives both halves
    const uint64_t p0 = uint64_t(0xD2511F53u) * c.x, p1 = uint64_t(0xCD9E8D57u) * c.z;
    const uint32_t lo0 = uint32_t(p0), hi0 = uint32_t(p0 >> 32);
    const uint32_t lo1 = uint32_t(p1), hi1 = uint32_t(p1 >> 32);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// The rng() of Alg. 1 for (seed, point index, tuple): top 24 bits of word 0.
__device__ __forceinline__ float sample_stream(uint64_t seed, uint64_t point, uint32_t index, uint32_t stream) {
  const uint4 o = philox4x32_10(make_uint4(uint32_t(point), uint32_t(point >> 32), index, stream),
                                make_uint2(uint32_t(seed), uint32_t(seed >> 32)));
  return float(o.x >> 8) * (1.0f / 16777216.0f);
}
// The rng() of Alg. 1 for one tuple (stream 0); the one-sample draws use
// stream 1 (index = draw) and the bins of the bin-packed sampler stream 2.
__device__ __forceinline__ float selection_uniform(uint64_t seed, uint64_t point, uint32_t tuple) {
  return sample_stream(seed, point, tuple, 0u);
}

}  // namespace bbc
