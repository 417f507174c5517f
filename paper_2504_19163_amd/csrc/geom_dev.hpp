// Scene geometry on the device: structure-of-arrays triangles, emitters and
// the planar receiver, and the per-tuple constants of the rational chain.
#pragma once
#include "dev_common.hpp"

namespace bbc {

template <class T>
struct V3 {
  T x, y, z;
};
template <class T>
__host__ __device__ __forceinline__ V3<T> mk(T x, T y, T z) {
  return V3<T>{x, y, z};
}
template <class T>
__host__ __device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) {
  return mk(a.x + b.x, a.y + b.y, a.z + b.z);
}
template <class T>
__host__ __device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) {
  return mk(a.x - b.x, a.y - b.y, a.z - b.z);
}
template <class T>
__host__ __device__ __forceinline__ V3<T> operator*(T s, V3<T> a) {
  return mk(s * a.x, s * a.y, s * a.z);
}
template <class T>
__host__ __device__ __forceinline__ T dot(V3<T> a, V3<T> b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class T>
__host__ __device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <class T>
__host__ __device__ __forceinline__ T comp(V3<T> a, int c) {
  return c == 0 ? a.x : (c == 1 ? a.y : a.z);
}

// Device-resident scene (library-owned copies, structure of arrays).
struct DevScene {
  int chain;
  int64_t n_tri;
  const float* pos;  // [9][n_tri]
  const float* nrm;  // [9][n_tri]
  int64_t n_emit;
  const float* epos;  // [3][n_emit]
  const float* eI;    // [n_emit]
  const float* eedge; // [6][n_emit] edges a, b of area lights, or null (point lights)
  float eta;
  float q0[3], f1[3], f2[3];
  // two reflections: the second surface, and the candidate pairs that survived
  // tuple construction (tuple k is tid[k] = (emitter * n_tri + t1) * n_tri2 + t2)
  int64_t n_tri2;
  const float* pos2;  // [9][n_tri2]
  const float* nrm2;  // [9][n_tri2]
  const uint32_t* tid;
};

// Constants of one (emitter, triangle) tuple.  Barycentric parameterisation of
// the specular vertex (Sec. 4.3, Eqs. eq_xi, eq_ni):
// x1 = p0 + u e1 + v e2, n = n0 + u dn1 + v dn2 (un-normalised).
template <class T>
struct TupleGeom {
  V3<T> p0, e1, e2, n0, dn1, dn2, x0, q0, f1, f2, ng;
  T I0, a1, ak, eta;
  bool front;  // light strictly in front of the triangle plane (n_g oriented with the vertex normals)
  // area light x0 + z1 ea + z2 eb, (z1, z2) in [0,1]^2 (front: any point of it)
  bool area;
  V3<T> ea, eb;
  // two reflections: x2 = p0b + u2 e1b + v2 e2b, n2 likewise, ngb oriented like ng
  V3<T> p0b, e1b, e2b, n0b, dn1b, dn2b, ngb;
};

__device__ __forceinline__ V3<float> load3(const float* a, int64_t n, int64_t i, int row) {
  return mk(a[(row + 0) * n + i], a[(row + 1) * n + i], a[(row + 2) * n + i]);
}

template <class T>
__device__ __forceinline__ V3<T> cvt3(V3<float> a) {
  return mk(T(a.x), T(a.y), T(a.z));
}

template <class T>
__device__ __forceinline__ void second_triangle(TupleGeom<T>& g, V3<T> q0, V3<T> q1, V3<T> q2, V3<T> m0, V3<T> m1,
                                                V3<T> m2) {
  g.p0b = q0;
  g.e1b = q1 - q0;
  g.e2b = q2 - q0;
  g.n0b = m0;
  g.dn1b = m1 - m0;
  g.dn2b = m2 - m0;
  const V3<T> c = cross(g.e1b, g.e2b);
  g.ngb = (T(1) / sqrt(dot(c, c))) * c;
  if (dot(g.ngb, m0 + m1 + m2) < T(0)) g.ngb = T(-1) * g.ngb;
}

// The first-surface part of a tuple: triangle t lit by emitter e.
template <class T>
__device__ TupleGeom<T> tuple_geom_first(const DevScene& s, int64_t t, int64_t e) {
  TupleGeom<T> g;
  const V3<T> p0 = cvt3<T>(load3(s.pos, s.n_tri, t, 0));
  const V3<T> p1 = cvt3<T>(load3(s.pos, s.n_tri, t, 3));
  const V3<T> p2 = cvt3<T>(load3(s.pos, s.n_tri, t, 6));
  const V3<T> n0 = cvt3<T>(load3(s.nrm, s.n_tri, t, 0));
  const V3<T> n1 = cvt3<T>(load3(s.nrm, s.n_tri, t, 3));
  const V3<T> n2 = cvt3<T>(load3(s.nrm, s.n_tri, t, 6));
  g.p0 = p0;
  g.e1 = p1 - p0;
  g.e2 = p2 - p0;
  g.n0 = n0;
  g.dn1 = n1 - n0;
  g.dn2 = n2 - n0;
  const V3<T> c = cross(g.e1, g.e2);
  g.a1 = sqrt(dot(c, c));
  g.ng = (T(1) / g.a1) * c;
  if (dot(g.ng, n0 + n1 + n2) < T(0)) g.ng = T(-1) * g.ng;
  g.x0 = mk(T(s.epos[e]), T(s.epos[s.n_emit + e]), T(s.epos[2 * s.n_emit + e]));
  g.I0 = T(s.eI[e]);
  g.q0 = mk(T(s.q0[0]), T(s.q0[1]), T(s.q0[2]));
  g.f1 = mk(T(s.f1[0]), T(s.f1[1]), T(s.f1[2]));
  g.f2 = mk(T(s.f2[0]), T(s.f2[1]), T(s.f2[2]));
  const V3<T> fk = cross(g.f1, g.f2);
  g.ak = sqrt(dot(fk, fk));
  g.eta = T(s.eta);
  g.front = dot(g.x0 - p0, g.ng) > T(0);
  g.area = s.eedge != nullptr;
  if (g.area) {
    const int64_t ne = s.n_emit;
    g.ea = mk(T(s.eedge[e]), T(s.eedge[ne + e]), T(s.eedge[2 * ne + e]));
    g.eb = mk(T(s.eedge[3 * ne + e]), T(s.eedge[4 * ne + e]), T(s.eedge[5 * ne + e]));
    for (int k = 1; k < 4; ++k)
      g.front = g.front || dot(g.x0 + T(k & 1) * g.ea + T(k >> 1) * g.eb - p0, g.ng) > T(0);
  }
  return g;
}

// Tuple `tuple` of the scene: emitter * n_tri + triangle for one vertex; for
// two reflections the index of a constructed pair, whose number tid[tuple] is
// (emitter * n_tri + t1) * n_tri2 + t2.
template <class T>
__device__ TupleGeom<T> tuple_geom(const DevScene& s, uint32_t tuple) {
  if (s.chain != 2) return tuple_geom_first<T>(s, int64_t(tuple) % s.n_tri, int64_t(tuple) / s.n_tri);
  const uint32_t dense = s.tid[tuple];
  const int64_t t2 = int64_t(dense) % s.n_tri2, m = s.n_tri2, first = int64_t(dense) / s.n_tri2;
  TupleGeom<T> g = tuple_geom_first<T>(s, first % s.n_tri, first / s.n_tri);
  second_triangle<T>(g, cvt3<T>(load3(s.pos2, m, t2, 0)), cvt3<T>(load3(s.pos2, m, t2, 3)),
                     cvt3<T>(load3(s.pos2, m, t2, 6)), cvt3<T>(load3(s.nrm2, m, t2, 0)),
                     cvt3<T>(load3(s.nrm2, m, t2, 3)), cvt3<T>(load3(s.nrm2, m, t2, 6)));
  return g;
}

// Packed per-tuple record read by the query stage (one 128-byte line per
// tuple instead of eighteen scattered structure-of-arrays loads):
//   [0..8] p0 p1 p2, [9..17] n0 n1 n2, [18..20] x0, [21] I0,
//   [22] first leaf, [23] end leaf (as uint bits), [24..27] root box, [28..31] 0;
// two reflections append the second triangle: [28..36] p0 p1 p2, [37..45] n0 n1
// n2, [46..47] 0 (192 bytes).
constexpr int kRecFloats = 32;
constexpr int kRecFloatsRR = 48;

template <class T, bool RR = false>
__device__ __forceinline__ TupleGeom<T> tuple_geom_rec(const float* rec, const DevScene& s) {
  const V3<T> p0 = mk(T(rec[0]), T(rec[1]), T(rec[2]));
  const V3<T> p1 = mk(T(rec[3]), T(rec[4]), T(rec[5]));
  const V3<T> p2 = mk(T(rec[6]), T(rec[7]), T(rec[8]));
  const V3<T> n0 = mk(T(rec[9]), T(rec[10]), T(rec[11]));
  const V3<T> n1 = mk(T(rec[12]), T(rec[13]), T(rec[14]));
  const V3<T> n2 = mk(T(rec[15]), T(rec[16]), T(rec[17]));
  TupleGeom<T> g;
  g.p0 = p0;
  g.e1 = p1 - p0;
  g.e2 = p2 - p0;
  g.n0 = n0;
  g.dn1 = n1 - n0;
  g.dn2 = n2 - n0;
  const V3<T> c = cross(g.e1, g.e2);
  g.a1 = sqrt(dot(c, c));
  g.ng = (T(1) / g.a1) * c;
  if (dot(g.ng, n0 + n1 + n2) < T(0)) g.ng = T(-1) * g.ng;
  g.x0 = mk(T(rec[18]), T(rec[19]), T(rec[20]));
  g.I0 = T(rec[21]);
  g.q0 = mk(T(s.q0[0]), T(s.q0[1]), T(s.q0[2]));
  g.f1 = mk(T(s.f1[0]), T(s.f1[1]), T(s.f1[2]));
  g.f2 = mk(T(s.f2[0]), T(s.f2[1]), T(s.f2[2]));
  const V3<T> fk = cross(g.f1, g.f2);
  g.ak = sqrt(dot(fk, fk));
  g.eta = T(s.eta);
  g.front = dot(g.x0 - p0, g.ng) > T(0);
  g.area = false;  // a query record carries the pair's light point in x0
  if constexpr (RR)
    second_triangle<T>(g, mk(T(rec[28]), T(rec[29]), T(rec[30])), mk(T(rec[31]), T(rec[32]), T(rec[33])),
                       mk(T(rec[34]), T(rec[35]), T(rec[36])), mk(T(rec[37]), T(rec[38]), T(rec[39])),
                       mk(T(rec[40]), T(rec[41]), T(rec[42])), mk(T(rec[43]), T(rec[44]), T(rec[45])));
  return g;
}

}  // namespace bbc
