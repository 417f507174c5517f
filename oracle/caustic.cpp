// FP64 CPU oracle of the bound-driven caustic estimator.
//
// TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct definition the
// GPU library is checked against (see oracle.h).  Every polynomial of a box is
// rebuilt from scratch from the box corners with the Bernstein toolkit of
// bern.cpp; nothing is blocked, fused or cached beyond what the method states.
//
// Section references are to "Bernstein Bounds for Caustics" (Sec. 4: bounds
// of specular paths; Sec. 5: bound-driven sampling; Sec. 6.1: implementation).
#include <algorithm>
#include <array>
#include <atomic>
#include <functional>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <thread>
#include <vector>

#include "bern.hpp"
#include "oracle.h"

namespace orc {

static const double kInf = std::numeric_limits<double>::infinity();

// ---------------------------------------------------------------- vectors
struct V3 {
  double x = 0, y = 0, z = 0;
};
static V3 v3(double x, double y, double z) { return V3{x, y, z}; }
static V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
static V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
static V3 operator*(double s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
static double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static V3 cross(V3 a, V3 b) { return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double norm(V3 a) { return std::sqrt(dot(a, a)); }

// ---------------------------------------------------------------- one tuple
// Geometry of one (emitter, triangle) tuple for the single-vertex chains.
// Barycentric parameterisation of the specular vertex (Sec. 4.3, Eqs. eq_xi, eq_ni):
// x1 = p0 + u e1 + v e2,  n = n0 + u (n1 - n0) + v (n2 - n0) (un-normalised).
struct Tuple {
  int chain = 0;
  double eta = 1.0;
  V3 p0, e1, e2, n0, dn1, dn2;
  V3 ng;           // unit geometric normal, oriented to agree with the vertex normals
  double a1 = 0;   // |e1 x e2| = |dx1/du1|
  V3 x0;           // point light, or the corner of an area light
  double I0 = 1;
  bool area = false;  // area light x0 + z1 ea + z2 eb, (z1, z2) in [0,1]^2
  V3 ea, eb;
  V3 q0, f1, f2;   // receiver
  double ak = 0;   // |f1 x f2| = 1 / |du_k/dx_k|
  bool front = false;  // light strictly on the front side of the triangle plane
  // two reflections: the second triangle, x2 = p0b + u2 e1b + v2 e2b
  V3 p0b, e1b, e2b, n0b, dn1b, dn2b, ngb;
};

static V3 col(const double* a, int64_t n, int64_t i, int row) {
  return v3(a[(row + 0) * n + i], a[(row + 1) * n + i], a[(row + 2) * n + i]);
}

// Number of tuples: emitters x triangles, and x second-surface triangles for
// two reflections (tuple = (emitter * n_tri + t1) * n_tri2 + t2).
static int64_t n_tuples_of(const orc_scene* s) {
  return s->chain == 2 ? s->n_emit * s->n_tri * s->n_tri2 : s->n_emit * s->n_tri;
}

static V3 orient(V3 g, V3 nsum) { return dot(g, nsum) < 0 ? -1.0 * g : g; }

static Tuple make_tuple(const orc_scene* s, int64_t tuple) {
  Tuple c;
  const int64_t n = s->n_tri;
  int64_t first = tuple;
  if (s->chain == 2) {
    const int64_t t2 = tuple % s->n_tri2;
    first = tuple / s->n_tri2;
    const int64_t m = s->n_tri2;
    const V3 q0 = col(s->pos2, m, t2, 0), q1 = col(s->pos2, m, t2, 3), q2 = col(s->pos2, m, t2, 6);
    const V3 m0 = col(s->nrm2, m, t2, 0), m1 = col(s->nrm2, m, t2, 3), m2 = col(s->nrm2, m, t2, 6);
    c.p0b = q0;
    c.e1b = q1 - q0;
    c.e2b = q2 - q0;
    c.n0b = m0;
    c.dn1b = m1 - m0;
    c.dn2b = m2 - m0;
    const V3 gb = cross(c.e1b, c.e2b);
    c.ngb = orient((1.0 / norm(gb)) * gb, m0 + m1 + m2);
  }
  const int64_t e = first / n, t = first % n;
  c.chain = s->chain;
  c.eta = s->eta;
  const V3 p0 = col(s->pos, n, t, 0), p1 = col(s->pos, n, t, 3), p2 = col(s->pos, n, t, 6);
  const V3 n0 = col(s->nrm, n, t, 0), n1 = col(s->nrm, n, t, 3), n2 = col(s->nrm, n, t, 6);
  c.p0 = p0;
  c.e1 = p1 - p0;
  c.e2 = p2 - p0;
  c.n0 = n0;
  c.dn1 = n1 - n0;
  c.dn2 = n2 - n0;
  const V3 g = cross(c.e1, c.e2);
  c.a1 = norm(g);
  c.ng = (1.0 / c.a1) * g;
  if (dot(c.ng, n0 + n1 + n2) < 0) c.ng = -1.0 * c.ng;
  c.x0 = col(s->epos, s->n_emit, e, 0);
  c.I0 = s->eI[e];
  c.q0 = v3(s->q0[0], s->q0[1], s->q0[2]);
  c.f1 = v3(s->f1[0], s->f1[1], s->f1[2]);
  c.f2 = v3(s->f2[0], s->f2[1], s->f2[2]);
  c.ak = norm(cross(c.f1, c.f2));
  c.front = dot(c.x0 - p0, c.ng) > 0.0;
  if (s->eedge) {
    // an area light faces the triangle when any point of it lies strictly in
    // front of the triangle's plane: the front side of its four corners
    c.area = true;
    c.ea = col(s->eedge, s->n_emit, e, 0);
    c.eb = col(s->eedge, s->n_emit, e, 3);
    for (int k = 1; k < 4; ++k) {
      const V3 xc = c.x0 + double(k & 1) * c.ea + double(k >> 1) * c.eb;
      c.front = c.front || dot(xc - p0, c.ng) > 0.0;
    }
  }
  return c;
}

// The tuple as lit from the point (z1, z2) of its area light.
static Tuple at_light_point(Tuple c, double z1, double z2) {
  if (c.area) {
    c.x0 = c.x0 + z1 * c.ea + z2 * c.eb;
    c.front = dot(c.x0 - c.p0, c.ng) > 0.0;
    c.area = false;
  }
  return c;
}

// ---------------------------------------------------------------- exact path evaluation
// Forward-mode derivative in (u, v): value and the two partials.
struct D {
  double v = 0, a = 0, b = 0;
};
static D dc(double v) { return D{v, 0, 0}; }
static D operator+(D x, D y) { return D{x.v + y.v, x.a + y.a, x.b + y.b}; }
static D operator-(D x, D y) { return D{x.v - y.v, x.a - y.a, x.b - y.b}; }
static D operator*(D x, D y) { return D{x.v * y.v, x.a * y.v + x.v * y.a, x.b * y.v + x.v * y.b}; }
static D operator/(D x, D y) {
  const double q = x.v / y.v;
  return D{q, (x.a - q * y.a) / y.v, (x.b - q * y.b) / y.v};
}
static D dsqrt(D x) {
  const double r = std::sqrt(x.v);
  return D{r, x.a / (2 * r), x.b / (2 * r)};
}
struct DV {
  D x, y, z;
};
static DV dv_lin(V3 base, V3 du, V3 dv, double u, double v) {
  DV r;
  r.x = D{base.x + u * du.x + v * dv.x, du.x, dv.x};
  r.y = D{base.y + u * du.y + v * dv.y, du.y, dv.y};
  r.z = D{base.z + u * du.z + v * dv.z, du.z, dv.z};
  return r;
}
static DV dvc(V3 a) { return DV{dc(a.x), dc(a.y), dc(a.z)}; }
static DV operator-(DV a, DV b) { return DV{a.x - b.x, a.y - b.y, a.z - b.z}; }
static DV operator*(D s, DV a) { return DV{s * a.x, s * a.y, s * a.z}; }
static D ddot(DV a, DV b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static DV dcross(DV a, DV b) {
  return DV{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

struct PathEval {
  double uk = 0, vk = 0, t = 0;
  double J[2][2] = {{0, 0}, {0, 0}};
  double detJ = 0, Ek = 0, beta = 0, dn = 0;
  V3 x1;
  bool admissible = false;
};

// The receiver vertex of the path through barycentric (u, v): outgoing direction
// by the unnormalised reflection / refraction law (Sec. 4.3, Eq. eq_refr_rational),
// receiver coordinates by the triple-product ratios of Eq. eq_rct, and the
// irradiance of the path E_k = I0 dOmega0/dA1 |dx1/du1| |du1/du_k| |du_k/dx_k|
// (Sec. 4.4, Eq. eq_dwda) with dOmega0/dA1 = |n_g . d0| / |d0|^3, visibility and
// Fresnel factors dropped (each is at most one).
static DV operator+(DV a, DV b) { return DV{a.x + b.x, a.y + b.y, a.z + b.z}; }

// Two reflections (Sec. 4.3, Eq. eq_rct applied twice): the reflected ray of
// x1 meets the second triangle's plane at barycentric u2(u1); there it is
// reflected again with the interpolated normal and meets the receiver.
static PathEval eval_path_rr(const Tuple& c, double u, double v) {
  PathEval r;
  const DV x1 = dv_lin(c.p0, c.e1, c.e2, u, v);
  const DV n1 = dv_lin(c.n0, c.dn1, c.dn2, u, v);
  const DV d0 = x1 - dvc(c.x0);
  const DV dt1 = ddot(n1, n1) * d0 - (dc(2.0) * ddot(d0, n1)) * n1;
  const DV sb = x1 - dvc(c.p0b);
  const DV c1 = dcross(dt1, dvc(c.e2b));
  const D Q2 = ddot(c1, dvc(c.e1b));
  const D u2 = ddot(c1, sb) / Q2;
  const D v2 = ddot(dcross(sb, dvc(c.e1b)), dt1) / Q2;
  const D s2 = ddot(dcross(sb, dvc(c.e1b)), dvc(c.e2b)) / Q2;  // x2 = x1 + s2 d~1
  const DV x2 = dvc(c.p0b) + u2 * dvc(c.e1b) + v2 * dvc(c.e2b);
  const DV n2 = dvc(c.n0b) + u2 * dvc(c.dn1b) + v2 * dvc(c.dn2b);
  const DV d1 = x2 - x1;
  const DV dt2 = ddot(n2, n2) * d1 - (dc(2.0) * ddot(d1, n2)) * n2;
  const DV s3 = x2 - dvc(c.q0);
  const DV c3 = dcross(dt2, dvc(c.f2));
  const D Q3 = ddot(c3, dvc(c.f1));
  const D uk = ddot(c3, s3) / Q3, vk = ddot(dcross(s3, dvc(c.f1)), dt2) / Q3;
  const D t3 = ddot(dcross(s3, dvc(c.f1)), dvc(c.f2)) / Q3;
  r.uk = uk.v;
  r.vk = vk.v;
  r.t = t3.v;
  r.J[0][0] = uk.a;
  r.J[0][1] = uk.b;
  r.J[1][0] = vk.a;
  r.J[1][1] = vk.b;
  r.detJ = uk.a * vk.b - uk.b * vk.a;
  r.x1 = v3(x1.x.v, x1.y.v, x1.z.v);
  const V3 d = r.x1 - c.x0;
  const double dl = norm(d);
  r.Ek = c.I0 * std::fabs(dot(c.ng, d)) / (dl * dl * dl) * c.a1 / (std::fabs(r.detJ) * c.ak);
  const V3 dt1v = v3(dt1.x.v, dt1.y.v, dt1.z.v);
  bool ok = c.front && u >= 0.0 && v >= 0.0 && u + v <= 1.0 && s2.v > 0.0 && u2.v >= 0.0 && v2.v >= 0.0 &&
            u2.v + v2.v <= 1.0 && dot(dt1v, c.ngb) < 0.0 && r.t > 0.0;
  r.admissible = ok && std::isfinite(r.uk) && std::isfinite(r.vk);
  return r;
}

static PathEval eval_path(const Tuple& c, double u, double v) {
  if (c.chain == 2) return eval_path_rr(c, u, v);
  PathEval r;
  const DV x1 = dv_lin(c.p0, c.e1, c.e2, u, v);
  const DV n = dv_lin(c.n0, c.dn1, c.dn2, u, v);
  const DV d0 = x1 - dvc(c.x0);
  const D nn = ddot(n, n), dn = ddot(d0, n);
  DV dt;
  if (c.chain == 0) {
    dt = nn * d0 - (dc(2.0) * dn) * n;
  } else {
    const D dd = ddot(d0, d0);
    const D beta = dc(1.0 - c.eta * c.eta) * nn * dd + dc(c.eta * c.eta) * dn * dn;
    r.beta = beta.v;
    if (!(beta.v > 0.0)) {
      r.x1 = v3(x1.x.v, x1.y.v, x1.z.v);
      return r;  // total internal reflection: no refracted path
    }
    const D sq = dsqrt(beta);
    dt = dc(c.eta) * (nn * d0 - dn * n) - sq * n;
  }
  const DV s = x1 - dvc(c.q0);
  const DV cc = dcross(dt, dvc(c.f2));
  const D Q = ddot(cc, dvc(c.f1));
  const D Pu = ddot(cc, s);
  const D Pv = ddot(dcross(s, dvc(c.f1)), dt);
  const D Tn = ddot(dcross(s, dvc(c.f1)), dvc(c.f2));
  const D uk = Pu / Q, vk = Pv / Q, t = Tn / Q;
  r.uk = uk.v;
  r.vk = vk.v;
  r.t = t.v;
  r.J[0][0] = uk.a;
  r.J[0][1] = uk.b;
  r.J[1][0] = vk.a;
  r.J[1][1] = vk.b;
  r.detJ = uk.a * vk.b - uk.b * vk.a;
  r.dn = dn.v;
  r.x1 = v3(x1.x.v, x1.y.v, x1.z.v);
  const V3 d = r.x1 - c.x0;
  const double dl = norm(d);
  r.Ek = c.I0 * std::fabs(dot(c.ng, d)) / (dl * dl * dl) * c.a1 / (std::fabs(r.detJ) * c.ak);
  bool ok = c.front && u >= 0.0 && v >= 0.0 && u + v <= 1.0 && r.t > 0.0;
  if (c.chain == 1) ok = ok && r.beta > 0.0 && r.dn < 0.0;
  r.admissible = ok && std::isfinite(r.uk) && std::isfinite(r.vk);
  return r;
}

// ---------------------------------------------------------------- polynomials of a box
struct BV {
  Bern x, y, z;
};
static BV lin3(V3 base, V3 du, V3 dv, double u0, double u1, double v0, double v1) {
  return BV{linear_on_box(base.x, du.x, dv.x, u0, u1, v0, v1), linear_on_box(base.y, du.y, dv.y, u0, u1, v0, v1),
            linear_on_box(base.z, du.z, dv.z, u0, u1, v0, v1)};
}
static Bern dotB(const BV& a, const BV& b) { return add(add(mul(a.x, b.x), mul(a.y, b.y)), mul(a.z, b.z)); }
static Bern dotC(const BV& a, V3 k) { return add(add(scale(a.x, k.x), scale(a.y, k.y)), scale(a.z, k.z)); }
static BV crossC(const BV& a, V3 k) {  // a x k, k constant
  return BV{sub(scale(a.y, k.z), scale(a.z, k.y)), sub(scale(a.z, k.x), scale(a.x, k.z)),
            sub(scale(a.x, k.y), scale(a.y, k.x))};
}
static BV mulSV(const Bern& s, const BV& a) { return BV{mul(s, a.x), mul(s, a.y), mul(s, a.z)}; }
static BV subV(const BV& a, const BV& b) { return BV{sub(a.x, b.x), sub(a.y, b.y), sub(a.z, b.z)}; }
static BV scaleV(const BV& a, double k) { return BV{scale(a.x, k), scale(a.y, k), scale(a.z, k)}; }

// Secant of sqrt on [blo, bhi]: r(x) = a x + b through both end points.  sqrt is
// concave, so sqrt(x) - r(x) >= 0 on the interval; its maximum is where the
// slope of sqrt equals a, i.e. sqrt(x*) = (sqrt(blo) + sqrt(bhi)) / 2, which gives
// delta_hi = (sqrt(bhi) - sqrt(blo))^2 / (4 (sqrt(blo) + sqrt(bhi))).  This is the
// on-the-fly linear approximant with remainder bounds of Sec. 4.3 (the paper
// leaves the closed form to its supplement; this is one valid choice).
static void sqrt_secant(double blo, double bhi, double* a, double* b, double* dlo, double* dhi) {
  const double sa = std::sqrt(blo), sb = std::sqrt(bhi);
  *a = 1.0 / (sa + sb);
  *b = sa * sb / (sa + sb);
  *dlo = 0.0;
  *dhi = (sb - sa) * (sb - sa) / (4.0 * (sa + sb));
}

struct BoxBound {
  bool live = false;
  double uk[4] = {0, 1, 0, 1};  // u_lo, u_hi, v_lo, v_hi (clipped to [0,1]^2)
  double E[2] = {0, kInf};
  bool universal = false;
  bool settled = false;  // unclipped position bound inside [0,1]^2 and t > 0 proven
};

// Clip a ratio bound to [0,1]; false if the intersection is empty.
static bool clip01(const RatioBound& rb, double* lo, double* hi) {
  if (rb.kind == kDirect) {
    *lo = std::max(rb.lo, 0.0);
    *hi = std::min(rb.hi, 1.0);
    return *lo <= *hi;
  }
  if (rb.kind == kSplit) {  // (-inf, L] U [H, inf)
    const bool left = rb.lo >= 0.0, right = rb.hi <= 1.0;
    if (!left && !right) return false;
    *lo = left ? 0.0 : std::max(rb.hi, 0.0);
    *hi = right ? 1.0 : std::min(rb.lo, 1.0);
    return true;
  }
  *lo = 0.0;
  *hi = 1.0;
  return true;
}

// Bound of |f| from a ratio bound of f.
static void abs_bound(const RatioBound& rb, double* lo, double* hi) {
  if (rb.kind == kDirect) {
    const double a = std::fabs(rb.lo), b = std::fabs(rb.hi);
    *lo = (rb.lo <= 0.0 && rb.hi >= 0.0) ? 0.0 : std::min(a, b);
    *hi = std::max(a, b);
  } else if (rb.kind == kSplit) {
    *hi = kInf;
    *lo = (rb.lo >= 0.0 || rb.hi <= 0.0) ? 0.0 : std::min(-rb.lo, rb.hi);
  } else {
    *lo = 0.0;
    *hi = kInf;
  }
}

static BV addV(const BV& a, const BV& b) { return BV{add(a.x, b.x), add(a.y, b.y), add(a.z, b.z)}; }
static BV vecB(const Bern& s, V3 k) { return BV{scale(s, k.x), scale(s, k.y), scale(s, k.z)}; }

// Tuple construction for two reflections (Sec. 6.1 implementation): the second
// triangle is a candidate when the bound of (x2 - x1) x d~1 covers zero, with
// x1 over the first triangle's bounding box, x2 over the second's, and d~1 the
// reflected direction bounded by its Bernstein coefficients over [0,1]^2; the
// second triangle must also lie ahead along d~1 somewhere.  Plain interval
// arithmetic on these boxes.
static bool pair_candidate(const Tuple& c) {
  const BV n = lin3(c.n0, c.dn1, c.dn2, 0, 1, 0, 1);
  const BV d0 = lin3(c.p0 - c.x0, c.e1, c.e2, 0, 1, 0, 1);
  const BV dt = subV(mulSV(dotB(n, n), d0), mulSV(scale(dotB(d0, n), 2.0), n));
  double dl[3], dh[3];
  coef_range(dt.x, &dl[0], &dh[0]);
  coef_range(dt.y, &dl[1], &dh[1]);
  coef_range(dt.z, &dl[2], &dh[2]);
  const V3 a0 = c.p0, a1 = c.p0 + c.e1, a2 = c.p0 + c.e2;
  const V3 b0 = c.p0b, b1 = c.p0b + c.e1b, b2 = c.p0b + c.e2b;
  double xl[3], xh[3];  // x2 - x1 over the two bounding boxes
  for (int k = 0; k < 3; ++k) {
    auto cmp = [k](V3 p) { return k == 0 ? p.x : (k == 1 ? p.y : p.z); };
    const double alo = std::min({cmp(a0), cmp(a1), cmp(a2)}), ahi = std::max({cmp(a0), cmp(a1), cmp(a2)});
    const double blo = std::min({cmp(b0), cmp(b1), cmp(b2)}), bhi = std::max({cmp(b0), cmp(b1), cmp(b2)});
    xl[k] = blo - ahi;
    xh[k] = bhi - alo;
  }
  auto imul = [](double a, double b, double c2, double d, double* lo, double* hi) {
    const double p[4] = {a * c2, a * d, b * c2, b * d};
    *lo = std::min({p[0], p[1], p[2], p[3]});
    *hi = std::max({p[0], p[1], p[2], p[3]});
  };
  for (int k = 0; k < 3; ++k) {
    const int i = (k + 1) % 3, j = (k + 2) % 3;
    double pl, ph, ql, qh;
    imul(xl[i], xh[i], dl[j], dh[j], &pl, &ph);
    imul(xl[j], xh[j], dl[i], dh[i], &ql, &qh);
    if (pl - qh > 0.0 || ph - ql < 0.0) return false;  // component k of the cross product cannot vanish
  }
  double fh = 0.0;
  for (int k = 0; k < 3; ++k) {
    double pl, ph;
    imul(xl[k], xh[k], dl[k], dh[k], &pl, &ph);
    fh += ph;
  }
  return fh > 0.0;
}

// Position bound of one box for two reflections: the second vertex's
// barycentric coordinates u2 = Pu2/Q2, v2 = Pv2/Q2 (Eq. eq_rct) must meet the
// second triangle with the ray going forward and arriving on its front side;
// with x2 = X2/Q2 and n2 = N2/Q2, the second reflection
// d~2 = (N2.N2) D1 - 2 (D1.N2) N2 (D1 = X2 - Q2 x1, the common factors of the
// reflection law dropped) and the receiver coordinates u_k = Pu3/(Q3 Q2) of
// degree (16, 16) over (15, 15).  The irradiance bound follows the box's
// position bound (see irradiance_from).
static void irradiance_from(const Tuple& c, const BV& d0, const Bern& Q, const Bern& Pu, const Bern& Pv,
                            const Bern& Qu, const Bern& Qv, const Bern& Puu, const Bern& Puv, const Bern& Pvu,
                            const Bern& Pvv, int flags, BoxBound* bb);

static void implicit_irradiance(const Tuple& c, const BV& d0, const BV& x1, const BV& n, double wu, double wv,
                                BoxBound* bb);

static BoxBound bound_box_rr(const Tuple& c, double u0, double u1, double v0, double v1, bool want_irr,
                             int flags) {
  BoxBound bb;
  if (!c.front) return bb;
  if (u0 + v0 >= 1.0) return bb;
  const BV n = lin3(c.n0, c.dn1, c.dn2, u0, u1, v0, v1);
  const BV d0 = lin3(c.p0 - c.x0, c.e1, c.e2, u0, u1, v0, v1);
  const BV x1 = lin3(c.p0, c.e1, c.e2, u0, u1, v0, v1);
  const BV sb = lin3(c.p0 - c.p0b, c.e1, c.e2, u0, u1, v0, v1);
  const BV dt1 = subV(mulSV(dotB(n, n), d0), mulSV(scale(dotB(d0, n), 2.0), n));
  const BV c1 = crossC(dt1, c.e2b);
  const Bern Q2 = dotC(c1, c.e1b);
  const Bern Pu2 = dotB(c1, sb);
  const BV sbe1 = crossC(sb, c.e1b);
  const Bern Pv2 = dotB(sbe1, dt1);
  const Bern Tn2 = dotC(sbe1, c.e2b);
  // the ray from x1 must go forward to the second triangle's plane
  const RatioBound sr = ratio_bound(Tn2, Q2);
  if (sr.kind == kDirect && sr.hi <= 0.0) return bb;
  // and arrive on its front side
  double fl, fh;
  coef_range(dotC(dt1, c.ngb), &fl, &fh);
  if (fl >= 0.0) return bb;
  // u2 must meet the second triangle
  const RatioBound ub2 = ratio_bound(Pu2, Q2), vb2 = ratio_bound(Pv2, Q2), wb2 = ratio_bound(add(Pu2, Pv2), Q2);
  if (ub2.kind == kDirect && ub2.hi < 0.0) return bb;
  if (vb2.kind == kDirect && vb2.hi < 0.0) return bb;
  if (wb2.kind == kDirect && wb2.lo > 1.0) return bb;
  const BV X2 = addV(addV(vecB(Q2, c.p0b), vecB(Pu2, c.e1b)), vecB(Pv2, c.e2b));
  const BV N2 = addV(addV(vecB(Q2, c.n0b), vecB(Pu2, c.dn1b)), vecB(Pv2, c.dn2b));
  const BV D1 = subV(X2, mulSV(Q2, x1));
  const BV dt2 = subV(mulSV(dotB(N2, N2), D1), mulSV(scale(dotB(D1, N2), 2.0), N2));
  const BV S3 = subV(X2, vecB(Q2, c.q0));
  const BV c3 = crossC(dt2, c.f2);
  const BV s3f1 = crossC(S3, c.f1);
  const Bern Den = mul(dotC(c3, c.f1), Q2);
  const Bern Pu3 = dotB(c3, S3), Pv3 = dotB(s3f1, dt2), Tn3 = dotC(s3f1, c.f2);
  const RatioBound tb = ratio_bound(Tn3, Den);
  if (tb.kind == kDirect && tb.hi <= 0.0) return bb;
  const RatioBound ub = ratio_bound(Pu3, Den), vb = ratio_bound(Pv3, Den);
  if (!clip01(ub, &bb.uk[0], &bb.uk[1])) return bb;
  if (!clip01(vb, &bb.uk[2], &bb.uk[3])) return bb;
  bb.universal = (ub.kind == kUnbounded) || (vb.kind == kUnbounded);
  const bool inside2 = ub2.kind == kDirect && vb2.kind == kDirect && wb2.kind == kDirect && ub2.lo >= 0.0 &&
                       vb2.lo >= 0.0 && wb2.hi <= 1.0 && sr.kind == kDirect && sr.lo > 0.0 && fh < 0.0;
  bb.settled = inside2 && ub.kind == kDirect && vb.kind == kDirect && ub.lo >= 0.0 && ub.hi <= 1.0 &&
               vb.lo >= 0.0 && vb.hi <= 1.0 && tb.kind == kDirect && tb.lo > 0.0;
  bb.live = true;
  if (!want_irr) return bb;
  // Irradiance bound of the chain parametrised by the first vertex (the
  // generalised geometric term of Sec. 4.4 holds for any chain whose receiver
  // point is a function of u1): det(du_k/du1) = det M / Den^3 with M built from
  // (Den, Pu3, Pv3) and their u-, v-derivatives; det M has degree (46, 46).
  const double wu = u1 - u0, wv = v1 - v0;
  irradiance_from(c, d0, Den, Pu3, Pv3, scale(deriv(Den, 0), 1.0 / wu), scale(deriv(Den, 1), 1.0 / wv),
                  scale(deriv(Pu3, 0), 1.0 / wu), scale(deriv(Pu3, 1), 1.0 / wv), scale(deriv(Pv3, 0), 1.0 / wu),
                  scale(deriv(Pv3, 1), 1.0 / wv), flags, &bb);
  return bb;
}

// Position and irradiance bound of one box of the barycentric domain of u1
// (Sec. 4.2: U_k and [E_lo, E_hi] from coefficient ratios).
static BoxBound bound_box(const Tuple& c, double u0, double u1, double v0, double v1, bool want_irr, int flags) {
  if (c.chain == 2) return bound_box_rr(c, u0, u1, v0, v1, want_irr, flags);
  BoxBound bb;
  if (!c.front) return bb;
  if (u0 + v0 >= 1.0) return bb;  // box lies outside the triangle u + v <= 1
  const double wu = u1 - u0, wv = v1 - v0;
  const BV x1 = lin3(c.p0, c.e1, c.e2, u0, u1, v0, v1);
  const BV n = lin3(c.n0, c.dn1, c.dn2, u0, u1, v0, v1);
  BV d0 = lin3(c.p0 - c.x0, c.e1, c.e2, u0, u1, v0, v1);
  if (c.area) {
    // area light: d0 = x1 - (x0 + z1 ea + z2 eb) over axes (u, v, z1, z2);
    // the bounds below then hold for every point of the light
    d0 = BV{add(d0.x, add(affine_axis(2, 0.0, -c.ea.x), affine_axis(3, 0.0, -c.eb.x))),
            add(d0.y, add(affine_axis(2, 0.0, -c.ea.y), affine_axis(3, 0.0, -c.eb.y))),
            add(d0.z, add(affine_axis(2, 0.0, -c.ea.z), affine_axis(3, 0.0, -c.eb.z)))};
  }
  const BV s = lin3(c.p0 - c.q0, c.e1, c.e2, u0, u1, v0, v1);
  const Bern nn = dotB(n, n), dn = dotB(d0, n);

  Bern Pu, Pv, Q;
  // rows of M for the irradiance bound: (Q, Pu, Pv) and their total u-, v-derivatives
  Bern Qu, Qv, Puu, Puv, Pvu, Pvv;
  if (c.chain == 0) {
    // reflection: d~ = (n.n) d0 - 2 (d0.n) n
    const BV dt = subV(mulSV(nn, d0), mulSV(scale(dn, 2.0), n));
    const BV cc = crossC(dt, c.f2);
    Pu = dotB(cc, s);
    Pv = dotB(crossC(s, c.f1), dt);
    Q = dotC(cc, c.f1);
    if (want_irr) {
      Qu = scale(deriv(Q, 0), 1.0 / wu);
      Qv = scale(deriv(Q, 1), 1.0 / wv);
      Puu = scale(deriv(Pu, 0), 1.0 / wu);
      Puv = scale(deriv(Pu, 1), 1.0 / wv);
      Pvu = scale(deriv(Pv, 0), 1.0 / wu);
      Pvv = scale(deriv(Pv, 1), 1.0 / wv);
    }
  } else {
    // refraction: d~ = eta ((n.n) d0 - (d0.n) n) - sqrt(beta) n,
    // beta = (1 - eta^2)(n.n)(d0.d0) + eta^2 (d0.n)^2
    double dnlo, dnhi;
    coef_range(dn, &dnlo, &dnhi);
    if (dnlo >= 0.0) return bb;  // light reaches the back of the shading normal everywhere
    const double eta = c.eta;
    const Bern beta = add(scale(mul(nn, dotB(d0, d0)), 1.0 - eta * eta), scale(mul(dn, dn), eta * eta));
    double blo, bhi;
    coef_range(beta, &blo, &bhi);
    if (bhi <= 0.0) return bb;  // total internal reflection everywhere
    if (blo <= 0.0) {           // the square root cannot be bounded here: universal bound
      bb.live = true;
      bb.universal = true;
      return bb;
    }
    // remainder variable xi1 on axis 2: sqrt(beta) -> a beta + b + (1 - xi1) dlo + xi1 dhi
    double a, b, dlo, dhi;
    sqrt_secant(blo, bhi, &a, &b, &dlo, &dhi);
    Bern rt = add(scale(beta, a), Bern::constant(b));
    if (!(flags & 2)) rt = add(rt, affine_axis(2, dlo, dhi));
    const BV dt0 = scaleV(subV(mulSV(nn, d0), mulSV(dn, n)), eta);
    const BV c0 = crossC(dt0, c.f2), c1 = crossC(n, c.f2);
    const BV sf1 = crossC(s, c.f1);
    const Bern P0u = dotB(c0, s), P1u = dotB(c1, s);
    const Bern P0v = dotB(sf1, dt0), P1v = dotB(sf1, n);
    const Bern Q0 = dotC(c0, c.f1), Q1 = dotC(c1, c.f1);
    Pu = sub(P0u, mul(rt, P1u));
    Pv = sub(P0v, mul(rt, P1v));
    Q = sub(Q0, mul(rt, Q1));
    if (want_irr) {
      // Derivative-aware remainder: d sqrt(beta)/du = beta_u w with
      // w = 1/(2 sqrt(beta)) in [1/(2 sqrt(bhi)), 1/(2 sqrt(blo))], carried by a
      // second remainder variable xi2 on axis 3 (4D superset of the true values).
      Bern w = affine_axis(3, 0.5 / std::sqrt(bhi), 0.5 / std::sqrt(blo));
      if (flags & 2) w = Bern::constant(a);
      const Bern bu = scale(deriv(beta, 0), 1.0 / wu), bv = scale(deriv(beta, 1), 1.0 / wv);
      const Bern wbu = mul(w, bu), wbv = mul(w, bv);
      auto total = [&](const Bern& X0, const Bern& X1, int axis, double width, const Bern& wb) {
        const Bern X0d = scale(deriv(X0, axis), 1.0 / width), X1d = scale(deriv(X1, axis), 1.0 / width);
        return sub(sub(X0d, mul(rt, X1d)), mul(wb, X1));
      };
      Qu = total(Q0, Q1, 0, wu, wbu);
      Qv = total(Q0, Q1, 1, wv, wbv);
      Puu = total(P0u, P1u, 0, wu, wbu);
      Puv = total(P0u, P1u, 1, wv, wbv);
      Pvu = total(P0v, P1v, 0, wu, wbu);
      Pvv = total(P0v, P1v, 1, wv, wbv);
    }
  }
  // ray parameter t = ((x1 - q0) x f1) . f2 / Q must be positive somewhere
  const Bern Tn = dotC(crossC(s, c.f1), c.f2);
  const RatioBound tb = ratio_bound(Tn, Q);
  if (tb.kind == kDirect && tb.hi <= 0.0) return bb;
  // position bound U_k (Sec. 4.2)
  const RatioBound ub = ratio_bound(Pu, Q), vb = ratio_bound(Pv, Q);
  if (!clip01(ub, &bb.uk[0], &bb.uk[1])) return bb;
  if (!clip01(vb, &bb.uk[2], &bb.uk[3])) return bb;
  bb.universal = (ub.kind == kUnbounded) || (vb.kind == kUnbounded);
  bb.settled = ub.kind == kDirect && vb.kind == kDirect && ub.lo >= 0.0 && ub.hi <= 1.0 && vb.lo >= 0.0 &&
               vb.hi <= 1.0 && tb.kind == kDirect && tb.lo > 0.0;
  bb.live = true;
  if (!want_irr) return bb;
  if (c.chain == 1 && (flags & 4))
    implicit_irradiance(c, d0, x1, n, wu, wv, &bb);
  else
    irradiance_from(c, d0, Q, Pu, Pv, Qu, Qv, Puu, Puv, Pvu, Pvv, flags, &bb);
  return bb;
}

// G1 = |n_g . d0| / |d0|^3 bounded factor-wise, times I0 A1 / A_k, applied to
// a bound [rlo, rhi] of |du1/du_k|.
static void irradiance_factor(const Tuple& c, const BV& d0, double rlo, double rhi, double* Elo, double* Ehi) {
  double glo, ghi, hlo, hhi;
  coef_range(dotC(d0, c.ng), &glo, &ghi);
  coef_range(dotB(d0, d0), &hlo, &hhi);
  const double aglo = (glo <= 0.0 && ghi >= 0.0) ? 0.0 : std::min(std::fabs(glo), std::fabs(ghi));
  const double aghi = std::max(std::fabs(glo), std::fabs(ghi));
  const double Glo = aglo / std::pow(hhi, 1.5);
  const double Ghi = hlo > 0.0 ? aghi / std::pow(hlo, 1.5) : kInf;
  const double k = c.I0 * c.a1 / c.ak;
  *Elo = (Glo == 0.0 || rlo == 0.0) ? 0.0 : k * Glo * rlo;
  *Ehi = (std::isinf(Ghi) || std::isinf(rhi)) ? kInf : k * Ghi * rhi;
}

// Irradiance bound [E_lo, E_hi] of a box from the receiver map u_k = (Pu/Q,
// Pv/Q) and its total derivatives: det(du_k/du1) = det M / Q^3 with
// M = [[Q, Pu, Pv], [Q_u, Pu_u, Pv_u], [Q_v, Pu_v, Pv_v]] (Sec. 4.4, Eq.
// eq_irr_term3a), |du1/du_k| bounded by the ratio of Q^3 to det M, and
// dOmega0/dA1 = |g| / h^(3/2) with g = n_g . d0 and h = d0 . d0 bounded
// factor-wise; E = I0 (A1 / A_k) G1 |Q^3 / det M|.
// Degree reduction (Sec. 6.1, "Degree reduction"; oracle flag 8): a polynomial
// whose degree along u or v exceeds kReduceAbove (the paper's example
// threshold, 40) is replaced by its least-squares approximant of degree
// kReduceTo along those axes (16, the degree of the chain's position
// numerators) plus a remainder variable:
// A = X + r (2 s - 1) for some s in [0, 1], r the largest residual coefficient,
// the remainder riding on a fresh axis `raxis` (each reduction starts from a
// polynomial without remainder variables, so none has to be absorbed).
static constexpr int kReduceAbove = 40, kReduceTo = 16;
static bool needs_reduction(const Bern& A) { return A.deg[0] > kReduceAbove || A.deg[1] > kReduceAbove; }
static Bern with_remainder(const Bern& A, int raxis) {
  Deg to = A.deg;
  to[0] = std::min(to[0], kReduceTo);
  to[1] = std::min(to[1], kReduceTo);
  double r = 0.0;
  const Bern X = reduce_degree(A, to, &r);
  return add(X, affine_axis(raxis, -r, r));
}

static void irradiance_from(const Tuple& c, const BV& d0, const Bern& Q, const Bern& Pu, const Bern& Pv,
                            const Bern& Qu, const Bern& Qv, const Bern& Puu, const Bern& Puv, const Bern& Pvu,
                            const Bern& Pvv, int flags, BoxBound* bb) {
  const Bern detM = add(sub(mul(Q, sub(mul(Puu, Pvv), mul(Pvu, Puv))), mul(Pu, sub(mul(Qu, Pvv), mul(Pvu, Qv)))),
                        mul(Pv, sub(mul(Qu, Puv), mul(Puu, Qv))));
  const Bern Q3 = mul(mul(Q, Q), Q);
  double rlo, rhi;
  if ((flags & 8) && (needs_reduction(detM) || needs_reduction(Q3))) {
    // Q^3 / det M over (u, v, s, t): Q^3's remainder on axis 2, det M's on 3
    abs_bound(ratio_bound(with_remainder(Q3, 2), with_remainder(detM, 3)), &rlo, &rhi);
  } else {
    abs_bound(ratio_bound(Q3, detM), &rlo, &rhi);
  }
  irradiance_factor(c, d0, rlo, rhi, &bb->E[0], &bb->E[1]);
}

static BV crossB(const BV& a, const BV& b) {
  return BV{sub(mul(a.y, b.z), mul(a.z, b.y)), sub(mul(a.z, b.x), mul(a.x, b.z)), sub(mul(a.x, b.y), mul(a.y, b.x))};
}

// Irradiance bound of a refraction box by implicit differentiation (Sec. 4.4,
// "Implicit differentiation").  The refraction at x1 is written as two
// polynomials in u1 and the receiver coordinates u_k (the multivariate
// specular polynomials of the footnote there):
//   F = |d0|^2 ((d1 x n).b)^2 - eta^2 |d1|^2 ((d0 x n).b)^2   (Snell's law along b),
//   G = (d0 x n).d1                                            (coplanarity),
// with d0 = x1 - x0, d1 = x_k - x1, n the interpolated normal and eta the
// ratio n_incident / n_transmitted of the refraction evaluator (reading R30).
// u1 and u_k are independent variables over the box times its position bound
// U_k (a 4-D superset of the path manifold, axes u, v, u_k, v_k); from
// F = G = 0, du1/du_k = -J_1^{-1} J_k with J_1 = d(F,G)/d(u1,v1) and
// J_k = d(F,G)/d(u_k,v_k), so |det du1/du_k| = |det J_k / det J_1| and
// E = I0 (A1/A_k) G1 |det J_k / det J_1|.  The bound is formed with b = (1,0,0)
// and b = (0,1,0) and the two intervals intersected.
static void implicit_irradiance(const Tuple& c, const BV& d0, const BV& x1, const BV& n, double wu, double wv,
                                BoxBound* bb) {
  bb->E[0] = 0.0;
  bb->E[1] = kInf;
  const double wk = bb->uk[1] - bb->uk[0], wl = bb->uk[3] - bb->uk[2];
  if (!(wk > 0.0 && wl > 0.0)) return;
  const Bern ukB = affine_axis(2, bb->uk[0], bb->uk[1]), vkB = affine_axis(3, bb->uk[2], bb->uk[3]);
  const BV q0{Bern::constant(c.q0.x), Bern::constant(c.q0.y), Bern::constant(c.q0.z)};
  const BV xk = addV(addV(q0, vecB(ukB, c.f1)), vecB(vkB, c.f2));
  const BV d1 = subV(xk, x1);
  const BV c0 = crossB(d0, n), c1 = crossB(d1, n);
  const Bern d0d0 = dotB(d0, d0), d1d1 = dotB(d1, d1);
  const Bern G = dotB(c0, d1);
  const Bern Gu = scale(deriv(G, 0), 1.0 / wu), Gv = scale(deriv(G, 1), 1.0 / wv);
  const Bern Gk = scale(deriv(G, 2), 1.0 / wk), Gl = scale(deriv(G, 3), 1.0 / wl);
  double Elo = 0.0, Ehi = kInf;
  for (int axis = 0; axis < 2; ++axis) {  // b = (1,0,0), then (0,1,0)
    const Bern& a0 = axis == 0 ? c0.x : c0.y;
    const Bern& a1 = axis == 0 ? c1.x : c1.y;
    const Bern F = sub(mul(d0d0, mul(a1, a1)), scale(mul(d1d1, mul(a0, a0)), c.eta * c.eta));
    const Bern Fu = scale(deriv(F, 0), 1.0 / wu), Fv = scale(deriv(F, 1), 1.0 / wv);
    const Bern Fk = scale(deriv(F, 2), 1.0 / wk), Fl = scale(deriv(F, 3), 1.0 / wl);
    const Bern detJ1 = sub(mul(Fu, Gv), mul(Fv, Gu));
    const Bern detJk = sub(mul(Fk, Gl), mul(Fl, Gk));
    double rlo, rhi, elo, ehi;
    abs_bound(ratio_bound(detJk, detJ1), &rlo, &rhi);
    irradiance_factor(c, d0, rlo, rhi, &elo, &ehi);
    Elo = std::max(Elo, elo);
    Ehi = std::min(Ehi, ehi);
  }
  bb->E[0] = Elo;
  bb->E[1] = Ehi;
}

// ---------------------------------------------------------------- build
struct Leaf {
  int64_t tuple;
  int32_t depth;
  int64_t iu, iv;
  double box[4];  // u0, u1, v0, v1
  double uk[4];
  double E[2];
  bool universal;
};

struct Root {
  int64_t tuple;
  double box[4];
};

struct Build {
  orc_params p;
  int64_t n_tuples = 0, n_tri = 0;
  std::vector<Root> roots;
  std::vector<Leaf> leaves;
  std::vector<int64_t> leaf_begin;  // per tuple, into leaves (size n_tuples + 1)
  std::vector<std::map<int64_t, double>> cells;  // per grid cell: tuple -> E~
  std::map<int64_t, double> cover;               // cover-all list: tuple -> largest E_hi of its leaves
  int64_t boxes = 0;
  const orc_scene* scene = nullptr;  // borrowed
  // deep copies so the build owns its geometry
  std::vector<double> pos, nrm, epos, eI, pos2, nrm2, eedge;
  orc_scene sc{};
};

static void parallel_for(int64_t n, int n_threads, const std::function<void(int64_t, int)>& fn);

// Domain initialisation (Sec. 6.1): breadth-first subdivision of [0,1]^2 keeping
// boxes whose position bound meets the receiver.  A box whose whole position
// bound already lies inside [0,1]^2 with the ray parameter proven positive is
// settled: it is kept without further refinement.  Descent stops when every
// kept box is settled, when more than init_pieces boxes would be kept, or after
// init_levels levels; the root box is the bounding box of the kept boxes.
static bool init_domain(const Tuple& c, const orc_params& p, double root[4], int64_t* boxes) {
  struct B {
    int level;
    int64_t iu, iv;
    bool settled;
  };
  auto test = [&](int level, int64_t iu, int64_t iv, B* out) {
    const double w = std::ldexp(1.0, -level);
    ++*boxes;
    const BoxBound bb = bound_box(c, iu * w, (iu + 1) * w, iv * w, (iv + 1) * w, false, p.flags);
    *out = B{level, iu, iv, bb.settled};
    return bb.live;
  };
  B b0;
  if (!test(0, 0, 0, &b0)) return false;
  std::vector<B> cur{b0};
  for (int L = 1; L <= p.init_levels; ++L) {
    bool all_settled = true;
    for (const B& b : cur) all_settled = all_settled && b.settled;
    if (all_settled) break;
    std::vector<B> next;
    for (const B& b : cur) {
      if (b.settled) {
        next.push_back(b);
        continue;
      }
      for (int a = 0; a < 2; ++a)
        for (int d = 0; d < 2; ++d) {
          B ch;
          if (test(b.level + 1, 2 * b.iu + a, 2 * b.iv + d, &ch)) next.push_back(ch);
        }
    }
    if (next.empty()) return false;
    if (int64_t(next.size()) > p.init_pieces) break;
    cur.swap(next);
  }
  root[0] = root[2] = kInf;
  root[1] = root[3] = -kInf;
  for (const B& b : cur) {
    const double w = std::ldexp(1.0, -b.level);
    root[0] = std::min(root[0], b.iu * w);
    root[1] = std::max(root[1], (b.iu + 1) * w);
    root[2] = std::min(root[2], b.iv * w);
    root[3] = std::max(root[3], (b.iv + 1) * w);
  }
  return true;
}

// Adaptive subdivision (Sec. 6.1): split a box into four at its midpoint until
// the clipped position bound is smaller than sigma, the irradiance bound is
// tighter than the ratio alpha, or the depth cap is reached.
static void subdivide(const Tuple& c, int64_t tuple, const double root[4], int depth, int64_t iu, int64_t iv,
                      const orc_params& p, std::vector<Leaf>* out, int64_t* boxes) {
  const double fu = (root[1] - root[0]) * std::ldexp(1.0, -depth);
  const double fv = (root[3] - root[2]) * std::ldexp(1.0, -depth);
  const double u0 = root[0] + iu * fu, u1 = root[0] + (iu + 1) * fu;
  const double v0 = root[2] + iv * fv, v1 = root[2] + (iv + 1) * fv;
  ++*boxes;
  const BoxBound bb = bound_box(c, u0, u1, v0, v1, true, p.flags);
  if (!bb.live) return;
  const double area = (bb.uk[1] - bb.uk[0]) * (bb.uk[3] - bb.uk[2]);
  bool stop = depth >= p.max_depth;
  if (!(p.flags & 1)) {
    stop = stop || area < p.sigma;
    stop = stop || (bb.E[0] > 0.0 && std::isfinite(bb.E[1]) && bb.E[1] < p.alpha * bb.E[0]);
  }
  if (stop) {
    Leaf l;
    l.tuple = tuple;
    l.depth = depth;
    l.iu = iu;
    l.iv = iv;
    l.box[0] = u0;
    l.box[1] = u1;
    l.box[2] = v0;
    l.box[3] = v1;
    std::memcpy(l.uk, bb.uk, sizeof(l.uk));
    l.E[0] = bb.E[0];
    l.E[1] = bb.E[1];
    l.universal = bb.universal;
    out->push_back(l);
    return;
  }
  for (int a = 0; a < 2; ++a)
    for (int d = 0; d < 2; ++d) subdivide(c, tuple, root, depth + 1, 2 * iu + a, 2 * iv + d, p, out, boxes);
}

static int cell_of(double x, int G) { return std::min(G - 1, int(std::floor(x * G))); }

static Build* build_all(const orc_scene* s, const orc_params* p, int n_threads) {
  Build* B = new Build;
  B->p = *p;
  // own a copy of the scene arrays
  const int64_t n = s->n_tri;
  B->pos.assign(s->pos, s->pos + 9 * n);
  B->nrm.assign(s->nrm, s->nrm + 9 * n);
  B->epos.assign(s->epos, s->epos + 3 * s->n_emit);
  B->eI.assign(s->eI, s->eI + s->n_emit);
  B->sc = *s;
  B->sc.pos = B->pos.data();
  B->sc.nrm = B->nrm.data();
  B->sc.epos = B->epos.data();
  B->sc.eI = B->eI.data();
  if (s->eedge) {
    B->eedge.assign(s->eedge, s->eedge + 6 * s->n_emit);
    B->sc.eedge = B->eedge.data();
  }
  B->scene = &B->sc;
  if (s->chain == 2) {
    B->pos2.assign(s->pos2, s->pos2 + 9 * s->n_tri2);
    B->nrm2.assign(s->nrm2, s->nrm2 + 9 * s->n_tri2);
    B->sc.pos2 = B->pos2.data();
    B->sc.nrm2 = B->nrm2.data();
  }
  B->n_tri = n;
  B->n_tuples = n_tuples_of(s);
  const int64_t T = B->n_tuples;
  std::vector<std::vector<Leaf>> per(T);
  std::vector<int> has_root(T, 0);
  std::vector<std::array<double, 4>> roots(T);
  std::vector<int64_t> boxes(std::max(1, n_threads), 0);
  parallel_for(T, n_threads, [&](int64_t t, int worker) {
    const Tuple c = make_tuple(&B->sc, t);
    if (!c.front) return;
    if (c.chain == 2 && !pair_candidate(c)) return;
    double root[4];
    if (!init_domain(c, *p, root, &boxes[worker])) return;
    has_root[t] = 1;
    std::memcpy(roots[t].data(), root, sizeof(root));
    subdivide(c, t, root, 0, 0, 0, *p, &per[t], &boxes[worker]);
  });
  for (int64_t b : boxes) B->boxes += b;
  B->leaf_begin.assign(T + 1, 0);
  for (int64_t t = 0; t < T; ++t) {
    if (has_root[t]) B->roots.push_back(Root{t, {roots[t][0], roots[t][1], roots[t][2], roots[t][3]}});
    B->leaf_begin[t] = int64_t(B->leaves.size());
    B->leaves.insert(B->leaves.end(), per[t].begin(), per[t].end());
  }
  B->leaf_begin[T] = int64_t(B->leaves.size());
  // Bound storage (Sec. 6.1): splat each leaf's irradiance bound into every grid
  // cell its closed position bound touches; per (cell, tuple) keep the maximum
  // (Eq. eq_pertuple_b with m = 1).  A tuple whose leaves would write at least
  // cover_frac * G^2 (leaf, cell) records (universal and very wide position
  // bounds) is stored once instead, in the cover-all list that every shading
  // point reads beside its cell, with the largest E_hi of all its leaves: a
  // larger per-tuple bound than its cells would hold, so still conservative.
  const int G = p->grid_res;
  B->cells.assign(size_t(G) * G, {});
  std::vector<char> in_cover(size_t(T), 0);
  if (p->cover_frac > 0.0) {
    const double thr = p->cover_frac * double(G) * double(G);
    for (int64_t t = 0; t < T; ++t) {
      int64_t cells = 0;
      double emax = 0.0;
      for (int64_t k = B->leaf_begin[t]; k < B->leaf_begin[t + 1]; ++k) {
        const Leaf& l = B->leaves[size_t(k)];
        cells += int64_t(cell_of(l.uk[1], G) - cell_of(l.uk[0], G) + 1) *
                 int64_t(cell_of(l.uk[3], G) - cell_of(l.uk[2], G) + 1);
        emax = std::max(emax, l.E[1]);
      }
      if (cells > 0 && double(cells) >= thr) {
        in_cover[size_t(t)] = 1;
        B->cover.emplace(t, emax);
      }
    }
  }
  for (const Leaf& l : B->leaves) {
    if (in_cover[size_t(l.tuple)]) continue;
    const int cu0 = cell_of(l.uk[0], G), cu1 = cell_of(l.uk[1], G);
    const int cv0 = cell_of(l.uk[2], G), cv1 = cell_of(l.uk[3], G);
    for (int cu = cu0; cu <= cu1; ++cu)
      for (int cv = cv0; cv <= cv1; ++cv) {
        auto& m = B->cells[size_t(cu) * G + cv];
        auto it = m.find(l.tuple);
        if (it == m.end())
          m.emplace(l.tuple, l.E[1]);
        else
          it->second = std::max(it->second, l.E[1]);
      }
  }
  return B;
}

// ---------------------------------------------------------------- threads
static void parallel_for(int64_t n, int n_threads, const std::function<void(int64_t, int)>& fn) {
  if (n_threads <= 1 || n < 2) {
    for (int64_t i = 0; i < n; ++i) fn(i, 0);
    return;
  }
  std::vector<std::thread> th;
  std::atomic<int64_t> next{0};
  for (int w = 0; w < n_threads; ++w)
    th.emplace_back([&, w]() {
      for (;;) {
        const int64_t i = next.fetch_add(1);
        if (i >= n) break;
        fn(i, w);
      }
    });
  for (auto& t : th) t.join();
}

// ---------------------------------------------------------------- sampling
// Bound-optimal probabilities (Sec. 5.4): P_T = min(gamma E~_T, 1) with gamma
// fixed by the expected sample count.  W' = min(W, |U|); unbounded entries take
// P = 1; the finite positive entries share max(W' - n_inf, 1) expected samples
// (at most one each), solved exactly by water-filling over the entries sorted
// in decreasing order; entries with E~ = 0 take P = 0.
static void probabilities(const double* Et, int64_t n, double W, double* P) {
  const double Wp = std::min(W, double(n));
  int64_t n_inf = 0;
  std::vector<int64_t> fin;
  for (int64_t i = 0; i < n; ++i) {
    if (std::isinf(Et[i])) {
      P[i] = 1.0;
      ++n_inf;
    } else if (Et[i] > 0.0) {
      fin.push_back(i);
    } else {
      P[i] = 0.0;
    }
  }
  if (fin.empty()) return;
  double Wf = std::max(Wp - double(n_inf), 1.0);
  Wf = std::min(Wf, double(fin.size()));
  if (Wf >= double(fin.size())) {
    for (int64_t i : fin) P[i] = 1.0;
    return;
  }
  std::vector<int64_t> ord = fin;
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return Et[a] > Et[b]; });
  const int64_t m = int64_t(ord.size());
  std::vector<double> tail(m + 1, 0.0);  // tail[k] = sum_{i >= k} E~_(i)
  for (int64_t k = m - 1; k >= 0; --k) tail[k] = tail[k + 1] + Et[ord[k]];
  int64_t k = 0;
  double gamma = 0.0;
  for (; k < m; ++k) {
    gamma = (Wf - double(k)) / tail[k];
    if (gamma * Et[ord[k]] <= 1.0) break;
  }
  for (int64_t i = 0; i < m; ++i) P[ord[i]] = i < k ? 1.0 : std::min(gamma * Et[ord[i]], 1.0);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy
// as 1, 2, 3", SC 2011): ten rounds of two 32x32->64 multiplies with the
// published multipliers and Weyl key increments.
static void philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c0;
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// The rng() of Alg. 1, keyed by (seed, index of the point in its request,
// tuple), so a result never depends on how requests are batched.  The other
// samplers draw from their own streams (last counter word): draw j of the
// one-sample estimator from stream 1, bin b of the bin-packed sampler from
// stream 2.  Values are multiples of 2^-24 in [0, 1), exact in FP32.
static double uniform_stream(uint64_t seed, uint64_t point, uint32_t index, uint32_t stream) {
  const uint32_t ctr[4] = {uint32_t(point), uint32_t(point >> 32), index, stream};
  const uint32_t key[2] = {uint32_t(seed), uint32_t(seed >> 32)};
  uint32_t o[4];
  philox(ctr, key, o);
  return double(o[0] >> 8) * (1.0 / 16777216.0);
}
static double uniform(uint64_t seed, uint64_t point, uint32_t tuple) { return uniform_stream(seed, point, tuple, 0u); }

// ---------------------------------------------------------------- other samplers
// The sampling schemes the paper compares with its multi-sample estimator
// (Sec. 5.2-5.3 and the sampling-scheme comparison figure), each as a list of
// selected candidates with the probability weight 1/P of its contribution.
// Every quantity is FP64, the sums run in list order, and each weight is the
// candidate's selection probability.
struct Pick {
  size_t k;  // index into U
  double P;  // contribution weight is 1 / P
};

// Uniform: every candidate of U with the same P = W' / |U|, W' = min(W, |U|)
// (position bound only; the irradiance bound is not consulted).
static std::vector<Pick> pick_uniform(size_t n, double W, uint64_t seed, uint64_t point, const int64_t* U) {
  std::vector<Pick> out;
  if (n == 0) return out;
  const double P = std::min(W, double(n)) / double(n);
  for (size_t k = 0; k < n; ++k)
    if (uniform(seed, point, uint32_t(U[k])) < P) out.push_back({k, P});
  return out;
}

// One-sample estimator repeated W times (Sec. 5.2): W independent draws with
// P1(T) = E~_T / sum E~ over the finite bounds, by inversion of the running
// sums in list order (draw j selects the first candidate whose running sum
// exceeds r_j times the total), and <E> = (1/W) sum_j E(T_j) / P1(T_j).  A
// candidate drawn c times enters once with weight c / (W P1).  Reading:
// candidates with an infinite bound have no finite P1; each is evaluated once
// with P = 1.  Candidates with E~ = 0 are never drawn (their E(T) is 0).
static std::vector<Pick> pick_one_sample(const std::vector<double>& Et, int W, uint64_t seed, uint64_t point) {
  const size_t n = Et.size();
  std::vector<Pick> out;
  std::vector<double> C(n, 0.0);
  double S = 0.0;
  size_t last = 0;
  for (size_t k = 0; k < n; ++k) {
    if (std::isinf(Et[k])) {
      out.push_back({k, 1.0});
    } else if (Et[k] > 0.0) {
      S += Et[k];
      last = k;
    }
    C[k] = S;
  }
  if (!(S > 0.0)) return out;
  std::vector<int> cnt(n, 0);
  for (int j = 0; j < W; ++j) {
    const double t = uniform_stream(seed, point, uint32_t(j), 1u) * S;
    size_t sel = last;
    for (size_t k = 0; k < n; ++k)
      if (std::isfinite(Et[k]) && Et[k] > 0.0 && t < C[k]) {
        sel = k;
        break;
      }
    ++cnt[sel];
  }
  for (size_t k = 0; k < n; ++k)
    if (cnt[k]) out.push_back({k, double(W) * (Et[k] / S) / double(cnt[k])});
  std::sort(out.begin(), out.end(), [](const Pick& a, const Pick& b) { return a.k < b.k; });
  return out;
}

// Bin-packed multi-sample estimator (Sec. 5.3): the bound-optimal P_T packed
// in list order into bins of total probability at most 1, one importance
// sample per bin.  Reading: next-fit packing (a candidate that does not fit
// the open bin closes it and opens the next), which is the greedy rule with
// O(|U|) time and approximation ratio 2 that the text states.  Candidate k
// of bin b owns [o_k, min(o_k + P_k, 1)) of that bin and is selected when the
// bin's draw r_b falls there; its weight is the length of that interval, its
// selection probability, and at most one candidate per bin is selected.
// The bound-optimal P sum to whole numbers in exact arithmetic, which their
// FP64 values reach only up to rounding, so "fits" means a running sum of at
// most 1 + 2^-40 (the part above 1 is cut), and a candidate whose interval
// would be empty (a full bin, or a P below the rounding of the sum) opens a
// new bin instead, so every candidate with P > 0 can be selected.
constexpr double kBinSlack = 1.0 / 1099511627776.0;  // 2^-40
static bool bin_fits(double fill, double p) { return fill + p <= 1.0 + kBinSlack && std::min(fill + p, 1.0) > fill; }
static std::vector<Pick> pick_bins(const std::vector<double>& P, uint64_t seed, uint64_t point) {
  std::vector<Pick> out;
  uint32_t b = 0;
  double fill = 0.0;
  double r = uniform_stream(seed, point, 0u, 2u);
  for (size_t k = 0; k < P.size(); ++k) {
    const double p = P[k];
    if (!(p > 0.0)) continue;
    if (!bin_fits(fill, p)) {
      ++b;
      fill = 0.0;
      r = uniform_stream(seed, point, b, 2u);
    }
    const double lo = fill;
    fill += p;
    const double hi = std::min(fill, 1.0);
    if (r >= lo && r < hi) out.push_back({k, hi - lo});
  }
  return out;
}

// Smallest distance between a quantity that decides a selection and its
// threshold, over the decisions one point's sampler takes (Alg. 1 and
// uniform: |r - P|; one-sample: |r S - C_k| / S over the running sums C_k;
// bins: |fill + P - 1| of every packing test and |r - o|, |r - o - P| of
// every interval).  Selections taken in another precision can differ only
// where this margin is below that precision's rounding.
static double sample_margin(const std::vector<double>& Et, const int64_t* U, double W, uint64_t seed,
                            uint64_t point, int sampler) {
  const size_t n = Et.size();
  double m = INFINITY;
  std::vector<double> P(n, 1.0);
  probabilities(Et.data(), int64_t(n), W, P.data());
  if (sampler == 0 || sampler == 1) {
    const double Pu = n ? std::min(W, double(n)) / double(n) : 0.0;
    for (size_t k = 0; k < n; ++k) {
      const double p = sampler == 1 ? Pu : P[k];
      if (p > 0.0 && p < 1.0) m = std::min(m, std::fabs(uniform(seed, point, uint32_t(U[k])) - p));
    }
  } else if (sampler == 2) {
    double S = 0.0;
    std::vector<double> C;
    for (size_t k = 0; k < n; ++k)
      if (std::isfinite(Et[k]) && Et[k] > 0.0) {
        S += Et[k];
        C.push_back(S);
      }
    if (S > 0.0)
      for (int j = 0; j < int(W); ++j) {
        const double t = uniform_stream(seed, point, uint32_t(j), 1u) * S;
        for (double c : C) m = std::min(m, std::fabs(t - c) / S);
      }
  } else {
    uint32_t b = 0;
    double fill = 0.0, r = uniform_stream(seed, point, 0u, 2u);
    for (size_t k = 0; k < n; ++k) {
      const double p = P[k];
      if (!(p > 0.0)) continue;
      m = std::min(m, std::fabs(fill + p - 1.0));
      if (!bin_fits(fill, p)) {
        ++b;
        fill = 0.0;
        r = uniform_stream(seed, point, b, 2u);
      }
      m = std::min(m, std::min(std::fabs(r - fill), std::fabs(r - std::min(fill + p, 1.0))));
      fill += p;
    }
  }
  return m;
}

// ---------------------------------------------------------------- roots
struct RootHit {
  double u, v, Ek, res;
};

static double residual(const Tuple& c, const PathEval& e, double us, double vs) {
  return norm((e.uk - us) * c.f1 + (e.vk - vs) * c.f2);
}

// Newton's method on u_k(u1) = u_k* in the local triangle domain (Sec. 6.1,
// root-finding).  Returns true when it converged to an admissible path.
static bool newton(const Tuple& c, double us, double vs, double u, double v, const double lim[4], int max_it,
                   double tol_stop, double tol_accept, RootHit* hit) {
  PathEval e = eval_path(c, u, v);
  for (int it = 0; it < max_it; ++it) {
    if (!std::isfinite(e.uk) || !std::isfinite(e.vk)) return false;
    if (residual(c, e, us, vs) < tol_stop) break;
    const double ru = e.uk - us, rv = e.vk - vs;
    const double det = e.detJ;
    if (det == 0.0 || !std::isfinite(det)) return false;
    const double du = (e.J[1][1] * ru - e.J[0][1] * rv) / det;
    const double dv = (-e.J[1][0] * ru + e.J[0][0] * rv) / det;
    u -= du;
    v -= dv;
    if (!(u >= lim[0] && u <= lim[1] && v >= lim[2] && v <= lim[3])) return false;
    e = eval_path(c, u, v);
  }
  const double res = residual(c, e, us, vs);
  if (!(res < tol_accept) || !e.admissible) return false;
  *hit = RootHit{u, v, e.Ek, res};
  return true;
}

static bool receiver_coords(const Tuple& c, V3 x, double* us, double* vs) {
  const V3 r = x - c.q0;
  const double a = dot(c.f1, c.f1), b = dot(c.f1, c.f2), d = dot(c.f2, c.f2);
  const double r1 = dot(c.f1, r), r2 = dot(c.f2, r);
  const double det = a * d - b * b;
  *us = (d * r1 - b * r2) / det;
  *vs = (a * r2 - b * r1) / det;
  return *us >= 0.0 && *us <= 1.0 && *vs >= 0.0 && *vs <= 1.0;
}

static void add_unique(std::vector<RootHit>* roots, const RootHit& h, double tol) {
  for (const RootHit& r : *roots)
    if (std::fabs(r.u - h.u) <= tol && std::fabs(r.v - h.v) <= tol) return;
  roots->push_back(h);
}

// Brute force: multi-start Newton from every point (i/L, j/L), i + j <= L, of a
// barycentric lattice; no bound is consulted.
static std::vector<RootHit> brute_roots(const Tuple& c, double us, double vs, int lattice) {
  std::vector<RootHit> roots;
  if (!c.front) return roots;
  const double lim[4] = {-2.0, 3.0, -2.0, 3.0};
  for (int i = 0; i <= lattice; ++i)
    for (int j = 0; i + j <= lattice; ++j) {
      RootHit h;
      if (newton(c, us, vs, double(i) / lattice, double(j) / lattice, lim, 50, 1e-13, 1e-9, &h))
        add_unique(&roots, h, 1e-9);
    }
  return roots;
}

// Deterministic initialisation from the bounds: one Newton start at the centre
// of every leaf of the tuple whose position bound contains u_k*; a start that
// moves farther than one box width outside its box is abandoned.
static std::vector<RootHit> leaf_roots(const Build& B, const Tuple& c, int64_t tuple, double us, double vs) {
  std::vector<RootHit> roots;
  for (int64_t k = B.leaf_begin[tuple]; k < B.leaf_begin[tuple + 1]; ++k) {
    const Leaf& l = B.leaves[k];
    if (!(us >= l.uk[0] && us <= l.uk[1] && vs >= l.uk[2] && vs <= l.uk[3])) continue;
    const double wu = l.box[1] - l.box[0], wv = l.box[3] - l.box[2];
    const double lim[4] = {l.box[0] - wu, l.box[1] + wu, l.box[2] - wv, l.box[3] + wv};
    RootHit h;
    if (newton(c, us, vs, 0.5 * (l.box[0] + l.box[1]), 0.5 * (l.box[2] + l.box[3]), lim, 20, 1e-13, 1e-6, &h))
      add_unique(&roots, h, 1e-7);
  }
  return roots;
}

}  // namespace orc

// ================================================================= C ABI
using namespace orc;

extern "C" {

int orc_eval_path(const orc_scene* s, int64_t tuple, double u, double v, double* out) {
  if (!s || !out || tuple < 0 || tuple >= n_tuples_of(s)) return -1;
  const Tuple c = make_tuple(s, tuple);
  const PathEval e = eval_path(c, u, v);
  out[0] = e.uk;
  out[1] = e.vk;
  out[2] = e.t;
  out[3] = e.Ek;
  out[4] = e.detJ;
  out[5] = e.admissible ? 1.0 : 0.0;
  out[6] = e.beta;
  out[7] = e.x1.x;
  out[8] = e.x1.y;
  out[9] = e.x1.z;
  return 0;
}

int orc_eval_path_at(const orc_scene* s, int64_t tuple, double u, double v, double z1, double z2, double* out) {
  if (!s || !out || tuple < 0 || tuple >= n_tuples_of(s)) return -1;
  const Tuple c = at_light_point(make_tuple(s, tuple), z1, z2);
  const PathEval e = eval_path(c, u, v);
  out[0] = e.uk;
  out[1] = e.vk;
  out[2] = e.t;
  out[3] = e.Ek;
  out[4] = e.detJ;
  out[5] = e.admissible ? 1.0 : 0.0;
  out[6] = e.beta;
  out[7] = e.x1.x;
  out[8] = e.x1.y;
  out[9] = e.x1.z;
  return 0;
}

int orc_box_bound(const orc_scene* s, int64_t tuple, const double* box, int want_irr, double* out) {
  return orc_box_bound_flags(s, tuple, box, want_irr, 0, out);
}

int orc_box_bound_flags(const orc_scene* s, int64_t tuple, const double* box, int want_irr, int flags,
                        double* out) {
  if (!s || !box || !out || tuple < 0 || tuple >= n_tuples_of(s)) return -1;
  const Tuple c = make_tuple(s, tuple);
  const BoxBound bb = bound_box(c, box[0], box[1], box[2], box[3], want_irr != 0, flags);
  out[0] = bb.live ? 1.0 : 0.0;
  for (int i = 0; i < 4; ++i) out[1 + i] = bb.uk[i];
  out[5] = bb.E[0];
  out[6] = bb.E[1];
  out[7] = bb.universal ? 1.0 : 0.0;
  return 0;
}

void* orc_build(const orc_scene* s, const orc_params* p, int n_threads) {
  if (!s || !p || s->chain < 0 || s->chain > 2 || p->grid_res < 1 || !(p->cover_frac >= 0.0)) return nullptr;
  if (s->chain == 2 && (!s->pos2 || !s->nrm2 || s->n_tri2 < 1)) return nullptr;
  if (s->eedge && s->chain != 0) return nullptr;  // area lights: one reflection only
  return build_all(s, p, n_threads);
}

void orc_free(void* h) { delete static_cast<Build*>(h); }

int64_t orc_n_leaves(const void* h) { return int64_t(static_cast<const Build*>(h)->leaves.size()); }

int orc_get_leaves(const void* h, int64_t* tuple, int32_t* code, double* box, double* ukbox, double* E) {
  const Build* B = static_cast<const Build*>(h);
  for (size_t i = 0; i < B->leaves.size(); ++i) {
    const Leaf& l = B->leaves[i];
    if (tuple) tuple[i] = l.tuple;
    if (code) {
      code[3 * i] = l.depth;
      code[3 * i + 1] = int32_t(l.iu);
      code[3 * i + 2] = int32_t(l.iv);
    }
    for (int k = 0; k < 4; ++k) {
      if (box) box[4 * i + k] = l.box[k];
      if (ukbox) ukbox[4 * i + k] = l.uk[k];
    }
    if (E) {
      E[2 * i] = l.E[0];
      E[2 * i + 1] = l.E[1];
    }
  }
  return 0;
}

int64_t orc_n_roots(const void* h) { return int64_t(static_cast<const Build*>(h)->roots.size()); }

int orc_get_roots(const void* h, int64_t* tuple, double* box) {
  const Build* B = static_cast<const Build*>(h);
  for (size_t i = 0; i < B->roots.size(); ++i) {
    tuple[i] = B->roots[i].tuple;
    for (int k = 0; k < 4; ++k) box[4 * i + k] = B->roots[i].box[k];
  }
  return 0;
}

int orc_build_stats(const void* h, double* st) {
  const Build* B = static_cast<const Build*>(h);
  int64_t entries = 0, inf = 0, uni = 0, maxl = 0;
  for (const auto& m : B->cells) entries += int64_t(m.size());
  entries += int64_t(B->cover.size());
  for (const Leaf& l : B->leaves) {
    inf += std::isinf(l.E[1]) ? 1 : 0;
    uni += l.universal ? 1 : 0;
  }
  for (int64_t t = 0; t < B->n_tuples; ++t) maxl = std::max(maxl, B->leaf_begin[t + 1] - B->leaf_begin[t]);
  st[0] = double(B->n_tuples);
  st[1] = double(B->roots.size());
  st[2] = double(B->boxes);
  st[3] = double(B->leaves.size());
  st[4] = double(entries);
  st[5] = double(inf);
  st[6] = double(uni);
  st[7] = double(maxl);
  st[8] = double(B->cover.size());
  return 0;
}

int64_t orc_cover_list(const void* h, int64_t* tuples, double* Et, int64_t cap) {
  const Build* B = static_cast<const Build*>(h);
  if (!B) return -1;
  int64_t k = 0;
  for (const auto& kv : B->cover) {
    if (k < cap) {
      tuples[k] = kv.first;
      Et[k] = kv.second;
    }
    ++k;
  }
  return k;
}

int64_t orc_cell_list(const void* h, int32_t cu, int32_t cv, int64_t* tuples, double* Et, int64_t cap) {
  const Build* B = static_cast<const Build*>(h);
  const int G = B->p.grid_res;
  if (cu < 0 || cv < 0 || cu >= G || cv >= G) return -1;
  const auto& m = B->cells[size_t(cu) * G + cv];
  int64_t k = 0;
  for (const auto& kv : m) {
    if (k < cap) {
      tuples[k] = kv.first;
      Et[k] = kv.second;
    }
    ++k;
  }
  return k;
}

int orc_query(const void* h, const double* pts, int64_t n, double W, uint64_t seed, int mode, double* E_out,
              double* stats, int n_threads) {
  const Build* B = static_cast<const Build*>(h);
  if (!B || !pts || !E_out || n < 0 || !(W >= 1.0) || mode < 0 || mode > 15) return -1;
  const int G = B->p.grid_res;
  const bool exhaustive = (mode & 1) != 0, brute = (mode & 2) != 0;
  const int sampler = (mode >> 2) & 3;  // 0 Alg. 1 with the bound-optimal P, 1 uniform, 2 one-sample, 3 bins
  if (exhaustive && sampler != 0) return -1;
  const Tuple ref = make_tuple(B->scene, 0);
  parallel_for(n, n_threads, [&](int64_t i, int) {
    const V3 x = v3(pts[i], pts[n + i], pts[2 * n + i]);
    double us, vs;
    double* st = stats ? stats + 4 * i : nullptr;
    if (st) st[0] = st[1] = st[2] = st[3] = 0.0;
    E_out[i] = 0.0;
    if (!receiver_coords(ref, x, &us, &vs)) return;
    // U: the cell's list, then the cover-all list (each ascending by tuple)
    const auto& m = B->cells[size_t(cell_of(us, G)) * G + cell_of(vs, G)];
    std::vector<int64_t> U;
    std::vector<double> Et;
    for (const auto& kv : m) {
      U.push_back(kv.first);
      Et.push_back(kv.second);
    }
    for (const auto& kv : B->cover) {
      U.push_back(kv.first);
      Et.push_back(kv.second);
    }
    std::vector<double> P(U.size(), 1.0);
    if (!exhaustive) probabilities(Et.data(), int64_t(U.size()), W, P.data());
    std::vector<Pick> S;
    double mu2 = 0.0;
    if (sampler == 1) {
      S = pick_uniform(U.size(), W, seed, uint64_t(i), U.data());
    } else if (sampler == 2) {
      S = pick_one_sample(Et, int(W), seed, uint64_t(i));
    } else if (sampler == 3) {
      S = pick_bins(P, seed, uint64_t(i));
      for (size_t k = 0; k < U.size(); ++k)
        if (P[k] > 0.0) mu2 += Et[k] * Et[k] / P[k];
    } else {
      for (size_t k = 0; k < U.size(); ++k) {
        if (P[k] > 0.0) mu2 += Et[k] * Et[k] / P[k];
        const double r = uniform(seed, uint64_t(i), uint32_t(U[k]));
        if (r < P[k]) S.push_back({k, P[k]});
      }
    }
    double E = 0.0;
    int64_t nroots = 0;
    for (const Pick& pk : S) {
      const size_t k = pk.k;
      Tuple c = make_tuple(B->scene, U[k]);
      if (c.area)  // one light point per selected pair, from streams 3 and 4
        c = at_light_point(c, uniform_stream(seed, uint64_t(i), uint32_t(U[k]), 3u),
                           uniform_stream(seed, uint64_t(i), uint32_t(U[k]), 4u));
      const std::vector<RootHit> roots = brute ? brute_roots(c, us, vs, 64) : leaf_roots(*B, c, U[k], us, vs);
      double ET = 0.0;
      for (const RootHit& rh : roots) ET += rh.Ek;
      nroots += int64_t(roots.size());
      E += sampler == 0 ? ET / P[k] : ET / pk.P;
    }
    E_out[i] = E;
    if (st) {
      st[0] = double(U.size());
      st[1] = double(S.size());
      st[2] = double(nroots);
      st[3] = mu2;
    }
  });
  return 0;
}

int orc_true_irradiance(const orc_scene* s, const double* pts, int64_t n, int lattice, double* E_out,
                        int n_threads) {
  if (!s || !pts || !E_out || n < 0 || lattice < 1 || s->eedge) return -1;
  const int64_t T = n_tuples_of(s);
  const Tuple ref = make_tuple(s, 0);
  parallel_for(n, n_threads, [&](int64_t i, int) {
    const V3 x = v3(pts[i], pts[n + i], pts[2 * n + i]);
    double us, vs;
    E_out[i] = 0.0;
    if (!receiver_coords(ref, x, &us, &vs)) return;
    double E = 0.0;
    for (int64_t t = 0; t < T; ++t) {
      const Tuple c = make_tuple(s, t);
      for (const RootHit& r : brute_roots(c, us, vs, lattice)) E += r.Ek;
    }
    E_out[i] = E;
  });
  return 0;
}

int64_t orc_pair_list(const orc_scene* s, int64_t emitter, int64_t t1, int64_t* t2_out, int64_t cap) {
  if (!s || s->chain != 2 || emitter < 0 || emitter >= s->n_emit || t1 < 0 || t1 >= s->n_tri) return -1;
  int64_t k = 0;
  for (int64_t t2 = 0; t2 < s->n_tri2; ++t2) {
    const Tuple c = make_tuple(s, (emitter * s->n_tri + t1) * s->n_tri2 + t2);
    if (!c.front || !pair_candidate(c)) continue;
    if (k < cap) t2_out[k] = t2;
    ++k;
  }
  return k;
}

int64_t orc_tuple_roots(const orc_scene* s, int64_t tuple, const double* x, int lattice, double* roots,
                        int64_t cap) {
  if (!s || !x || tuple < 0 || tuple >= n_tuples_of(s)) return -1;
  const Tuple c = make_tuple(s, tuple);
  double us, vs;
  if (!receiver_coords(c, v3(x[0], x[1], x[2]), &us, &vs)) return 0;
  const auto r = brute_roots(c, us, vs, lattice);
  for (int64_t k = 0; k < int64_t(r.size()) && k < cap; ++k) {
    roots[4 * k] = r[k].u;
    roots[4 * k + 1] = r[k].v;
    roots[4 * k + 2] = r[k].Ek;
    roots[4 * k + 3] = r[k].res;
  }
  return int64_t(r.size());
}

int64_t orc_tuple_roots_leaves(const void* h, int64_t tuple, const double* x, double* roots, int64_t cap) {
  const Build* B = static_cast<const Build*>(h);
  if (!B || !x || tuple < 0 || tuple >= B->n_tuples) return -1;
  const Tuple c = make_tuple(B->scene, tuple);
  double us, vs;
  if (!receiver_coords(c, v3(x[0], x[1], x[2]), &us, &vs)) return 0;
  const auto r = leaf_roots(*B, c, tuple, us, vs);
  for (int64_t k = 0; k < int64_t(r.size()) && k < cap; ++k) {
    roots[4 * k] = r[k].u;
    roots[4 * k + 1] = r[k].v;
    roots[4 * k + 2] = r[k].Ek;
    roots[4 * k + 3] = r[k].res;
  }
  return int64_t(r.size());
}

int orc_probabilities(const double* Et, int64_t n, double W, double* P) {
  if ((!Et && n) || (!P && n) || n < 0 || !(W >= 1.0)) return -1;
  probabilities(Et, n, W, P);
  return 0;
}

int64_t orc_sample(const double* Et, const int64_t* U, int64_t n, double W, uint64_t seed, uint64_t point,
                   int sampler, int64_t* k_out, double* P_out, int64_t cap) {
  if ((!Et && n) || (!U && n) || n < 0 || !(W >= 1.0) || sampler < 0 || sampler > 3) return -1;
  std::vector<double> E(Et, Et + n), P(size_t(n), 1.0);
  probabilities(E.data(), n, W, P.data());
  std::vector<Pick> S;
  if (sampler == 1) {
    S = pick_uniform(size_t(n), W, seed, point, U);
  } else if (sampler == 2) {
    S = pick_one_sample(E, int(W), seed, point);
  } else if (sampler == 3) {
    S = pick_bins(P, seed, point);
  } else {
    for (int64_t k = 0; k < n; ++k)
      if (uniform(seed, point, uint32_t(U[k])) < P[size_t(k)]) S.push_back({size_t(k), P[size_t(k)]});
  }
  for (size_t j = 0; j < S.size() && int64_t(j) < cap; ++j) {
    k_out[j] = int64_t(S[j].k);
    P_out[j] = S[j].P;
  }
  return int64_t(S.size());
}

double orc_sample_margin(const double* Et, const int64_t* U, int64_t n, double W, uint64_t seed, uint64_t point,
                         int sampler) {
  if ((!Et && n) || (!U && n) || n < 0 || !(W >= 1.0) || sampler < 0 || sampler > 3) return -1.0;
  return sample_margin(std::vector<double>(Et, Et + n), U, W, seed, point, sampler);
}

void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox(ctr, key, out); }

double orc_uniform(uint64_t seed, uint64_t point, uint32_t tuple) { return uniform(seed, point, tuple); }

static Bern from_flat(const int32_t* d, const double* a) {
  Bern b(Deg{d[0], d[1], d[2], d[3]});
  for (size_t i = 0; i < b.size(); ++i) b.c[i] = a[i];
  return b;
}
static void to_flat(const Bern& b, double* out) {
  for (size_t i = 0; i < b.size(); ++i) out[i] = b.c[i];
}

int orc_bern_mul(const int32_t* da, const double* a, const int32_t* db, const double* b, double* out) {
  to_flat(mul(from_flat(da, a), from_flat(db, b)), out);
  return 0;
}
int orc_bern_elevate(const int32_t* da, const double* a, const int32_t* dto, double* out) {
  to_flat(elevate(from_flat(da, a), Deg{dto[0], dto[1], dto[2], dto[3]}), out);
  return 0;
}
int orc_bern_deriv(const int32_t* da, const double* a, int axis, double* out) {
  to_flat(deriv(from_flat(da, a), axis), out);
  return 0;
}
int orc_bern_split(const int32_t* da, const double* a, int axis, double t, double* left, double* right) {
  Bern l, r;
  split(from_flat(da, a), axis, t, &l, &r);
  to_flat(l, left);
  to_flat(r, right);
  return 0;
}
int orc_bern_reduce(const int32_t* da, const double* a, const int32_t* dto, double* out, double* rem) {
  const Deg to{dto[0], dto[1], dto[2], dto[3]};
  for (int k = 0; k < kAxes; ++k)
    if (to[k] < 0 || to[k] > da[k]) return -1;
  to_flat(reduce_degree(from_flat(da, a), to, rem), out);
  return 0;
}
double orc_bern_eval(const int32_t* da, const double* a, const double* x) {
  return eval(from_flat(da, a), {x[0], x[1], x[2], x[3]});
}
int orc_ratio_bound(const int32_t* dp, const double* p, const int32_t* dq, const double* q, double* out) {
  const RatioBound rb = ratio_bound(from_flat(dp, p), from_flat(dq, q));
  out[0] = rb.kind;
  out[1] = rb.lo;
  out[2] = rb.hi;
  return 0;
}
int orc_sqrt_secant(double blo, double bhi, double* out) {
  if (!(blo > 0.0) || !(bhi >= blo)) return -1;
  sqrt_secant(blo, bhi, &out[0], &out[1], &out[2], &out[3]);
  return 0;
}

}  // extern "C"
