// FP64 Bernstein toolkit of the oracle (test infrastructure only; see bern.hpp).
#include "bern.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <stdexcept>
#include <vector>

namespace orc {

double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return std::round(r);
}

static size_t count_of(const Deg& d) {
  size_t n = 1;
  for (int a = 0; a < kAxes; ++a) n *= size_t(d[a] + 1);
  return n;
}

Bern::Bern(const Deg& d, double fill) : deg(d), c(count_of(d), fill) {}

Bern Bern::constant(double v) {
  Bern b;
  b.c[0] = v;
  return b;
}

size_t Bern::index(const std::array<int, kAxes>& i) const {
  size_t f = 0;
  for (int a = 0; a < kAxes; ++a) f = f * size_t(deg[a] + 1) + size_t(i[a]);
  return f;
}

std::array<int, kAxes> Bern::multi(size_t flat) const {
  std::array<int, kAxes> i{};
  for (int a = kAxes - 1; a >= 0; --a) {
    i[a] = int(flat % size_t(deg[a] + 1));
    flat /= size_t(deg[a] + 1);
  }
  return i;
}

Bern linear_on_box(double a, double b, double c, double u0, double u1, double v0, double v1) {
  Bern r(Deg{1, 1, 0, 0});
  const double us[2] = {u0, u1}, vs[2] = {v0, v1};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.at({i, j, 0, 0}) = a + b * us[i] + c * vs[j];
  return r;
}

Bern affine_axis(int axis, double lo, double hi) {
  Deg d{0, 0, 0, 0};
  d[axis] = 1;
  Bern r(d);
  std::array<int, kAxes> i{0, 0, 0, 0};
  r.at(i) = lo;
  i[axis] = 1;
  r.at(i) = hi;
  return r;
}

// Product of two Bernstein polynomials: the coefficient of B_{k,m+n} collects
// a_i b_j C(m,i) C(n,j) / C(m+n,k) over i + j = k, axis by axis.
Bern mul(const Bern& A, const Bern& B) {
  Deg d;
  for (int a = 0; a < kAxes; ++a) d[a] = A.deg[a] + B.deg[a];
  Bern C(d);
  // the binomials and multi-indices the sum below uses, tabulated once per
  // call (the same values binom() returns, in the same order of operations)
  std::array<std::vector<double>, kAxes> bA, bB, bC;
  for (int a = 0; a < kAxes; ++a) {
    for (int i = 0; i <= A.deg[a]; ++i) bA[a].push_back(binom(A.deg[a], i));
    for (int i = 0; i <= B.deg[a]; ++i) bB[a].push_back(binom(B.deg[a], i));
    for (int i = 0; i <= d[a]; ++i) bC[a].push_back(binom(d[a], i));
  }
  std::vector<std::array<int, kAxes>> MB(B.size());
  for (size_t ib = 0; ib < B.size(); ++ib) MB[ib] = B.multi(ib);
  for (size_t ia = 0; ia < A.size(); ++ia) {
    const auto mi = A.multi(ia);
    for (size_t ib = 0; ib < B.size(); ++ib) {
      const auto& mj = MB[ib];
      std::array<int, kAxes> mk;
      double w = 1.0;
      for (int a = 0; a < kAxes; ++a) {
        mk[a] = mi[a] + mj[a];
        w *= bA[a][size_t(mi[a])] * bB[a][size_t(mj[a])] / bC[a][size_t(mk[a])];
      }
      C.at(mk) += w * A.c[ia] * B.c[ib];
    }
  }
  return C;
}

// Raise the degree along one axis by one: b'_i = (i/(n+1)) b_{i-1} + (1 - i/(n+1)) b_i.
static Bern elevate_once(const Bern& A, int axis) {
  Deg d = A.deg;
  d[axis] += 1;
  Bern R(d);
  const int n = A.deg[axis];
  for (size_t f = 0; f < R.size(); ++f) {
    auto mi = R.multi(f);
    const int i = mi[axis];
    double v = 0.0;
    if (i >= 1) {
      auto mp = mi;
      mp[axis] = i - 1;
      v += double(i) / double(n + 1) * A.at(mp);
    }
    if (i <= n) v += (1.0 - double(i) / double(n + 1)) * A.at(mi);
    R.c[f] = v;
  }
  return R;
}

Bern elevate(const Bern& A, const Deg& to) {
  Bern R = A;
  for (int a = 0; a < kAxes; ++a) {
    if (to[a] < R.deg[a]) throw std::invalid_argument("elevate: target degree below current");
    while (R.deg[a] < to[a]) R = elevate_once(R, a);
  }
  return R;
}

static Deg max_deg(const Deg& a, const Deg& b) {
  Deg d;
  for (int k = 0; k < kAxes; ++k) d[k] = std::max(a[k], b[k]);
  return d;
}

Bern add(const Bern& A, const Bern& B) {
  const Deg d = max_deg(A.deg, B.deg);
  Bern X = elevate(A, d), Y = elevate(B, d);
  for (size_t f = 0; f < X.size(); ++f) X.c[f] += Y.c[f];
  return X;
}

Bern sub(const Bern& A, const Bern& B) { return add(A, scale(B, -1.0)); }

Bern scale(const Bern& A, double s) {
  Bern R = A;
  for (double& v : R.c) v *= s;
  return R;
}

// d/dx of sum b_i B_{i,n}(x) = n * sum (b_{i+1} - b_i) B_{i,n-1}(x).
Bern deriv(const Bern& A, int axis) {
  const int n = A.deg[axis];
  if (n == 0) {
    Deg d = A.deg;
    return Bern(d, 0.0);
  }
  Deg d = A.deg;
  d[axis] = n - 1;
  Bern R(d);
  for (size_t f = 0; f < R.size(); ++f) {
    auto mi = R.multi(f);
    auto mp = mi;
    mp[axis] += 1;
    R.c[f] = double(n) * (A.at(mp) - A.at(mi));
  }
  return R;
}

// de Casteljau subdivision at x_axis = t: the left piece re-parameterises
// [0, t] to [0, 1], the right piece [t, 1].
void split(const Bern& A, int axis, double t, Bern* left, Bern* right) {
  const int n = A.deg[axis];
  *left = Bern(A.deg);
  *right = Bern(A.deg);
  // iterate over every line of coefficients along `axis`
  Deg line_deg = A.deg;
  line_deg[axis] = 0;
  Bern lines(line_deg);
  for (size_t f = 0; f < lines.size(); ++f) {
    auto base = lines.multi(f);
    std::vector<double> w(n + 1);
    for (int i = 0; i <= n; ++i) {
      auto mi = base;
      mi[axis] = i;
      w[i] = A.at(mi);
    }
    for (int r = 0; r <= n; ++r) {
      auto ml = base, mr = base;
      ml[axis] = r;
      mr[axis] = n - r;
      left->at(ml) = w[0];
      right->at(mr) = w[n - r];
      for (int i = 0; i < n - r; ++i) w[i] = (1.0 - t) * w[i] + t * w[i + 1];
    }
  }
}

// Elevation matrix of one axis from degree m to degree n >= m:
// b'_i = sum_j E_ij b_j with E_ij = C(n-m, i-j) C(m, j) / C(n, i).
static std::vector<double> elevation_matrix(int m, int n) {
  std::vector<double> E(size_t(n + 1) * size_t(m + 1), 0.0);
  for (int i = 0; i <= n; ++i)
    for (int j = 0; j <= m; ++j)
      if (i - j >= 0 && i - j <= n - m) E[size_t(i) * (m + 1) + j] = binom(n - m, i - j) * binom(m, j) / binom(n, i);
  return E;
}

// Pseudo-inverse (m+1) x (n+1) of the (n+1) x (m+1) elevation matrix by its
// singular-value decomposition E = U S V^T (one-sided Jacobi: plane rotations
// of the columns until they are mutually orthogonal), E+ = V S^-1 U^T.
static std::vector<double> elevation_pinv(int m, int n) {
  const int R = n + 1, C = m + 1;
  std::vector<double> W = elevation_matrix(m, n), V(size_t(C) * C, 0.0);
  for (int j = 0; j < C; ++j) V[size_t(j) * C + j] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < C; ++p)
      for (int q = p + 1; q < C; ++q) {
        double a = 0, b = 0, g = 0;
        for (int i = 0; i < R; ++i) {
          const double wp = W[size_t(i) * C + p], wq = W[size_t(i) * C + q];
          a += wp * wp;
          b += wq * wq;
          g += wp * wq;
        }
        if (std::fabs(g) <= 1e-15 * std::sqrt(a * b)) continue;
        off = std::max(off, std::fabs(g) / std::sqrt(a * b));
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < R; ++i) {
          const double wp = W[size_t(i) * C + p], wq = W[size_t(i) * C + q];
          W[size_t(i) * C + p] = cs * wp - sn * wq;
          W[size_t(i) * C + q] = sn * wp + cs * wq;
        }
        for (int i = 0; i < C; ++i) {
          const double vp = V[size_t(i) * C + p], vq = V[size_t(i) * C + q];
          V[size_t(i) * C + p] = cs * vp - sn * vq;
          V[size_t(i) * C + q] = sn * vp + cs * vq;
        }
      }
    if (off < 1e-15) break;
  }
  // W = U S: column j has norm s_j; E+ = V S^-1 U^T = V S^-2 W^T
  std::vector<double> P(size_t(C) * R, 0.0);
  for (int j = 0; j < C; ++j) {
    double s2 = 0;
    for (int i = 0; i < R; ++i) s2 += W[size_t(i) * C + j] * W[size_t(i) * C + j];
    for (int r = 0; r < C; ++r)
      for (int i = 0; i < R; ++i) P[size_t(r) * R + i] += V[size_t(r) * C + j] * W[size_t(i) * C + j] / s2;
  }
  return P;
}

Bern reduce_degree(const Bern& A, const Deg& to, double* rem) {
  Bern X = A;
  for (int ax = 0; ax < kAxes; ++ax) {
    if (to[ax] > A.deg[ax]) throw std::invalid_argument("reduce_degree: target degree above current");
    if (to[ax] == A.deg[ax]) continue;
    const int n = X.deg[ax], m = to[ax];
    const std::vector<double> P = elevation_pinv(m, n);
    Deg d = X.deg;
    d[ax] = m;
    Bern Y(d);
    for (size_t f = 0; f < Y.size(); ++f) {
      auto mi = Y.multi(f);
      const int r = mi[ax];
      double v = 0.0;
      for (int i = 0; i <= n; ++i) {
        auto mx = mi;
        mx[ax] = i;
        v += P[size_t(r) * (n + 1) + i] * X.at(mx);
      }
      Y.c[f] = v;
    }
    X = Y;
  }
  const Bern back = elevate(X, A.deg);
  double r = 0.0;
  for (size_t f = 0; f < A.size(); ++f) r = std::max(r, std::fabs(A.c[f] - back.c[f]));
  *rem = r;
  return X;
}

double eval(const Bern& A, const std::array<double, kAxes>& x) {
  double s = 0.0;
  for (size_t f = 0; f < A.size(); ++f) {
    const auto mi = A.multi(f);
    double b = 1.0;
    for (int a = 0; a < kAxes; ++a) {
      const int n = A.deg[a], i = mi[a];
      b *= binom(n, i) * std::pow(x[a], i) * std::pow(1.0 - x[a], n - i);
    }
    s += A.c[f] * b;
  }
  return s;
}

void coef_range(const Bern& A, double* lo, double* hi) {
  *lo = *std::min_element(A.c.begin(), A.c.end());
  *hi = *std::max_element(A.c.begin(), A.c.end());
}

static int strict_sign(const Bern& A) {
  bool pos = true, neg = true;
  for (double v : A.c) {
    if (!(v > 0.0)) pos = false;
    if (!(v < 0.0)) neg = false;
  }
  return pos ? 1 : (neg ? -1 : 0);
}

static void direct_ratio(const Bern& P, const Bern& Q, double* lo, double* hi) {
  *lo = std::numeric_limits<double>::infinity();
  *hi = -std::numeric_limits<double>::infinity();
  for (size_t f = 0; f < P.size(); ++f) {
    const double r = P.c[f] / Q.c[f];
    *lo = std::min(*lo, r);
    *hi = std::max(*hi, r);
  }
}

RatioBound ratio_bound(const Bern& P0, const Bern& Q0) {
  const Deg d = max_deg(P0.deg, Q0.deg);
  const Bern P = elevate(P0, d), Q = elevate(Q0, d);
  RatioBound rb;
  if (strict_sign(Q) != 0) {
    rb.kind = kDirect;
    direct_ratio(P, Q, &rb.lo, &rb.hi);
    return rb;
  }
  if (strict_sign(P) != 0) {
    double a, b;  // q/p in [a, b]; invert
    direct_ratio(Q, P, &a, &b);
    const double inf = std::numeric_limits<double>::infinity();
    if (a > 0.0 || b < 0.0) {
      rb.kind = kDirect;
      rb.lo = 1.0 / b;
      rb.hi = 1.0 / a;
    } else if (a < 0.0 && b > 0.0) {
      rb.kind = kSplit;
      rb.lo = 1.0 / a;
      rb.hi = 1.0 / b;
    } else if (a == 0.0 && b > 0.0) {
      rb.kind = kDirect;
      rb.lo = 1.0 / b;
      rb.hi = inf;
    } else if (b == 0.0 && a < 0.0) {
      rb.kind = kDirect;
      rb.lo = -inf;
      rb.hi = 1.0 / a;
    } else {
      rb.kind = kUnbounded;
    }
    return rb;
  }
  rb.kind = kUnbounded;
  return rb;
}

}  // namespace orc
