// FP64 tensor-product Bernstein toolkit of the oracle.
//
// TEST INFRASTRUCTURE ONLY: the oracle is the plain, slow, obviously correct CPU
// definition that the GPU library is checked against.  Only the tests, the
// smoke check and the CPU-baseline leg of the benchmark may load it; the
// product path never does.  It shares no code with the HIP library.
//
// A polynomial over the unit box [0,1]^4 (unused axes have degree 0) is held
// by its Bernstein coefficients b_i, p(x) = sum_i b_i B_{i,n}(x), with
// B_{i,n}(x) = prod_j C(n_j,i_j) x_j^{i_j} (1-x_j)^{n_j-i_j}  (Sec. 4.1, Eq. 1).
#pragma once
#include <array>
#include <cstddef>
#include <vector>

namespace orc {

constexpr int kAxes = 4;
using Deg = std::array<int, kAxes>;

double binom(int n, int k);

struct Bern {
  Deg deg{0, 0, 0, 0};
  std::vector<double> c;  // row-major, axis 0 slowest

  Bern() : c(1, 0.0) {}
  explicit Bern(const Deg& d, double fill = 0.0);
  static Bern constant(double v);
  size_t size() const { return c.size(); }
  size_t index(const std::array<int, kAxes>& i) const;
  std::array<int, kAxes> multi(size_t flat) const;
  double& at(const std::array<int, kAxes>& i) { return c[index(i)]; }
  double at(const std::array<int, kAxes>& i) const { return c[index(i)]; }
};

// Linear form a + b*u + c*v restricted to the box [u0,u1] x [v0,v1] of the
// (u, v) plane, in local coordinates (s, t) in [0,1]^2 of that box: its
// degree-(1,1) coefficients are the values at the four box corners.
Bern linear_on_box(double a, double b, double c, double u0, double u1, double v0, double v1);
// An affine function of one local axis: lo + (hi - lo) * x_axis.
Bern affine_axis(int axis, double lo, double hi);

Bern mul(const Bern& A, const Bern& B);            // product (degrees add)
Bern elevate(const Bern& A, const Deg& to);        // degree elevation to `to` (>= A.deg)
Bern add(const Bern& A, const Bern& B);            // sum at the common (max) degree
Bern sub(const Bern& A, const Bern& B);
Bern scale(const Bern& A, double s);
Bern deriv(const Bern& A, int axis);               // d/dx_axis in local coordinates
void split(const Bern& A, int axis, double t, Bern* left, Bern* right);  // de Casteljau
double eval(const Bern& A, const std::array<double, kAxes>& x);         // sum b_i B_i(x)
void coef_range(const Bern& A, double* lo, double* hi);                 // min/max coefficient

// Degree reduction (Sec. 6.1, "Degree reduction"): the polynomial of degree
// `to` whose degree-elevated coefficients are closest to A's in the least-
// squares sense (a linear regression solved through the singular-value
// decomposition of the elevation matrix of each reduced axis), and in *rem
// the largest coefficient of the difference at A's degree, which bounds
// |A - reduced| everywhere on the box (convex hull of the Bernstein
// coefficients): A = reduced + xi * rem for some xi in [-1, 1].
Bern reduce_degree(const Bern& A, const Deg& to, double* rem);

// Range bound of p/q from coefficient ratios (Sec. 4.1, Eq. eq_bbound) with the
// sign-failure rules of the same section: when q's coefficients are not all of
// one strict sign, bound q/p instead and invert (possibly two intervals); when
// both fail the bound is the whole real line.
enum BoundKind { kDirect = 0, kSplit = 1, kUnbounded = 2 };
struct RatioBound {
  int kind = kUnbounded;
  double lo = 0, hi = 0;  // kDirect: [lo, hi];  kSplit: (-inf, lo] U [hi, +inf)
};
RatioBound ratio_bound(const Bern& P, const Bern& Q);

}  // namespace orc
