// Polynomial accelerator of Sec. 5: psi_d is the degree-d polynomial that
// interpolates f_d(t) = max(0, t)^(10 d) (eq. def:fN) at the d+1 Chebyshev
// points of the second kind t_j = -cos(j pi / d).
//
// The points are the Chebyshev-Lobatto nodes x_j = cos(j pi / d) (same set),
// so the interpolant's Chebyshev coefficients follow from the discrete
// orthogonality of T_k on those nodes:
//   c_k = (2/d) sum''_j f(x_j) T_k(x_j),  with T_k(x_j) = cos(k j pi / d),
// where the double prime halves the j = 0 and j = d terms, and c_0, c_d are
// halved as well. The monomial coefficients Gamma_d of eq. chebfun-f follow by
// expanding T_k with T_{k+1} = 2 t T_k - T_{k-1}.
//
// Product form: psi_d has d real simple roots in [-1, 1). It vanishes at the
// nodes t_j <= 0 (f_d is zero there), and each other root lies next to a
// positive node t_j < 1, where f_d is tiny. So psi_d(t) = lead prod (t - r_i),
// with lead = 2^(d-1) c_d the leading monomial coefficient. The roots are
// the nonpositive nodes, exactly, and Newton iterates with Maehly's deflation
// started at the positive nodes, on the Chebyshev series in long double. They
// are returned in Leja order (each next root maximizes the product of its
// distances to the earlier ones), which keeps partial products well scaled.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace arr {

std::vector<double> filter_chebyshev_coefficients(int d) {
  ARR_REQUIRE(d >= 1 && d <= 64, "filter degree must be in [1, 64]");
  const double pi = 3.14159265358979323846;
  std::vector<double> f(d + 1), c(d + 1);
  for (int j = 0; j <= d; ++j) {
    const double x = std::cos(j * pi / d);
    f[j] = x > 0.0 ? std::pow(x, 10.0 * d) : 0.0;
  }
  for (int k = 0; k <= d; ++k) {
    double s = 0.0;
    for (int j = 0; j <= d; ++j) {
      const double wj = (j == 0 || j == d) ? 0.5 : 1.0;
      s += wj * f[j] * std::cos((double)k * j * pi / d);
    }
    c[k] = (2.0 / d) * s;
  }
  c[0] *= 0.5;
  c[d] *= 0.5;
  return c;
}

std::vector<double> filter_coefficients(int d) {
  const std::vector<double> c = filter_chebyshev_coefficients(d);
  // ascending-power coefficients of T_{k-1}, T_k
  std::vector<double> tm(d + 1, 0.0), tk(d + 1, 0.0), acc(d + 1, 0.0);
  tm[0] = 1.0;  // T_0
  acc[0] += c[0];
  if (d >= 1) {
    tk[1] = 1.0;  // T_1
    acc[1] += c[1];
  }
  for (int k = 1; k < d; ++k) {
    std::vector<double> tn(d + 1, 0.0);
    for (int p = 0; p < d; ++p) tn[p + 1] += 2.0 * tk[p];
    for (int p = 0; p <= d; ++p) tn[p] -= tm[p];
    for (int p = 0; p <= d; ++p) acc[p] += c[k + 1] * tn[p];
    tm = tk;
    tk = tn;
  }
  std::vector<double> g(d + 1);
  for (int i = 0; i <= d; ++i) g[i] = acc[d - i];  // leading coefficient first
  return g;
}

FilterPoly filter_poly(int d) {
  FilterPoly fp;
  fp.gamma = filter_coefficients(d);
  const std::vector<double> c = filter_chebyshev_coefficients(d);
  typedef long double R;
  auto eval = [&](R t, R &p, R &dp) {
    // T_k and T_k' by the three-term recurrences
    R t0 = 1, t1 = t, d0 = 0, d1 = 1;
    p = c[0] * t0 + (d >= 1 ? c[1] * t1 : 0);
    dp = (d >= 1 ? c[1] * d1 : 0);
    for (int k = 1; k < d; ++k) {
      const R t2 = 2 * t * t1 - t0, d2 = 2 * t1 + 2 * t * d1 - d0;
      p += c[k + 1] * t2;
      dp += c[k + 1] * d2;
      t0 = t1, t1 = t2, d0 = d1, d1 = d2;
    }
  };
  const R pi = 3.141592653589793238462643383279502884L;
  std::vector<R> roots;
  for (int j = 0; j < d; ++j) {
    const R x = -std::cos((R)j * pi / d);
    if (x <= 0) {
      roots.push_back(x);
      continue;
    }
    R t = x;
    for (int it = 0; it < 200; ++it) {
      R p, dp;
      eval(t, p, dp);
      R sdef = 0;
      for (R r : roots) sdef += 1 / (t - r);
      const R den = dp - p * sdef;
      if (den == 0) break;
      const R step = p / den;
      t -= step;
      if (std::fabs(step) <= 1e-30L * std::max((R)1, std::fabs(t))) break;
    }
    roots.push_back(t);
  }
  // Leja order
  std::vector<R> left = roots, ord;
  while (!left.empty()) {
    size_t best = 0;
    R bv = -1;
    for (size_t i = 0; i < left.size(); ++i) {
      R v = 1;
      if (ord.empty())
        v = std::fabs(left[i]);
      else
        for (R r : ord) v *= std::fabs(left[i] - r);
      if (v > bv) bv = v, best = i;
    }
    ord.push_back(left[best]);
    left.erase(left.begin() + best);
  }
  fp.roots.assign(ord.begin(), ord.end());
  fp.lead = std::ldexp(c[d], d - 1);
  // check: the product form reproduces the Chebyshev series at the nodes and at 1.1
  for (int j = 0; j <= d + 1; ++j) {
    const R t = j <= d ? -std::cos((R)j * pi / d) : (R)1.1;
    R p, dp, q = fp.lead;
    eval(t, p, dp);
    for (R r : ord) q *= (t - r);
    ARR_REQUIRE(std::fabs((double)(q - p)) <= 1e-9 * std::max(1.0, std::fabs((double)p)),
                "filter roots do not reproduce the interpolant");
  }
  return fp;
}

}  // namespace arr
