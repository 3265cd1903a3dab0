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

}  // namespace arr
