// Sinc quadrature of Bonito and Pasciak (the comparison method of Section 5.3)
// as a partial-fraction form for the shifted-solve engine.  Host code only.
//
// The rule approximates B^-alpha for an SPD B by
//   (2 k' sin(pi alpha)/pi) sum_{l=-m}^{M} exp(2(alpha-1) l k') (exp(-2 l k') I + B)^-1,
//   m = ceil(pi^2/(4 alpha k'^2)),  M = ceil(pi^2/(4 (1-alpha) k'^2)).
// With B = scale * A it becomes sum_l w_l (A + s_l I)^-1 after dividing each
// system by scale; multiplying by scale^alpha makes it an approximation of
// A^-alpha itself:  w_l = scale^(alpha-1) (2k' sin(pi alpha)/pi) exp(2(alpha-1) l k'),
// s_l = exp(-2 l k') / scale.
#include <cmath>

#include "../../include/bura.h"

namespace {

// ceil(x), except that a value within 1e-9 (relative) of an integer counts as
// that integer: with k' derived from an integer k_Q the arguments are exact
// rationals such as 4 = (1 - 0.5) * 8, which rounding may push just above.
long long ceil_reading(long double x) {
  const long double r = std::nearbyint(x);
  if (std::fabs(x - r) <= 1e-9L * std::fabs(x)) return (long long)r;
  return (long long)std::ceil(x);
}

}  // namespace

extern "C" int bura_sinc_coefficients(double alpha, double kprime, double scale, int max_terms, double* weights,
                                      double* shifts, int* nterms) {
  if (!(alpha > 0.0 && alpha < 1.0) || !(kprime > 0.0) || !std::isfinite(kprime) || !(scale > 0.0) ||
      !std::isfinite(scale) || !nterms)
    return BURA_EINVAL;
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double a = alpha, kp = kprime, sc = scale;
  const long long m = ceil_reading(pi * pi / (4.0L * a * kp * kp));
  const long long M = ceil_reading(pi * pi / (4.0L * (1.0L - a) * kp * kp));
  const long long count = m + M + 1;
  if (count > (1LL << 30)) return BURA_EINVAL;
  *nterms = (int)count;
  if (count > max_terms) return BURA_EINVAL;   // *nterms tells the caller how many it needs
  if (!weights || !shifts) return BURA_EINVAL;
  const long double pref = 2.0L * kp * std::sin(pi * a) / pi * std::pow(sc, a - 1.0L);
  for (long long l = -m; l <= M; ++l) {
    const long double y = (long double)l * kp;
    weights[l + m] = (double)(pref * std::exp(2.0L * (a - 1.0L) * y));
    shifts[l + m] = (double)(std::exp(-2.0L * y) / sc);
    if (!std::isfinite(weights[l + m]) || !std::isfinite(shifts[l + m])) return BURA_EINVAL;
  }
  return BURA_OK;
}

// Section 5.3 parametrises the rule by k_Q = pi^2/(4 alpha (1-alpha) k'^2), the
// nominal count m + M of its systems; this inverts that relation.
extern "C" int bura_sinc_kprime(double alpha, double kq, double* kprime) {
  if (!(alpha > 0.0 && alpha < 1.0) || !(kq > 0.0) || !std::isfinite(kq) || !kprime) return BURA_EINVAL;
  const long double pi = 3.141592653589793238462643383279502884L;
  *kprime = (double)(pi / (2.0L * std::sqrt((long double)alpha * (1.0L - alpha) * kq)));
  return BURA_OK;
}
