// Host-side rational approximation (no HIP dependency; built by the host compiler).
#pragma once
#include <string>
#include <vector>

namespace bura {
// (k,k) best uniform rational approximation r of t^(1-alpha) on [0,1] and its
// partial fractions r(t)/t = sum_j c_j/(t - d_j), d_0 = 0 > d_1 > ... > d_k.
int remez_bura(double alpha, int k, std::vector<double>& c, std::vector<double>& d, double& E, std::string& why);
// the same for beta = 1 (type (k,k)) or 2 (type (k+1,k), c gains c_{0,2} at
// index k+1), plus for beta = 1 the zeros zeta_1 > ... > zeta_k of r (Lemma 2.5)
// and the leading constant C of r(t) = C prod_j (t - zeta_j)/(t - d_j)
int remez_bura_full(double alpha, int beta, int k, std::vector<double>& c, std::vector<double>& d, double& E,
                    std::vector<double>& zeta, double& C, std::string& why);
}  // namespace bura
