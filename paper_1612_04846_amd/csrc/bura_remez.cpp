// Host computation of the (k,k) best uniform rational approximation r of
// t^(1-alpha) on [0,1] (Definition 2.1) and of its partial fractions
// r(t)/t = sum_{j=0..k} c_j/(t - d_j), d_0 = 0 > d_1 > ... > d_k (eq. (15),
// Lemma 2.5), in __float128 arithmetic; and of the (k+1,k) 2-BURA of
// t^(2-alpha) with r(t)/t^2 = c_{0,2}/t^2 + c_{0,1}/t + sum_j c_j/(t - d_j)
// (Section 4.1, eq. (22)-(25)).
//
// Same mathematics as the modified Remez algorithm of Section 3.2 (levelled
// equations f(x_i) - r(x_i) = (-1)^i E on 2k+2 reference points, Step 3;
// exchange of the reference set for the local extrema of the error, Step 1;
// stop when the extremal values agree, Step 2), with a different
// representation: the paper's Chebyshev basis needs ~k log10(1/eta_2) digits
// because the alternation points cluster geometrically at t = 0 (Table 5), so
// here r = N/D is kept in barycentric form
//     N(t) = sum_j a_j/(t - z_j),  D(t) = sum_j b_j/(t - z_j)
// with the support points z_j at every other reference point (for type
// (k+1,k) N has one more term, a constant).  Then
//   * the levelled system is a (k+1)x(k+1) pencil (L + 2E C) b = 0 (L a Loewner,
//     C a Cauchy matrix), solved for the E nearest the current estimate by
//     inverse iteration with Rayleigh-quotient updates;
//   * a pole-free solution has weights b_j alternating in sign;
//   * the poles are the zeros of D on t < 0 (bracketed on a log grid, then
//     bisected), and c_j = N(d_j) / (d_j D'(d_j)), c_0 = r(0) = E (eq. (23));
//   * the zeros of r (for the product form of Section 2.2's remark) are the
//     zeros of N on t < 0, found the same way, and the leading constant is
//     lim r(t) = sum a_j / sum b_j as t -> infinity.
// Initial reference set: interpolation at 2k+1 nodes placed by a model of
// the extremal-point distribution (sqrt(-log t) about equispaced, smallest
// ~30 E^(1/(1-alpha)) with E from the asymptotic formula eq. (14)), moved by
// local-error equalisation of the interval lengths until the local maxima agree
// to a few per cent.
#include <quadmath.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "../../include/bura.h"
#include "bura_remez.h"

namespace bura {
namespace {

typedef __float128 Q;

inline Q qabs(Q x) { return x < 0 ? -x : x; }

struct Bary {
  std::vector<Q> z, a, b;   // support points, numerator and denominator weights
  Q ainf = 0;               // constant numerator term: type (k+1, k) instead of (k, k)
  Q eval(Q t) const {
    Q n = ainf, d = 0;
    for (size_t j = 0; j < z.size(); ++j) {
      const Q dt = t - z[j];
      if (dt == 0) return a[j] / b[j];
      n += a[j] / dt;
      d += b[j] / dt;
    }
    return n / d;
  }
};

struct Problem {
  Q g;        // exponent beta - alpha
  int ex = 0;  // numerator degree minus denominator degree: 0 (beta = 1) or 1 (beta = 2)
  Q f(Q t) const { return t <= 0 ? Q(0) : powq(t, g); }
};

// Solve the n x n system M x = rhs (row-major) by Gaussian elimination with partial pivoting.
bool lu_solve(std::vector<Q> M, std::vector<Q>& x, int n) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (qabs(M[r * (n + 1) + c]) > qabs(M[piv * (n + 1) + c])) piv = r;
    if (M[piv * (n + 1) + c] == 0) return false;
    if (piv != c)
      for (int q = 0; q <= n; ++q) std::swap(M[c * (n + 1) + q], M[piv * (n + 1) + q]);
    for (int r = c + 1; r < n; ++r) {
      const Q fac = M[r * (n + 1) + c] / M[c * (n + 1) + c];
      if (fac == 0) continue;
      for (int q = c; q <= n; ++q) M[r * (n + 1) + q] -= fac * M[c * (n + 1) + q];
    }
  }
  x.assign(n, 0);
  for (int r = n - 1; r >= 0; --r) {
    Q s = M[r * (n + 1) + n];
    for (int q = r + 1; q < n; ++q) s -= M[r * (n + 1) + q] * x[q];
    x[r] = s / M[r * (n + 1) + r];
  }
  return true;
}

// Null vector of the m x (m+1) matrix L (row-major) by elimination with complete pivoting.
bool null_vector(std::vector<Q> L, int m, std::vector<Q>& v) {
  const int ncol = m + 1;
  std::vector<int> col(ncol);
  for (int c = 0; c < ncol; ++c) col[c] = c;
  for (int r = 0; r < m; ++r) {
    int pr = r, pc = r;
    Q best = -1;
    for (int i = r; i < m; ++i)
      for (int c = r; c < ncol; ++c)
        if (qabs(L[i * ncol + c]) > best) { best = qabs(L[i * ncol + c]); pr = i; pc = c; }
    if (best <= 0) return false;
    if (pr != r)
      for (int c = 0; c < ncol; ++c) std::swap(L[r * ncol + c], L[pr * ncol + c]);
    if (pc != r) {
      for (int i = 0; i < m; ++i) std::swap(L[i * ncol + r], L[i * ncol + pc]);
      std::swap(col[r], col[pc]);
    }
    for (int i = r + 1; i < m; ++i) {
      const Q fac = L[i * ncol + r] / L[r * ncol + r];
      for (int c = r; c < ncol; ++c) L[i * ncol + c] -= fac * L[r * ncol + c];
    }
  }
  // free variable: the last column
  std::vector<Q> y(ncol, 0);
  y[m] = 1;
  for (int r = m - 1; r >= 0; --r) {
    Q s = -L[r * ncol + m];
    for (int c = r + 1; c < m; ++c) s -= L[r * ncol + c] * y[c];
    y[r] = s / L[r * ncol + r];
  }
  v.assign(ncol, 0);
  for (int c = 0; c < ncol; ++c) v[col[c]] = y[c];
  return true;
}

// ---- extremum and zero localisation in the variable u = log t ---------------

template <class F>
Q golden_max(const F& absval, Q lo, Q hi, int iters) {   // lo, hi: log t
  const Q gr = (sqrtq(Q(5)) - 1) / 2;
  Q x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
  Q f1 = absval(expq(x1)), f2 = absval(expq(x2));
  for (int i = 0; i < iters; ++i) {
    if (f1 > f2) {
      hi = x2; x2 = x1; f2 = f1; x1 = hi - gr * (hi - lo); f1 = absval(expq(x1));
    } else {
      lo = x1; x1 = x2; f1 = f2; x2 = lo + gr * (hi - lo); f2 = absval(expq(x2));
    }
  }
  return expq(f1 > f2 ? x1 : x2);
}

// local maximiser of |e| on [lo, hi] (lo may be 0); endpoints are candidates
template <class F>
Q local_max(const F& e, Q lo, Q hi, bool with_lo, bool with_hi, int iters) {
  auto ab = [&](Q t) { return qabs(e(t)); };
  // coarse scan in log t, then golden section around the best sample
  const Q ulo = lo > 0 ? logq(lo) : logq(hi) - 140;
  const Q uhi = logq(hi);
  const int ns = 24;
  int jb = 0;
  Q vb = -1;
  for (int j = 0; j <= ns; ++j) {
    const Q v = ab(expq(ulo + (uhi - ulo) * j / ns));
    if (v > vb) { vb = v; jb = j; }
  }
  const Q a = ulo + (uhi - ulo) * std::max(jb - 1, 0) / ns;
  const Q b = ulo + (uhi - ulo) * std::min(jb + 1, ns) / ns;
  Q best = golden_max(ab, a, b, iters);
  Q bestv = ab(best);
  if (with_lo && ab(lo) >= bestv) { best = lo; bestv = ab(lo); }
  if (with_hi && ab(hi) >= bestv) { best = hi; }
  return best;
}

template <class F>
Q zero_between(const F& e, Q lo, Q hi) {
  Q elo = e(lo);
  for (int i = 0; i < 200; ++i) {
    const Q mid = lo > 0 ? sqrtq(lo * hi) : hi * Q(1e-6);
    const Q em = e(mid);
    if ((em > 0) == (elo > 0)) { lo = mid; elo = em; }
    else hi = mid;
    if (hi - lo <= Q(1e-32) * hi) break;
  }
  return lo > 0 ? sqrtq(lo * hi) : (lo + hi) / 2;
}

// ---- stage 1: interpolation and node equalisation ---------------------------

bool interpolant(const Problem& P, const std::vector<Q>& X, int k, Bary& r) {
  // support: X[0], X[2], ..., X[2k]; test nodes X[1], X[3], ..., X[2k-1] and,
  // for type (k+1, k), X[2k+1].  At a test node y: ainf + sum_j (f(z_j) - f(y)) b_j/(y - z_j) = 0.
  r.z.clear(); r.a.clear(); r.b.clear();
  r.ainf = 0;
  std::vector<Q> y, fy, fz;
  for (int i = 0; i < 2 * k + 1 + P.ex; ++i) {
    if (i % 2 == 0 && i <= 2 * k) { r.z.push_back(X[i]); fz.push_back(P.f(X[i])); }
    else { y.push_back(X[i]); fy.push_back(P.f(X[i])); }
  }
  const int rows = k + P.ex, cols = k + 1 + P.ex;
  std::vector<Q> L(rows * cols);
  for (int i = 0; i < rows; ++i) {
    for (int j = 0; j <= k; ++j) L[i * cols + j] = (fy[i] - fz[j]) / (y[i] - r.z[j]);
    if (P.ex) L[i * cols + k + 1] = -1;
  }
  std::vector<Q> v;
  if (!null_vector(L, rows, v)) return false;
  r.b.assign(v.begin(), v.begin() + k + 1);
  if (P.ex) r.ainf = v[k + 1];
  r.a.resize(k + 1);
  for (int j = 0; j <= k; ++j) r.a[j] = fz[j] * r.b[j];
  return true;
}

Q stahl(Q g, int k) {   // eq. (14) with beta = 1
  return powq(Q(4), 1 + g) * qabs(sinq(acosq(Q(-1)) * g)) * expq(-2 * acosq(Q(-1)) * sqrtq(g * k));
}

bool initial_reference(const Problem& P, int k, std::vector<Q>& ref, Q& E0, std::string& why) {
  const int n = 2 * k + 1 + P.ex;   // interpolation nodes = degrees of freedom
  const Q tmin = 30 * powq(stahl(P.g, k), 1 / P.g);
  const Q a_ = sqrtq(-logq(tmin)) / n;
  std::vector<Q> eta(n + 1);
  for (int i = 0; i <= n; ++i) eta[i] = expq(-(a_ * (n - i)) * (a_ * (n - i)));
  std::vector<Q> X(n);
  X[0] = eta[0] / 10;
  for (int i = 1; i < n; ++i) X[i] = sqrtq(eta[i - 1] * eta[i]);
  Q tau = Q(0.25);
  std::vector<Q> prevX;
  std::vector<Q> prevd;
  Q prevmax = -1;
  for (int it = 0; it < 600; ++it) {
    Bary r;
    if (!interpolant(P, X, k, r)) { why = "singular interpolation"; return false; }
    auto e = [&](Q t) { return P.f(t) - r.eval(t); };
    std::vector<Q> B;
    B.push_back(0);
    for (Q x : X) B.push_back(x);
    B.push_back(1);
    std::vector<Q> loc(n + 1), dl(n + 1);
    for (int j = 0; j <= n; ++j) {
      loc[j] = local_max(e, B[j], B[j + 1], j == 0, j == n, 40);
      dl[j] = qabs(e(loc[j]));
    }
    Q mx = 0, mn = dl[0];
    bool finite = true;
    for (Q d : dl) { mx = std::max(mx, d); mn = std::min(mn, d); if (!(d == d) || isinfq(d)) finite = false; }
    if (finite && (mx - mn) < Q(0.02) * mx) {
      ref = loc;
      E0 = expq([&] { Q s = 0; for (Q d : dl) s += logq(d); return s / (n + 1); }());
      return true;
    }
    if (!finite || (prevmax > 0 && mx > 4 * prevmax)) {
      if (prevX.empty()) { why = "initial interpolant has poles"; return false; }
      X = prevX;
      dl = prevd;
      tau /= 2;
      if (tau < Q(1e-4)) { why = "node equalisation stalled"; return false; }
      B.assign(1, Q(0));
      for (Q x : X) B.push_back(x);
      B.push_back(1);
    } else {
      prevX = X;
      prevd = dl;
      prevmax = mx;
    }
    Q gm = 0;
    for (Q d : dl) gm += logq(d);
    gm = expq(gm / (n + 1));
    std::vector<Q> len(n + 1);
    Q tot = 0;
    for (int j = 0; j <= n; ++j) {
      len[j] = (B[j + 1] - B[j]) * powq(dl[j] / gm, -tau);
      tot += len[j];
    }
    Q acc = 0;
    for (int j = 0; j < n; ++j) { acc += len[j] / tot; X[j] = acc; }
  }
  why = "node equalisation did not converge";
  return false;
}

// ---- stage 2: levelled barycentric solve + exchange ---------------------------

// reference x[0..2k+1+ex] (x[0] = 0, last = 1); support = even positions
// 0..2k.  Solve (L + 2E C) v = 0 for the E nearest Eguess, v = (b, ainf).
bool levelled(const Problem& P, const std::vector<Q>& x, int k, Q& E, Bary& r) {
  const int nb = k + 1, m = k + 1 + P.ex;   // weights b; unknowns (and rows) incl. ainf
  std::vector<Q> z, y, fz, fy;
  std::vector<int> ty;   // 1: test point of opposite sign to the supports; 0: same sign
  for (int i = 0; i < 2 * k + 2 + P.ex; ++i) {
    if (i % 2 == 0 && i <= 2 * k) { z.push_back(x[i]); fz.push_back(P.f(x[i])); }
    else { y.push_back(x[i]); fy.push_back(P.f(x[i])); ty.push_back(i % 2); }
  }
  // sigma(support) = -1 (odd 1-based index), sigma(odd-position test) = +1, the
  // extra last point of type (k+1, k) has the supports' sign:
  // ainf + sum_j b_j [(f(z_j) - f(y_i)) + (sigma_i + 1) E] / (y_i - z_j) = 0
  std::vector<Q> L(m * m, 0), C(m * m, 0);
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < nb; ++j) {
      const Q dd = y[i] - z[j];
      L[i * m + j] = (fz[j] - fy[i]) / dd;
      C[i * m + j] = ty[i] ? 1 / dd : Q(0);
    }
    if (P.ex) L[i * m + nb] = 1;
  }
  std::vector<Q> b(m, 0), w;
  for (int j = 0; j < nb; ++j) b[j] = (j % 2 == 0) ? 1 : -1;
  Q Ec = E;
  for (int it = 0; it < 60; ++it) {
    std::vector<Q> M(m * (m + 1));
    for (int i = 0; i < m; ++i) {
      Q cb = 0;
      for (int j = 0; j < m; ++j) {
        M[i * (m + 1) + j] = L[i * m + j] + 2 * Ec * C[i * m + j];
        cb += C[i * m + j] * b[j];
      }
      M[i * (m + 1) + m] = cb;
    }
    if (!lu_solve(M, w, m)) break;   // exactly singular: Ec is the eigenvalue
    Q nrm = 0;
    for (Q v : w) nrm += v * v;
    nrm = sqrtq(nrm);
    for (int j = 0; j < m; ++j) b[j] = w[j] / nrm;
    // E minimising ||(L + 2E C) b||
    std::vector<Q> Lb(m, 0), Cb(m, 0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) { Lb[i] += L[i * m + j] * b[j]; Cb[i] += C[i * m + j] * b[j]; }
    Q num = 0, den = 0;
    for (int i = 0; i < m; ++i) { num += Cb[i] * Lb[i]; den += Cb[i] * Cb[i]; }
    const Q En = -num / (2 * den);
    const bool done = qabs(En - Ec) <= Q(1e-30) * qabs(En);
    Ec = En;
    if (done) break;
  }
  // pole-free on [0,1] needs alternating weights
  for (int j = 0; j + 1 < nb; ++j)
    if ((b[j] > 0) == (b[j + 1] > 0)) return false;
  E = Ec;
  r.z = z;
  r.b.assign(b.begin(), b.begin() + nb);
  r.ainf = P.ex ? b[nb] : Q(0);
  r.a.resize(nb);
  for (int j = 0; j < nb; ++j) r.a[j] = (fz[j] + E) * b[j];   // r(z_j) = f(z_j) - sigma E = f + E
  return true;
}

// The beta-BURA of t^(beta - alpha), beta = 1 (type (k,k)) or 2 (type (k+1,k)).
int remez_q(double alpha, int beta, int k, std::vector<double>& c_out, std::vector<double>& d_out,
            double& E_out, std::vector<double>& zeta_out, double& C_out, std::string& why) {
  Problem P;
  P.g = Q(beta) - Q(alpha);
  P.ex = beta - 1;
  const int nref = 2 * k + 2 + P.ex;   // m + k + 2 reference points
  std::vector<Q> ref;
  Q E0;
  if (!initial_reference(P, k, ref, E0, why)) return BURA_EREMEZ;
  ref[0] = 0;
  ref[nref - 1] = 1;
  Q E = E0;
  Bary r;
  bool ok = false;
  for (int it = 0; it < 40; ++it) {
    if (!levelled(P, ref, k, E, r)) { why = "levelled system has no pole-free solution"; return BURA_EREMEZ; }
    auto e = [&](Q t) { return P.f(t) - r.eval(t); };
    // zeros of the error between consecutive reference points
    std::vector<Q> Z;
    Z.push_back(0);
    for (int i = 0; i + 1 < nref; ++i) {
      const Q e0 = e(ref[i]), e1 = e(ref[i + 1]);
      if ((e0 > 0) == (e1 > 0)) { why = "alternation lost"; return BURA_EREMEZ; }
      Z.push_back(zero_between(e, ref[i], ref[i + 1]));
    }
    Z.push_back(1);
    std::vector<Q> next(nref);
    Q mx = 0, mn = -1;
    for (int i = 0; i < nref; ++i) {
      next[i] = local_max(e, Z[i], Z[i + 1], i == 0, i == nref - 1, 110);
      const Q v = qabs(e(next[i]));
      mx = std::max(mx, v);
      mn = (mn < 0) ? v : std::min(mn, v);
    }
    ref = next;
    if (mx - mn <= Q(1e-16) * mx) { ok = true; break; }
  }
  if (!ok) { why = "exchange did not level"; return BURA_EREMEZ; }
  if (!levelled(P, ref, k, E, r)) { why = "final levelled solve failed"; return BURA_EREMEZ; }
  // poles: zeros of D(t) on t < 0; zeros of r: zeros of N(t) on t < 0 (no
  // support point lies there, so N and D have no common singularity)
  auto D = [&](Q t) { Q s = 0; for (size_t j = 0; j < r.z.size(); ++j) s += r.b[j] / (t - r.z[j]); return s; };
  auto Dp = [&](Q t) { Q s = 0; for (size_t j = 0; j < r.z.size(); ++j) { Q dt = t - r.z[j]; s -= r.b[j] / (dt * dt); } return s; };
  auto N = [&](Q t) { Q s = r.ainf; for (size_t j = 0; j < r.z.size(); ++j) s += r.a[j] / (t - r.z[j]); return s; };
  auto negative_roots = [](auto&& fn) {
    std::vector<Q> roots;
    const Q u0 = -200, u1 = 30, du = Q(0.01);   // t = -exp(u)
    Q uprev = u0, fprev = fn(-expq(u0));
    for (Q u = u0 + du; u <= u1; u += du) {
      const Q fv = fn(-expq(u));
      if ((fv > 0) != (fprev > 0)) {
        Q lo = uprev, hi = u, flo = fprev;
        for (int i = 0; i < 200; ++i) {
          const Q mid = (lo + hi) / 2;
          const Q fm = fn(-expq(mid));
          if ((fm > 0) == (flo > 0)) { lo = mid; flo = fm; } else hi = mid;
          if (hi - lo < Q(1e-33)) break;
        }
        roots.push_back(-expq((lo + hi) / 2));
      }
      uprev = u;
      fprev = fv;
    }
    std::sort(roots.begin(), roots.end(), [](Q a, Q b) { return a > b; });   // descending
    return roots;
  };
  std::vector<Q> poles = negative_roots(D);
  if ((int)poles.size() != k) { why = "pole count differs from k"; return BURA_EREMEZ; }
  if (beta == 2) {
    // Section 4.1 / eq. (22): residues c*_j = N(d_j)/D'(d_j) of r, c_j = c*_j / d_j^2,
    // c_{0,2} = r(0) (eq. (23)); c_{0,1} from the identity
    // r(t)/t^2 = c_{0,2}/t^2 + c_{0,1}/t + sum_j c_j/(t - d_j) at t = 1
    c_out.assign(k + 2, 0.0);
    d_out.assign(k + 1, 0.0);
    const Q c02 = r.eval(0);
    Q sum = 0;
    std::vector<Q> cj(k);
    for (int j = 0; j < k; ++j) {
      const Q dj = poles[j];
      cj[j] = N(dj) / Dp(dj) / (dj * dj);
      if (!(cj[j] > 0)) { why = "non-positive weight"; return BURA_EREMEZ; }
      sum += cj[j] / (1 - dj);
      c_out[j + 1] = (double)cj[j];
      d_out[j + 1] = (double)dj;
    }
    const Q c01 = r.eval(1) - c02 - sum;
    c_out[0] = (double)c01;
    c_out[k + 1] = (double)c02;
    zeta_out.clear();
    C_out = 0.0;
    E_out = (double)qabs(E);
    return BURA_OK;
  }
  std::vector<Q> zeros = negative_roots(N);
  if ((int)zeros.size() != k) { why = "zero count differs from k"; return BURA_EREMEZ; }
  // Lemma 2.5: 0 > zeta_1 > d_1 > zeta_2 > ... > zeta_k > d_k
  for (int j = 0; j < k; ++j)
    if (!(zeros[j] > poles[j]) || (j > 0 && !(zeros[j] < poles[j - 1]))) {
      why = "zeros and poles do not interlace";
      return BURA_EREMEZ;
    }
  {
    Q sa = 0, sb = 0;   // r(t) -> sum a / sum b as t -> infinity: the leading constant
    for (size_t j = 0; j < r.z.size(); ++j) { sa += r.a[j]; sb += r.b[j]; }
    C_out = (double)(sa / sb);
  }
  zeta_out.assign(k, 0.0);
  for (int j = 0; j < k; ++j) zeta_out[j] = (double)zeros[j];
  c_out.assign(k + 1, 0.0);
  d_out.assign(k + 1, 0.0);
  c_out[0] = (double)r.eval(0);   // = E, eq. (23)
  for (int j = 0; j < k; ++j) {
    const Q dj = poles[j];
    const Q cj = N(dj) / (dj * Dp(dj));
    if (!(cj > 0)) { why = "non-positive weight"; return BURA_EREMEZ; }
    c_out[j + 1] = (double)cj;
    d_out[j + 1] = (double)dj;
  }
  E_out = (double)qabs(E);
  return BURA_OK;
}

struct Cached {
  std::vector<double> c, d, zeta;
  double E = 0.0, C = 0.0;
};
std::mutex g_mu;
std::map<std::pair<uint64_t, int>, Cached> g_cache;

}  // namespace

int remez_bura_full(double alpha, int beta, int k, std::vector<double>& c, std::vector<double>& d, double& E,
                    std::vector<double>& zeta, double& C, std::string& why) {
  uint64_t bits;
  std::memcpy(&bits, &alpha, 8);
  const auto key = std::make_pair(bits, k * 4 + beta);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      c = it->second.c;
      d = it->second.d;
      E = it->second.E;
      zeta = it->second.zeta;
      C = it->second.C;
      return BURA_OK;
    }
  }
  const int rc = remez_q(alpha, beta, k, c, d, E, zeta, C, why);
  if (rc == BURA_OK) {
    std::lock_guard<std::mutex> lk(g_mu);
    Cached& e = g_cache[key];
    e.c = c;
    e.d = d;
    e.E = E;
    e.zeta = zeta;
    e.C = C;
  }
  return rc;
}

int remez_bura(double alpha, int k, std::vector<double>& c, std::vector<double>& d, double& E, std::string& why) {
  std::vector<double> zeta;
  double C = 0.0;
  return remez_bura_full(alpha, 1, k, c, d, E, zeta, C, why);
}

}  // namespace bura

extern "C" int bura_coefficients(double alpha, int beta, int k, double* c, double* d, double* E) {
  if (!(alpha > 0 && alpha < 1) || k < 1 || k > 16 || !c || !d || !E) return BURA_EINVAL;
  if (beta != 1 && beta != 2) return BURA_EUNSUPPORTED;
  std::vector<double> cc, dd, zz;
  double C = 0.0;
  std::string why;
  const int rc = bura::remez_bura_full(alpha, beta, k, cc, dd, *E, zz, C, why);
  if (rc) return rc;
  if (beta == 2) c[k + 1] = cc[k + 1];   // c_{0,2}, the weight of A^-2 f
  for (int j = 0; j <= k; ++j) {
    c[j] = cc[j];
    d[j] = dd[j];
  }
  return BURA_OK;
}

extern "C" int bura_zeros(double alpha, int beta, int k, double* zeta, double* C) {
  if (!(alpha > 0 && alpha < 1) || k < 1 || k > 16 || !zeta || !C) return BURA_EINVAL;
  if (beta != 1) return BURA_EUNSUPPORTED;
  std::vector<double> cc, dd, zz;
  double E = 0.0;
  std::string why;
  const int rc = bura::remez_bura_full(alpha, 1, k, cc, dd, E, zz, *C, why);
  if (rc) return rc;
  for (int j = 0; j < k; ++j) zeta[j] = zz[j];
  return BURA_OK;
}
