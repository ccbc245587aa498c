"""O1: the beta-BURA of t^(beta-alpha) on [0,1] by the modified Remez algorithm.

TEST INFRASTRUCTURE (see the package docstring): slow, multiprecision, plain.

What is computed (arXiv:1612.04846):

* Definition 2.1 / eq. (11): r = P_m/Q_k minimises max_[0,1] |t^(beta-alpha) - r|;
  E_alpha(m,k;beta) is that maximum.  By the equioscillation theorem quoted in
  Section 3.1 the error reaches +-E with alternating signs at m+k+2 points, and
  that property is the test of every result.
* eq. (18): P and Q are written in the shifted Chebyshev basis T_j(2t-1); the
  iteration works with s = 2t-1 in [-1,1] and f(s) = ((1+s)/2)^(beta-alpha),
  with the denominator normalised to qbar_0 = 1.
* The iteration is the modified Remez algorithm of Section 3.2 (Algorithm 3.1):
  from the current rational function, move the reference set to the extrema
  of the error between its sign changes; stop when those extrema are level;
  otherwise solve the levelled equations f(s_i) - r(s_i) = (-1)^i E on the new
  set for r and E, by the paper's linear solves with E of the previous sweep
  frozen in the denominator term, accelerated by Aitken-Steffensen.
* Lemma 2.5 and eq. (15): for m = k, beta = 1 the poles are real, negative and
  simple; r(t)/t = sum_{j=0..k} c_j/(t - d_j) with d_0 = 0.  The weights are the
  residues of P/(t Q): c_0 = P(0)/Q(0) = r(0) and c_j = P(d_j)/(d_j Q'(d_j)).
* Section 4.1 for beta > 1 (m - k < beta): polynomial part and simple
  fractions of P/Q, then the relations of eq. (22) give the weights of
  eq. (25), c_{0,i} for A^-i f (i = 1..beta) and c_j for (A - d_j)^-1 f.

Readings where the paper is silent (also listed in the design notes):

* Initial reference set and r_0 (the paper only asks for an admissible r_0 and
  mentions least squares).  Here: interpolation nodes placed by a model of the
  extremal-point distribution (sqrt(-log t) roughly equispaced, smallest point
  ~ E^(1/(beta-alpha)) from the asymptotic formula eq. (14)), then the nodes
  are moved by repeated local-error equalisation of the interpolant (each
  node interval is rescaled by its local maximum error) until the local
  maxima agree to a few per cent.  That interpolant is r_0 (its error
  alternates at the extrema, so it is admissible) and the extrema are s^(0).
* Which solution of the levelled equations.  They have k+1 solutions E (after
  eliminating pbar they are a (k+1) x (k+1) eigenproblem for E), and the
  frozen-E iteration can settle on any of them; only one has a denominator of
  one sign on the reference set, the admissible one that the algorithm
  requires of r_0 and of every later iterate.  When the iteration ends
  elsewhere (it does for alpha = 0.9, k = 8, 10, 11, 12 from the start above),
  the iteration is restarted from that admissible root, found from the
  eigenproblem.
* Extremum localisation: zoomed grid search in log t (the remarks after
  Algorithm 3.1 describe the same idea), endpoints t = 0 and t = 1 included.
* delta is relative: max eta - min eta < delta_rel * max eta.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import mpmath as mp


_VERBOSE = False


class RemezError(RuntimeError):
    """Raised when Algorithm 3.1 loses alternation or does not level."""


# ----------------------------------------------------------------------------
# Chebyshev basis of eq. (18)
# ----------------------------------------------------------------------------

def _cheb(s, n):
    """T_0(s) .. T_n(s) by the three-term recurrence below eq. (18)."""
    T = [mp.mpf(1), s]
    for _ in range(2, n + 1):
        T.append(2 * s * T[-1] - T[-2])
    return T[: n + 1]


def _ratval(pbar, qbar, s):
    n = max(len(pbar), len(qbar)) - 1
    T = _cheb(s, n)
    num = mp.fsum(pbar[j] * T[j] for j in range(len(pbar)))
    den = mp.fsum(qbar[j] * T[j] for j in range(len(qbar)))
    return num / den


def stahl_estimate(alpha, k, beta=1):
    """Asymptotic error formula eq. (14)."""
    g = mp.mpf(beta) - mp.mpf(alpha)
    return 4 ** (1 + g) * abs(mp.sin(mp.pi * g)) * mp.exp(-2 * mp.pi * mp.sqrt(g * k))


@dataclass
class Bura:
    """Result of Algorithm 3.1 and of the partial-fraction step eq. (15)."""

    alpha: float
    beta: int
    m: int
    k: int
    dps: int
    E: mp.mpf                      # E_alpha(m,k;beta) (signed levelled value)
    pbar: List[mp.mpf]             # numerator in T_j(2t-1), qbar_0 = 1
    qbar: List[mp.mpf]
    eta: List[mp.mpf]              # final reference / alternation points in t
    eta_err: List[mp.mpf]          # t^(b-a) - r at eta
    iterations: int
    p: List[mp.mpf] = field(default_factory=list)   # monomial coefficients, q_k = 1
    q: List[mp.mpf] = field(default_factory=list)
    d: List[mp.mpf] = field(default_factory=list)   # poles, d_0 = 0 > d_1 > ... (beta=1, m=k)
    c: List[mp.mpf] = field(default_factory=list)   # residues of r(t)/t
    # beta > 1 (eq. (25)): c0[i-1] = c_{0,i} multiplies A^-i f, i = 1..beta; then
    # c = [c_{0,1}, c_1, ..., c_k] and d = [0, d_1, ..., d_k] as for beta = 1
    c0: List[mp.mpf] = field(default_factory=list)

    # -- evaluation helpers (multiprecision) -------------------------------
    def r(self, t):
        """r(t) from the Chebyshev form eq. (18)."""
        return _ratval(self.pbar, self.qbar, 2 * mp.mpf(t) - 1)

    def r_from_fractions(self, t):
        """r(t) = t * sum_j c_j/(t - d_j), eq. (15)."""
        t = mp.mpf(t)
        return mp.fsum(self.c[j] * (t / (t - self.d[j]) if j else 1) for j in range(len(self.c)))

    def err(self, t):
        t = mp.mpf(t)
        return t ** (self.beta - mp.mpf(self.alpha)) - self.r(t)

    # -- float views ---------------------------------------------------------
    @property
    def c_f64(self):
        return [float(x) for x in self.c]

    @property
    def d_f64(self):
        return [float(x) for x in self.d]

    @property
    def E_f64(self):
        return float(abs(self.E))


# ----------------------------------------------------------------------------
# the levelled equations f(s_i) - r(s_i) = (-1)^i E on a reference set
# ----------------------------------------------------------------------------

def _sigma(i):
    """(-1)^i for the i-th reference point counted from 1 (i = 0 here is the first)."""
    return -1 if i % 2 == 0 else 1


def _level_sweeps(Ts, fS, m, k, E0, tol):
    """The paper's iteration for the levelled equations: with E_old frozen in the
    denominator term,

        sum_j pbar_j T_j(s_i) - (f_i - (-1)^i E_old) sum_{j>=1} qbar_j T_j(s_i)
            + (-1)^i E_new = f_i

    is linear in (pbar, qbar_1..k, E_new); the map E_old -> E_new is iterated
    from E0 with Aitken-Steffensen acceleration.  Returns (E, pbar, qbar)."""
    L = len(fS)

    def sweep(E):
        A = mp.matrix(L, L)
        b = mp.matrix(L, 1)
        for i in range(L):
            sg = _sigma(i)
            for j in range(m + 1):
                A[i, j] = Ts[i][j]
            for j in range(1, k + 1):
                A[i, m + j] = -(fS[i] - sg * E) * Ts[i][j]
            A[i, L - 1] = sg
            b[i] = fS[i]
        x = mp.lu_solve(A, b)
        return x[L - 1], x

    E = E0
    best = None
    for _ in range(100):
        E1, x = sweep(E)
        ch = abs(E1 - E)
        if ch <= tol * abs(E1):
            E = E1
            break
        if best is None or ch < best[0]:
            best = (ch, E1)
        E2, x = sweep(E1)
        den = E2 - 2 * E1 + E
        E = E - (E1 - E) ** 2 / den if den != 0 else E2
    else:
        # stagnation at the working precision's noise floor is accepted when
        # the fixed point is already resolved far below the levelling tolerance
        if best[0] > mp.sqrt(tol) * abs(best[1]):
            raise RemezError("levelled equations: the iteration did not converge")
        E = best[1]
    E, x = sweep(E)
    pbar = [x[j] for j in range(m + 1)]
    qbar = [mp.mpf(1)] + [x[m + j] for j in range(1, k + 1)]
    return E, pbar, qbar


def _admissible(Ts, qbar):
    """The denominator has one sign on the reference set."""
    Q = [mp.fsum(qbar[j] * T[j] for j in range(len(qbar))) for T in Ts]
    return all(v > 0 for v in Q) or all(v < 0 for v in Q)


def _admissible_root(Ts, fS, m, k):
    """The levelled equations as an eigenproblem: P(s_i) = (f_i - (-1)^i E) Q(s_i).
    With N spanning the left null space of [T_j(s_i)]_{j<=m}, pbar drops out:
    N^T F V qbar = E N^T Sigma V qbar, V = [T_j(s_i)]_{j<=k}, F = diag(f_i),
    Sigma = diag((-1)^i).  Returns the real eigenvalue whose eigenvector gives a
    denominator of one sign on the reference set."""
    L = len(fS)
    VP = mp.matrix(L, m + 1)
    for i in range(L):
        for j in range(m + 1):
            VP[i, j] = Ts[i][j]
    Qf, _ = mp.qr(VP, mode="full")
    N = Qf[:, m + 1:L]
    FV = mp.matrix(L, k + 1)
    SV = mp.matrix(L, k + 1)
    for i in range(L):
        for j in range(k + 1):
            FV[i, j] = fS[i] * Ts[i][j]
            SV[i, j] = _sigma(i) * Ts[i][j]
    vals, vecs = mp.eig(mp.inverse(N.T * SV) * (N.T * FV))
    scale = max(abs(v) for v in vals)
    found = []
    for c, lam in enumerate(vals):
        if abs(mp.im(lam)) > mp.mpf(10) ** (-(mp.mp.dps // 3)) * scale:
            continue
        q = [mp.re(vecs[j, c]) for j in range(k + 1)]
        if _admissible(Ts, q):
            found.append(mp.re(lam))
    if len(found) != 1:
        raise RemezError(f"levelled equations: {len(found)} admissible solutions")
    return found[0]


def _level(S, fS, m, k, E0, tol):
    """Solve f(s_i) - r(s_i) = (-1)^i E (i = 1..l) for an admissible r and E,
    starting the paper's iteration from E0 (the previous levelled value)."""
    Ts = [_cheb(s, max(m, k)) for s in S]
    E, pbar, qbar = _level_sweeps(Ts, fS, m, k, E0, tol)
    if not _admissible(Ts, qbar):
        E, pbar, qbar = _level_sweeps(Ts, fS, m, k, _admissible_root(Ts, fS, m, k), tol)
        if not _admissible(Ts, qbar):
            raise RemezError("levelled equations: no admissible solution")
    return pbar, qbar, E


# ----------------------------------------------------------------------------
# extremum / zero localisation on [-1,1], working in u = log(1+s) = log(2t)
# ----------------------------------------------------------------------------

def _zero_between(e, lo, hi, elo, rel):
    """Bisection (in log(1+s) when lo > -1) for a sign change of e on (lo, hi)."""
    for _ in range(400):
        if lo == -1:
            mid = (lo + hi) / 2 if hi - lo > mp.mpf(10) ** (-mp.mp.dps // 2) else -1 + (1 + hi) / 2 ** 20
        else:
            mid = mp.sqrt((1 + lo) * (1 + hi)) - 1
        em = e(mid)
        if (em > 0) == (elo > 0):
            lo, elo = mid, em
        else:
            hi = mid
        if (hi - lo) <= rel * (1 + hi):
            break
    return (lo + hi) / 2


def _argmax_abs(e, a, b, include_a, include_b, span_floor, zooms=9, n=24):
    """Zoomed grid search for argmax |e| on [a,b] in the variable u = log(1+s)."""
    ua = mp.log(1 + a) if a > -1 else mp.log(1 + b) - span_floor
    ub = mp.log(1 + b)
    lo, hi = ua, ub
    best_u = None
    for _ in range(zooms):
        pts = [lo + (hi - lo) * j / n for j in range(n + 1)]
        vals = [abs(e(mp.exp(u) - 1)) for u in pts]
        jb = max(range(n + 1), key=lambda j: vals[j])
        best_u = pts[jb]
        lo, hi = pts[max(jb - 1, 0)], pts[min(jb + 1, n)]
    cands = [mp.exp(best_u) - 1]
    if include_a:
        cands.append(a)
    if include_b:
        cands.append(b)
    return max(cands, key=lambda s: abs(e(s)))


# ----------------------------------------------------------------------------
# initial reference set (reading: the paper leaves the initialisation open)
# ----------------------------------------------------------------------------

def _interp(X, fX, m, k):
    """Rational interpolant of type (m,k) through m+k+1 nodes, qbar_0 = 1."""
    n = len(X)
    A = mp.matrix(n, n)
    b = mp.matrix(n, 1)
    for i, x in enumerate(X):
        T = _cheb(2 * x - 1, max(m, k))
        for j in range(m + 1):
            A[i, j] = T[j]
        for j in range(1, k + 1):
            A[i, m + j] = -fX[i] * T[j]
        b[i] = fX[i]
    sol = mp.lu_solve(A, b)
    return [sol[j] for j in range(m + 1)], [mp.mpf(1)] + [sol[m + j] for j in range(1, k + 1)]


def _initial_reference(alpha, beta, m, k, X=None, iters=400, tau=0.25, target=0.05):
    g = mp.mpf(beta) - mp.mpf(alpha)
    n = m + k + 1
    if X is None:
        # model of the extremal points: sqrt(-log eta) about equispaced, with the
        # smallest nonzero point ~ 30 * E^(1/g), E from eq. (14)
        Es = stahl_estimate(alpha, k, beta)
        tmin = 30 * Es ** (1 / g)
        a_ = mp.sqrt(-mp.log(tmin)) / n
        eta = [mp.exp(-(a_ * (n - i)) ** 2) for i in range(n + 1)]  # eta[0]=tmin .. eta[n]=1
        X = [eta[0] / 10] + [mp.sqrt(eta[i] * eta[i + 1]) for i in range(n)]
        X = X[:n]
    fX = None
    prev = None
    for _ in range(iters):
        fX = [x ** g for x in X]
        pbar, qbar = _interp(X, fX, m, k)
        e = lambda s: ((1 + s) / 2) ** g - _ratval(pbar, qbar, s)
        B = [mp.mpf(-1)] + [2 * x - 1 for x in X] + [mp.mpf(1)]
        loc, dl = [], []
        for j in range(n + 1):
            s_ = _argmax_abs(e, B[j], B[j + 1], j == 0, j == n, 80, zooms=5, n=16)
            loc.append(s_)
            dl.append(abs(e(s_)))
        mx, mn = max(dl), min(dl)
        if (mx - mn) / mx < target:
            return loc, mx, pbar, qbar
        if prev is not None and mx > 4 * prev[0]:
            # overshoot: go back and take a smaller step
            X, dl_prev = prev[1], prev[2]
            tau = tau / 2
            dl = dl_prev
        else:
            prev = (mx, X, dl)
        lengths = [(B[j + 1] - B[j]) / 2 for j in range(n + 1)]
        gmean = mp.exp(mp.fsum(mp.log(d) for d in dl) / len(dl))
        lengths = [Lj * (d / gmean) ** (-tau) for Lj, d in zip(lengths, dl)]
        tot = mp.fsum(lengths)
        acc = mp.mpf(0)
        X = []
        for Lj in lengths[:-1]:
            acc += Lj / tot
            X.append(acc)
    raise RemezError("initial node equalisation did not converge")


# ----------------------------------------------------------------------------
# Algorithm 3.1
# ----------------------------------------------------------------------------

def required_dps(alpha, k, m=None, beta=1, tmin=None):
    """Working precision needed by the Chebyshev-basis systems (Table 5 reading).

    Near t = 0 the basis functions T_j(2t-1) differ from (-1)^j only by
    O(j^2 t), so resolving a reference point at t ~ eta_2 costs about
    log10(1/eta_2) digits per degree.  eta_2 ~ 30 E^(1/(beta-alpha)) with E from
    eq. (14) unless the caller supplies it.
    """
    m = k if m is None else m
    with mp.workdps(30):
        if tmin is None:
            g = mp.mpf(beta) - mp.mpf(alpha)
            tmin = 30 * stahl_estimate(alpha, k, beta) ** (1 / g)
        digits = -mp.log10(tmin)
    return int(40 + max(m, k) * max(float(digits), 1.0))


def _exchange(e, S, dps):
    """New reference set from the current error e = f - r: the point of largest
    |e| between each pair of consecutive sign changes (the first interval
    starts at s = -1, the last ends at s = 1, both included).  The error must
    alternate on the old set; the largest |e| on [-1,1] is then one of the new
    points."""
    L = len(S)
    ev = [e(s) for s in S]
    for i in range(L - 1):
        if (ev[i] > 0) == (ev[i + 1] > 0):
            raise RemezError("the error does not alternate on the reference set")
    Z = [mp.mpf(-1)]
    Z += [_zero_between(e, S[i], S[i + 1], ev[i], mp.mpf(10) ** (-(dps // 2))) for i in range(L - 1)]
    Z.append(mp.mpf(1))
    return [_argmax_abs(e, Z[i], Z[i + 1], i == 0, i == L - 1, 2 * dps) for i in range(L)]


def remez(alpha, k, m=None, beta=1, dps=None, delta_rel=1e-20, max_iter=60,
          start: Optional[Sequence] = None) -> Bura:
    """Modified Remez algorithm (Section 3.2, Algorithm 3.1) for the beta-BURA
    of t^(beta-alpha): exchange, level check, levelled solve, until level.

    ``start`` optionally gives interpolation nodes in t (m+k+1 of them) for the
    initialisation, e.g. taken from a neighbouring (alpha, k).  ``dps`` defaults
    to :func:`required_dps`.
    """
    m = k if m is None else m
    if dps is None:
        dps = required_dps(alpha, k, m, beta)
    with mp.workdps(dps):
        g = mp.mpf(beta) - mp.mpf(alpha)
        f = lambda s: ((1 + s) / 2) ** g
        delta = mp.mpf(delta_rel)
        ltol = mp.mpf(10) ** (-(dps * 2) // 3)
        X0 = [mp.mpf(x) for x in start] if start is not None else None
        # admissible r_0 (the equalised interpolant), s^(0) = its error's extrema
        S, E, pbar, qbar = _initial_reference(alpha, beta, m, k, X=X0)
        S = sorted(S)
        S[0], S[-1] = mp.mpf(-1), mp.mpf(1)
        it = 0
        for it in range(1, max_iter + 1):
            e = lambda s: f(s) - _ratval(pbar, qbar, s)
            S = _exchange(e, S, dps)
            etas = [abs(e(s)) for s in S]
            if _VERBOSE:
                print("remez it", it, mp.nstr(E, 12), mp.nstr((max(etas) - min(etas)) / max(etas), 3), flush=True)
            if max(etas) - min(etas) < delta * max(etas):
                break
            pbar, qbar, E = _level(S, [f(s) for s in S], m, k, E, ltol)
        else:
            raise RemezError("Algorithm 3.1 reached its iteration limit")
        eta = [(s + 1) / 2 for s in S]
        res = Bura(alpha=alpha, beta=beta, m=m, k=k, dps=dps, E=E, pbar=pbar, qbar=qbar,
                   eta=eta, eta_err=[eta_i ** g - _ratval(pbar, qbar, 2 * eta_i - 1) for eta_i in eta],
                   iterations=it)
        _monomial(res)
        if beta == 1 and m == k:
            _partial_fractions(res)
        elif beta > 1 and 0 <= m - k < beta:
            # eq. (25) needs simple real negative poles; some (m, k, beta) of
            # Table 1 do not have them, and only E is used there
            try:
                _partial_fractions_beta(res)
            except RemezError:
                res.c0, res.c, res.d = [], [], []
        return res


# ----------------------------------------------------------------------------
# eq. (18) -> monomials in t, and eq. (15) partial fractions
# ----------------------------------------------------------------------------

def _shifted_cheb_monomials(n):
    """Monomial coefficients (in t) of T_j(2t - 1), j = 0..n."""
    rows = [[mp.mpf(1)], [mp.mpf(-1), mp.mpf(2)]]
    for _ in range(2, n + 1):
        a, b = rows[-1], rows[-2]
        new = [mp.mpf(0)] * (len(a) + 1)
        for i, v in enumerate(a):        # 2(2t-1) a(t)
            new[i + 1] += 4 * v
            new[i] -= 2 * v
        for i, v in enumerate(b):
            new[i] -= v
        rows.append(new)
    return rows[: n + 1]


def _monomial(res: Bura):
    n = max(res.m, res.k)
    rows = _shifted_cheb_monomials(n)
    p = [mp.mpf(0)] * (res.m + 1)
    q = [mp.mpf(0)] * (res.k + 1)
    for j, a in enumerate(res.pbar):
        for i, v in enumerate(rows[j]):
            p[i] += a * v
    for j, a in enumerate(res.qbar):
        for i, v in enumerate(rows[j]):
            q[i] += a * v
    lead = q[res.k]               # the coefficient tables normalise q_k = 1
    res.p = [x / lead for x in p]
    res.q = [x / lead for x in q]


def _poly(coefs, t):
    return mp.fsum(cf * t ** i for i, cf in enumerate(coefs))


def _polydiv(num, den):
    """Quotient and remainder of num/den (ascending monomial coefficients)."""
    num = list(num)
    dq = len(den) - 1
    quo = [mp.mpf(0)] * max(1, len(num) - dq)
    for i in range(len(num) - 1, dq - 1, -1):
        f = num[i] / den[dq]
        quo[i - dq] = f
        for j in range(dq + 1):
            num[i - dq + j] -= f * den[j]
    return quo, num[:dq]


def _partial_fractions_beta(res: Bura):
    """Section 4.1 for beta > 1 with m - k < beta: P/Q = sum_{j<beta} b_j t^j +
    sum_j c*_j/(t - d_j) (polynomial division, simple real poles), then eq. (22):
    c_{0,i} = b_{beta-i} - sum_j c*_j / d_j^(beta-i+1) and c_j = c*_j / d_j^beta."""
    beta = res.beta
    roots = mp.polyroots(list(reversed(res.q)), maxsteps=400, extraprec=4 * res.dps)
    d = []
    for z in roots:
        if abs(mp.im(z)) > mp.mpf(10) ** (-(res.dps // 3)) * (1 + abs(z)):
            raise RemezError("complex pole: partial fractions with p_2 > 0 are not covered")
        d.append(mp.re(z))
    if any(x >= 0 for x in d):
        raise RemezError("non-negative pole")
    d = sorted(d, reverse=True)
    quo, _ = _polydiv(res.p, res.q)
    b = [quo[j] if j < len(quo) else mp.mpf(0) for j in range(beta)]
    dq = [i * res.q[i] for i in range(1, len(res.q))]
    cstar = [_poly(res.p, dj) / _poly(dq, dj) for dj in d]
    c0 = [b[beta - i] - mp.fsum(cs / dj ** (beta - i + 1) for cs, dj in zip(cstar, d)) for i in range(1, beta + 1)]
    res.c0 = c0
    res.d = [mp.mpf(0)] + d
    res.c = [c0[0]] + [cs / dj ** beta for cs, dj in zip(cstar, d)]


def _partial_fractions(res: Bura):
    """Steps 1-2 of the method (Section 2.2): poles d_j and weights c_j of eq. (15)."""
    # roots of Q(t) = sum q_j t^j (Lemma 2.5: real, negative, simple)
    roots = mp.polyroots(list(reversed(res.q)), maxsteps=400, extraprec=4 * res.dps)
    d = []
    for z in roots:
        if abs(mp.im(z)) > mp.mpf(10) ** (-(res.dps // 3)) * (1 + abs(z)):
            raise RemezError("complex pole: partial fractions with p_2 > 0 are not covered")
        d.append(mp.re(z))
    if any(x >= 0 for x in d):
        raise RemezError("non-negative pole")
    d = sorted(d, reverse=True)            # 0 > d_1 > d_2 > ... > d_k
    dq = [i * res.q[i] for i in range(1, len(res.q))]
    c0 = _poly(res.p, 0) / _poly(res.q, 0)     # = r(0) = E, eq. (23)
    c = [c0] + [_poly(res.p, dj) / (dj * _poly(dq, dj)) for dj in d]
    res.d = [mp.mpf(0)] + d
    res.c = c
