"""The certified error bound of every report and its enforcement (opts.err_tol).

A residual test alone does not bound the error of u_r = sum_j c_j (A - d_j)^-1 f:
a residual left in the lowest mode is amplified by 1/(lambda_min + s_j), and
the poles next to 0 carry large weights for alpha = 0.75.  The report's
err_bound is sum_j |c_j| |r_j| / (lam_lb + s_j) / |u| with a guaranteed lower
bound lam_lb of the spectrum; these tests check that it is a true upper bound
of the error against the oracle, and that err_tol makes the solve meet it.
"""


import numpy as np
import pytest

import synth
from conftest import oracle_coeffs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _B():
    import paper_1612_04846_amd as B
    return B


def _solve(B, n, alpha, k, F, **kw):
    plan = B.Plan(2, n, alpha, k, **kw)
    res = plan.solve(torch.from_numpy(np.ascontiguousarray(F)).cuda(), ok=(B.BURA_OK, B.BURA_ENOCONV))
    torch.cuda.synchronize()
    u = res.u.cpu().numpy()
    plan.close()
    return u, res.report


def test_lowest_mode_alpha075_k9_1023():
    """f = the lowest sine mode psi_1 at 1023^2, alpha = 0.75, k = 9, tol 1e-10:
    u_r = r(lambda_1)/lambda_1 psi_1 exactly (Section 5.1's eigenvector input,
    eq. (16) in the eigenbasis), and the solve with err_tol = 1e-8 certifies and
    meets 1e-8 against it."""
    from oracle import spectral
    B = _B()
    n, alpha, k = 1023, 0.75, 9
    psi = synth.sine_mode(n, (1, 1))[None]
    b = oracle_coeffs(alpha, k)
    lam1 = float(spectral.eigenvalues(n, 2)[0, 0])
    rho = sum(c / (lam1 - d) for c, d in zip(b.c_f64, b.d_f64))
    ref = rho * psi
    for prec in (B.BURA_MIXED, B.BURA_FP64):
        kw = dict(precision=prec, tol=1e-10)
        if prec == B.BURA_MIXED:
            kw["err_tol"] = 1e-8
        u, rep = _solve(B, n, alpha, k, psi, **kw)
        err = float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
        print(f"lowest mode prec={prec}: rel err {err:.2e}, bound {rep.err_bound:.2e}, status {rep.status}")
        assert rep.status == B.BURA_OK
        assert err <= 1e-8
        # (the plan's coefficients are the library's, within 1e-11 of the oracle's)
        assert err <= rep.err_bound + 1e-10
        if prec == B.BURA_MIXED:
            assert rep.err_bound <= 1e-8


@pytest.mark.parametrize("prec", ["MIXED", "FP64"])
def test_bound_holds_on_random_rhs(prec):
    """The reported bound is an upper bound of the actual error against the
    oracle's DST evaluation of the same terms (alpha = 0.75, k = 9, 511^2)."""
    from oracle import spectral
    B = _B()
    n, alpha, k = 511, 0.75, 9
    F = synth.normal_rhs(n, 2, nrhs=2, tag=171)
    u, rep = _solve(B, n, alpha, k, F, precision=getattr(B, "BURA_" + prec), tol=1e-10, nrhs_max=2)
    b = oracle_coeffs(alpha, k)
    ref = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    err = max(float(np.linalg.norm(u[r] - ref[r]) / np.linalg.norm(u[r])) for r in range(2))
    print(f"random rhs {prec}: rel err {err:.2e}, bound {rep.err_bound:.2e}")
    assert rep.status == B.BURA_OK
    assert 0.0 < rep.err_bound and err <= rep.err_bound + 1e-10


def test_err_tol_tightens_the_refinement():
    """Random f at 511^2, alpha = 0.75, k = 9, tol 1e-4: the residual test alone
    stops after one refinement step with a bound far above 1e-8; with err_tol =
    1e-8 the refinement continues on the systems that need it until the
    certified bound is met, and the error against the oracle is within it."""
    from oracle import spectral
    B = _B()
    n, alpha, k = 511, 0.75, 9
    F = synth.normal_rhs(n, 2, nrhs=1, tag=172)
    u0, rep0 = _solve(B, n, alpha, k, F, precision=B.BURA_MIXED, tol=1e-4)
    u1, rep1 = _solve(B, n, alpha, k, F, precision=B.BURA_MIXED, tol=1e-4, err_tol=1e-8)
    b = oracle_coeffs(alpha, k)
    ref = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    e0 = float(np.linalg.norm(u0 - ref) / np.linalg.norm(u0))
    e1 = float(np.linalg.norm(u1 - ref) / np.linalg.norm(u1))
    print(f"tol 1e-4: err {e0:.2e} bound {rep0.err_bound:.2e} outer {list(rep0.outer)[:k + 1]}; "
          f"err_tol 1e-8: err {e1:.2e} bound {rep1.err_bound:.2e} outer {list(rep1.outer)[:k + 1]}")
    assert rep0.err_bound > 1e-8
    assert rep1.status == B.BURA_OK and rep1.err_bound <= 1e-8
    assert e1 <= rep1.err_bound + 1e-10 and e0 <= rep0.err_bound + 1e-10
    assert max(list(rep1.outer)[:k + 1]) > max(list(rep0.outer)[:k + 1])


def test_err_tol_on_slot_plan():
    """Per-rhs terms (slot plans): the bound is formed per rhs from its own
    weights and shifts, and err_tol is met for each."""
    from oracle import spectral
    B = _B()
    n, K = 255, 12
    F = synth.normal_rhs(n, 2, nrhs=2, tag=173)
    terms = []
    pairs = ((0.75, 9), (0.3, 6))
    for a, k in pairs:
        c, d, _ = B.bura_coefficients(a, k)
        terms.append((c, [-x for x in d]))
    plan = B.bura_plan_create_slots(2, n, K, B.bura_opts_default(nrhs_max=2, tol=1e-4, err_tol=1e-9))
    Fd = torch.from_numpy(F).cuda()
    U = torch.empty_like(Fd)
    rep = B.bura_solve_slots(plan, K, Fd, U, terms)
    torch.cuda.synchronize()
    u = U.cpu().numpy()
    B.bura_plan_destroy(plan)
    assert rep.status == B.BURA_OK and rep.err_bound <= 1e-9
    for r, (a, k) in enumerate(pairs):
        b = oracle_coeffs(a, k)
        ref = spectral.bura_spectral(F[r:r + 1], 2, b.c_f64, b.d_f64)[0]
        assert float(np.linalg.norm(u[r] - ref) / np.linalg.norm(u[r])) <= 1e-9 + 1e-10
