"""GPU parity of the sinc-quadrature plans (the comparison method of Section 5.3) against the oracle."""

import json

import numpy as np
import pytest

import synth
from conftest import golden_path, oracle_coeffs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _B():
    import paper_1612_04846_amd as B
    return B


def _rel(u, ref):
    nb = u.shape[0]
    a, b = u.reshape(nb, -1), ref.reshape(nb, -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_table7_quadratures_1023(prec):
    """1023^2 checkerboard, k_Q = 9, 7, 6 in one plan (28 systems): each output
    against the oracle's eigenbasis evaluation, and Table 7's two rows recomputed
    from the GPU results."""
    from oracle import quadrature, spectral
    B = _B()
    g = json.load(open(golden_path("table7_2d_sinc.json")))
    n = g["h_inv"] - 1
    F = synth.checkerboard_rhs(n)[None]
    alphas = [r["alpha"] for r in g["rows"]]
    kps = [B.sinc_kprime(r["alpha"], r["kq"]) for r in g["rows"]]
    plan = B.Plan(2, n, alphas, kprime=kps, precision=getattr(B, "BURA_" + prec), tol=1e-10)
    Lam = plan.info[0]
    assert Lam == 8.0 * (n + 1) ** 2
    nout, begins = B.bura_plan_outputs(plan.handle)
    assert nout == 3 and begins == [0, 11, 20, 28]
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    plan.close()
    bplan = B.Plan(2, n, alphas, [r["k_bura"] for r in g["rows"]], precision=getattr(B, "BURA_" + prec), tol=1e-10)
    UR = bplan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    bplan.close()
    fn = np.linalg.norm(F)
    for i, (row, kp) in enumerate(zip(g["rows"], kps)):
        a = row["alpha"]
        ref = quadrature.sinc_spectral(F, 2, a, kp, Lam)
        err = _rel(U[i], ref)
        print(f"sinc 1023^2 alpha={a} k_Q={row['kq']} {prec}: rel err {err:.2e}")
        assert err <= 1e-8
        # Table 7: errors of u_Q and of the (k,k) 1-BURA against u_ref (the rule at
        # k' = 1/3), in the unscaled problem (outputs times Lambda^-alpha)
        uref = quadrature.sinc_spectral(F, 2, a, g["kprime_ref"], Lam)
        eq = np.linalg.norm(uref - U[i]) * Lam ** -a / fn
        assert abs(eq - row["err_q"]) <= 1e-3 * row["err_q"], (a, eq)
        b = oracle_coeffs(a, row["k_bura"])
        assert _rel(UR[i], spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)) <= 1e-8
        er = np.linalg.norm(uref - UR[i]) * Lam ** -a / fn
        assert er < eq
        print(f"   Table 7: BURA {er:.4e}, quadrature {eq:.4e}")


def test_quadrature_that_beats_bura_255():
    """alpha 0.25, k_Q = 38: 40 systems in one plan, N(0,1) rhs, two right-hand sides."""
    from oracle import quadrature
    B = _B()
    n, a, kq = 255, 0.25, 38
    F = synth.normal_rhs(n, 2, nrhs=2, tag=21)
    kp = B.sinc_kprime(a, kq)
    plan = B.Plan(2, n, a, kprime=kp, nrhs_max=2, precision=B.BURA_FP64, tol=1e-11)
    assert B.bura_plan_outputs(plan.handle)[1] == [0, 40]
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    ref = quadrature.sinc_spectral(F, 2, a, kp, plan.info[0])
    plan.close()
    assert _rel(U, ref) <= 1e-8


def test_variable_coefficient_sinc_against_sparse_solves():
    """127^2 a = exp(g), alpha 0.5, k_Q = 7: Lambda is the Gershgorin bound, same as the oracle's."""
    from oracle import operators, quadrature, shifted
    B = _B()
    n, a, kq = 127, 0.5, 7
    coeff = synth.lognormal_coefficient(n, 2, tag=22)
    F = synth.normal_rhs(n, 2, nrhs=1, tag=22)
    kp = B.sinc_kprime(a, kq)
    plan = B.Plan(2, n, a, kprime=kp, coeff=coeff, precision=B.BURA_MIXED, tol=1e-11)
    A, lam = operators.scaled_operator(n, 2, coeff)
    assert plan.info[0] == pytest.approx(lam, rel=1e-13)
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    plan.close()
    w, s = quadrature.sinc_terms(a, kp, lam)
    ref = shifted.bura_by_solves(A, w, -s, F)
    assert _rel(U, ref) <= 1e-8


def test_rational_multi_with_library_terms_equals_sinc_plan():
    """The same terms given explicitly through bura_plan_create_rational_multi give
    the same bits as the sinc plan."""
    B = _B()
    n = 63
    F = torch.from_numpy(synth.normal_rhs(n, 2, nrhs=1, tag=23)).cuda()
    alphas, kqs = [0.3, 0.7], [6, 9]
    kps = [B.sinc_kprime(a, q) for a, q in zip(alphas, kqs)]
    p1 = B.Plan(2, n, alphas, kprime=kps, precision=B.BURA_FP64, tol=1e-11)
    Lam = p1.info[0]
    ws, ss, nt = [], [], []
    for a, kp in zip(alphas, kps):
        w, s = B.bura_sinc_coefficients(a, kp, Lam)
        ws += w
        ss += s
        nt.append(len(w))
    p2 = B.Plan(2, n, weights=ws, shifts=ss, nterms=nt, precision=B.BURA_FP64, tol=1e-11)
    u1 = p1.solve(F).u
    u2 = p2.solve(F).u
    torch.cuda.synchronize()
    assert u1.shape == (2,) + tuple(F.shape)
    assert torch.equal(u1, u2)
    p1.close()
    p2.close()


def test_sinc_rejects_too_many_terms():
    B = _B()
    with pytest.raises(B.BuraError):
        B.Plan(2, 63, 0.5, kprime=0.2)      # 249 systems
