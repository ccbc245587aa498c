"""GPU parity of the sequential forms: multi-step BURA (Section 4.4) and the
zero-pole product form (remark in Section 2.2), against the oracle."""

import numpy as np
import pytest

import synth
from conftest import oracle_bura, oracle_coeffs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _B():
    import paper_1612_04846_amd as B
    return B


def _rel(u, ref):
    nb = u.shape[0]
    a, b = u.reshape(nb, -1), ref.reshape(nb, -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def _steps(alphas, ks):
    out = []
    for a, k in zip(alphas, ks):
        b = oracle_coeffs(a, k)
        out.append((b.c_f64, b.d_f64))
    return out


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
@pytest.mark.parametrize("alphas,ks", [((0.5, 0.25), (7, 7)), ((0.25, 0.25, 0.25), (5, 5, 5))])
def test_multistep_matches_oracle(prec, alphas, ks):
    from oracle import multistep
    B = _B()
    n = 255
    F = synth.normal_rhs(n, 2, nrhs=2, tag=51)
    plan = B.Plan(2, n, list(alphas), list(ks), form="multistep", nrhs_max=2,
                  precision=getattr(B, "BURA_" + prec), tol=1e-11)
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    plan.close()
    ref = multistep.multistep_spectral(F, 2, _steps(alphas, ks))
    err = _rel(U, ref)
    print(f"multistep {alphas} {prec}: rel err {err:.2e}")
    assert err <= 1e-8


def test_multistep_variable_coefficient_and_fewer_rhs():
    """127^2 a = exp(g), steps (0.3, 0.4); one right-hand side in a two-slot plan."""
    from oracle import multistep, operators
    B = _B()
    n = 127
    coeff = synth.lognormal_coefficient(n, 2, tag=52)
    F = synth.normal_rhs(n, 2, nrhs=1, tag=52)
    plan = B.Plan(2, n, [0.3, 0.4], [6, 6], form="multistep", coeff=coeff, nrhs_max=2,
                  precision=B.BURA_FP64, tol=1e-11)
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    plan.close()
    A, _ = operators.scaled_operator(n, 2, coeff)
    ref = multistep.multistep_by_solves(A, _steps([0.3, 0.4], [6, 6]), F)
    assert _rel(U, ref) <= 1e-8


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_product_form_matches_oracle_and_fractions(prec):
    from oracle import product, spectral
    B = _B()
    n, alpha, k = 255, 0.5, 7
    F = synth.normal_rhs(n, 2, nrhs=1, tag=53)
    plan = B.Plan(2, n, alpha, k, form="product", precision=getattr(B, "BURA_" + prec), tol=1e-11)
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    plan.close()
    b = oracle_bura(alpha, k)
    z, C = product.zeros_and_constant(b)
    assert _rel(U, product.product_spectral(F, 2, C, z, b.d)) <= 1e-8
    assert _rel(U, spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)) <= 1e-8


def test_product_form_3d_and_zero_rhs():
    from oracle import product
    B = _B()
    n, alpha, k = 31, 0.25, 6
    F = synth.normal_rhs(n, 3, nrhs=2, tag=54)
    F[1] = 0.0
    plan = B.Plan(3, n, alpha, k, form="product", nrhs_max=2, precision=B.BURA_MIXED, tol=1e-11)
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    plan.close()
    b = oracle_bura(alpha, k)
    z, C = product.zeros_and_constant(b)
    assert _rel(U[:1], product.product_spectral(F[:1], 3, C, z, b.d)) <= 1e-8
    assert np.all(U[1] == 0.0)


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_beta2_matches_oracle(prec):
    """2-BURA (Section 4.1), alpha 0.5, (m,k) = (7,6): 8 systems, the last one chained."""
    from oracle import remez, spectral
    B = _B()
    n, alpha, k = 255, 0.5, 6
    F = synth.normal_rhs(n, 2, nrhs=2, tag=55)
    plan = B.Plan(2, n, alpha, k, beta=2, nrhs_max=2, precision=getattr(B, "BURA_" + prec), tol=1e-12)
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    plan.close()
    o = remez.remez(alpha, k, m=k + 1, beta=2)
    ref = spectral.bura_beta_spectral(F, 2, o.c0, o.c, o.d)
    err = _rel(U, ref)
    print(f"beta=2 255^2 {prec}: rel err {err:.2e}")
    assert err <= 1e-8
    # and the 2-BURA approximates A^-alpha f within Lemma 2.1's bound
    Ue = spectral.exact_fractional(F, 2, alpha)
    A2f = spectral.apply_function(F, 2, lambda lam: lam ** -2.0)
    for r in range(2):
        assert np.linalg.norm(U[r] - Ue[r]) <= abs(float(o.E)) * np.linalg.norm(A2f[r]) * 1.001


def test_beta2_variable_coefficient_against_sparse_solves():
    from oracle import operators, remez, shifted
    B = _B()
    n, alpha, k = 127, 0.25, 4
    coeff = synth.lognormal_coefficient(n, 2, tag=56)
    F = synth.normal_rhs(n, 2, nrhs=1, tag=56)
    plan = B.Plan(2, n, alpha, k, beta=2, coeff=coeff, precision=B.BURA_FP64, tol=1e-12)
    U = plan.solve(torch.from_numpy(F).cuda()).u.cpu().numpy()
    plan.close()
    o = remez.remez(alpha, k, m=k + 1, beta=2)
    A, _ = operators.scaled_operator(n, 2, coeff)
    Fm = F.reshape(1, -1)
    v1 = shifted.shifted_solve_direct(A, 0.0, Fm)
    v2 = shifted.shifted_solve_direct(A, 0.0, v1)
    ref = float(o.c0[0]) * v1 + float(o.c0[1]) * v2
    for cj, dj in zip(o.c[1:], o.d[1:]):
        ref = ref + float(cj) * shifted.shifted_solve_direct(A, -float(dj), Fm)
    assert _rel(U, ref.reshape(F.shape)) <= 1e-8
