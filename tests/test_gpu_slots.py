"""Slot plans: per-right-hand-side partial-fraction terms and tolerances in one batched solve.

Right-hand side r of a slot-plan solve is mapped to
u_r = sum_j w_rj (A + s_rj I)^-1 f_r (eq. (16) with its own weights and
shifts).  Checked against the oracle (spectral for constant coefficients,
sparse direct shifted solves for variable ones), and bit for bit against the
ordinary plan for the same (alpha, k, tol) solved alone: a system's
arithmetic does not depend on its slot or on the other systems of the batch.
"""

import numpy as np
import pytest

import synth
from conftest import oracle_coeffs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K = 13   # term slots per rhs (k <= 12)


def _B():
    import paper_1612_04846_amd as B
    return B


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(u, ref):
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))


MIX = [  # alpha, k, tol
    (0.25, 5, 1e-11),
    (0.5, 9, 1e-12),
    (0.75, 9, 1e-10),
]


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_slots_match_oracle_and_single_plans_bitwise(prec):
    from oracle import spectral
    B = _B()
    n = 127
    P = getattr(B, "BURA_" + prec)
    F = synth.normal_rhs(n, 2, nrhs=len(MIX), tag=501)
    terms = []
    for a, k, _ in MIX:
        c, d, _E = B.bura_coefficients(a, k)
        terms.append((c, [-x for x in d]))
    plan = B.bura_plan_create_slots(2, n, K, B.bura_opts_default(precision=P, nrhs_max=4))
    Fd = _dev(F)
    U = torch.empty_like(Fd)
    rep = B.bura_solve_slots(plan, K, Fd, U, terms, tols=[t for _, _, t in MIX])
    u = _host(U)
    assert rep.nterms == max(k for _, k, _ in MIX) + 1
    for r, (a, k, tol) in enumerate(MIX):
        b = oracle_coeffs(a, k)
        ref = spectral.bura_spectral(F[r:r + 1], 2, b.c_f64, b.d_f64)[0]
        err = _rel(u[r], ref)
        print(f"{prec} slot rhs {r}: alpha={a} k={k} tol={tol:g} rel err vs oracle {err:.2e}")
        assert err <= 1e-8
        single = B.Plan(2, n, a, k, precision=P, tol=tol)
        us = _host(single.solve(_dev(F[r:r + 1])).u)[0]
        single.close()
        assert np.array_equal(us, u[r])
    # a second solve on the same plan with fewer rhs and fewer terms: no state leaks
    U2 = torch.empty_like(Fd[:1])
    B.bura_solve_slots(plan, K, Fd[1:2].contiguous(), U2, [terms[0]], tols=[MIX[0][2]])
    single = B.Plan(2, n, MIX[0][0], MIX[0][1], precision=P, tol=MIX[0][2])
    assert np.array_equal(_host(U2)[0], _host(single.solve(_dev(F[1:2])).u)[0])
    single.close()
    B.bura_plan_destroy(plan)


def test_slots_variable_coefficient_and_arbitrary_terms():
    """Caller-given terms (not a BURA) on a variable-coefficient grid, against direct solves."""
    from oracle import operators, shifted
    B = _B()
    n = 63
    coeff = synth.lognormal_coefficient(n, 2, tag=511)
    A, _ = operators.scaled_operator(n, 2, coeff)
    F = synth.normal_rhs(n, 2, nrhs=2, tag=512)
    terms = [([0.7, 0.2, 0.1], [0.0, 0.05, 2.0]), ([1.5], [0.3])]
    plan = B.bura_plan_create_slots(2, n, 4, B.bura_opts_default(precision=B.BURA_FP64, nrhs_max=2), coeff=coeff)
    Fd = _dev(F)
    U = torch.empty_like(Fd)
    B.bura_solve_slots(plan, 4, Fd, U, terms)
    u = _host(U)
    for r, (w, s) in enumerate(terms):
        ref = shifted.bura_by_solves(A, w, [-x for x in s], F[r:r + 1])[0]
        assert _rel(u[r], ref) <= 1e-9
    B.bura_plan_destroy(plan)


def test_slots_async_submit_and_poll():
    import time
    from oracle import spectral
    B = _B()
    n = 63
    F = synth.normal_rhs(n, 2, nrhs=2, tag=521)
    terms = []
    for a, k in ((0.3, 6), (0.6, 8)):
        c, d, _ = B.bura_coefficients(a, k)
        terms.append((c, [-x for x in d]))
    plan = B.bura_plan_create_slots(2, n, K, B.bura_opts_default(nrhs_max=2))
    Fd = _dev(F)
    U = torch.empty_like(Fd)
    ticket = B.bura_submit_slots(plan, K, Fd, U, terms, tols=[1e-12, 1e-12])
    t0 = time.time()
    while True:
        code, rep = B.bura_poll(ticket)
        if code != B.BURA_PENDING:
            break
        assert time.time() - t0 < 60
        time.sleep(0.001)
    assert code == B.BURA_OK
    u = _host(U)
    for r, (a, k) in enumerate(((0.3, 6), (0.6, 8))):
        b = oracle_coeffs(a, k)
        ref = spectral.bura_spectral(F[r:r + 1], 2, b.c_f64, b.d_f64)[0]
        assert _rel(u[r], ref) <= 1e-9
    B.bura_plan_destroy(plan)


def test_slots_argument_errors():
    B = _B()
    n = 31
    plan = B.bura_plan_create_slots(2, n, 4, B.bura_opts_default(nrhs_max=2))
    F = _dev(synth.normal_rhs(n, 2, nrhs=1, tag=531))
    U = torch.empty_like(F)
    with pytest.raises(B.BuraError) as ei:    # an ordinary solve on a slot plan
        B.bura_solve(plan, F, U, 1)
    assert ei.value.code == B.BURA_EINVAL
    with pytest.raises(B.BuraError) as ei:    # more terms than the plan's 4 slots (arrays laid out for 5)
        B.bura_solve_slots(plan, 5, F, U, [([1.0] * 5, [0.0] * 5)])
    assert ei.value.code == B.BURA_EINVAL
    with pytest.raises(B.BuraError):          # negative shift
        B.bura_solve_slots(plan, 4, F, U, [([1.0], [-0.5])])
    with pytest.raises(B.BuraError):          # non-positive tolerance
        B.bura_solve_slots(plan, 4, F, U, [([1.0], [0.5])], tols=[0.0])
    B.bura_plan_destroy(plan)
    with pytest.raises(B.BuraError) as ei:
        B.bura_plan_create_slots(2, n, 4, B.bura_opts_default(schedule=B.BURA_PER_POLE))
    assert ei.value.code == B.BURA_EUNSUPPORTED
    p = B.Plan(2, n, 0.5, 5)
    with pytest.raises(B.BuraError):          # a slot solve on an ordinary plan
        B.bura_solve_slots(p.handle, 6, F, U, [([1.0], [0.5])])
    p.close()
