"""The allocation-free entry point bura_solve_static against the ordinary
bura_plan_create_rational + bura_solve path, through the C ABI.

Two calls in a row on one GPU (the second on a smaller problem, reusing the
same static scratch array), each compared with the plan-based result on the
same inputs and checked against the oracle's spectral evaluation of the same
partial fractions (eq. (16) in the sine eigenbasis); then a request whose
workspace does not fit the array is refused before anything runs.
"""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(u, ref):
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))


def _plan_result(B, dim, n, w, s, F, opts):
    plan = B.bura_plan_create_rational(dim, n, w, s, opts)
    try:
        f = _dev(F.reshape(F.shape[0], -1))
        u = torch.empty_like(f)
        B.bura_solve(plan, f, u, F.shape[0])
        return _host(u)
    finally:
        B._lib.bura_plan_destroy(plan)


def _static_result(B, dim, n, w, s, F, opts):
    f = _dev(F.reshape(F.shape[0], -1))
    u = torch.full_like(f, float("nan"))
    rep = B.bura_solve_static(dim, n, w, s, f, u, opts)
    return _host(u), rep


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_solve_matches_plan_solve_twice(order):
    import paper_1612_04846_amd as B
    from conftest import oracle_coeffs
    from oracle import spectral

    cases = [
        # (dim, n, alpha, k, precision, nrhs, tag): the second is smaller
        (2, 127, 0.5, 7, B.BURA_FP64, 2, 701),
        (2, 63, 0.25, 5, B.BURA_MIXED, 1, 702),
    ]
    for dim, n, alpha, k, prec, nrhs, tag in cases:
        print(f"static solve: dim={dim} n={n} alpha={alpha} k={k} prec={prec} nrhs={nrhs}", flush=True)
        b = oracle_coeffs(alpha, k)
        w, s = b.c_f64, [-x for x in b.d_f64]
        F = synth.normal_rhs(n, dim, nrhs=nrhs, tag=tag)
        opts = B.bura_opts_default(precision=prec, tol=1e-11, nrhs_max=nrhs)
        u_static, rep = _static_result(B, dim, n, w, s, F, opts)
        u_plan = _plan_result(B, dim, n, w, s, F, opts)
        assert rep.status == B.BURA_OK
        assert np.isfinite(u_static).all()
        # same kernels, launch shapes and reduction order as the plan path
        assert _rel(u_static.ravel(), u_plan.ravel()) <= 1e-12
        ref = spectral.bura_spectral(F, dim, w, b.d_f64)
        assert _rel(u_static.reshape(F.shape), ref) <= 1e-8


def test_static_solve_refuses_a_workspace_beyond_the_array():
    import paper_1612_04846_amd as B
    n, dim = 1023, 2
    w, s = [0.5, 0.5], [0.0, 1.0]
    F = np.ones((1, n * n))
    f = _dev(F)
    u = torch.full_like(f, 7.0)
    opts = B.bura_opts_default(precision=B.BURA_FP64, tol=1e-10)
    rep = B.bura_solve_static(dim, n, w, s, f, u, opts, ok=(B.BURA_ETOOBIG,))
    assert rep.status == B.BURA_ETOOBIG
    assert float(_host(u).min()) == 7.0 and float(_host(u).max()) == 7.0
