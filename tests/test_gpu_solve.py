"""GPU parity: the HIP path (through the C ABI) against the oracle.

Tolerances: the solver stops on the FP64 relative residual (tol); the
combined result is compared with the oracle's u_r for the same c_j, d_j
element by element through the relative l2 error and the max-norm error
relative to max |u_r|.
"""

import numpy as np
import pytest

import synth
from conftest import oracle_coeffs as oracle_bura

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _B():
    import paper_1612_04846_amd as B
    return B


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _errs(u, ref):
    rel2 = np.linalg.norm((u - ref).reshape(u.shape[0], -1), axis=1) / np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)
    relinf = np.abs(u - ref).max() / np.abs(ref).max()
    return float(rel2.max()), float(relinf)


# ----------------------------------------------------------------------------
# operator and scaling (Section 1.4 eq. (10), Section 5.3)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,var", [(2, 31, False), (3, 15, False), (2, 33, True), (3, 9, True), (2, 64, False)])
def test_apply_matches_oracle_operator(dim, n, var):
    from oracle import operators
    B = _B()
    coeff = synth.lognormal_coefficient(n, dim, tag=21) if var else None
    A, lam = operators.scaled_operator(n, dim, coeff)
    plan = B.Plan(dim, n, weights=[1.0], shifts=[0.0], coeff=coeff, precision=B.BURA_FP64)
    lam_gpu, nlev, _ = plan.info
    assert lam_gpu == pytest.approx(lam, rel=1e-13)
    X = synth.normal_rhs(n, dim, nrhs=2, tag=22)
    for shift in (0.0, 0.37):
        y = _host(plan.apply(_dev(X), shift))
        ref = np.stack([A @ X[i].ravel() + shift * X[i].ravel() for i in range(2)]).reshape(X.shape)
        assert np.max(np.abs(y - ref)) <= 1e-14 * np.max(np.abs(ref)) * 8
    plan.close()


# ----------------------------------------------------------------------------
# full solve with the oracle's coefficients (isolates the solver)
# ----------------------------------------------------------------------------

CASES = [
    # dim, n, alpha, k, precision, schedule
    (2, 63, 0.5, 5, "FP64", "BATCHED"),
    (2, 63, 0.5, 5, "MIXED", "BATCHED"),
    (2, 64, 0.5, 5, "FP64", "BATCHED"),      # 64x64 grid: no coarsening, Jacobi-PCG
    (2, 37, 0.25, 7, "MIXED", "PER_POLE"),   # ragged: 37 -> 18, coarse level not 1 point
    (3, 31, 0.25, 8, "MIXED", "BATCHED"),
    (3, 15, 0.75, 7, "FP64", "PER_POLE"),
    (2, 127, 0.75, 9, "MIXED", "BATCHED"),
]


@pytest.mark.parametrize("dim,n,alpha,k,prec,sched", CASES)
def test_solve_matches_spectral_oracle(dim, n, alpha, k, prec, sched):
    from oracle import spectral
    B = _B()
    b = oracle_bura(alpha, k)
    c, d = b.c_f64, b.d_f64
    F = synth.normal_rhs(n, dim, nrhs=2, tag=31)
    plan = B.Plan(dim, n, weights=c, shifts=[-x for x in d], nrhs_max=2,
                  precision=getattr(B, "BURA_" + prec), schedule=getattr(B, "BURA_" + sched), tol=1e-12)
    res = plan.solve(_dev(F))
    u = _host(res.u)
    ref = spectral.bura_spectral(F, dim, c, d)
    rel2, relinf = _errs(u, ref)
    print(f"dim={dim} n={n} a={alpha} k={k} {prec} {sched} rel2={rel2:.2e} relinf={relinf:.2e} "
          f"iters={list(res.report.iters)[:k+1]} outer={list(res.report.outer)[:k+1]}")
    assert rel2 <= 1e-9 and relinf <= 1e-9
    plan.close()


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_variable_coefficient_matches_direct_solves(prec):
    from oracle import operators, shifted
    B = _B()
    n, dim, alpha, k = 63, 2, 0.6, 7
    b = oracle_bura(alpha, k)
    coeff = synth.lognormal_coefficient(n, dim, tag=41)
    A, _ = operators.scaled_operator(n, dim, coeff)
    F = synth.normal_rhs(n, dim, nrhs=3, tag=42)
    ref = shifted.bura_by_solves(A, b.c_f64, b.d_f64, F)
    plan = B.Plan(dim, n, weights=b.c_f64, shifts=[-x for x in b.d_f64], coeff=coeff, nrhs_max=3,
                  precision=getattr(B, "BURA_" + prec), tol=1e-12)
    res = plan.solve(_dev(F))
    rel2, relinf = _errs(_host(res.u), ref)
    print(f"var {prec} rel2={rel2:.2e} relinf={relinf:.2e} iters={list(res.report.iters)[:k+1]}")
    assert rel2 <= 1e-9 and relinf <= 1e-9
    plan.close()


@pytest.mark.parametrize("prec", ["FP64", "MIXED"])
def test_variable_coefficient_3d_matches_direct_solves(prec):
    """3D, variable coefficients: the first fine sweep forms (A + s) p from p
    with the face weights while marching along z (no q stored)."""
    from oracle import operators, shifted
    B = _B()
    n, dim, alpha, k = 23, 3, 0.6, 5   # 23 -> 11 -> 5 -> 2: the fine level is outside LDS
    b = oracle_bura(alpha, k)
    coeff = synth.lognormal_coefficient(n, dim, tag=43)
    A, _ = operators.scaled_operator(n, dim, coeff)
    F = synth.normal_rhs(n, dim, nrhs=2, tag=44)
    ref = shifted.bura_by_solves(A, b.c_f64, b.d_f64, F)
    plan = B.Plan(dim, n, weights=b.c_f64, shifts=[-x for x in b.d_f64], coeff=coeff, nrhs_max=2,
                  precision=getattr(B, "BURA_" + prec), tol=1e-12)
    _, nlev, _ = plan.info
    assert nlev >= 2
    res = plan.solve(_dev(F))
    rel2, relinf = _errs(_host(res.u), ref)
    print(f"var 3D {prec} levels={nlev} rel2={rel2:.2e} relinf={relinf:.2e} iters={list(res.report.iters)[:k+1]}")
    assert rel2 <= 1e-9 and relinf <= 1e-9
    plan.close()


@pytest.mark.parametrize("n,prec", [(191, "FP64"), (95, "MIXED")])
def test_3d_march_widths_with_ragged_tiles(n, prec):
    """3D marching workgroups are 256, 128 or 64 columns wide by grid size:
    191 -> 95 -> 47 -> 23 runs 128-column workgroups over a ragged second tile
    (63 columns) and 64-column ones below, 95 starts at 64 columns."""
    from oracle import spectral
    B = _B()
    alpha, k = 0.5, 5
    b = oracle_bura(alpha, k)
    F = synth.normal_rhs(n, 3, nrhs=1, tag=71)
    plan = B.Plan(3, n, weights=b.c_f64, shifts=[-x for x in b.d_f64], precision=getattr(B, "BURA_" + prec),
                  tol=1e-12)
    res = plan.solve(_dev(F))
    u = _host(res.u)
    ref = spectral.bura_spectral(F, 3, b.c_f64, b.d_f64)
    err = float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    print(f"3D {n} {prec}: rel err {err:.2e}, iters {list(res.report.iters)[:k + 1]}")
    assert err <= 1e-9
    plan.close()


FUSED3D_CASES = [
    # n, precision, sweeps: 63 -> 31 -> 15 (whole tiles at the top level are
    # ragged: 31 coarse columns of 32, 31 coarse rows of 8, one z segment),
    # 127 (four coarse rows of tiles, one segment of 16 coarse planes and a
    # short one), 47 (an even coarsest level), one sweep
    (63, "FP64", 2), (63, "MIXED", 2), (127, "MIXED", 2), (47, "MIXED", 2), (63, "MIXED", 1), (31, "FP64", 1),
]


@pytest.mark.parametrize("n,prec,nu", FUSED3D_CASES)
def test_fused_3d_levels_match_unfused_and_oracle(n, prec, nu):
    """The z-marching fused 3D level kernels (constant coefficients) against
    the one-kernel-per-step V-cycle (BURA_VARIANT_UNFUSED) and the oracle: the
    same preconditioner up to rounding, so both solutions agree to the solver
    tolerance and match the DST evaluation of eq. (16); with and without the
    PCG updates folded into the level kernels."""
    from oracle import spectral
    B = _B()
    alpha, k = 0.75, 7
    b = oracle_bura(alpha, k)
    F = synth.normal_rhs(n, 3, nrhs=2, tag=97)
    ref = spectral.bura_spectral(F, 3, b.c_f64, b.d_f64)
    kw = dict(weights=b.c_f64, shifts=[-x for x in b.d_f64], precision=getattr(B, "BURA_" + prec), nrhs_max=2,
              tol=1e-12, nu_pre=nu, nu_post=nu)
    out = {}
    for name, v in (("fused", 0), ("fused-sep", B.BURA_VARIANT_NO_FOLDXR), ("unfused", B.BURA_VARIANT_UNFUSED)):
        plan = B.Plan(3, n, variant=v, **kw)
        res = plan.solve(_dev(F))
        out[name] = (_host(res.u), list(res.report.iters)[:k + 1])
        plan.close()
    for name, (u, it) in out.items():
        err = float(np.max(np.linalg.norm((u - ref).reshape(2, -1), axis=1) / np.linalg.norm(ref.reshape(2, -1), axis=1)))
        print(f"3D {n} {prec} nu={nu} {name}: rel err {err:.2e}, iters {it}")
        assert err <= 1e-9
    # same preconditioner: the iteration counts agree within one per pole
    assert all(abs(a - c) <= 1 for a, c in zip(out["fused"][1], out["unfused"][1]))


def test_q_buffer_only_where_a_kernel_reads_q():
    """Plans whose residual update forms q = (A + s) p from p (fused 2D down
    kernel) hold one vector per system less than the 2D unfused plan, whose
    first sweep reads q; nothing else differs between the two."""
    B = _B()
    n, k = 255, 5
    fused = B.Plan(2, n, 0.5, k, nrhs_max=2, precision=B.BURA_FP64)
    unfused = B.Plan(2, n, 0.5, k, nrhs_max=2, precision=B.BURA_FP64, variant=B.BURA_VARIANT_UNFUSED)
    try:
        bf, bu = fused.info[2], unfused.info[2]
        assert bu - bf == (k + 1) * 2 * n * n * 8
    finally:
        fused.close()
        unfused.close()


def test_batched_equals_per_pole_and_alone_equals_mixed():
    """The same system gives bit-identical results whatever else is in the launch."""
    B = _B()
    b = oracle_bura(0.5, 5)
    n = 63
    F = synth.normal_rhs(n, 2, nrhs=3, tag=51)
    kw = dict(weights=b.c_f64, shifts=[-x for x in b.d_f64], precision=B.BURA_MIXED, tol=1e-12)
    p3 = B.Plan(2, n, nrhs_max=3, **kw)
    u3 = _host(p3.solve(_dev(F)).u)
    pp = B.Plan(2, n, nrhs_max=3, schedule=B.BURA_PER_POLE, **kw)
    upp = _host(pp.solve(_dev(F)).u)
    p1 = B.Plan(2, n, nrhs_max=1, **kw)
    u1 = np.stack([_host(p1.solve(_dev(F[i:i + 1])).u)[0] for i in range(3)])
    assert np.array_equal(u3, upp)
    assert np.array_equal(u3, u1)
    for p in (p3, pp, p1):
        p.close()


def test_zero_rhs_gives_zero():
    B = _B()
    b = oracle_bura(0.5, 5)
    plan = B.Plan(2, 31, weights=b.c_f64, shifts=[-x for x in b.d_f64], nrhs_max=2)
    F = np.zeros((2, 31, 31))
    F[1] = synth.normal_rhs(31, 2, tag=61)[0]
    u = _host(plan.solve(_dev(F)).u)
    assert np.all(u[0] == 0.0)
    assert np.abs(u[1]).max() > 0
    plan.close()


def test_fewer_rhs_than_slots():
    from oracle import spectral
    B = _B()
    b = oracle_bura(0.5, 5)
    plan = B.Plan(2, 31, weights=b.c_f64, shifts=[-x for x in b.d_f64], nrhs_max=4)
    F = synth.normal_rhs(31, 2, nrhs=2, tag=62)
    u = _host(plan.solve(_dev(F)).u)
    ref = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    assert _errs(u, ref)[0] <= 1e-9
    plan.close()


def test_nan_input_reports_enan():
    B = _B()
    b = oracle_bura(0.5, 5)
    plan = B.Plan(2, 15, weights=b.c_f64, shifts=[-x for x in b.d_f64])
    F = synth.normal_rhs(15, 2, tag=63)
    F[0, 3, 3] = np.nan
    res = plan.solve(_dev(F), ok=(B.BURA_OK, B.BURA_ENAN, B.BURA_ENOCONV))
    assert res.report.status == B.BURA_ENAN
    plan.close()


# ----------------------------------------------------------------------------
# full path: coefficients from the library's own Remez (bura_plan_create)
# ----------------------------------------------------------------------------

FULL = [
    (2, 63, 0.5, 5, "MIXED"),
    (2, 127, 0.25, 9, "FP64"),
    (2, 255, 0.75, 9, "MIXED"),
    (3, 31, 0.25, 8, "MIXED"),
    (2, 64, 0.5, 5, "FP64"),
]


@pytest.mark.parametrize("dim,n,alpha,k,prec", FULL)
def test_full_path_matches_oracle(dim, n, alpha, k, prec):
    """u from bura_plan_create (library Remez + GPU solves) vs the oracle's own u_r."""
    from oracle import metrics, spectral
    B = _B()
    b = oracle_bura(alpha, k)
    F = synth.uniform_rhs(n, dim, nrhs=1, tag=71)
    plan = B.Plan(dim, n, alpha, k, precision=getattr(B, "BURA_" + prec), tol=1e-12)
    c_lib, d_lib, E_lib = plan.coeffs
    assert E_lib == pytest.approx(float(b.E), rel=1e-10)
    res = plan.solve(_dev(F))
    u = _host(res.u)
    ref = spectral.bura_spectral(F, dim, b.c_f64, b.d_f64)
    rel2, relinf = _errs(u, ref)
    # and the BURA error bound of Lemma 2.1 (gamma = 0) against the exact A^-alpha f
    exact = spectral.exact_fractional(F, dim, alpha)
    lhs, rhs = metrics.lemma_bound_sides(F, u, dim, alpha, float(b.E), 0.0)
    print(f"full dim={dim} n={n} a={alpha} k={k} {prec}: rel2={rel2:.2e} relinf={relinf:.2e} "
          f"bura_err={metrics.rel_err(u, exact):.2e} lemma lhs/rhs={float(lhs[0] / rhs[0]):.3f}")
    assert rel2 <= 1e-9 and relinf <= 1e-9
    assert np.all(lhs <= rhs * (1 + 1e-6))
    plan.close()


def test_tickets_several_in_flight_on_one_plan():
    """Three solves queued on one plan before the first completes (two
    right-hand-side batches, one with its own tolerance): each ticket's result
    is bit-identical to the synchronous solve of the same inputs, tickets are
    distinct and released by the poll that returns them."""
    B = _B()
    n = 63
    F1 = _dev(synth.normal_rhs(n, 2, nrhs=2, tag=81))
    F2 = _dev(synth.normal_rhs(n, 2, nrhs=2, tag=82))
    plan = B.Plan(2, n, 0.5, 5, nrhs_max=2, precision=B.BURA_FP64, tol=1e-12)
    loose = B.Plan(2, n, 0.5, 5, nrhs_max=2, precision=B.BURA_FP64, tol=1e-8)
    u1 = _host(plan.solve(F1).u)
    u2 = _host(plan.solve(F2).u)
    u3 = _host(loose.solve(F1).u)
    U = [torch.empty_like(F1) for _ in range(3)]
    torch.cuda.synchronize()
    t1 = B.bura_submit(plan.handle, F1, U[0], 2)
    t2 = B.bura_submit(plan.handle, F2, U[1], 2)
    t3 = B.bura_submit(plan.handle, F1, U[2], 2, tol=1e-8)
    assert len({t1, t2, t3}) == 3 and 0 not in (t1, t2, t3)
    code3, rep3 = B.bura_wait(t3)        # the last one: the others ran before it
    assert code3 == B.BURA_OK and max(rep3.relres[:6]) <= 1e-8
    code1, rep1 = B.bura_poll(t1)
    code2, rep2 = B.bura_wait(t2)
    assert code1 == B.BURA_OK and code2 == B.BURA_OK
    assert max(rep1.relres[:6]) <= 1e-12
    assert B.bura_poll(t1)[0] == B.BURA_EINVAL   # released
    assert np.array_equal(_host(U[0]), u1)
    assert np.array_equal(_host(U[1]), u2)
    assert np.array_equal(_host(U[2]), u3)
    plan.close()
    loose.close()


def test_unscaled_rhs_returns_lambda_scaled_result():
    """rhs_unscaled = 1: f is f~ of the unscaled A~^alpha u = f~, and the plan
    returns Lambda^-alpha A^-alpha f~ (Section 1.4, eq. (10)), Lambda = 4 dim/h^2
    for the Laplacian (Section 5.3's scaling); for the BURA, the multi-step and
    the product forms, in FP64 and mixed precision."""
    from conftest import oracle_coeffs
    from oracle import spectral
    B = _B()
    n, dim = 127, 2
    lam = 4.0 * dim * (n + 1) ** 2
    F = synth.normal_rhs(n, dim, nrhs=1, tag=83)
    cases = [
        ("bura", dict(alpha=0.5, k=7), 0.5, [(0.5, 7)]),
        ("product", dict(alpha=0.25, k=6, form="product"), 0.25, [(0.25, 6)]),
        ("multistep", dict(alpha=[0.5, 0.25], k=[7, 6], form="multistep"), 0.75, [(0.5, 7), (0.25, 6)]),
    ]
    for name, kw, alpha, steps in cases:
        for prec in (B.BURA_FP64, B.BURA_MIXED):
            alpha_arg = kw.pop("alpha")
            k_arg = kw.pop("k")
            plan = B.Plan(dim, n, alpha_arg, k_arg, precision=prec, tol=1e-12, rhs_unscaled=1, **kw)
            kw.update(alpha=alpha_arg, k=k_arg)
            u = _host(plan.solve(_dev(F)).u)
            ref = F
            for a, k in steps:
                b = oracle_coeffs(a, k)
                ref = spectral.bura_spectral(ref, dim, b.c_f64, b.d_f64)
            ref = lam ** (-alpha) * ref
            err = float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
            print(f"unscaled {name} prec={prec}: rel err {err:.2e}")
            assert err <= 1e-9
            plan.close()


def test_multi_alpha_plan_equals_single_plans():
    """All poles of several alphas in one batch: each output bit-identical to its own plan."""
    from oracle import spectral
    B = _B()
    n = 63
    alphas, k = [0.25, 0.5, 0.75], 7
    F = synth.normal_rhs(n, 2, nrhs=2, tag=91)
    pm = B.Plan(2, n, alphas, k, nrhs_max=2, precision=B.BURA_FP64, tol=1e-12)
    um = _host(pm.solve(_dev(F)).u)
    assert um.shape == (3, 2, n, n)
    for i, a in enumerate(alphas):
        p1 = B.Plan(2, n, a, k, nrhs_max=2, precision=B.BURA_FP64, tol=1e-12)
        u1 = _host(p1.solve(_dev(F)).u)
        assert np.array_equal(um[i], u1)
        b = oracle_bura(a, k)
        assert _errs(um[i], spectral.bura_spectral(F, 2, b.c_f64, b.d_f64))[0] <= 1e-9
        p1.close()
    nout, tb = B.bura_plan_outputs(pm.handle)
    assert nout == 3 and tb == [0, 8, 16, 24]
    pm.close()


def test_folded_scalars_match_separate_launches():
    """Scalar updates folded into the producing kernels (opt-in) give the same bits as separate launches,
    with and without graph replay."""
    B = _B()
    n = 63
    F = _dev(synth.normal_rhs(n, 2, nrhs=1, tag=92))
    u_sep = _host(B.Plan(2, n, 0.5, 5, precision=B.BURA_MIXED).solve(F).u)
    u_fold = _host(B.Plan(2, n, 0.5, 5, precision=B.BURA_MIXED, variant=B.BURA_VARIANT_FOLD_SCALARS).solve(F).u)
    u_eager = _host(B.Plan(2, n, 0.5, 5, precision=B.BURA_MIXED,
                           variant=B.BURA_VARIANT_FOLD_SCALARS | B.BURA_VARIANT_NO_GRAPH).solve(F).u)
    assert np.array_equal(u_fold, u_sep)
    assert np.array_equal(u_eager, u_sep)


FOLD_CASES = [  # dim, n, precision, one kernel per V-cycle step (BURA_VARIANT_UNFUSED)
    (2, 255, "FP64", False), (2, 255, "MIXED", False),
    (3, 63, "FP64", False), (3, 63, "MIXED", False), (2, 127, "MIXED", True),
]


@pytest.mark.parametrize("dim,n,prec,unfused", FOLD_CASES)
def test_folded_vector_updates_match_separate_pass(dim, n, prec, unfused):
    """x += alpha p deferred into the stencil-product pass and r -= alpha q done by the
    first fine pre-smoothing kernel (fused down kernel in 2D, the zero-guess Jacobi
    sweep in 3D or unfused) give the same result as the separate update pass; both
    match the oracle.  Ragged tiles, several systems converging at different
    iterations (so the last deferred update lands in both p buffers)."""
    from oracle import spectral
    B = _B()
    alpha, k = 0.75, 9
    v = B.BURA_VARIANT_UNFUSED if unfused else 0
    F = synth.normal_rhs(n, dim, nrhs=2, tag=93)
    pr = getattr(B, "BURA_" + prec)
    u_fold = _host(B.Plan(dim, n, alpha, k, precision=pr, nrhs_max=2, tol=1e-11, variant=v).solve(_dev(F)).u)
    u_sep = _host(B.Plan(dim, n, alpha, k, precision=pr, nrhs_max=2, tol=1e-11,
                         variant=v | B.BURA_VARIANT_NO_FOLDXR).solve(_dev(F)).u)
    b = oracle_bura(alpha, k)
    ref = spectral.bura_spectral(F, dim, b.c_f64, b.d_f64)
    d = np.linalg.norm((u_fold - u_sep).reshape(2, -1), axis=1) / np.linalg.norm(ref.reshape(2, -1), axis=1)
    assert np.max(d) <= 1e-12
    for u in (u_fold, u_sep):
        e = np.linalg.norm((u - ref).reshape(2, -1), axis=1) / np.linalg.norm(ref.reshape(2, -1), axis=1)
        assert np.max(e) <= 1e-9
