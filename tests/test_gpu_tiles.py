"""GPU parity of every tile-shape variant of the 2D kernels, and the plan-time tuner.

The variants (bura_plan_set_tiles) change only the launch shape of the
stencil product and of the fused down/up level kernels: each computes the
same value at every grid point, and only the grouping of the per-block
partial sums of the PCG dot products differs.  So every variant, and the
tuner's choice, must match the oracle at the same tolerance as the default
shape.  The grids are chosen so that every variant has ragged edge tiles
(255 -> 127 -> 63 ...: 127 is not a multiple of 6 or 8 coarse rows or of 32
or 64 coarse columns, 255 not a multiple of 8, 16 or 24 fine rows or of 64 or
128 columns; 191 -> 95 -> 47 ... stops at an even level).
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


def _rel2(u, ref):
    return float((np.linalg.norm((u - ref).reshape(u.shape[0], -1), axis=1) /
                  np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)).max())


def _reference(n, var, alpha, k, F, tag):
    from oracle import operators, shifted, spectral
    b = oracle_bura(alpha, k)
    if not var:
        return None, spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    coeff = synth.lognormal_coefficient(n, 2, tag=tag)
    A, _ = operators.scaled_operator(n, 2, coeff)
    return coeff, shifted.bura_by_solves(A, b.c_f64, b.d_f64, F)


def _rows(n, nsys, segments):
    return 255 <= n <= 1023 and nsys * segments >= 1024


def _default_tiles(n, nsys, levels):
    """The documented default: the row-marching variant 3 for a kernel of a
    level of 255..1023 points per axis whose launch makes at least 1024 row
    segments over all systems (128 fine rows for the stencil product and the
    up kernel, 64 coarse rows for the down kernel); otherwise variant 0,
    except the down kernel on levels whose 64 x 6 launch (coarse points per
    workgroup) would make fewer than 1024 workgroups, which take the 32 x 8
    tile (1)."""
    out = [3 if _rows(n, nsys, -(-n // 128)) else 0]
    for _ in range(levels):
        nc = (n - 1) // 2
        blocks = -(-nc // 64) * -(-nc // 6)
        down = 3 if _rows(n, nsys, -(-nc // 64)) else (0 if nsys * blocks >= 1024 else 1)
        out += [down, 3 if _rows(n, nsys, -(-n // 128)) else 0]
        n = nc
    return out


def test_default_down_tile_follows_launch_width():
    B = _B()
    b = oracle_bura(0.5, 9)
    one = B.Plan(2, 1023, weights=[1.0], shifts=[0.25])
    wide = B.Plan(2, 1023, weights=b.c_f64, shifts=[-x for x in b.d_f64], nrhs_max=3)
    try:
        t1, t30 = one.tiles, wide.tiles
        print("1 system:", t1, " 30 systems:", t30)
        assert t1 == _default_tiles(1023, 1, len(t1) // 2)
        assert t30 == _default_tiles(1023, 30, len(t30) // 2)
        assert t1[1] == 1 and t30[1] == 0   # the fine level: 688 workgroups per system
    finally:
        one.close()
        wide.close()


CASES = [
    # n, variable coefficients, precision, alpha, k
    (255, False, "FP64", 0.5, 5),
    (255, True, "MIXED", 0.6, 7),
    (191, False, "MIXED", 0.25, 6),
]


@pytest.mark.parametrize("n,var,prec,alpha,k", CASES)
def test_every_tile_variant_matches_oracle(n, var, prec, alpha, k):
    B = _B()
    b = oracle_bura(alpha, k)
    F = synth.normal_rhs(n, 2, nrhs=2, tag=401)
    coeff, ref = _reference(n, var, alpha, k, F, tag=402)
    plan = B.Plan(2, n, weights=b.c_f64, shifts=[-x for x in b.d_f64], coeff=coeff, nrhs_max=2,
                  precision=getattr(B, "BURA_" + prec), tol=1e-12)
    default = plan.tiles
    assert len(default) % 2 == 1 and len(default) >= 3
    assert default == _default_tiles(n, 2 * (k + 1), len(default) // 2)
    settings = [[v] * len(default) for v in range(B.BURA_TILE_VARIANTS)]
    settings.append([(i % B.BURA_TILE_VARIANTS) for i in range(len(default))])   # mixed per level
    u0 = None
    for tv in settings:
        plan.tiles = tv
        assert plan.tiles == tv
        res = plan.solve(_dev(F))
        u = _host(res.u)
        err = _rel2(u, ref)
        print(f"n={n} var={var} {prec} tiles={tv}: rel2 vs oracle {err:.2e}, iters {list(res.report.iters)[:k + 1]}")
        assert err <= 1e-9
        if u0 is None:
            u0 = u
        else:
            assert _rel2(u, u0) <= 1e-9
    plan.close()


ROW_CASES = [
    # n, variable coefficients, precision, smoothing sweeps
    (95, False, "FP64", 1),
    (127, True, "MIXED", 3),
    (191, False, "MIXED", 3),
    (255, True, "FP64", 1),
    (127, True, "FP64", 3),
    (191, True, "FP64", 2),
    # FP32 inner solves with one and two sweeps (the up kernel's register
    # budget is fixed for these), 159 -> 79 -> 39 ...
    (159, True, "MIXED", 2),
    (79, True, "MIXED", 1),
    (79, False, "MIXED", 2),
]


@pytest.mark.parametrize("n,var,prec,nu", ROW_CASES)
def test_row_variants_with_one_and_three_sweeps(n, var, prec, nu):
    """The row-marching variants (3: segments of 128 fine rows, 4: of 32) on
    every level with one, two and three smoothing sweeps, FP64 and mixed,
    constant and variable coefficients; no grid's rows are a multiple of a
    segment (95 -> 47 -> 23 -> 11 -> 5 ..., 191 -> 95 ...).  Each matches the
    oracle at the tiles' tolerance, and the tiles' result to rounding."""
    B = _B()
    alpha, k = 0.5, 6
    b = oracle_bura(alpha, k)
    F = synth.normal_rhs(n, 2, nrhs=2, tag=441)
    coeff, ref = _reference(n, var, alpha, k, F, tag=442)
    plan = B.Plan(2, n, weights=b.c_f64, shifts=[-x for x in b.d_f64], coeff=coeff, nrhs_max=2,
                  precision=getattr(B, "BURA_" + prec), tol=1e-12, nu_pre=nu, nu_post=nu)
    try:
        nt = len(plan.tiles)
        outs = {}
        for v in (0, 3, 4):
            plan.tiles = [v] * nt
            res = plan.solve(_dev(F))
            outs[v] = _host(res.u)
            err = _rel2(outs[v], ref)
            print(f"n={n} var={var} {prec} nu={nu} variant {v}: rel2 vs oracle {err:.2e}, "
                  f"iters {list(res.report.iters)[:k + 1]}")
            assert err <= 1e-9
        assert _rel2(outs[3], outs[0]) <= 1e-9 and _rel2(outs[4], outs[0]) <= 1e-9
    finally:
        plan.close()


def test_wide_launch_defaults_to_rows_and_matches_oracle():
    """512 systems of a 255^2 grid (8 poles x 64 right-hand sides): the stencil
    product and the fine down and up kernels default to the row-marching
    variant 3 (2 row segments per system, 1024 per launch), the coarser levels
    to the tiles.  The solve matches the spectral oracle for every right-hand
    side, and the all-tiles shape to rounding."""
    from oracle import spectral
    B = _B()
    n, alpha, k, R = 255, 0.5, 7, 64
    b = oracle_bura(alpha, k)
    F = synth.normal_rhs(n, 2, nrhs=R, tag=431)
    ref = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    plan = B.Plan(2, n, weights=b.c_f64, shifts=[-x for x in b.d_f64], nrhs_max=R, precision=B.BURA_MIXED,
                  tol=1e-12)
    try:
        t = plan.tiles
        print("default tiles at 512 systems:", t)
        assert t == _default_tiles(n, R * (k + 1), len(t) // 2)
        assert t[:3] == [3, 3, 3] and all(v != 3 for v in t[3:])
        u_rows = _host(plan.solve(_dev(F)).u)
        err = _rel2(u_rows, ref)
        plan.tiles = [0] * len(t)
        u_tiles = _host(plan.solve(_dev(F)).u)
        print(f"rows rel2 vs oracle {err:.2e}; rows vs tiles {_rel2(u_rows, u_tiles):.2e}")
        assert err <= 1e-9
        assert _rel2(u_rows, u_tiles) <= 1e-9
    finally:
        plan.close()


def test_tuner_choice_is_valid_cached_and_correct():
    B = _B()
    n, alpha, k = 255, 0.6, 7
    b = oracle_bura(alpha, k)
    F = synth.normal_rhs(n, 2, nrhs=4, tag=411)
    coeff, ref = _reference(n, True, alpha, k, F, tag=412)
    kw = dict(weights=b.c_f64, shifts=[-x for x in b.d_f64], coeff=coeff, nrhs_max=4, precision=B.BURA_MIXED,
              tol=1e-12, autotune=1)
    p1 = B.Plan(2, n, **kw)
    t1 = p1.tiles
    assert len(t1) >= 3 and all(0 <= v < B.BURA_TILE_VARIANTS for v in t1)
    u = _host(p1.solve(_dev(F)).u)
    err = _rel2(u, ref)
    print(f"tuned tiles {t1}: rel2 vs oracle {err:.2e}")
    assert err <= 1e-9
    p2 = B.Plan(2, n, **kw)   # same shape: the cached choice
    assert p2.tiles == t1
    p1.close()
    p2.close()


def test_set_tiles_rejects_bad_input():
    B = _B()
    b = oracle_bura(0.5, 5)
    plan = B.Plan(2, 63, weights=b.c_f64, shifts=[-x for x in b.d_f64])
    t = plan.tiles
    with pytest.raises(B.BuraError) as ei:
        plan.tiles = t + [0]
    assert ei.value.code == B.BURA_EINVAL
    with pytest.raises(B.BuraError) as ei:
        plan.tiles = [B.BURA_TILE_VARIANTS] + t[1:]
    assert ei.value.code == B.BURA_EINVAL
    with pytest.raises(B.BuraError):
        plan.tiles = [-1] + t[1:]
    assert plan.tiles == t
    plan.close()
    p3 = B.Plan(3, 15, weights=b.c_f64, shifts=[-x for x in b.d_f64])
    assert p3.tiles == []   # one launch shape in 3D
    p3.close()


def test_tiles_of_jacobi_pcg_grid():
    """A 64 x 64 grid has no hierarchy: only the stencil product has variants."""
    from oracle import spectral
    B = _B()
    b = oracle_bura(0.5, 5)
    F = synth.normal_rhs(64, 2, nrhs=1, tag=421)
    ref = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    plan = B.Plan(2, 64, weights=b.c_f64, shifts=[-x for x in b.d_f64], precision=B.BURA_FP64, autotune=1)
    assert len(plan.tiles) == 1
    for v in range(B.BURA_TILE_VARIANTS):
        plan.tiles = [v]
        assert _rel2(_host(plan.solve(_dev(F)).u), ref) <= 1e-9
    plan.close()


@pytest.mark.parametrize("variant", [0, "NO_FOLDXR"])
def test_wide_mixed_refinement_fuses_the_x64_update(variant):
    """Mixed refinement on a wide launch (255^2, 8 poles x 64 right-hand
    sides: the FP64 residual marches rows, 2 segments per system) folds
    x64 += e into the residual pass (the first update assigns x64 = e, the
    first residual having left x64 uncleared), with the inner solve's
    pending update (default) and without it (separate vector updates).
    Every right-hand side matches the spectral oracle (a zero one gives
    exactly 0), and the first four match a narrow launch of the same terms
    (4 right-hand sides: two separate passes, x64 cleared first)."""
    from oracle import spectral
    B = _B()
    n, alpha, k, R = 255, 0.5, 7, 64
    b = oracle_bura(alpha, k)
    v = 0 if variant == 0 else getattr(B, "BURA_VARIANT_" + variant)
    F = synth.normal_rhs(n, 2, nrhs=R, tag=451)
    F[5] = 0.0   # a zero right-hand side: its systems stay inactive, and their x64 must read 0
    ref = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    kw = dict(weights=b.c_f64, shifts=[-x for x in b.d_f64], precision=B.BURA_MIXED, tol=1e-12, variant=v)
    wide = B.Plan(2, n, nrhs_max=R, **kw)
    narrow = B.Plan(2, n, nrhs_max=4, **kw)
    try:
        res = wide.solve(_dev(F))
        u_wide = _host(res.u)
        u_narrow = _host(narrow.solve(_dev(F[:4])).u)
        assert np.all(u_wide[5] == 0.0)
        keep = [r for r in range(R) if r != 5]
        err = _rel2(u_wide[keep], ref[keep])
        print(f"variant {variant}: wide rel2 vs oracle {err:.2e}, outer steps {list(res.report.outer)[:k + 1]}, "
              f"wide vs narrow {_rel2(u_wide[:4], u_narrow):.2e}")
        assert err <= 1e-9
        assert _rel2(u_narrow, ref[:4]) <= 1e-9
        assert _rel2(u_wide[:4], u_narrow) <= 1e-9
    finally:
        wide.close()
        narrow.close()
