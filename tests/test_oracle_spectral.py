"""Pins of the oracle's operators, closed-form spectral paths and shifted solves."""

import json

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from conftest import golden_path, oracle_bura
from oracle import metrics, operators, shifted, spectral


@pytest.mark.parametrize("n,dim", [(7, 2), (5, 3), (8, 2), (1, 2), (2, 2), (1, 3), (2, 3)])
def test_scaled_laplacian_matches_paper_scaling(n, dim):
    """Section 5.3: A = h^2 A~ / 8 (2D); 3D: h^2/12.  Diagonal 1/2, off-diagonals -1/(4d)."""
    A, lam = operators.scaled_operator(n, dim)
    h = 1.0 / (n + 1)
    assert lam == pytest.approx(4 * dim / h ** 2, rel=1e-14)
    Ad = A.toarray()
    assert np.allclose(np.diag(Ad), 0.5)
    off = Ad - np.diag(np.diag(Ad))
    vals = np.unique(off)
    assert all(abs(v) < 1e-15 or abs(v + 1.0 / (4 * dim)) < 1e-15 for v in vals)
    assert np.allclose(Ad, Ad.T)


@pytest.mark.parametrize("n,dim", [(3, 2), (4, 3), (9, 2)])
def test_paper_scaling_is_gershgorin_from_n_3(n, dim):
    """For n >= 3 an interior node with all neighbours inside attains Gershgorin's
    bound, which then equals the paper's 4d/h^2; below that it is smaller."""
    At = operators.unscaled_operator(n, dim)
    assert operators.gershgorin_bound(At) == pytest.approx(4 * dim * (n + 1) ** 2, rel=1e-14)
    assert operators.gershgorin_bound(operators.unscaled_operator(2, dim)) < 4 * dim * 3 ** 2


@pytest.mark.parametrize("n,dim", [(7, 2), (5, 3), (1, 2), (2, 2), (1, 3), (2, 3)])
def test_eigenvalues_against_dense_eigh(n, dim):
    A, _ = operators.scaled_operator(n, dim)
    w = np.linalg.eigvalsh(A.toarray())
    assert np.allclose(np.sort(spectral.eigenvalues(n, dim).ravel()), w, atol=1e-13)
    assert w.min() > 0 and w.max() <= 1.0


@pytest.mark.parametrize("idx", [(1, 1), (3, 5), (7, 2)])
def test_eigenvector_input(idx):
    """A psi = lambda psi for the sine modes (generalises Section 5.1)."""
    n = 9
    A, _ = operators.scaled_operator(n, 2)
    psi = synth.sine_mode(n, idx)
    lam = spectral.eigenvalues(n, 2)[idx[0] - 1, idx[1] - 1]
    assert np.allclose(A @ psi.ravel(), lam * psi.ravel(), atol=1e-13)
    # and the fractional power: A^-alpha psi = lambda^-alpha psi
    u = spectral.exact_fractional(psi[None], 2, 0.3)[0]
    assert np.allclose(u, lam ** -0.3 * psi, atol=1e-12)


@pytest.mark.parametrize("n,dim,alpha", [(7, 2, 0.5), (5, 3, 0.25), (6, 2, 0.75)])
def test_exact_fractional_brute_force(n, dim, alpha):
    """eq. (9) by dense eigendecomposition vs the DST closed form."""
    A, _ = operators.scaled_operator(n, dim)
    F = synth.uniform_rhs(n, dim, nrhs=2, tag=11)
    w, V = np.linalg.eigh(A.toarray())
    brute = (V @ np.diag(w ** -alpha) @ V.T @ F.reshape(2, -1).T).T
    assert np.allclose(spectral.exact_fractional(F, dim, alpha).reshape(2, -1), brute, rtol=1e-11, atol=1e-11)


def test_composition_half_powers():
    """A^-1/2 (A^-1/2 f) = A^-1 f, the latter by a sparse direct solve."""
    n = 15
    A, _ = operators.scaled_operator(n, 2)
    F = synth.normal_rhs(n, 2, tag=12)
    half = spectral.exact_fractional(spectral.exact_fractional(F, 2, 0.5), 2, 0.5)
    inv = spla.spsolve(A.tocsc(), F.ravel())
    assert np.allclose(half.ravel(), inv, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("n,dim,alpha,k", [(15, 2, 0.5, 5), (7, 3, 0.25, 5), (20, 2, 0.75, 7)])
def test_shifted_solves_match_spectral(n, dim, alpha, k):
    """O3 (k+1 sparse solves, eq. (16)) against O2 (eigenbasis) -- two independent routes."""
    b = oracle_bura(alpha, k)
    A, _ = operators.scaled_operator(n, dim)
    F = synth.uniform_rhs(n, dim, nrhs=3, tag=13)
    u_spec = spectral.bura_spectral(F, dim, b.c_f64, b.d_f64)
    u_dir = shifted.bura_by_solves(A, b.c_f64, b.d_f64, F)
    assert metrics.rel_err(u_dir, u_spec) < 1e-12


def test_cg_matches_direct():
    n = 9
    A, _ = operators.scaled_operator(n, 3)
    f = synth.normal_rhs(n, 3, tag=14).ravel()
    x, it = shifted.cg(A, f, shift=1e-3, rtol=1e-14)
    xd = shifted.shifted_solve_direct(A, 1e-3, f[None])[0]
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12


@pytest.mark.parametrize("gamma", [0.0, 1.0])
@pytest.mark.parametrize("alpha,k", [(0.5, 5), (0.25, 7)])
def test_error_lemma_bound(alpha, k, gamma):
    """Lemma 2.1: ||u_r - u||_{A^g} <= E ||f||_{A^(g-2)} on random and eigenvector inputs."""
    b = oracle_bura(alpha, k)
    n = 31
    F = np.concatenate([synth.normal_rhs(n, 2, nrhs=4, tag=15),
                        synth.sine_mode(n, (1, 1))[None], synth.sine_mode(n, (n, n))[None]])
    U_r = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64)
    lhs, rhs = metrics.lemma_bound_sides(F, U_r, 2, alpha, float(b.E), gamma)
    assert np.all(lhs <= rhs * (1 + 1e-9))
    # the bound is attained up to a modest factor at the lowest mode (t -> 0 is an
    # extremal point, Lemma 2.5)
    assert lhs[4] >= 0.2 * rhs[4]


def test_table7_2d_checkerboard():
    """Table 7 (loose pin, reference u_ref there carries ~1e-7 error of its own)."""
    ref = json.load(open(golden_path("table7_2d_checkerboard.json")))
    n = ref["h_inv"] - 1
    F = synth.checkerboard_rhs(n)
    h = 1.0 / (n + 1)
    Lam = 8 / h ** 2
    for alpha, k, printed in ref["rows"]:
        b = oracle_bura(alpha, k)
        # u = A~^-alpha f~ = Lambda^-alpha A^-alpha f~ (eq. (10))
        ue = spectral.exact_fractional(F, 2, alpha) * Lam ** -alpha
        ur = spectral.bura_spectral(F, 2, b.c_f64, b.d_f64) * Lam ** -alpha
        got = np.linalg.norm(ue - ur) / np.linalg.norm(F)
        tol = 1e-2 if alpha == 0.75 else 2e-3
        assert abs(got - printed) <= tol * printed, (alpha, got, printed)


def test_variable_coefficient_operator():
    """Flux form with harmonic face means; a = const reduces to the Laplacian."""
    n = 5
    a1 = np.full((n + 2, n + 2), 3.0)
    A1, lam1 = operators.scaled_operator(n, 2, a1)
    A0, lam0 = operators.scaled_operator(n, 2)
    assert np.allclose(A1.toarray(), A0.toarray())
    assert lam1 == pytest.approx(3 * lam0)
    # one interior node (n = 1): four faces to boundary nodes with values 1,2,4,8
    a = np.ones((3, 3))
    a[1, 1] = 2.0
    a[0, 1], a[2, 1], a[1, 0], a[1, 2] = 1.0, 2.0, 4.0, 8.0
    At = operators.unscaled_operator(1, 2, a).toarray()
    hm = lambda x, y: 2 * x * y / (x + y)
    h = 0.5
    expect = (hm(2, 1) + hm(2, 2) + hm(2, 4) + hm(2, 8)) / h ** 2
    assert At[0, 0] == pytest.approx(expect)
    # Gershgorin bound >= largest eigenvalue, for a rough field
    field = synth.lognormal_coefficient(15, 2, tag=16)
    A, lam = operators.scaled_operator(15, 2, field)
    w = np.linalg.eigvalsh(A.toarray())
    assert w.max() <= 1.0 + 1e-12 and w.min() > 0


def test_gaussian_field_statistics():
    g = synth.gaussian_field(127, 2, corr_len=0.1, sigma=1.0, tag=4)
    assert g.shape == (129, 129)
    assert abs(g.std() - 1.0) < 0.5
    # smooth on the scale of h: neighbouring nodes are strongly correlated
    c = np.corrcoef(g[:, :-1].ravel(), g[:, 1:].ravel())[0, 1]
    assert c > 0.95
