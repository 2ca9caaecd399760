"""Pins of the oracle's CG solves against facts fixed outside its code:
the free-field FFT closed form, termination in at most (number of distinct
eigenvalues) steps, dense LU solves on tiny lattices, and the Krylov
orthogonality that every CG iterate must satisfy."""

import numpy as np
import pytest

import oracle
from oracle import dense, free_field
from paper_1311_2719_amd import inputs


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_fft_solver_matches_lu_free_field():
    dims, m = (4, 4, 4, 4), 0.1
    b = inputs.gaussian_source(dims, 1)
    x_lu = dense.lu_solve(dims, inputs.unit_links(dims), m, b)
    assert _rel(free_field.solve(dims, m, b), x_lu) < 1e-13


@pytest.mark.parametrize("par", [oracle.EVEN, oracle.ODD])
def test_free_field_terminates_in_four_steps(par):
    # On 4^4 the free A has 4 distinct eigenvalues (m^2 + k + 1/2), so CG on
    # either parity system stops after at most 4 iterations in exact arithmetic.
    dims, m = (4, 4, 4, 4), 0.1
    U = inputs.unit_links(dims)
    b = inputs.gaussian_source(dims, 2)
    x, res = oracle.cg_pass(dims, U, m, b, tol=1e-12, maxiter=100, parity=par)
    assert res["iters"] <= 4
    odd = dense.parity_mask(dims)
    sel = odd if par == oracle.ODD else ~odd
    bp = np.where(sel[:, None], b, 0)
    assert _rel(x[sel], free_field.solve(dims, m, bp)[sel]) < 1e-12


def test_plane_wave_converges_in_one_step():
    dims, m = (4, 4, 4, 4), 0.2
    U = inputs.unit_links(dims)
    v, lam = free_field.plane_wave(dims, (1, 0, 3, 2), [1.0, 0.5j, -0.25])
    x, y, info = oracle.cg_solve(dims, U, m, v, tol=1e-12)
    assert info["iters"] == 1
    assert _rel(x, v / (m * m + lam)) < 1e-14


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (4, 6, 8, 10)])
def test_free_field_fft_at_larger_sizes(dims):
    m = 0.05
    b = inputs.gaussian_source(dims, 3)
    x, _, info = oracle.cg_solve(dims, inputs.unit_links(dims), m, b, tol=1e-12)
    assert info["status"] == 0
    assert _rel(x, free_field.solve(dims, m, b)) < 1e-10


@pytest.mark.parametrize("dims,m", [((2, 2, 2, 2), 0.3), ((4, 4, 4, 4), 0.1), ((2, 4, 6, 8), 0.05)])
def test_cg_matches_lu_on_haar(dims, m):
    U = inputs.haar_su3(dims, seed=101)
    b = inputs.gaussian_source(dims, 201)
    x_lu = dense.lu_solve(dims, U, m, b)
    x, y, info = oracle.cg_solve(dims, U, m, b, tol=1e-10, want_y=True)
    assert info["status"] == 0 and info["true_rel"] <= 1e-10
    # error <= condition number x residual; kappa(4^4 Haar, m=0.1) ~ 7e2
    A = dense.dense_normal(dense.dense_dslash(dims, U), m)
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0]
    assert _rel(x, x_lu) <= kappa * 1e-10
    # y = D x on the opposite parity of each system = D x everywhere
    D = dense.dense_dslash(dims, U)
    assert _rel(y, (D @ x.reshape(-1)).reshape(-1, 3)) < 1e-13


def test_full_lattice_cg_matches_lu():
    dims, m = (4, 4, 4, 4), 0.1
    U = inputs.haar_su3(dims, seed=101)
    b = inputs.gaussian_source(dims, 201)
    x_lu = dense.lu_solve(dims, U, m, b)
    x, info = oracle.cg_full(dims, U, m, b, tol=1e-13)
    assert info["true_rel"] < 1e-12
    assert _rel(x, x_lu) < 1e-10


@pytest.mark.parametrize("par", [oracle.EVEN, oracle.ODD])
def test_cg_iterates_are_krylov_orthogonal(par):
    # CG's k-th residual is orthogonal to the Krylov space K_k(A, b): a
    # property of the method, independent of how the loop is written.
    dims, m = (4, 4, 4, 4), 0.15
    U = inputs.haar_su3(dims, seed=61)
    b = inputs.gaussian_source(dims, 62)
    odd = dense.parity_mask(dims)
    sel = np.repeat(odd if par == oracle.ODD else ~odd, 3)
    A = dense.dense_normal(dense.dense_dslash(dims, U), m)[np.ix_(sel, sel)]
    bp = b.reshape(-1)[sel]
    K = [bp]
    for _ in range(5):
        K.append(A @ K[-1])
    for k in range(1, 6):
        x, res = oracle.cg_pass(dims, U, m, b, tol=0.0, maxiter=k, parity=par)
        assert res["iters"] == k
        r = bp - A @ x.reshape(-1)[sel]
        for j in range(k):
            kj = K[j] / np.linalg.norm(K[j])
            assert abs(np.vdot(kj, r)) < 1e-10 * np.linalg.norm(r) * 10 ** j
        # and the iterate minimises the A-norm error over x0 + K_k
        B = np.stack(K[:k], axis=1)
        coef = np.linalg.solve(B.conj().T @ A @ B, B.conj().T @ bp)
        assert _rel(x.reshape(-1)[sel], B @ coef) < 1e-8


def test_even_odd_spectra_agree():
    dims, m = (4, 4, 4, 4), 0.1
    U = inputs.haar_su3(dims, seed=71)
    odd = np.repeat(dense.parity_mask(dims), 3)
    A = dense.dense_normal(dense.dense_dslash(dims, U), m)
    e1 = np.linalg.eigvalsh(A[np.ix_(~odd, ~odd)])
    e2 = np.linalg.eigvalsh(A[np.ix_(odd, odd)])
    assert np.max(np.abs(e1 - e2)) < 1e-12
    # A is block diagonal in parity
    assert np.max(np.abs(A[np.ix_(~odd, odd)])) < 1e-14


def test_apply_normal_and_true_residual():
    dims, m = (2, 4, 6, 8), 0.2
    U = inputs.haar_su3(dims, seed=81)
    v = inputs.gaussian_source(dims, 82)
    A = dense.dense_normal(dense.dense_dslash(dims, U), m)
    assert _rel(oracle.apply_normal(dims, U, m, v), (A @ v.reshape(-1)).reshape(-1, 3)) < 1e-13
    b = (A @ v.reshape(-1)).reshape(-1, 3)
    assert oracle.true_residual(dims, U, m, b, v) < 1e-13


def test_zero_source_and_iteration_limit():
    dims = (4, 4, 4, 4)
    U = inputs.haar_su3(dims, seed=91)
    x, _, info = oracle.cg_solve(dims, U, 0.1, np.zeros((256, 3), np.complex128))
    assert info["status"] == 0 and info["iters"] == 0 and not np.any(x)
    b = inputs.gaussian_source(dims, 92)
    x, _, info = oracle.cg_solve(dims, U, 0.1, b, maxiter=3)
    assert info["status"] == 1 and info["iters"] == 3


def test_bad_arguments_rejected():
    dims = (4, 4, 4, 4)
    U = inputs.unit_links(dims)
    b = inputs.gaussian_source(dims, 1)
    with pytest.raises(ValueError):
        oracle.cg_solve(dims, U, 0.0, b)
    with pytest.raises(ValueError):
        oracle.cg_solve(dims, U, 0.1, b, tol=0.0)


def test_ritz_values_free_field_exact():
    # the free 4^4 parity operator has the four eigenvalues m^2 + {1/2, 3/2,
    # 5/2, 7/2} (the hand-derived spectrum of -D^2): CG stops after four
    # iterations and the Lanczos matrix of its coefficients has exactly them
    dims, m = (4, 4, 4, 4), 0.1
    b = inputs.gaussian_source(dims, 11)
    for par in (oracle.EVEN, oracle.ODD):
        _, al, be, info = oracle.cg_coefficients(dims, inputs.unit_links(dims), m, b, tol=1e-14, parity=par)
        assert info["iters"] == 4
        th = oracle.ritz_values(al, be)
        assert np.max(np.abs(th - (m * m + np.array([0.5, 1.5, 2.5, 3.5])))) < 1e-12


def test_kappa_estimate_against_dense_spectrum():
    # Haar 4^4: the extreme Ritz values of a converged CG run approach the
    # extreme eigenvalues of the parity operator from the inside; the
    # reference spectrum comes from the independent dense builder
    dims, m = (4, 4, 4, 4), 0.1
    U = inputs.haar_su3(dims, 101)
    A = dense.dense_normal(dense.dense_dslash(dims, U), m)
    even = np.repeat(~dense.parity_mask(dims), 3)
    lam = np.linalg.eigvalsh(A[np.ix_(even, even)])
    lmax, lmin, kappa = oracle.kappa_estimate(dims, U, m, inputs.gaussian_source(dims, 201), tol=1e-12, parity=0)
    assert lmin >= lam[0] * (1 - 1e-12) and lmax <= lam[-1] * (1 + 1e-12)
    # the largest converges first; the smallest to a few 1e-4 at this residual
    assert abs(lmax / lam[-1] - 1) < 1e-8 and abs(lmin / lam[0] - 1) < 2e-3
    assert abs(kappa / (lam[-1] / lam[0]) - 1) < 2e-3
    # a planted mistake: coefficients of a run on a different mass give a
    # spectrum shifted by the mass difference, which the pin sees
    _, al, be, _ = oracle.cg_coefficients(dims, U, 0.2, inputs.gaussian_source(dims, 201), tol=1e-12, parity=0)
    assert abs(oracle.ritz_values(al, be)[0] - lam[0]) > 0.02
