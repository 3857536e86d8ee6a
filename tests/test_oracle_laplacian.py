"""Pins for L_k (Section 3.1) and its Fourier diagonalization (eq. 7)."""

import numpy as np
import pytest

from oracle import laplacian, sylvester


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8, 31, 50])
@pytest.mark.parametrize("delta", [0.0, 0.3, 0.5])
def test_closed_form_eigenvalues(n, delta):
    L = laplacian.matrix(n, delta)
    closed = delta + 4.0 * np.sin(np.pi * np.arange(n) / n) ** 2
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(L)), np.sort(closed), atol=1e-12)
    np.testing.assert_allclose(laplacian.fourier_eigenvalues(n, delta), closed, atol=1e-12)


def test_pure_laplacian_eigenvalues_4sin2():
    n = 12
    ev = laplacian.fourier_eigenvalues(n, 0.0)
    for j in range(n):
        assert abs(ev[j] - 4.0 * np.sin(np.pi * j / n) ** 2) < 1e-13


@pytest.mark.parametrize("n", [3, 8, 9, 144])
def test_dft_diagonalizes(n):
    L = laplacian.matrix(n, 0.5)
    F = laplacian.dft_matrix(n)
    Lam = laplacian.fourier_eigenvalues(n, 0.5)
    np.testing.assert_allclose(F.conj().T @ np.diag(Lam) @ F, L, atol=1e-11)
    np.testing.assert_allclose(F.conj().T @ F, np.eye(n), atol=1e-12)


def test_structure_small_cases():
    # n = 3: circulant with 2+delta on the diagonal and -1 elsewhere
    L = laplacian.matrix(3, 0.5)
    np.testing.assert_allclose(L, [[2.5, -1, -1], [-1, 2.5, -1], [-1, -1, 2.5]])
    # n = 2: both neighbours are the same entry, so the off-diagonal is -2
    np.testing.assert_allclose(laplacian.matrix(2, 0.5), [[2.5, -2], [-2, 2.5]])
    np.testing.assert_allclose(laplacian.matrix(1, 0.5), [[0.5]])


def test_quadratic_form_is_periodic_difference_energy():
    # tr(A^T L A) = delta ||A||^2 + sum of squared periodic first differences
    #             = delta ||A||^2 - <A, periodic second difference of A>
    rng = np.random.default_rng(0)
    n, s, delta = 11, 5, 0.4
    A = rng.standard_normal((n, s))
    first = np.roll(A, -1, axis=0) - A
    second = np.roll(A, 1, axis=0) - 2 * A + np.roll(A, -1, axis=0)
    tr = sylvester.trace_term(A, delta)
    assert abs(tr - (delta * np.sum(A * A) + np.sum(first ** 2))) < 1e-11
    assert abs(tr - (delta * np.sum(A * A) - np.sum(A * second))) < 1e-11


def test_squared_second_differences_are_L_squared():
    # the sum of squared periodic second differences of A is tr(A^T L0^2 A),
    # L0 the delta = 0 matrix; its eigenvalues are (4 sin^2)^2
    rng = np.random.default_rng(1)
    n = 9
    A = rng.standard_normal((n, 3))
    second = np.roll(A, 1, axis=0) - 2 * A + np.roll(A, -1, axis=0)
    L0 = laplacian.matrix(n, 0.0)
    assert abs(np.sum(second ** 2) - np.trace(A.T @ L0 @ L0 @ A)) < 1e-11


def test_printed_sign_is_negative_definite():
    # the matrix as printed has every eigenvalue <= -delta < 0: with it the
    # trace term rewards large factors and the model is unbounded below, which
    # is why the oracle uses the negated (positive definite) matrix
    for n in (3, 8, 31):
        ev = np.linalg.eigvalsh(laplacian.printed_matrix(n, 0.5))
        assert ev.max() <= -0.5 + 1e-12
