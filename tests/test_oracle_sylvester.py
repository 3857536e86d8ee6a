"""Pins for the factor subproblem: Theorem 1 / eq. 8 against the dense
Kronecker system of eq. 6, the residual of eq. 5, and the lambda = 0 ridge."""

import numpy as np
import pytest
import scipy.linalg

from oracle import sylvester, laplacian


def _case(q, s, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((s, 3 * s + 2))
    G = M @ M.T
    Y = rng.standard_normal((q, s))
    return G, Y


@pytest.mark.parametrize("q,s", [(3, 4), (8, 9), (7, 6), (16, 12), (1, 3), (2, 5)])
@pytest.mark.parametrize("lam", [1e-2, 0.45, 3.0])
def test_fast_equals_kronecker(q, s, lam):
    G, Y = _case(q, s, q * 100 + s)
    A1 = sylvester.solve_fast(G, Y, lam, 0.5, 0.1)
    A2 = sylvester.solve_kronecker(G, Y, lam, 0.5, 0.1)
    np.testing.assert_allclose(A1, A2, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("q,s", [(31, 64), (144, 27), (50, 40)])
def test_residual_eq5(q, s):
    G, Y = _case(q, s, 7)
    A = sylvester.solve_fast(G, Y, 1e-2, 0.5, 0.1)
    r = sylvester.residual(A, G, Y, 1e-2, 0.5, 0.1)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(Y) * max(1.0, np.linalg.norm(G, 2))


def test_lambda_zero_is_ridge():
    G, Y = _case(10, 8, 3)
    A = sylvester.solve_fast(G, Y, 0.0, 0.5, 0.1)
    c = scipy.linalg.cho_factor(G + 0.1 * np.eye(8))
    ref = scipy.linalg.cho_solve(c, Y.T).T          # Y (G + rho I)^{-1}
    np.testing.assert_allclose(A, ref, rtol=1e-10)


def test_zero_gram_is_laplacian_solve():
    q, s = 9, 4
    _, Y = _case(q, s, 4)
    A = sylvester.solve_fast(np.zeros((s, s)), Y, 0.7, 0.3, 0.1)
    ref = np.linalg.solve(0.7 * laplacian.matrix(q, 0.3) + 0.1 * np.eye(q), Y)
    np.testing.assert_allclose(A, ref, rtol=1e-11)


def test_solution_is_subproblem_minimizer():
    # perturbing the solution can only raise the eq. 4 objective
    rng = np.random.default_rng(9)
    q, s, n = 6, 4, 30
    M = rng.standard_normal((s, n)); Xk = rng.standard_normal((q, n)); Ap = rng.standard_normal((q, s))
    lam, delta, rho = 0.3, 0.5, 0.1
    L = laplacian.matrix(q, delta)

    def obj(A):
        return (0.5 * np.sum((Xk - A @ M) ** 2) + 0.5 * lam * np.trace(A.T @ L @ A)
                + 0.5 * rho * np.sum((A - Ap) ** 2))
    A = sylvester.solve_fast(M @ M.T, sylvester.rhs(Xk, M, Ap, rho), lam, delta, rho)
    f0 = obj(A)
    for _ in range(20):
        assert obj(A + 1e-3 * rng.standard_normal(A.shape)) > f0
