"""The factor subproblem (oracle; test infrastructure).

Section 3.2: the A_k update minimizes (eq. 4)
    1/2 ||X_(k) - A M||^2 + lambda/2 tr(A^T L A) + rho/2 ||A - A^t||^2,
whose stationarity condition is the Sylvester equation (eq. 5)
    A (M M^T) + lambda L A + rho A = X_(k) M^T + rho A^t.
eq. 6 is its Kronecker form; eq. 7-8 (Theorem 1) solve it by diagonalizing
M M^T = C Phi C^T (symmetric eigendecomposition) and L = F^H Lambda F (DFT):
    A = F^H ( (1 ./ T) .* (F Y C) ) C^T,   T_ij = lambda Lambda_i + Phi_j + rho,
with Y the right-hand side.  (The theorem's text swaps the names of the
elementwise product and division; the formula is unambiguous.)
"""

import numpy as np

from . import laplacian


def rhs(Xk, M, A_prev, rho):
    """Y = X_(k) M^T + rho A^t (right-hand side of eq. 5)."""
    return Xk @ M.T + rho * A_prev


def solve_fast(G, Y, lam, delta, rho):
    """eq. 8: the Theorem 1 solution with an eigendecomposition of G = M M^T
    and the DFT along mode k.  Returns the real I_k x s_k solution."""
    n = Y.shape[0]
    Phi, C = np.linalg.eigh(G)
    Lam = laplacian.fourier_eigenvalues(n, delta)
    T = lam * Lam[:, None] + Phi[None, :] + rho
    FYC = np.fft.fft(Y @ C, axis=0, norm="ortho")
    A = np.fft.ifft(FYC / T, axis=0, norm="ortho") @ C.T
    return np.real(A)


def solve_kronecker(G, Y, lam, delta, rho):
    """eq. 6 solved densely: (lam I_s (x) L + G (x) I_q + rho I) vec(A) = vec(Y).
    vec stacks columns (column-major), as in the paper.  Small sizes only."""
    q, s = Y.shape
    L = laplacian.matrix(q, delta)
    K = lam * np.kron(np.eye(s), L) + np.kron(G, np.eye(q)) + rho * np.eye(q * s)
    vecA = np.linalg.solve(K, Y.reshape(-1, order="F"))
    return vecA.reshape((q, s), order="F")


def residual(A, G, Y, lam, delta, rho):
    """Residual of eq. 5: A G + lam L A + rho A - Y."""
    L = laplacian.matrix(A.shape[0], delta)
    return A @ G + lam * (L @ A) + rho * A - Y


def trace_term(A, delta):
    """tr(A^T L A) for the mode-k unfolding A (Section 3.1)."""
    L = laplacian.matrix(A.shape[0], delta)
    return float(np.trace(A.T @ L @ A))
