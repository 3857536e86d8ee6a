"""The periodically modified negative Laplacian L_k (oracle; test infrastructure).

Section 3.1 prints L_k as the circulant with diagonal -2-delta and periodic
off-diagonals +1.  That matrix is negative definite, which makes the model
unbounded below (scale A_1 by c and A_2 by 1/c) and contradicts the
convergence proof, which needs every eigenvalue of the Kronecker system to be
at least rho (Section 3.5, proof of condition 1).  The reading used throughout is the
negation, L = (2 + delta) I - S - S^T with S the cyclic shift: positive
definite, eigenvalues delta + 4 sin^2(pi j / n), and the "negative Laplacian"
in the usual sense (minus the periodic second difference).  ``printed_matrix``
keeps the literal print for the test that documents this reading.

eq. 7 diagonalizes L_k by the one-dimensional DFT: L = F^H Lambda F.
"""

import numpy as np


def first_column(n, delta):
    """First column of the circulant L for size n (n = 1, 2 handled as sums)."""
    c = np.zeros(n)
    c[0] += 2.0 + delta
    c[1 % n] -= 1.0
    c[(n - 1) % n] -= 1.0
    return c


def matrix(n, delta):
    """Dense L = (2 + delta) I - S - S^T (circulant, symmetric)."""
    c = first_column(n, delta)
    return np.array([[c[(i - j) % n] for j in range(n)] for i in range(n)])


def printed_matrix(n, delta):
    """The matrix exactly as printed in Section 3.1 (diag -2-delta, +1 off)."""
    return -matrix(n, delta)


def dft_matrix(n):
    """Unitary DFT matrix F with F[j, i] = exp(-2 pi i j i / n) / sqrt(n)."""
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n) / np.sqrt(n)


def fourier_eigenvalues(n, delta):
    """diag(Lambda) of eq. 7: the DFT of the first column of the circulant."""
    return np.real(np.fft.fft(first_column(n, delta)))
