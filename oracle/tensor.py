"""Tensor algebra of the paper, in float64 NumPy (oracle; test infrastructure).

Indices are 0-based here; the paper's are 1-based.  Unfoldings follow
Definition 2 literally: the first listed mode varies fastest (column-major).

FCTN rank bookkeeping: the rank vector lists R_{12}, R_{13}, ..., R_{1N},
R_{23}, ..., R_{N-1,N} (Section 1, definition of r_FCTN).  Factor k has modes
(R_{1k}, ..., R_{k-1,k}, I_k, R_{k,k+1}, ..., R_{kN}) (Section 1, FCTN
factor shapes; Section 3.1 after eq. model_1).
"""

import itertools
import string

import numpy as np


# ----------------------------------------------------------------------------
# rank / shape bookkeeping (Section 1, r_FCTN and factor shapes)
# ----------------------------------------------------------------------------

def bond_pairs(N):
    """Pairs (i, j), i < j, in r_FCTN order: (0,1), (0,2), ..., (N-2, N-1)."""
    return [(i, j) for i in range(N) for j in range(i + 1, N)]


def rank_matrix(ranks, N):
    """Symmetric N x N matrix R with R[i][j] = R_{ij} from the r_FCTN vector."""
    pairs = bond_pairs(N)
    if len(ranks) != len(pairs):
        raise ValueError(f"need {len(pairs)} ranks for N={N}, got {len(ranks)}")
    R = [[0] * N for _ in range(N)]
    for (i, j), r in zip(pairs, ranks):
        R[i][j] = R[j][i] = int(r)
    return R


def factor_shape(dims, R, k):
    """Shape of A_k: (R_{1k}, ..., I_k, ..., R_{kN})."""
    return tuple(dims[k] if j == k else R[k][j] for j in range(len(dims)))


def factor_shapes(dims, ranks):
    N = len(dims)
    R = rank_matrix(ranks, N)
    return [factor_shape(dims, R, k) for k in range(N)]


# ----------------------------------------------------------------------------
# Definitions 1-3
# ----------------------------------------------------------------------------

def gtranspose(X, n):
    """Definition 1: the n-mode transposition; mode n[m] of X becomes mode m."""
    return np.transpose(X, tuple(n))


def gunfold(X, rows, cols):
    """Definition 2: X_[rows | cols], first listed mode fastest in both indices."""
    rows, cols = list(rows), list(cols)
    if sorted(rows + cols) != list(range(X.ndim)):
        raise ValueError("rows and cols must partition the modes")
    Xt = gtranspose(X, rows + cols)
    nr = int(np.prod([X.shape[m] for m in rows], dtype=np.int64))
    nc = int(np.prod([X.shape[m] for m in cols], dtype=np.int64))
    return Xt.reshape((nr, nc), order="F")


def gfold(Mat, rows, cols, shape):
    """Inverse of gunfold: rebuild the tensor of the given shape."""
    rows, cols = list(rows), list(cols)
    perm = rows + cols
    tshape = [shape[m] for m in perm]
    Xt = np.asarray(Mat).reshape(tshape, order="F")
    inv = np.argsort(perm)
    return np.transpose(Xt, tuple(inv))


def unfold(X, k):
    """Mode-k unfolding X_(k) = X_[k | 1..k-1, k+1..N]."""
    return gunfold(X, [k], [m for m in range(X.ndim) if m != k])


def fold(Mat, k, shape):
    """Inverse of unfold (eq. 9: GFold(A, k | 1..k-1, k+1..N))."""
    return gfold(Mat, [k], [m for m in range(len(shape)) if m != k], shape)


def contract(X, Y, n_modes, m_modes):
    """Definition 3: contract modes n_modes of X with modes m_modes of Y.

    The result keeps the free modes of X (in increasing order) followed by the
    free modes of Y (in increasing order); the definition's matricized form
    Z = X_[free|n] Y_[m|free] is literally what ``np.tensordot`` evaluates.
    """
    return np.tensordot(X, Y, axes=(list(n_modes), list(m_modes)))


# ----------------------------------------------------------------------------
# FCTN (Section 1 element formula) and the sub-network of Property 1
# ----------------------------------------------------------------------------

def _labels(N):
    """einsum labels: uppercase for physical modes i_k, lowercase for bonds
    (then the unused uppercase letters: N = 8 has 28 bonds)."""
    phys = string.ascii_uppercase[:N]
    lower = iter(string.ascii_lowercase + string.ascii_uppercase[N:])
    bond = {}
    for (i, j) in bond_pairs(N):
        bond[(i, j)] = bond[(j, i)] = next(lower)
    return phys, bond


def factor_labels(N, k):
    phys, bond = _labels(N)
    return "".join(phys[k] if j == k else bond[(k, j)] for j in range(N))


def fctn(factors):
    """FCTN({A_k}): the element formula of Section 1 evaluated by einsum.

    X(i_1..i_N) = sum over every bond r_{ij} (1 <= i < j <= N, r_{ij} < R_{ij})
    of prod_k A_k(r_{1k}, .., i_k, .., r_{kN}).
    """
    N = len(factors)
    phys, _ = _labels(N)
    spec = ",".join(factor_labels(N, k) for k in range(N)) + "->" + phys
    return np.einsum(spec, *factors, optimize="greedy")


def fctn_bruteforce(factors):
    """FCTN by explicit loops over every index and every bond (tiny inputs)."""
    N = len(factors)
    dims = [factors[k].shape[k] for k in range(N)]
    pairs = bond_pairs(N)
    R = [[0] * N for _ in range(N)]
    for (i, j) in pairs:
        R[i][j] = R[j][i] = factors[i].shape[j]
    X = np.zeros(dims)
    for idx in itertools.product(*[range(d) for d in dims]):
        total = 0.0
        for rs in itertools.product(*[range(R[i][j]) for (i, j) in pairs]):
            r = {}
            for (i, j), v in zip(pairs, rs):
                r[(i, j)] = r[(j, i)] = v
            term = 1.0
            for k in range(N):
                sub = tuple(idx[k] if j == k else r[(k, j)] for j in range(N))
                term *= factors[k][sub]
            total += term
        X[idx] = total
    return X


def subnetwork_modes(N, k):
    """Mode list of M_k (Property 1): for each other factor j in increasing order
    the pair (I_j, R_jk) if j < k, and (R_kj, I_j) if j > k.  Returns
    (labels, row_positions, col_positions) where rows are the bond modes
    (the index vector i of Property 1) and cols the physical modes (n)."""
    phys, bond = _labels(N)
    labels, rows, cols = [], [], []
    for j in range(N):
        if j == k:
            continue
        if j < k:
            pair = [phys[j], bond[(j, k)]]
            cols.append(len(labels)); rows.append(len(labels) + 1)
        else:
            pair = [bond[(k, j)], phys[j]]
            rows.append(len(labels)); cols.append(len(labels) + 1)
        labels.extend(pair)
    return "".join(labels), rows, cols


def subnetwork(factors, k):
    """M_k = FCTN({A}, /A_k) as the order-2(N-1) tensor of Property 1."""
    N = len(factors)
    out, _, _ = subnetwork_modes(N, k)
    spec = ",".join(factor_labels(N, j) for j in range(N) if j != k) + "->" + out
    ops = [factors[j] for j in range(N) if j != k]
    return np.einsum(spec, *ops, optimize="greedy")


def subnetwork_unfolded(factors, k):
    """M_k = GUnfold(M_k, i | n): s_k x prod_{j != k} I_j (Property 1)."""
    N = len(factors)
    _, rows, cols = subnetwork_modes(N, k)
    return gunfold(subnetwork(factors, k), rows, cols)
