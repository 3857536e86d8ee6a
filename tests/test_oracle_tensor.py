"""Pins for the oracle's tensor algebra: the FCTN element formula against a
brute-force index sum, Definitions 2-3 against explicit index maps, Property 1
for every mode, and the Gram of M_k against an independent route."""

import itertools

import numpy as np
import pytest

from oracle import tensor


def _factors(dims, ranks, seed=0):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) for s in tensor.factor_shapes(dims, ranks)]


@pytest.mark.parametrize("dims,ranks", [
    ((4, 5, 3), (2, 3, 2)),
    ((3, 4, 2, 3), (2, 2, 2, 2, 2, 2)),
    ((3, 2, 4, 2), (1, 2, 3, 2, 1, 2)),
    ((2, 3, 2, 2, 2), (2, 1, 2, 2, 1, 2, 1, 2, 2, 1)),
    ((2, 2, 1, 2, 2, 2), (2, 1, 1, 2, 1, 1, 2, 1, 2, 2, 1, 1, 2, 1, 2)),
    # orders 7 and 8 (8 has more bonds than lowercase einsum labels)
    ((2, 1, 2, 2, 1, 2, 2), (2, 1, 1, 1, 1, 2, 1, 1, 2, 1, 1, 1, 1, 2, 1, 1, 1, 1, 1, 2, 1)),
    ((2, 2, 1, 2, 1, 2, 1, 2), (2, 1, 1, 1, 1, 1, 2, 1, 1, 2, 1, 1, 1, 1, 1, 1, 1, 2, 1,
                                1, 1, 1, 1, 1, 2, 1, 1, 2)),
])
def test_fctn_matches_bruteforce(dims, ranks):
    fs = _factors(dims, ranks)
    np.testing.assert_allclose(tensor.fctn(fs), tensor.fctn_bruteforce(fs), rtol=1e-12, atol=1e-12)


def test_fctn_order2_is_matrix_product():
    fs = _factors((5, 7), (3,))
    np.testing.assert_allclose(tensor.fctn(fs), fs[0] @ fs[1], rtol=1e-13)


def test_fctn_order3_explicit_sum():
    # X(i,j,k) = sum_{a,b,c} A1(i,a,b) A2(a,j,c) A3(b,c,k): the Section 1 formula for N = 3
    fs = _factors((3, 4, 5), (2, 3, 2))
    A1, A2, A3 = fs
    X = np.zeros((3, 4, 5))
    for i, j, k in itertools.product(range(3), range(4), range(5)):
        for a, b, c in itertools.product(range(2), range(3), range(2)):
            X[i, j, k] += A1[i, a, b] * A2[a, j, c] * A3[b, c, k]
    np.testing.assert_allclose(tensor.fctn(fs), X, rtol=1e-12)


def test_gunfold_index_map_definition2():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((2, 3, 4, 5))
    rows, cols = [2, 0], [3, 1]
    M = tensor.gunfold(X, rows, cols)
    shp = X.shape
    for idx in itertools.product(*[range(d) for d in shp]):
        # j1 = i_{n1} + (i_{n2}) I_{n1}; j2 likewise (0-based form of Definition 2)
        j1 = idx[rows[0]] + idx[rows[1]] * shp[rows[0]]
        j2 = idx[cols[0]] + idx[cols[1]] * shp[cols[0]]
        assert M[j1, j2] == X[idx]
    np.testing.assert_array_equal(tensor.gfold(M, rows, cols, shp), X)


def test_unfold_fold_roundtrip_and_mode_k():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3, 4, 5))
    for k in range(3):
        U = tensor.unfold(X, k)
        assert U.shape == (X.shape[k], X.size // X.shape[k])
        np.testing.assert_array_equal(tensor.fold(U, k, X.shape), X)
    # mode-2 unfolding: column index i1 + i3 * I1 (first remaining mode fastest)
    U = tensor.unfold(X, 1)
    assert U[2, 1 + 3 * 3] == X[1, 2, 3]


def test_contract_definition3_explicit():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((2, 3, 4))
    Y = rng.standard_normal((4, 5, 3))
    Z = tensor.contract(X, Y, [1, 2], [2, 0])
    ref = np.zeros((2, 5))
    for a, b, c, d in itertools.product(range(2), range(3), range(4), range(5)):
        ref[a, d] += X[a, b, c] * Y[c, d, b]
    np.testing.assert_allclose(Z, ref, rtol=1e-13)


@pytest.mark.parametrize("dims,ranks", [
    ((4, 5, 3), (2, 3, 2)),
    ((3, 4, 2, 3), (2, 3, 2, 1, 2, 2)),
    ((2, 3, 2, 2, 3), (2, 1, 2, 2, 1, 2, 1, 2, 2, 1)),
    ((2, 2, 3, 2, 2, 2), (2, 1, 1, 2, 1, 1, 2, 1, 2, 2, 1, 1, 2, 1, 2)),
])
def test_property1_every_mode(dims, ranks):
    fs = _factors(dims, ranks, seed=4)
    X = tensor.fctn(fs)
    for k in range(len(dims)):
        Mk = tensor.subnetwork_unfolded(fs, k)
        Ak = tensor.unfold(fs[k], k)
        np.testing.assert_allclose(Ak @ Mk, tensor.unfold(X, k), rtol=1e-11, atol=1e-12)


def test_subnetwork_bruteforce_order3():
    # M_1(r12, i2, r13, i3) = sum_c A2(r12, i2, c) A3(r13, c, i3), Property 1 mode order
    fs = _factors((3, 4, 5), (2, 3, 2), seed=5)
    _, A2, A3 = fs
    M = tensor.subnetwork(fs, 0)
    ref = np.zeros((2, 4, 3, 5))
    for a, j, b, k, c in itertools.product(range(2), range(4), range(3), range(5), range(2)):
        ref[a, j, b, k] += A2[a, j, c] * A3[b, c, k]
    np.testing.assert_allclose(M, ref, rtol=1e-13)


def test_gram_by_factor_grams_order3():
    # G_1 = M_1 M_1^T equals sum_{c,c'} W2[a,c,a',c'] W3[b,c,b',c'] with
    # W_j the per-factor Gram over its physical index: an O(prod R) route.
    fs = _factors((6, 5, 4), (3, 2, 2), seed=6)
    _, A2, A3 = fs
    M = tensor.subnetwork_unfolded(fs, 0)
    W2 = np.einsum("ajc,xjy->acxy", A2, A2)
    W3 = np.einsum("bck,xyk->bcxy", A3, A3)
    Gt = np.einsum("acxy,bcwy->abxw", W2, W3)           # (r12, r13, r12', r13')
    G = Gt.reshape((6, 6), order="F")                    # first bond fastest
    np.testing.assert_allclose(M @ M.T, G, rtol=1e-11)


def test_gram_by_factor_grams_order4():
    fs = _factors((3, 4, 2, 3), (2, 3, 2, 2, 1, 2), seed=7)
    A1, A2, A3, A4 = fs
    k = 2   # M_3: rows (r13, r23, r34), the other factors A1, A2, A4
    M = tensor.subnetwork_unfolded(fs, k)
    # bonds: r12=a r13=b r14=c r23=d r24=e r34=f; primed copies in uppercase
    W1 = np.einsum("iabc,iABC->abcABC", A1, A1)
    W2 = np.einsum("ajde,AjDE->adeADE", A2, A2)
    W4 = np.einsum("cefl,CEFl->cefCEF", A4, A4)
    # contract r12, r14, r24 (and their primes) between the three Grams
    Gt = np.einsum("abcABC,adeADE,cefCEF->bdfBDF", W1, W2, W4)
    s = M.shape[0]
    G = Gt.reshape((s, s), order="F")
    np.testing.assert_allclose(M @ M.T, G, rtol=1e-11)
