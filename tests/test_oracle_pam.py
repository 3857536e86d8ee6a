"""Pins for the oracle's PAM loop (Algorithms 1-2): exact block-decrease
identities (Section 3.5, condition 4), monotone objective, observed entries
bit-exact, reuse on == reuse off, the Eckart-Young limit for N = 2, the
stopping rule, and the per-sweep flop counts of Tables 1-2."""

import numpy as np
import pytest

from oracle import pam, tensor, sylvester, laplacian, metrics
from workloads import make_problem, init_factors, factor_shapes_of


def _rand_problem(dims, ranks, sr=0.3, seed=0):
    rng = np.random.default_rng(seed)
    truth = rng.random(dims)
    mask = rng.random(dims) < sr
    Y = np.where(mask, truth, 0.0)
    A0 = init_factors(rng, dims, ranks)
    return truth, Y, mask, A0


def _objective(X, fs, lam, delta):
    return pam.objective(X, fs, [lam] * len(fs), [delta] * len(fs))


@pytest.mark.parametrize("dims,ranks,k", [
    ((6, 5, 4), (3, 2, 2), 0), ((6, 5, 4), (3, 2, 2), 2),
    ((4, 3, 3, 5), (2, 2, 3, 1, 2, 2), 1), ((4, 3, 3, 5), (2, 2, 3, 1, 2, 2), 3),
    ((4, 3, 3, 2, 3), (2, 1, 2, 2, 2, 1, 2, 2, 1, 2), 0),
    ((4, 3, 3, 2, 3), (2, 1, 2, 2, 2, 1, 2, 2, 1, 2), 2),
    ((4, 3, 3, 2, 3), (2, 1, 2, 2, 2, 1, 2, 2, 1, 2), 4),
])
def test_factor_block_exact_decrease(dims, ranks, k):
    # f_old - f_new = rho ||D||^2 + 1/2 (tr(D G D^T) + lam tr(D^T L D)), D = A_new - A_old
    lam, delta, rho = 0.3, 0.5, 0.1
    _, Y, mask, A0 = _rand_problem(dims, ranks, seed=k)
    X = np.where(mask, Y, 0.0)
    fs = [a.copy() for a in A0]
    f_old = _objective(X, fs, lam, delta)
    M = tensor.subnetwork_unfolded(fs, k)
    G = M @ M.T
    A_old = tensor.unfold(fs[k], k)
    A_new = sylvester.solve_fast(G, sylvester.rhs(tensor.unfold(X, k), M, A_old, rho), lam, delta, rho)
    fs[k] = tensor.fold(A_new, k, fs[k].shape)
    f_new = _objective(X, fs, lam, delta)
    D = A_new - A_old
    L = laplacian.matrix(dims[k], delta)
    pred = rho * np.sum(D * D) + 0.5 * (np.trace(D @ G @ D.T) + lam * np.trace(D.T @ L @ D))
    assert abs((f_old - f_new) - pred) <= 1e-9 * max(1.0, abs(f_old))
    assert f_old - f_new >= rho * np.sum(D * D) * (1 - 1e-9)


def test_x_block_exact_decrease():
    # f(A, X_old) - f(A, X_new) = (1/2 + rho) ||X_new - X_old||^2 (eq. 10 is the prox step)
    dims, ranks, rho = (5, 6, 4), (2, 3, 2), 0.1
    _, Y, mask, A0 = _rand_problem(dims, ranks, seed=3)
    X = np.where(mask, Y, 0.0)
    Z = tensor.fctn(A0)
    Xn = pam.x_update(X, Z, mask, rho)
    f_old = 0.5 * np.sum((X - Z) ** 2)
    f_new = 0.5 * np.sum((Xn - Z) ** 2)
    assert abs((f_old - f_new) - (0.5 + rho) * np.sum((Xn - X) ** 2)) < 1e-10 * f_old


@pytest.mark.parametrize("reuse", [False, True])
@pytest.mark.parametrize("dims,ranks,policy", [
    ((8, 7, 5), (3, 2, 2), 0),
    ((5, 4, 3, 6), (2, 2, 3, 2, 2, 2), 1),
    ((4, 3, 3, 2, 3), (2, 1, 2, 2, 2, 1, 2, 2, 1, 2), 1),
])
def test_objective_monotone_blockwise(reuse, dims, ranks, policy):
    _, Y, mask, A0 = _rand_problem(dims, ranks, seed=1)
    _, _, st = pam.complete(Y, mask, ranks, 1e-2, 0.5, 0.1, 6, A0, reuse=reuse,
                            order_policy=policy, record_blocks=True)
    vals = [v for (_, _, v) in st["blocks"]]
    assert all(b <= a * (1 + 1e-12) + 1e-12 for a, b in zip(vals, vals[1:]))


def test_observed_bit_exact_and_nan_off_omega():
    dims, ranks = (6, 5, 4), (2, 2, 2)
    truth, Y, mask, A0 = _rand_problem(dims, ranks, seed=2)
    X1, f1, _ = pam.complete(Y, mask, ranks, 1e-2, 0.5, 0.1, 4, A0)
    np.testing.assert_array_equal(X1[mask], Y[mask])
    Ynan = np.where(mask, Y, np.nan)
    X2, f2, _ = pam.complete(Ynan, mask, ranks, 1e-2, 0.5, 0.1, 4, A0)
    np.testing.assert_array_equal(X1, X2)
    for a, b in zip(f1, f2):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("dims,ranks,policy", [
    ((9, 8, 5), (3, 2, 2), 0),
    ((5, 4, 3, 6), (2, 2, 3, 2, 2, 2), 0),
    ((5, 4, 3, 6), (2, 2, 3, 2, 2, 2), 1),
    ((4, 3, 5, 2, 3), (2, 1, 2, 2, 3, 1, 2, 2, 1, 2), 0),
    ((3, 2, 3, 2, 2, 3), (2, 1, 2, 1, 2, 2, 1, 2, 1, 2, 1, 2, 2, 1, 2), 0),
])
def test_reuse_on_equals_off(dims, ranks, policy):
    _, Y, mask, A0 = _rand_problem(dims, ranks, seed=5)
    Xa, fa, sa = pam.complete(Y, mask, ranks, 1e-2, 0.5, 0.1, 5, A0, reuse=False, order_policy=policy)
    Xb, fb, sb = pam.complete(Y, mask, ranks, 1e-2, 0.5, 0.1, 5, A0, reuse=True, order_policy=policy)
    assert np.linalg.norm(Xa - Xb) <= 1e-12 * np.linalg.norm(Xa)
    for a, b in zip(fa, fb):
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)


@pytest.mark.parametrize("dims,ranks", [
    ((4, 5, 3), (2, 3, 2)),
    ((3, 4, 2, 3), (2, 1, 2, 3, 2, 2)),
    ((3, 2, 3, 2, 2), (2, 1, 2, 2, 2, 1, 2, 2, 1, 2)),
])
def test_loop_subnetwork_equals_property1_unfolding(dims, ranks):
    # the PAM loop's M_k (pair-cache route for N = 4 with reuse, factor chain
    # otherwise) against tensor.subnetwork_unfolded, itself pinned to the
    # brute-force index sum; then, after a factor changes, the cache must hand
    # out the M_k of the new factors (version bump) and keep the old ones
    # while no version moves
    rng = np.random.default_rng(3)
    fs = init_factors(rng, dims, ranks)
    N = len(dims)
    for reuse in (False, True):
        cache = pam.PairCache()
        gcache = pam.GroupCache()
        versions = [0] * N
        for k in range(N):
            M = pam.subnetwork_M(fs, k, reuse, cache, versions, None, gcache)
            Mo = tensor.subnetwork_unfolded(fs, k)
            assert M.shape == Mo.shape
            assert np.max(np.abs(M - Mo)) <= 1e-12 * np.max(np.abs(Mo)), (reuse, k)
        changed = [f.copy() for f in fs]
        j = N - 1
        changed[j] = rng.standard_normal(fs[j].shape)
        k = 0
        stale = pam.subnetwork_M(changed, k, reuse, cache, versions, None, gcache)
        fresh_versions = list(versions)
        fresh_versions[j] += 1
        fresh = pam.subnetwork_M(changed, k, reuse, cache, fresh_versions, None, gcache)
        Mo_new = tensor.subnetwork_unfolded(changed, k)
        assert np.max(np.abs(fresh - Mo_new)) <= 1e-12 * np.max(np.abs(Mo_new))
        if reuse and N >= 4:
            # the group holding the last factor (pair (3, 4) for N = 4, the
            # group {3..N} for N = 5) cached from the old factors: still the
            # old M_1 while no version moves
            Mo_old = tensor.subnetwork_unfolded(fs, k)
            assert np.max(np.abs(stale - Mo_old)) <= 1e-12 * np.max(np.abs(Mo_old))
        else:
            assert np.max(np.abs(stale - Mo_new)) <= 1e-12 * np.max(np.abs(Mo_new))


def test_order2_full_observation_reaches_eckart_young():
    # N = 2, every entry observed, lambda = 0: PAM on ||X - A1 A2||^2 converges
    # to the best rank-R approximation, whose error is the tail singular values
    rng = np.random.default_rng(11)
    I1, I2, R = 12, 10, 3
    U, _ = np.linalg.qr(rng.standard_normal((I1, I1)))
    V, _ = np.linalg.qr(rng.standard_normal((I2, I2)))
    sig = np.array([10.0, 8.0, 6.0, 1.0, 0.5, 0.2, 0.1, 0.05, 0.02, 0.01])
    Y = U[:, :10] @ np.diag(sig) @ V.T
    mask = np.ones_like(Y, dtype=bool)
    A0 = init_factors(rng, (I1, I2), (R,))
    X, fs, st = pam.complete(Y, mask, (R,), 0.0, 0.5, 0.1, 400, A0)
    err = np.linalg.norm(Y - fs[0] @ fs[1])
    assert abs(err - np.sqrt(np.sum(sig[R:] ** 2))) < 1e-6


def test_stopping_rule():
    dims, ranks = (8, 7, 5), (2, 2, 2)
    _, Y, mask, A0 = _rand_problem(dims, ranks, seed=6)
    _, _, st = pam.complete(Y, mask, ranks, 1e-2, 0.5, 0.1, 500, A0, tol=1e-3)
    assert st["sweeps_done"] < 500
    assert st["rel_change"][-1] <= 1e-3
    assert all(r > 1e-3 for r in st["rel_change"][:-1])


def _counts(dims, ranks, reuse, policy, sweeps):
    _, Y, mask, A0 = _rand_problem(dims, ranks, seed=7)
    cs = []
    pam.complete(Y, mask, ranks, 1e-2, 0.5, 0.1, sweeps, A0, reuse=reuse,
                 order_policy=policy, counters=cs)
    return [c.flops for c in cs]


def test_table1_counts_order4():
    # Table 1 (N = 4, every I and R equal): the printed per-sweep complexities
    I, R = 6, 2
    dims, ranks = (I,) * 4, (R,) * 6
    alg1 = _counts(dims, ranks, False, 0, 3)
    alg2 = _counts(dims, ranks, True, 1, 3)
    for c in alg1:
        assert c["M"] == 8 * (I**2 + I**3) * R**5
        assert c["X"] == 2 * (I**2 + I**3) * R**5 + 2 * I**4 * R**3
        assert c["gram"] + c["rhs"] == 8 * (I**3 * R**6 + I**4 * R**3)
    assert alg2[0]["M"] == 4 * I**2 * R**5 + 8 * I**3 * R**5
    for c in alg2[1:]:
        assert c["M"] == 2 * I**2 * R**5 + 8 * I**3 * R**5
    for c in alg2:
        assert c["X"] == 2 * I**4 * R**3
        assert c["gram"] + c["rhs"] == 8 * (I**3 * R**6 + I**4 * R**3)


def test_table1_needs_the_alternating_order():
    # with the fixed order (1,2,3,4) the cached pair A_1 x A_2 is stale at the
    # start of every sweep, so t >= 2 costs as much as t = 1: the order
    # alternation is what produces Table 1's t >= 2 row
    I, R = 6, 2
    c = _counts((I,) * 4, (R,) * 6, True, 0, 3)
    assert c[1]["M"] == 4 * I**2 * R**5 + 8 * I**3 * R**5


@pytest.mark.parametrize("N,I,R", [(3, 5, 2), (5, 3, 2)])
def test_table2_counts_algorithm1(N, I, R):
    dims, ranks = (I,) * N, (R,) * (N * (N - 1) // 2)
    c = _counts(dims, ranks, False, 0, 1)[0]
    m = 2 * N * sum(I**K * R**(K * (N - K) + K - 1) for K in range(2, N))
    x = 2 * sum(I**K * R**(K * (N - K) + K - 1) for K in range(2, N + 1))
    mm = 2 * N * (I**(N - 1) * R**(2 * (N - 1)) + I**N * R**(N - 1))
    assert c["M"] == m and c["X"] == x and c["gram"] + c["rhs"] == mm


@pytest.mark.parametrize("N,I,R", [(5, 3, 2), (6, 2, 2)])
def test_table2_counts_algorithm2(N, I, R):
    # Table 2, Algorithm 2 column for the N-th order case: computing M_k costs
    # 4I^2R^{2N-3} + 6I^3R^{3N-7} + .. + 2N I^{N-1}R^{2N-3} per sweep (the
    # j-factor groups for j = 2 .. N-2, then N final contractions), every
    # sweep; the X step reuses M'_last
    dims, ranks = (I,) * N, (R,) * (N * (N - 1) // 2)
    m = sum(2 * j * I**j * R**(j * (N - j) + j - 1) for j in range(2, N - 1))
    m += 2 * N * I**(N - 1) * R**(2 * N - 3)
    for c in _counts(dims, ranks, True, 0, 3):
        assert c["M"] == m
        assert c["X"] == 2 * I**N * R**(N - 1)
    # and it is below Algorithm 1's count
    a1 = _counts(dims, ranks, False, 0, 1)[0]["M"]
    assert m < a1


def test_table2_x_count_algorithm2_order3():
    I, R = 5, 2
    c = _counts((I,) * 3, (R,) * 3, True, 0, 2)
    for cc in c:
        assert cc["X"] == 2 * I**3 * R**2
        assert cc["M"] == 6 * I**2 * R**3     # no M saving at N = 3 (Table 2 rule)


def test_psnr_definition():
    truth = np.zeros((4, 5, 3))
    recon = truth.copy()
    recon[..., 0] += 0.1          # slice MSE 1e-2 -> 20 dB
    recon[..., 1] += 0.01         # 1e-4 -> 40 dB
    recon[..., 2] += 0.001        # 1e-6 -> 60 dB
    assert abs(metrics.psnr(truth, recon) - 40.0) < 1e-9


def test_generators_shapes_and_ranges():
    p = make_problem("c1", seed=0)
    assert p.Y.shape == (32, 32, 8) and p.Y.dtype == np.float64
    assert 0.0 <= p.truth.min() and p.truth.max() <= 1.0
    assert [a.shape for a in p.A0] == factor_shapes_of(p.dims, p.ranks)
    assert abs(p.mask.mean() - 0.3) < 0.03
    np.testing.assert_array_equal(p.Y[p.mask == 0], 0)
    q = make_problem("c3", seed=1, dims=(24, 28, 3, 6))
    assert q.Y.dtype == np.float32 and q.Y.shape == (24, 28, 3, 6)
    r = make_problem("c4", seed=2, dims=(40, 36, 31))
    assert r.truth.min() == 0.0 and r.truth.max() == 1.0
    m = make_problem("c6", seed=3, dims=(30, 28, 4, 5))
    assert m.Y.shape == (30, 28, 4, 5) and m.truth.min() == 0.0 and m.truth.max() == 1.0
    assert [a.shape for a in m.A0] == factor_shapes_of(m.dims, m.ranks)
    # dates differ (blobs drift and change amplitude between acquisitions)
    assert np.abs(m.truth[..., 0] - m.truth[..., 4]).max() > 1e-3
    o5 = make_problem("c7", seed=5, dims=(4, 5, 3, 4, 2))
    assert o5.Y.shape == (4, 5, 3, 4, 2) and o5.truth.min() == 0.0 and o5.truth.max() == 1.0
    assert [a.shape for a in o5.A0] == factor_shapes_of(o5.dims, o5.ranks)
    v = make_problem("c5", seed=4, dims=(20, 22, 3, 4))
    assert v.Y.shape == (20, 22, 3, 4) and abs(v.mask.mean() - 0.05) < 0.03


def test_c1_quality_improves():
    # on the low-rank C1 tensor the completion beats the zero-filled input
    p = make_problem("c1", seed=0, sweeps=15)
    X, _, st = pam.complete(p.Y, p.mask != 0, p.ranks, p.lam, p.delta, p.rho, p.sweeps, p.A0)
    assert metrics.psnr(p.truth, X) > metrics.psnr(p.truth, p.Y) + 5.0
    assert all(b <= a * (1 + 1e-12) for a, b in zip(st["objective"], st["objective"][1:]))


# --- asymmetric extrapolation (Section 4.2) --------------------------------

def _small(seed=5, dims=(6, 5, 4), ranks=(2, 3, 2)):
    rng = np.random.default_rng(seed)
    Y = rng.random(dims)
    mask = rng.random(dims) < 0.4
    A0 = init_factors(rng, dims, ranks)
    return Y, mask, ranks, A0


def test_extrapolation_alpha_zero_is_plain():
    Y, mask, ranks, A0 = _small()
    X0, F0, s0 = pam.complete(Y, mask, ranks, 0.3, 0.5, 0.1, 3, A0)
    X1, F1, s1 = pam.complete(Y, mask, ranks, 0.3, 0.5, 0.1, 3, A0, extrapolation=(0.0, 0.7))
    # equal up to the summation order of BLAS on a differently strided copy
    np.testing.assert_allclose(X1, X0, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(s1["objective"], s0["objective"], rtol=1e-12)


@pytest.mark.parametrize("alpha,beta", [(0.5, 0.5), (0.3, 0.6), (0.4, 1.0), (0.7, 0.0)])
def test_extrapolation_proximal_limit(alpha, beta):
    # rho -> infinity pins every subproblem to its proximal centre
    # (A_new = A^t + O(1/rho)), so after one sweep each factor is
    # (1 + alpha - alpha beta) times its initial value; beta = 1 leaves it
    # unchanged and beta = 0 scales it by 1 + alpha.
    Y, mask, ranks, A0 = _small()
    rho = 1e10
    _, F, _ = pam.complete(Y, mask, ranks, 0.3, 0.5, rho, 1, A0,
                           extrapolation=(alpha, beta))
    c = 1.0 + alpha - alpha * beta
    for a, a0 in zip(F, A0):
        np.testing.assert_allclose(a, c * a0, rtol=1e-6, atol=1e-8)


def test_extrapolation_first_order_weight():
    # to first order in 1/rho the plain update moves the first factor by D/rho;
    # the extrapolated factor is c A^t plus (1 + alpha) times that move (the
    # extrapolation acts on the new factor, not on the proximal centre, which
    # would give alpha times the move)
    Y, mask, ranks, A0 = _small(seed=8)
    rho, alpha, beta = 1e6, 0.5, 0.5
    _, Fp, _ = pam.complete(Y, mask, ranks, 0.3, 0.5, rho, 1, A0)
    _, Fe, _ = pam.complete(Y, mask, ranks, 0.3, 0.5, rho, 1, A0,
                            extrapolation=(alpha, beta))
    move = Fp[0] - A0[0]
    extra = Fe[0] - (1.0 + alpha - alpha * beta) * A0[0]
    assert np.abs(move).max() > 1e-7
    np.testing.assert_allclose(extra, (1.0 + alpha) * move, rtol=1e-4,
                               atol=1e-4 * np.abs(move).max())


# --- rank-increasing schedule ----------------------------------------------

from workloads import rank_growth_draws  # noqa: E402


@pytest.mark.parametrize("dims,r_old,r_new", [
    ((3, 4, 2), (1, 1, 1), (2, 2, 2)),
    ((3, 4, 2), (1, 2, 1), (2, 2, 3)),
    ((2, 3, 2, 2), (1, 1, 1, 1, 1, 1), (2, 1, 2, 2, 1, 2)),
])
def test_grow_factors_leaves_fctn_unchanged(dims, r_old, r_new):
    # the embedded network equals the old one entry by entry (brute-force
    # index sum over every bond value), old entries are kept, and the draws
    # land only where no bond (j, k), j < k, takes a new value
    rng = np.random.default_rng(3)
    old = init_factors(rng, dims, r_old)
    fills = rank_growth_draws(4, dims)(0, r_new)
    new = pam.grow_factors(old, dims, r_old, r_new, fills)
    np.testing.assert_allclose(tensor.fctn_bruteforce(new), tensor.fctn_bruteforce(old),
                               rtol=1e-12, atol=1e-12)
    N = len(dims)
    Ro = tensor.rank_matrix(r_old, N)
    for k in range(N):
        assert new[k].shape == factor_shapes_of(dims, r_new)[k]
        np.testing.assert_array_equal(new[k][tuple(slice(0, n) for n in old[k].shape)], old[k])
        for idx in np.ndindex(new[k].shape):
            if all(idx[j] < old[k].shape[j] for j in range(N)):
                continue
            lower_new = any(idx[j] >= Ro[j][k] for j in range(k))
            assert new[k][idx] == (0.0 if lower_new else fills[k][idx]), (k, idx)


def test_rank_schedule_never_growing_is_fixed_rank():
    Y, mask, _, _ = _small()
    dims = Y.shape
    ones = (1, 1, 1)
    A0 = init_factors(np.random.default_rng(2), dims, ones)
    fill = rank_growth_draws(9, dims)
    X0, F0, s0 = pam.complete(Y, mask, ones, 0.3, 0.5, 0.1, 4, A0)
    X1, F1, s1 = pam.complete_rank_increasing(Y, mask, (2, 3, 2), 0.3, 0.5, 0.1, 4, A0, fill,
                                              tau=0.0)
    np.testing.assert_allclose(X1, X0, rtol=1e-12, atol=1e-14)
    assert s1["ranks"] == [ones] * 4


def test_rank_schedule_grows_to_the_maximum():
    # tau = inf grows after every sweep: ones, then +1 per bond, capped
    Y, mask, _, _ = _small()
    dims = Y.shape
    A0 = init_factors(np.random.default_rng(2), dims, (1, 1, 1))
    fill = rank_growth_draws(9, dims)
    X, F, st = pam.complete_rank_increasing(Y, mask, (2, 4, 3), 0.3, 0.5, 0.1, 6, A0, fill,
                                            tau=np.inf)
    assert st["ranks"] == [(1, 1, 1), (2, 2, 2), (2, 3, 3), (2, 4, 3), (2, 4, 3), (2, 4, 3)]
    assert [f.shape for f in F] == factor_shapes_of(dims, (2, 4, 3))
    np.testing.assert_array_equal(X[mask], Y[mask])
    # at fixed ranks the objective does not increase
    obj = st["objective"]
    assert obj[4] <= obj[3] * (1 + 1e-12) and obj[5] <= obj[4] * (1 + 1e-12)
