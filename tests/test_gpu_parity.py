"""GPU parity: every step of a PAM sweep and whole completions through the C
ABI (libfctn.so) against the FP64 oracle on identical seeded inputs.

Tolerances: float64 plans follow the oracle to 1e-9 relative (the two sides
use different exact routes for the factor solve: Cholesky per Fourier class
on the GPU, eigendecomposition + DFT in the oracle); float32 plans to 1e-5
relative (float32 products, float64 reductions and solves).  Observed
entries are compared bit for bit.
"""

import numpy as np
import pytest
import torch

from oracle import tensor, pam, sylvester
from workloads import make_problem, init_factors, factor_shapes_of

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-9, "f32": 1e-5}
STEP_TOL = {"f64": 1e-12, "f32": 1e-5}

SHAPES = [
    ((37, 29, 6), (5, 3, 4)),                 # ragged tiles on every axis
    ((40, 24, 5), (12, 12, 4)),               # s_1 = 144, 72 output tiles
    ((150, 24, 5), (12, 12, 4)),              # s_1 = 144, 135 tiles: one group of 16 waves x 10
    ((500, 8, 3), (12, 12, 4)),               # s_1 = 144, 333 tiles: two groups of 16 waves x 12
    ((13, 11, 3, 7), (4, 2, 3, 2, 3, 2)),     # order 4, small ranks
    ((24, 28, 3, 6), (8, 3, 8, 3, 8, 3)),     # order 4 with the C3 ranks (s = 192)
    ((31, 29, 3, 20), (2, 2, 4, 2, 4, 4)),    # mode 4: 16-byte slab staging, ragged last tile
    ((9, 7, 3, 4, 5), (2, 3, 1, 2, 3, 1, 2, 2, 1, 3)),            # order 5
    ((4, 3, 5, 2, 3, 4), (2, 1, 2, 2, 1, 2, 1, 2, 3, 1, 2, 2, 2, 1, 2)),  # order 6
]


def _plan(dims, ranks, prec, **kw):
    from paper_2510_22506_amd import Plan
    return Plan(dims, ranks, precision=prec, **kw)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _max_rel(a, b):
    """Largest entry error relative to the largest oracle magnitude: catches a
    few badly wrong entries (a ragged tile edge, a padding row) that a norm
    over the whole matrix would hide."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _bonds(dims, ranks, k):
    return [s for j, s in enumerate(factor_shapes_of(dims, ranks)[k]) if j != k]


def _c_order(mat, lead, bonds):
    """Oracle unfolding (first index fastest) -> the library's (last fastest)."""
    return np.asarray(mat).reshape(list(lead) + list(bonds), order="F").reshape(mat.shape)


def _inputs(dims, ranks, prec, seed):
    rng = np.random.default_rng(seed)
    A = init_factors(rng, dims, ranks)
    store = np.float64 if prec == "f64" else np.float32
    X = rng.random(dims).astype(store)
    mask = (rng.random(dims) < 0.3).astype(np.uint8)
    if prec == "f32":   # the oracle sees the factors the GPU rounds to float
        A = [a.astype(np.float32).astype(np.float64) for a in A]
    return A, X, mask


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_gram_rhs_step(prec, dims, ranks):
    A, X, mask = _inputs(dims, ranks, prec, 1)
    p = _plan(dims, ranks, prec)
    p.set_factors(A)
    p.set_observed(X, mask)
    p.set_x(X)
    Xo = X.astype(np.float64)
    for k in range(len(dims)):
        G, B = p.step_gram_rhs(k)
        M = tensor.subnetwork_unfolded(A, k)
        Go = M @ M.T
        Bo = tensor.unfold(Xo, k) @ M.T + 0.1 * tensor.unfold(A[k], k)
        bonds = _bonds(dims, ranks, k)
        Go = _c_order(Go, bonds, bonds)
        Bo = _c_order(Bo, [dims[k]], bonds)
        Gg, Bg = G.cpu().numpy(), B.cpu().numpy()
        assert _rel(Gg, Go) <= STEP_TOL[prec], (k, _rel(Gg, Go))
        assert _rel(Bg, Bo) <= STEP_TOL[prec], (k, _rel(Bg, Bo))
        assert _max_rel(Gg, Go) <= STEP_TOL[prec], (k, _max_rel(Gg, Go))
        assert _max_rel(Bg, Bo) <= STEP_TOL[prec], (k, _max_rel(Bg, Bo))
        np.testing.assert_array_equal(Gg, Gg.T)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_solve_step(prec, dims, ranks):
    A, X, mask = _inputs(dims, ranks, prec, 2)
    p = _plan(dims, ranks, prec, lam=0.3, delta=0.4)
    p.set_factors(A)
    Xo = X.astype(np.float64)
    for k in range(len(dims)):
        M = tensor.subnetwork_unfolded(A, k)
        Go = M @ M.T
        Bo = tensor.unfold(Xo, k) @ M.T + 0.1 * tensor.unfold(A[k], k)
        Ao = sylvester.solve_fast(Go, Bo, 0.3, 0.4, 0.1)
        bonds = _bonds(dims, ranks, k)
        tr = p.step_solve(k, _c_order(Go, bonds, bonds), _c_order(Bo, [dims[k]], bonds))
        Ag = p.factor(k).cpu().numpy()
        Af = tensor.fold(Ao, k, A[k].shape)
        assert _rel(Ag, Af) <= 1e-9
        assert _max_rel(Ag, Af) <= 1e-9, (k, _max_rel(Ag, Af))
        assert abs(tr - sylvester.trace_term(Ao, 0.4)) <= 1e-9 * abs(tr)


# s_k = R_ka * R_kb at the panel edges of the blocked factorization (1, 31-33,
# 64, 66, 96, 128, 160, 191, 192) with I_k of both parities and I_k = 1, 2
SOLVE_EDGES = [
    ((4, 3, 2), (1, 1, 1)),
    ((9, 8, 2), (8, 4, 4)),
    ((7, 10, 1), (11, 3, 6)),
    ((6, 5, 4), (16, 4, 8)),
    ((5, 4, 3), (16, 12, 10)),
    ((3, 2, 2), (191, 1, 1)),
    ((6, 7, 5), (31, 1, 3)),
    ((5, 6, 4), (12, 8, 8)),
]


@pytest.mark.parametrize("dims,ranks", SOLVE_EDGES)
def test_solve_step_panel_edges(dims, ranks):
    test_solve_step("f64", dims, ranks)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims,ranks", SHAPES)
def test_reconstruct_step(prec, dims, ranks):
    A, X, mask = _inputs(dims, ranks, prec, 3)
    p = _plan(dims, ranks, prec)
    p.set_factors(A)
    Zo = tensor.fctn(A)
    for k in range(len(dims)):
        Z = p.step_reconstruct(k).cpu().numpy()
        assert _rel(Z, Zo) <= STEP_TOL[prec], (k, _rel(Z, Zo))
        assert _max_rel(Z, Zo) <= STEP_TOL[prec], (k, _max_rel(Z, Zo))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(37, 29, 6), (13, 11, 3, 7), (5, 3, 3)])
def test_x_update_step(prec, dims):
    rng = np.random.default_rng(4)
    store = np.float64 if prec == "f64" else np.float32
    X = rng.random(dims).astype(store)
    Z = rng.standard_normal(dims).astype(store)
    mask = (rng.random(dims) < 0.4).astype(np.uint8)
    ranks = (2,) * (len(dims) * (len(dims) - 1) // 2)
    p = _plan(dims, ranks, prec)
    p.set_factors(init_factors(rng, dims, ranks))
    p.set_observed(X, mask)
    p.set_x(X)
    st = p.step_x_update(Z)
    Xg = p.x().cpu().numpy()
    obs = mask != 0
    np.testing.assert_array_equal(Xg[obs], X[obs])
    Xo = pam.x_update(X.astype(np.float64), Z.astype(np.float64), obs, 0.1)
    # rounding bound of (z + rho x) / (1 + rho) with or without a fused multiply-add:
    # a few units in the last place of the operands' magnitude
    eps = np.finfo(store).eps
    scale = (np.abs(Z.astype(np.float64)) + 0.1 * np.abs(X.astype(np.float64))) / 1.1
    assert np.all(np.abs(Xg - Xo)[~obs] <= 4 * eps * scale[~obs])
    Xn = Xg.astype(np.float64)
    rel = np.linalg.norm(Xn - X) / np.linalg.norm(X.astype(np.float64))
    fd = 0.5 * np.sum((Xn - Z.astype(np.float64)) ** 2)
    assert abs(st["rel_change"] - rel) <= 1e-12 * rel
    assert abs(st["f_data"] - fd) <= 1e-12 * fd


def _run_gpu(prob, prec, sweeps, reuse, policy):
    p = _plan(prob.dims, prob.ranks, prec, lam=prob.lam, delta=prob.delta, rho=prob.rho,
              reuse=reuse, order_policy=policy)
    p.set_factors(prob.A0)
    p.set_observed(prob.Y, prob.mask)
    p.sweep(sweeps)
    return p


def _run_oracle(prob, prec, sweeps, reuse, policy):
    A0 = prob.A0
    if prec == "f32":
        A0 = [a.astype(np.float32).astype(np.float64) for a in A0]
    return pam.complete(prob.Y.astype(np.float64), prob.mask != 0, prob.ranks, prob.lam,
                        prob.delta, prob.rho, sweeps, A0, reuse=reuse, order_policy=policy)


@pytest.mark.parametrize("reuse,policy", [(True, 1), (False, 0), (True, 0)])
@pytest.mark.parametrize("name,dims", [("c1", (20, 18, 6)), ("c3", (12, 14, 3, 5))])
def test_sweeps_f64(name, dims, reuse, policy):
    prob = make_problem(name, seed=5, dims=dims, precision="f64", sr=0.3)
    sweeps = 8
    p = _run_gpu(prob, "f64", sweeps, reuse, policy)
    Xo, fo, so = _run_oracle(prob, "f64", sweeps, reuse, policy)
    Xg = p.x().cpu().numpy()
    assert _rel(Xg, Xo) <= TOL["f64"], _rel(Xg, Xo)
    for k in range(len(dims)):
        assert _rel(p.factor(k).cpu().numpy(), fo[k]) <= TOL["f64"]
    obs = prob.mask != 0
    np.testing.assert_array_equal(Xg[obs], prob.Y[obs])
    h = p.history(0, sweeps)
    for t in range(sweeps):
        assert abs(h[t]["rel_change"] - so["rel_change"][t]) <= 1e-8 * so["rel_change"][t]
        assert abs(h[t]["objective"] - so["objective"][t]) <= 1e-8 * so["objective"][t]


@pytest.mark.parametrize("name,dims,sweeps", [
    ("c2", (64, 48, 3), 20), ("c3", (24, 28, 3, 6), 10), ("c4", (40, 36, 31), 10)])
def test_sweeps_f32(name, dims, sweeps):
    prob = make_problem(name, seed=6, dims=dims, precision="f32", sr=0.2)
    p = _run_gpu(prob, "f32", sweeps, True, 1)
    Xo, _, so = _run_oracle(prob, "f32", sweeps, True, 1)
    Xg = p.x().cpu().numpy()
    assert _rel(Xg, Xo) <= TOL["f32"], _rel(Xg, Xo)
    obs = prob.mask != 0
    np.testing.assert_array_equal(Xg[obs], prob.Y[obs])


@pytest.mark.parametrize("dims,ranks", [((2, 5, 3), (2, 3, 2)), ((1, 6, 4), (1, 2, 3)),
                                        ((5, 3, 3), (2, 2, 2)), ((3, 2, 1, 4), (2, 1, 2, 1, 2, 2))])
def test_sweeps_degenerate_modes(dims, ranks):
    # modes of size 1 and 2 (a single Fourier class, the n = 2 Laplacian) and
    # tensors smaller than one tile
    prob = make_problem("c1", seed=8, dims=(4, 4, 4), precision="f64", sr=0.5)
    rng = np.random.default_rng(9)
    prob.dims, prob.ranks = dims, ranks
    prob.truth = rng.random(dims)
    prob.mask = (rng.random(dims) < 0.5).astype(np.uint8)
    prob.Y = np.where(prob.mask != 0, prob.truth, 0.0)
    prob.A0 = init_factors(rng, dims, ranks)
    p = _run_gpu(prob, "f64", 5, True, 1)
    Xo, _, _ = _run_oracle(prob, "f64", 5, True, 1)
    assert _rel(p.x().cpu().numpy(), Xo) <= TOL["f64"]


def test_c1_full_reuse_on_and_off():
    prob = make_problem("c1", seed=0)
    for reuse in (True, False):
        p = _run_gpu(prob, "f64", prob.sweeps, reuse, 0)
        Xo, _, so = _run_oracle(prob, "f64", prob.sweeps, reuse, 0)
        Xg = p.x().cpu().numpy()
        assert _rel(Xg, Xo) <= TOL["f64"], (reuse, _rel(Xg, Xo))
        obj = [h["objective"] for h in p.history(0, prob.sweeps)]
        assert all(b <= a * (1 + 1e-12) for a, b in zip(obj, obj[1:]))


def test_reuse_on_off_bitwise_and_deterministic():
    prob = make_problem("c3", seed=7, dims=(16, 18, 3, 5), precision="f32", sr=0.2)
    xs = []
    for reuse in (True, False, True):
        p = _run_gpu(prob, "f32", 6, reuse, 1)
        xs.append(p.x().cpu().numpy())
    np.testing.assert_array_equal(xs[0], xs[1])
    np.testing.assert_array_equal(xs[0], xs[2])


def test_nan_off_omega_and_numeric_error():
    from paper_2510_22506_amd import FctnError
    prob = make_problem("c1", seed=1, dims=(16, 12, 5))
    Ynan = np.where(prob.mask != 0, prob.Y, np.nan)
    a = _run_gpu(prob, "f64", 4, True, 0).x().cpu().numpy()
    prob2 = make_problem("c1", seed=1, dims=(16, 12, 5))
    prob2.Y = Ynan
    b = _run_gpu(prob2, "f64", 4, True, 0).x().cpu().numpy()
    np.testing.assert_array_equal(a, b)
    Ybad = prob.Y.copy()
    Ybad[np.argwhere(prob.mask != 0)[0][0], ...] = np.inf
    p = _plan(prob.dims, prob.ranks, "f64")
    p.set_factors(prob.A0)
    with pytest.raises(FctnError) as e:
        p.set_observed(np.where(prob.mask != 0, Ybad, 0), prob.mask)
    assert e.value.status == 4
