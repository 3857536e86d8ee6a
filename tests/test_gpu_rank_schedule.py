"""GPU parity of rank growth (fctn_regrow) and of the rank-increasing
schedule against the FP64 oracle: the embedded factors bit for bit, X
carried over bit for bit, FCTN(A) unchanged by the growth, whole schedules
(ranks per sweep, X, per-sweep objective) in float64 to 1e-9 and float32 to
1e-5, and the rejected argument combinations."""

import numpy as np
import pytest

from oracle import pam
from workloads import make_problem, init_factors, rank_growth_draws

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dims,r_old,r_new", [
    ((20, 18, 6), (1, 1, 1), (2, 2, 2)),
    ((20, 18, 6), (2, 3, 1), (3, 3, 4)),
    ((12, 10, 3, 5), (1, 1, 1, 1, 1, 1), (2, 2, 2, 2, 2, 2)),
    ((12, 10, 3, 5), (2, 1, 3, 1, 2, 1), (3, 2, 3, 2, 2, 3)),
])
def test_regrow_embeds_factors_and_keeps_fctn(dims, r_old, r_new):
    from paper_2510_22506_amd import Plan
    rng = np.random.default_rng(21)
    Y = rng.random(dims)
    mask = (rng.random(dims) < 0.4).astype(np.uint8)
    A = init_factors(rng, dims, r_old)
    p = Plan(dims, r_old, precision="f64")
    p.set_factors(A)
    p.set_observed(np.where(mask != 0, Y, 0.0), mask)
    p.sweep(2)
    X_old = p.x().cpu().numpy()
    F_old = [p.factor(k).cpu().numpy() for k in range(len(dims))]
    Z_old = p.step_reconstruct(0).cpu().numpy()
    fills = rank_growth_draws(5, dims)(0, r_new)
    q = Plan(dims, r_new, precision="f64")
    q.regrow_from(p, fills)
    p.close()
    ref = pam.grow_factors(F_old, dims, r_old, r_new, fills)
    for k in range(len(dims)):
        np.testing.assert_array_equal(q.factor(k).cpu().numpy(), ref[k])
    np.testing.assert_array_equal(q.x().cpu().numpy(), X_old)
    assert _rel(q.step_reconstruct(0).cpu().numpy(), Z_old) <= 1e-13
    q.close()


def test_regrow_rejects_bad_pairs():
    from paper_2510_22506_amd import Plan, FctnError
    dims = (10, 9, 4)
    A = init_factors(np.random.default_rng(1), dims, (2, 2, 2))
    p = Plan(dims, (2, 2, 2), precision="f64")
    p.set_factors(A)
    fills_small = rank_growth_draws(1, dims)(0, (1, 2, 2))
    smaller = Plan(dims, (1, 2, 2), precision="f64")
    with pytest.raises(FctnError):
        smaller.regrow_from(p, fills_small)
    other = Plan((10, 9, 5), (2, 2, 2), precision="f64")
    with pytest.raises(FctnError):
        other.regrow_from(p, rank_growth_draws(1, (10, 9, 5))(0, (2, 2, 2)))
    f32 = Plan(dims, (2, 2, 2), precision="f32")
    with pytest.raises(FctnError):
        f32.regrow_from(p, rank_growth_draws(1, dims)(0, (2, 2, 2)))
    for q in (p, smaller, other, f32):
        q.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 1e-5)])
@pytest.mark.parametrize("name,dims,rmax,tau", [
    ("c1", (24, 20, 6), (3, 3, 3), np.inf),
    ("c3", (16, 14, 3, 6), (4, 3, 4, 3, 4, 3), np.inf),
    ("c1", (24, 20, 6), (3, 3, 3), 0.06),     # one growth, then no more (margin > 10%)
])
def test_schedule_matches_oracle(prec, tol, name, dims, rmax, tau):
    from paper_2510_22506_amd import complete_rank_increasing
    prob = make_problem(name, seed=22, dims=dims, precision=prec, sr=0.3)
    ones = (1,) * len(rmax)
    A0 = init_factors(np.random.default_rng(23), dims, ones)
    fill = rank_growth_draws(24, dims)
    sweeps = 8
    p, hist = complete_rank_increasing(dims, rmax, prob.Y, prob.mask, A0, fill, sweeps, tau=tau,
                                       lam=prob.lam, delta=prob.delta, rho=prob.rho,
                                       precision=prec)
    Xg = p.x().cpu().numpy()
    p.close()
    if prec == "f32":
        A0 = [a.astype(np.float32).astype(np.float64) for a in A0]
    Xo, _, so = pam.complete_rank_increasing(prob.Y.astype(np.float64), prob.mask != 0, rmax,
                                             prob.lam, prob.delta, prob.rho, sweeps, A0, fill,
                                             tau=tau, order_policy=1)
    print(name, prec, tau, [h["ranks"] for h in hist], f"rel err {_rel(Xg, Xo):.2e}")
    assert [h["ranks"] for h in hist] == so["ranks"]
    assert len(set(so["ranks"])) > 1        # the schedule did grow
    assert _rel(Xg, Xo) <= tol
    for t in range(sweeps):
        assert abs(hist[t]["objective"] - so["objective"][t]) <= 10 * tol * so["objective"][t]
    obs = prob.mask != 0
    np.testing.assert_array_equal(Xg[obs], prob.Y[obs])
