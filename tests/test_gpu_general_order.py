"""GPU parity at orders 5 to 8 (Table 2's N-th order case): whole PAM sweeps
through the C ABI against the FP64 oracle on the same seeded inputs.  Each
mode's sub-network is generated from two operand runs of consecutive factors:
a run of one factor is read in place, a longer one is a cached prefix or
suffix group, grown one factor at a time from its neighbour group and rebuilt
only when one of its factors changed (Algorithm 2's reuse, Section 3.4).
float64 to 1e-9, float32 to 1e-5, split bf16 to 2e-4; observed entries bit
for bit; per-sweep objective and relative change.  With reuse each group is
contracted once per sweep; Algorithm 1 (reuse off) rebuilds the chains for
every mode and gives the same iterates bit for bit."""

import numpy as np
import pytest

from oracle import pam
from workloads import init_factors

pytestmark = pytest.mark.gpu

CASES = [
    ((9, 7, 3, 4, 5), (2, 3, 1, 2, 3, 1, 2, 2, 1, 3)),
    ((6, 5, 4, 3, 7), (3, 2, 2, 3, 2, 1, 2, 3, 2, 2)),
    ((4, 3, 5, 2, 3, 4), (2, 1, 2, 2, 1, 2, 1, 2, 3, 1, 2, 2, 2, 1, 2)),
    ((3, 4, 2, 3, 2, 3, 4), (2, 1, 2, 2, 1, 1, 2, 1, 2, 2, 1, 2, 1, 2, 2, 1, 1, 2, 2, 1, 2)),
    ((2, 3, 2, 2, 3, 2, 2, 3), (1, 2, 1, 2, 2, 1, 1, 2, 1, 2, 1, 1, 2, 2, 1, 2, 1, 1, 2, 1, 2,
                                2, 1, 1, 2, 1, 2, 1)),
]
TOL = {"f64": 1e-9, "f32": 1e-5, "bf16x3": 2e-4}


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("dims,ranks", CASES)
def test_sweeps_general_order(dims, ranks, prec):
    from paper_2510_22506_amd import Plan
    rng = np.random.default_rng(31)
    truth = rng.random(dims)
    mask = (rng.random(dims) < 0.3).astype(np.uint8)
    store = np.float64 if prec == "f64" else np.float32
    Y = np.where(mask != 0, truth, 0.0).astype(store)
    A0 = init_factors(rng, dims, ranks)
    sweeps = 6
    p = Plan(dims, ranks, 1e-2, 0.5, 0.1, precision=prec)
    p.set_factors(A0)
    p.set_observed(Y, mask)
    p.sweep(sweeps)
    Xg = p.x().cpu().numpy()
    h = p.history(0, sweeps)
    p.close()
    if prec != "f64":
        A0 = [a.astype(np.float32).astype(np.float64) for a in A0]
    Xo, _, so = pam.complete(Y.astype(np.float64), mask != 0, ranks, 1e-2, 0.5, 0.1, sweeps, A0,
                             order_policy=1)
    tol = TOL[prec]
    print(dims, prec, f"rel err {_rel(Xg, Xo):.2e}")
    assert _rel(Xg, Xo) <= tol
    obs = mask != 0
    np.testing.assert_array_equal(Xg[obs], Y[obs])
    for t in range(sweeps):
        assert abs(h[t]["objective"] - so["objective"][t]) <= 10 * tol * so["objective"][t]
        assert abs(h[t]["rel_change"] - so["rel_change"][t]) <= 10 * tol * so["rel_change"][t]


def test_order5_extrapolation_and_rank_growth():
    # the options built on top of the sweep work at order 5 as well
    from paper_2510_22506_amd import complete_rank_increasing
    from workloads import rank_growth_draws
    dims, rmax = (6, 5, 4, 3, 7), (2, 2, 2, 2, 2, 1, 2, 2, 2, 2)
    rng = np.random.default_rng(32)
    truth = rng.random(dims)
    mask = (rng.random(dims) < 0.3).astype(np.uint8)
    Y = np.where(mask != 0, truth, 0.0)
    A0 = init_factors(rng, dims, (1,) * 10)
    fill = rank_growth_draws(33, dims)
    p, hist = complete_rank_increasing(dims, rmax, Y, mask, A0, fill, 5, tau=np.inf,
                                       precision="f64", extrapolation=(0.5, 0.5))
    Xg = p.x().cpu().numpy()
    p.close()
    Xo, _, so = pam.complete_rank_increasing(Y, mask != 0, rmax, 1e-2, 0.5, 0.1, 5, A0, fill,
                                             tau=np.inf, order_policy=1,
                                             extrapolation=(0.5, 0.5))
    assert [h["ranks"] for h in hist] == so["ranks"]
    assert _rel(Xg, Xo) <= 1e-9


@pytest.mark.parametrize("dims,ranks", CASES[:2] + CASES[3:4])
def test_group_chain_builds(dims, ranks):
    # with reuse every one of the 2(N-3) prefix/suffix groups is contracted
    # exactly once per sweep in the order 1..N; without reuse the chains are
    # contracted again for every mode (and the X step), with the same iterates
    from paper_2510_22506_amd import Plan
    N = len(dims)
    rng = np.random.default_rng(35)
    mask = (rng.random(dims) < 0.3).astype(np.uint8)
    Y = np.where(mask != 0, rng.random(dims), 0.0)
    A0 = init_factors(rng, dims, ranks)
    xs, launches = [], []
    for reuse in (True, False):
        p = Plan(dims, ranks, 1e-2, 0.5, 0.1, precision="f64", reuse=reuse)
        p.set_factors(A0)
        p.set_observed(Y, mask)
        p.sweep(1)
        p.profile_enable(True)
        p.sweep(3)
        launches.append(p.profile_read(reset=True)["pair"]["launches"])
        xs.append(p.x().cpu().numpy())
        p.close()
    assert launches[0] == 3 * 2 * (N - 3), launches
    assert launches[1] > launches[0], launches
    np.testing.assert_array_equal(xs[0], xs[1])
