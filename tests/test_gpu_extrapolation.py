"""GPU parity of the asymmetric extrapolation (Section 4.2: after each
factor's subproblem, A_k <- A_k + alpha (A_k - beta A_k^t)) through the C ABI
against the FP64 oracle: whole sweeps in float64 (1e-9) and float32 (1e-5) on
orders 3 and 4, with the pair caches on and off, the factors themselves, the
per-sweep objective (whose trace term is recomputed for the extrapolated
factor) and a single solve step."""

import numpy as np
import pytest

from oracle import pam, tensor, sylvester
from workloads import make_problem

pytestmark = pytest.mark.gpu

EXT = [(0.5, 0.5), (0.3, 0.7)]


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _run(prob, prec, sweeps, reuse, policy, ext):
    from paper_2510_22506_amd import Plan
    p = Plan(prob.dims, prob.ranks, prob.lam, prob.delta, prob.rho, precision=prec,
             reuse=reuse, order_policy=policy, extrapolation=ext)
    p.set_factors(prob.A0)
    p.set_observed(prob.Y, prob.mask)
    p.sweep(sweeps)
    A0 = prob.A0
    if prec != "f64":
        A0 = [a.astype(np.float32).astype(np.float64) for a in A0]
    ref = pam.complete(prob.Y.astype(np.float64), prob.mask != 0, prob.ranks, prob.lam,
                       prob.delta, prob.rho, sweeps, A0, reuse=reuse, order_policy=policy,
                       extrapolation=ext)
    return p, ref


@pytest.mark.parametrize("ext", EXT)
@pytest.mark.parametrize("reuse,policy", [(True, 1), (False, 0)])
@pytest.mark.parametrize("name,dims", [("c1", (20, 18, 6)), ("c6", (14, 12, 4, 5))])
def test_sweeps_f64(name, dims, reuse, policy, ext):
    prob = make_problem(name, seed=11, dims=dims, precision="f64", sr=0.3)
    sweeps = 6
    p, (Xo, Fo, so) = _run(prob, "f64", sweeps, reuse, policy, ext)
    assert _rel(p.x().cpu().numpy(), Xo) <= 1e-9
    for k in range(len(dims)):
        assert _rel(p.factor(k).cpu().numpy(), Fo[k]) <= 1e-9, k
    h = p.history(0, sweeps)
    for t in range(sweeps):
        assert abs(h[t]["objective"] - so["objective"][t]) <= 1e-8 * so["objective"][t]
        assert abs(h[t]["rel_change"] - so["rel_change"][t]) <= 1e-8 * so["rel_change"][t]
    obs = prob.mask != 0
    np.testing.assert_array_equal(p.x().cpu().numpy()[obs], prob.Y[obs])
    p.close()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("bf16x3", 2e-4)])
def test_sweeps_multitemporal_f32(prec, tol):
    prob = make_problem("c6", seed=12, dims=(60, 50, 4, 5), precision="f32", sr=0.1)
    p, (Xo, _, so) = _run(prob, prec, 10, True, 1, (0.5, 0.5))
    assert _rel(p.x().cpu().numpy(), Xo) <= tol
    h = p.history(0, 10)
    for t in range(10):
        assert abs(h[t]["objective"] - so["objective"][t]) <= 10 * tol * so["objective"][t]
    p.close()


def test_step_solve_extrapolates_and_reports_its_trace():
    # one subproblem through the single-step entry points.  Factor 1 is the
    # first block of the sweep (order 1..N), so the oracle's factor 1 after one
    # sweep is the extrapolated solution from the initial factors; the trace
    # returned is that of the stored (extrapolated) factor.
    from paper_2510_22506_amd import Plan
    prob = make_problem("c1", seed=13, dims=(16, 12, 5), precision="f64", sr=0.4)
    ext = (0.5, 0.5)
    Fo = pam.complete(prob.Y, prob.mask != 0, prob.ranks, prob.lam, prob.delta, prob.rho, 1,
                      prob.A0, order_policy=0, extrapolation=ext)[1]
    for k in (0, 2):
        p = Plan(prob.dims, prob.ranks, prob.lam, prob.delta, prob.rho, precision="f64",
                 extrapolation=ext)
        p.set_factors(prob.A0)
        p.set_observed(prob.Y, prob.mask)
        G, B = p.step_gram_rhs(k)
        tr = p.step_solve(k, G, B)
        A = p.factor(k).cpu().numpy()
        if k == 0:
            assert _rel(A, Fo[0]) <= 1e-10
        ref = sylvester.trace_term(tensor.unfold(A, k), prob.delta)
        assert abs(tr - ref) <= 1e-10 * abs(ref), k
        p.close()
