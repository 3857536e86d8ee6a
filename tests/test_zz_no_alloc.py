"""fctn_sweep_noalloc (the sweep with its split-K partial products in the
library's static device array, for callers that cannot allocate) against
fctn_sweep on the same inputs: X and the per-sweep scalars bit for bit, for
two calls in a row on different plans, the second one smaller; and the
documented refusal of a plan whose partial products exceed the array."""

import numpy as np
import pytest

from workloads import make_problem

pytestmark = pytest.mark.gpu


def _plan(prob, prec):
    from paper_2510_22506_amd import Plan
    p = Plan(prob.dims, prob.ranks, prob.lam, prob.delta, prob.rho, precision=prec,
             reuse=True, order_policy=1)
    p.set_factors(prob.A0)
    p.set_observed(prob.Y, prob.mask)
    return p


def test_noalloc_equals_sweep_two_calls_second_smaller():
    cases = [("c3", (48, 44, 3, 10), "f32", 4), ("c2", (40, 36, 3), "bf16x3", 3)]
    for name, dims, prec, sweeps in cases:
        prob = make_problem(name, seed=31, dims=dims, precision="f32", sr=0.2)
        ref = _plan(prob, prec)
        ref.sweep(sweeps)
        na = _plan(prob, prec)
        na.sweep_noalloc(sweeps)
        np.testing.assert_array_equal(na.x().cpu().numpy(), ref.x().cpu().numpy(),
                                      err_msg=f"{name} {dims} {prec}")
        assert na.history(0, sweeps) == ref.history(0, sweeps)
        ref.close()
        na.close()


def test_noalloc_refuses_partials_beyond_the_array():
    from paper_2510_22506_amd import FctnError
    prob = make_problem("c1", seed=32, dims=(500, 550, 24), ranks=(16, 8, 8), precision="f64",
                        sr=0.05)
    p = _plan(prob, "f64")
    with pytest.raises(FctnError) as e:
        p.sweep_noalloc(1)
    assert e.value.status == 2
