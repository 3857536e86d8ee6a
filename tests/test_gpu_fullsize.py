"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (reuse on, alternating order): two PAM sweeps of the image-shaped
256x256x3, video-shaped 144x176x3x50 and multispectral-shaped 512x512x31
configurations, and of the paper's second workload set (a 500x550x3x24 video
and a 300x300x4x5 multi-temporal image, run with the asymmetric extrapolation
at alpha = beta = 0.5 as the paper runs it), and an order-5 32x32x32x32x8
low-rank tensor, against the FP64 oracle on the same
seeded inputs (the oracle finishes the two sweeps in seconds, the 500x550x3x24
case in under a minute; its result is shared by the two precisions).  float32 to 1e-5 relative, split
bf16 to 2e-4, observed entries bit for bit, and the per-sweep objective and
relative change to the same tolerance."""

import functools

import numpy as np
import pytest

from oracle import pam
from workloads import make_problem

pytestmark = pytest.mark.gpu

SWEEPS = 2


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@functools.lru_cache(maxsize=1)
def _oracle(name, ext):
    prob = make_problem(name, seed=0, precision="f32")
    A0 = [a.astype(np.float32).astype(np.float64) for a in prob.A0]
    Xo, _, st = pam.complete(prob.Y.astype(np.float64), prob.mask != 0, prob.ranks, prob.lam,
                             prob.delta, prob.rho, SWEEPS, A0, reuse=True, order_policy=1,
                             extrapolation=ext)
    return Xo, st


@pytest.mark.parametrize("name,prec,tol,ext", [
    ("c2", "f32", 1e-5, None), ("c3", "f32", 1e-5, None), ("c3", "bf16x3", 2e-4, None),
    ("c4", "f32", 1e-5, None), ("c4", "bf16x3", 2e-4, None),
    ("c5", "f32", 1e-5, None), ("c5", "bf16x3", 2e-4, None),
    ("c6", "f32", 1e-5, (0.5, 0.5)), ("c6", "bf16x3", 2e-4, (0.5, 0.5)),
    ("c7", "f32", 1e-5, None),
])
def test_full_size_sweeps(name, prec, tol, ext):
    from paper_2510_22506_amd import Plan
    prob = make_problem(name, seed=0, precision="f32")
    p = Plan(prob.dims, prob.ranks, prob.lam, prob.delta, prob.rho, precision=prec,
             reuse=True, order_policy=1, extrapolation=ext)
    p.set_factors(prob.A0)
    p.set_observed(prob.Y, prob.mask)
    p.sweep(SWEEPS)
    hist = p.history(0, SWEEPS)
    Xg = p.x().cpu().numpy()
    p.close()
    Xo, st = _oracle(name, ext)
    print(f"{name} {prob.dims} {prec}: rel err {_rel(Xg, Xo):.3e}")
    assert _rel(Xg, Xo) <= tol, _rel(Xg, Xo)
    obs = prob.mask != 0
    np.testing.assert_array_equal(Xg[obs], prob.Y[obs])
    for t in range(SWEEPS):
        assert abs(hist[t]["objective"] - st["objective"][t]) <= 10 * tol * abs(st["objective"][t])
        assert abs(hist[t]["rel_change"] - st["rel_change"][t]) <= 10 * tol * st["rel_change"][t]
