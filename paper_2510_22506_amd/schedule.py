"""Rank-increasing PAM on the GPU.

Algorithms 1-2 take a maximal FCTN-rank and start from rank ones; the growth
rule is deferred to the paper's reference [Zheng2022].  The rule here: after a
sweep whose relative change ||X^{t+1} - X^t||_F / ||X^t||_F is below `tau`,
every bond rank below its maximum grows by one.  A growth builds a plan at the
new ranks and moves the state into it with fctn_regrow (X and the mask are
copied; each grown bond (i, j), i < j, gets fresh draws in factor i and zeros
in factor j, so FCTN(A) and X are unchanged); the new plan starts at sweep 0.
"""

from .fctn import Plan


def complete_rank_increasing(dims, rmax, Y, mask, A0, fill, sweeps, tau=1e-2, r0=None,
                             lam=1e-2, delta=0.5, rho=0.1, precision="f32", reuse=True,
                             order_policy=1, extrapolation=None, device="cuda:0"):
    """Run `sweeps` PAM sweeps from factors A0 at ranks r0 (default all ones),
    growing towards rmax.  fill(g, ranks) gives the float64 draws (one array
    per factor at `ranks`) for growth event g = 0, 1, ...  Returns the plan of
    the last run (its X and factors are the result; close it when done) and a
    per-sweep list of {"ranks", "rel_change", "objective"}."""
    rmax = [int(r) for r in rmax]
    ranks = [1] * len(rmax) if r0 is None else [int(r) for r in r0]
    kw = dict(lam=lam, delta=delta, rho=rho, precision=precision, reuse=reuse,
              order_policy=order_policy, device=device, extrapolation=extrapolation)
    p = Plan(dims, ranks, **kw)
    p.set_factors(A0)
    p.set_observed(Y, mask)
    hist = []
    grown = 0
    for t in range(sweeps):
        st = p.sweep(1, stats=True)
        hist.append({"ranks": tuple(ranks), "rel_change": st["rel_change"],
                     "objective": st["objective"]})
        if st["rel_change"] < tau and ranks != rmax and t + 1 < sweeps:
            new = [min(r + 1, m) for r, m in zip(ranks, rmax)]
            q = Plan(dims, new, **kw)
            q.regrow_from(p, fill(grown, tuple(new)))
            p.close()
            p, ranks = q, new
            grown += 1
    return p, hist
