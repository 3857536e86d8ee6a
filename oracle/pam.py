"""Algorithms 1 and 2 (PAM-FCTNLR / PAM-AFCTNLR) in float64 (oracle; test
infrastructure).

One sweep (Section 3.2, Algorithms 1-2): for each k in the sweep order,
  M_k   = FCTN({A}, /A_k) unfolded as in Property 1 (eq. 4),
  G     = M_k M_k^T, Y = X_(k) M_k^T + rho A_k^t (eq. 5),
  A_k   = the eq. 8 solution, folded back by eq. 9;
then X^{t+1} = P_Omega^c((FCTN(A^{t+1}) + rho X^t)/(1 + rho)) + P_Omega(Y) (eq. 10),
stopping when ||X^{t+1} - X^t||_F / ||X^t||_F <= eps or after the sweep limit.

Sub-networks are built by binary contractions of labelled tensors, each one
counted as 2 * (output entries) * (contracted size) flops, so that the
per-sweep counts can be checked against Tables 1-2:

* reuse off (Algorithm 1): every M_k, and FCTN(A) for the X update, is a
  chain contraction of the factors in increasing index order.
* reuse on (Algorithm 2, Section 3.3): for N = 4 the pair tensors
  A_3 x A_4 (contracted over R_34; shared by M_1 and M_2) and A_1 x A_2
  (over R_12; shared by M_3 and M_4) are cached and rebuilt only when one of
  their factors has changed; FCTN(A^{t+1}) is A_last times the sub-network of
  the last-updated factor, which is then already current (M'_last).  For
  N = 3 only the X step is reused (Table 2 gives no M_k saving at N = 3).
  For N >= 5 (Table 2's N-th order case; the figures that would show the
  schedule are missing, so the schedule is a reading of ours that reproduces
  Table 2's Algorithm 2 counts): every M_k is a cached group of N - 2
  factors contracted with the one remaining factor, and groups grow one
  factor at a time from a cached smaller group.  Modes 1 and 2 share the
  group {3..N}, grown from the pair {N-1, N} downwards; mode 3 grows the pair
  {1, 2} by N, N-1, .., 5 (contracting with A_4); mode k >= 4 extends the
  cached group {1, 2, k+1..N} by 3, .., k-2 (contracting with A_{k-1}).  Per
  sweep that is 2 pairs, 3 groups of three, .., N-2 groups of N-2 factors
  and N final contractions: Table 2's 4I^2R^{2N-3} + 6I^3R^{3N-7} + .. +
  2N I^{N-1}R^{2N-3} (1-based modes here; the code is 0-based).

Sweep order (Algorithm 2's "unordered permutation"; Figure 6 is missing from
the source): order_policy 0 keeps (1, .., N); order_policy 1 alternates
(1, 2, 3, 4) and (3, 4, 1, 2) for N = 4, so that the pair built last in one
sweep is still current for the first two updates of the next.  With reuse on
this gives exactly Table 1's counts (t = 1: 4I^2R^5 + 8I^3R^5; t >= 2:
2I^2R^5 + 8I^3R^5; X: 2I^4R^3).  For N != 4 policy 1 equals policy 0.

Asymmetric extrapolation (Section 4.2, used there for the multi-temporal
images; off unless `extrapolation=(alpha, beta)` is given): right after factor
k's subproblem is solved, the new factor A is replaced by
A + alpha (A - beta A^t), with A^t the factor the subproblem started from (its
proximal centre).  The paper states the update but not where it sits in the
loop; it is read here as part of each factor's block, so the factors updated
later in the sweep, FCTN(A^{t+1}) in the X step and the next sweep's proximal
centre all see the extrapolated factor.  The PAM objective is then no longer
monotone.

Rank-increasing schedule (Algorithms 1-2 take a maximal FCTN-rank and start
from rank ones; the growth rule itself is deferred to the paper's reference
[Zheng2022], so the rule here is a reading of ours): after a sweep whose
relative change is below tau, every bond rank below its maximum grows by one.
Each grown bond (i, j), i < j, gets a new slice in both factors: factor i's new
entries are fresh draws (standard normal, like the initial factors), factor
j's are zero, so FCTN(A) and X are unchanged by the growth itself; the next
sweep starts a new run (sweep counter, and with it the alternating order,
restarting at zero).

Initial X is P_Omega(Y): the observed tensor is zero off Omega by definition
of a partial observation (Section 1), so Algorithm 1's X^(1) = Y is read as
P_Omega(Y); values of Y off Omega never enter any arithmetic.
"""

import numpy as np

from . import tensor, laplacian, sylvester


class FlopCounter:
    """Per-category flop totals for the current sweep ('M', 'X', 'gram', 'rhs')."""

    def __init__(self):
        self.flops = {}

    def add(self, cat, n):
        self.flops[cat] = self.flops.get(cat, 0) + int(n)


def _contract2(a, la, b, lb, out, counter, cat):
    """Binary contraction of labelled tensors; counts 2*|out|*|contracted|."""
    size = {}
    for t, l in ((a, la), (b, lb)):
        for ch, d in zip(l, t.shape):
            size[ch] = d
    shared = [c for c in la if c in lb and c not in out]
    n_out = int(np.prod([size[c] for c in out], dtype=np.int64))
    n_con = int(np.prod([size[c] for c in shared], dtype=np.int64)) if shared else 1
    if counter is not None:
        counter.add(cat, 2 * n_out * n_con)
    return np.einsum(f"{la},{lb}->{out}", a, b, optimize=True)


def _free_labels(N, group, labs):
    """Labels that survive after contracting the factors in `group`: their
    physical modes plus every bond to a factor outside the group."""
    phys, bond = tensor._labels(N)
    out = []
    for j in sorted(group):
        for ch in labs[j]:
            if ch == phys[j]:
                out.append(ch)
            else:
                other = [m for m in range(N) if m != j and bond[(j, m)] == ch][0]
                if other not in group and ch not in out:
                    out.append(ch)
    return "".join(out)


def chain(factors, members, counter, cat):
    """Contract the factors in `members` one by one in increasing index order
    (the from-scratch route of Algorithm 1).  Returns (tensor, labels)."""
    N = len(factors)
    labs = [tensor.factor_labels(N, j) for j in range(N)]
    members = sorted(members)
    T, lt = factors[members[0]], labs[members[0]]
    for n, j in enumerate(members[1:], start=2):
        out = _free_labels(N, members[:n], labs)
        T = _contract2(T, lt, factors[j], labs[j], out, counter, cat)
        lt = out
    return T, lt


def to_property1(T, lt, N, k):
    """Permute a labelled M_k into Property 1's mode order and unfold it."""
    order, rows, cols = tensor.subnetwork_modes(N, k)
    T = np.einsum(f"{lt}->{order}", T)
    return tensor.gunfold(T, rows, cols)


class PairCache:
    """Cached pair tensors for N = 4 (Section 3.3, Figures 2-3)."""

    def __init__(self):
        self.pairs = {}            # (p, q) -> (tensor, labels, versions)

    def get(self, factors, versions, p, q, counter):
        key = (p, q)
        hit = self.pairs.get(key)
        if hit is not None and hit[2] == (versions[p], versions[q]):
            return hit[0], hit[1]
        T, lt = chain(factors, [p, q], counter, "M")
        self.pairs[key] = (T, lt, (versions[p], versions[q]))
        return T, lt


class GroupCache:
    """Contracted factor groups of the general-N reuse chain (N >= 5), each
    kept with the versions of its members when it was built."""

    def __init__(self):
        self.groups = {}            # frozenset(members) -> (tensor, labels, versions)

    def get(self, members, versions):
        hit = self.groups.get(frozenset(members))
        if hit is not None and hit[2] == tuple(versions[m] for m in sorted(members)):
            return hit[0], hit[1]
        return None

    def put(self, members, T, lt, versions):
        self.groups[frozenset(members)] = (T, lt, tuple(versions[m] for m in sorted(members)))


def group_sequence(N, k):
    """For N >= 5: the factors whose contraction, grown in this order, is the
    group of N - 2 factors for M_k, and the remaining factor (0-based modes)."""
    if k in (0, 1):
        return [N - 2, N - 1] + list(range(N - 3, 1, -1)), 1 - k
    if k == 2:
        return [0, 1] + list(range(N - 1, 3, -1)), 3
    return [0, 1] + list(range(N - 1, k, -1)) + list(range(2, k - 1)), k - 1


def grown_group(factors, seq, gcache, versions, counter):
    """The contraction of the factors in seq, reusing the longest cached
    prefix group of seq and caching every group it builds."""
    N = len(factors)
    labs = [tensor.factor_labels(N, j) for j in range(N)]
    have, T, lt = 0, None, None
    for j in range(len(seq), 1, -1):
        hit = gcache.get(seq[:j], versions)
        if hit is not None:
            have, (T, lt) = j, hit
            break
    if have == 0:
        T, lt = chain(factors, seq[:2], counter, "M")
        gcache.put(seq[:2], T, lt, versions)
        have = 2
    for j in range(have, len(seq)):
        m = seq[j]
        out = _free_labels(N, seq[:j + 1], labs)
        T = _contract2(T, lt, factors[m], labs[m], out, counter, "M")
        lt = out
        gcache.put(seq[:j + 1], T, lt, versions)
    return T, lt


def subnetwork_M(factors, k, reuse, cache, versions, counter, gcache=None):
    """M_k (Property 1 unfolding), with or without the reuse mechanism."""
    N = len(factors)
    if reuse and N >= 5 and gcache is not None:
        seq, f = group_sequence(N, k)
        G, lg = grown_group(factors, seq, gcache, versions, counter)
        labs = [tensor.factor_labels(N, j) for j in range(N)]
        out = _free_labels(N, seq + [f], labs)
        T = _contract2(G, lg, factors[f], labs[f], out, counter, "M")
        return to_property1(T, out, N, k)
    if reuse and N == 4:
        p, q = (2, 3) if k in (0, 1) else (0, 1)
        P, lp = cache.get(factors, versions, p, q, counter)
        other = [m for m in range(4) if m != k and m not in (p, q)][0]
        labs = tensor.factor_labels(4, other)
        out = _free_labels(4, [p, q, other], [tensor.factor_labels(4, j) for j in range(4)])
        T = _contract2(P, lp, factors[other], labs, out, counter, "M")
        return to_property1(T, out, N, k)
    T, lt = chain(factors, [j for j in range(N) if j != k], counter, "M")
    return to_property1(T, lt, N, k)


def sweep_order(N, t, order_policy):
    """Factor order for sweep t (0-based); see the module docstring."""
    if order_policy == 1 and N == 4 and t % 2 == 1:
        return [2, 3, 0, 1]
    return list(range(N))


def objective(X, factors, lam, delta):
    """f = 1/2 ||X - FCTN(A)||^2 + sum_k lam_k/2 tr(A_k(k)^T L_k A_k(k))
    (Section 3.5, f without the indicator, which is zero on feasible X)."""
    Z = tensor.fctn(factors)
    f = 0.5 * float(np.sum((X - Z) ** 2))
    for k, A in enumerate(factors):
        f += 0.5 * lam[k] * sylvester.trace_term(tensor.unfold(A, k), delta[k])
    return f


def x_update(X, Z, mask, rho):
    """eq. 10 with X already equal to Y on Omega: a select, Y never re-read."""
    return np.where(mask, X, (Z + rho * X) / (1.0 + rho))


def complete(Y, mask, ranks, lam, delta, rho, sweeps, A0, tol=0.0, reuse=True,
             order_policy=0, record_blocks=False, counters=None, extrapolation=None,
             X0=None, t0=0):
    """Run PAM (Algorithm 1 if reuse is False, Algorithm 2 if True).

    Y, mask: observed tensor and boolean Omega of shape I_1 x .. x I_N.
    ranks: r_FCTN vector; lam, delta: per-mode lambda_k, delta_k; rho: proximal
    weight; A0: initial factors (list of arrays with the factor shapes).
    Returns (X, factors, stats) where stats holds per-sweep rel_change,
    objective and, with record_blocks, the objective after every block.
    counters: optional list that receives one FlopCounter per sweep.
    extrapolation: None, or (alpha, beta) of the asymmetric extrapolation.
    X0: the starting X (equal to Y on Omega); None starts from P_Omega(Y).
    t0: index of the first sweep (selects the sweep order).
    """
    Y = np.asarray(Y, dtype=np.float64)
    mask = np.asarray(mask, dtype=bool)
    N = Y.ndim
    dims = Y.shape
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (N,))
    delta = np.broadcast_to(np.asarray(delta, dtype=np.float64), (N,))
    shapes = tensor.factor_shapes(dims, ranks)
    factors = [np.array(a, dtype=np.float64).reshape(s) for a, s in zip(A0, shapes)]
    X = np.where(mask, Y, 0.0) if X0 is None else np.array(X0, dtype=np.float64)
    cache = PairCache()
    gcache = GroupCache()
    versions = [0] * N
    stats = {"rel_change": [], "objective": [], "blocks": [], "sweeps_done": 0}

    for t in range(sweeps):
        counter = FlopCounter()
        order = sweep_order(N, t0 + t, order_policy)
        Mk = None
        for k in order:
            Mk = subnetwork_M(factors, k, reuse, cache, versions, counter, gcache)
            Xk = tensor.unfold(X, k)
            Ak = tensor.unfold(factors[k], k)
            G = Mk @ Mk.T
            counter.add("gram", 2 * Mk.shape[0] ** 2 * Mk.shape[1])
            Yk = sylvester.rhs(Xk, Mk, Ak, rho)
            counter.add("rhs", 2 * Xk.shape[0] * Mk.shape[0] * Mk.shape[1])
            Anew = sylvester.solve_fast(G, Yk, lam[k], delta[k], rho)
            if extrapolation is not None:
                alpha, beta = extrapolation
                Anew = Anew + alpha * (Anew - beta * Ak)
            factors[k] = tensor.fold(Anew, k, shapes[k])
            versions[k] += 1
            if record_blocks:
                stats["blocks"].append(("A", k, objective(X, factors, lam, delta)))
        last = order[-1]
        if reuse:
            Zl = tensor.unfold(factors[last], last) @ Mk
            counter.add("X", 2 * Zl.shape[0] * Mk.shape[0] * Mk.shape[1])
            Z = tensor.fold(Zl, last, dims)
        else:
            Z, lz = chain(factors, list(range(N)), counter, "X")
        Xn = x_update(X, Z, mask, rho)
        rel = float(np.linalg.norm(Xn - X) / np.linalg.norm(X))
        X = Xn
        f = 0.5 * float(np.sum((X - Z) ** 2))
        for k in range(N):
            f += 0.5 * lam[k] * sylvester.trace_term(tensor.unfold(factors[k], k), delta[k])
        stats["rel_change"].append(rel)
        stats["objective"].append(f)
        stats["sweeps_done"] = t + 1
        if record_blocks:
            stats["blocks"].append(("X", -1, f))
        if counters is not None:
            counters.append(counter)
        if tol > 0 and rel <= tol:
            break
    return X, factors, stats


def grow_factors(factors, dims, ranks_old, ranks_new, fills):
    """Embed factors of FCTN-rank ranks_old into ranks_new (elementwise >=).
    Factor k keeps its old entries; an entry whose index along some bond
    (j, k), j < k, is a new one is zero; every other new entry (new only along
    bonds (k, j), j > k) is taken from fills[k], an array of the new shape."""
    N = len(dims)
    Ro = tensor.rank_matrix(ranks_old, N)
    new_shapes = tensor.factor_shapes(dims, ranks_new)
    out = []
    for k in range(N):
        a = np.array(fills[k], dtype=np.float64).reshape(new_shapes[k]).copy()
        for j in range(k):
            idx = [slice(None)] * N
            idx[j] = slice(Ro[j][k], None)
            a[tuple(idx)] = 0.0
        a[tuple(slice(0, n) for n in factors[k].shape)] = factors[k]
        out.append(a)
    return out


def complete_rank_increasing(Y, mask, rmax, lam, delta, rho, sweeps, A0, fill, tau=1e-2,
                             r0=None, reuse=True, order_policy=0, extrapolation=None):
    """PAM with the rank-increasing schedule above.  A0: factors at the start
    ranks r0 (default all ones); fill(g, ranks) returns the list of draws for
    growth event g (0, 1, ..) to ranks `ranks`.  Returns (X, factors, stats)
    with stats["ranks"][t] the ranks sweep t ran at."""
    Y = np.asarray(Y, dtype=np.float64)
    mask = np.asarray(mask, dtype=bool)
    dims = Y.shape
    rmax = [int(r) for r in rmax]
    ranks = [1] * len(rmax) if r0 is None else [int(r) for r in r0]
    factors = [np.array(a, dtype=np.float64) for a in A0]
    X = None
    stats = {"rel_change": [], "objective": [], "ranks": [], "sweeps_done": 0}
    run_t = 0
    grown = 0
    for t in range(sweeps):
        X, factors, st = complete(Y, mask, ranks, lam, delta, rho, 1, factors, reuse=reuse,
                                  order_policy=order_policy, extrapolation=extrapolation,
                                  X0=X, t0=run_t)
        stats["rel_change"].append(st["rel_change"][0])
        stats["objective"].append(st["objective"][0])
        stats["ranks"].append(tuple(ranks))
        stats["sweeps_done"] = t + 1
        run_t += 1
        if st["rel_change"][0] < tau and ranks != rmax and t + 1 < sweeps:
            new = [min(r + 1, m) for r, m in zip(ranks, rmax)]
            factors = grow_factors(factors, dims, ranks, new, fill(grown, tuple(new)))
            ranks = new
            grown += 1
            run_t = 0
    return X, factors, stats
