"""Continuous-batching server (fctn_server_*): each result of a mixed batch
equals the same request run alone on a plan, bit for bit (the plans share no
state and every kernel is deterministic), for orders 3, 4 and 5, four
precisions and the asymmetric extrapolation; the float64 requests in the mix
match the oracle; a small arena still admits every request by footprint;
a request larger than the arena is rejected; a non-finite observed value is
reported on the completion; a cancelled request completes as cancelled,
queued ones at once and resident ones after the sweeps already queued, whose
X equals a plan run alone for that many sweeps."""

import numpy as np
import pytest
import torch

from oracle import pam
from paper_2510_22506_amd import fctn, serve
from workloads import make_problem

pytestmark = pytest.mark.gpu

# (generator, dims, ranks or None for the config's, precision)
MIX = [
    ("c2", (24, 20, 3), None, "f32"),
    ("c3", (12, 10, 3, 5), (4, 2, 3, 2, 3, 2), "f32"),
    ("c2", (30, 18, 3), None, "bf16x3"),
    ("c1", (10, 9, 6), None, "f64"),
    ("c3", (9, 11, 3, 4), (3, 2, 3, 2, 3, 2), "bf16"),
    ("c4", (16, 14, 7), (6, 4, 4), "bf16x3"),
    ("c2", (20, 20, 3), (6, 3, 3), "f32"),
    ("c1", (8, 7, 5), None, "f64"),
    ("c7", (6, 5, 4, 3, 4), (2,) * 10, "f32"),                # order 5
    ("c6", (18, 16, 4, 5), (4, 3, 3, 3, 3, 2), "f64"),       # with extrapolation
]
# the paper runs its multi-temporal images with the asymmetric extrapolation
EXTRAP = {"c6": (0.5, 0.5)}


def _request(tag, name, dims, ranks, prec, sweeps=6):
    p = make_problem(name, seed=100 + tag, dims=dims, ranks=ranks, precision=prec,
                     sweeps=sweeps)
    elem = torch.float64 if prec == "f64" else torch.float32
    r = dict(tag=tag, dims=p.dims, ranks=p.ranks,
             Y=torch.from_numpy(np.ascontiguousarray(p.Y)).to("cuda", elem),
             mask=torch.from_numpy(np.ascontiguousarray(p.mask.astype(np.uint8))).cuda(),
             A0=torch.from_numpy(np.concatenate([a.ravel() for a in p.A0])).cuda(),
             sweeps=sweeps, lam=p.lam, delta=p.delta, rho=p.rho, precision=prec,
             extrapolation=EXTRAP.get(name))
    return p, r


def _alone(r):
    pl = fctn.Plan(r["dims"], r["ranks"], r["lam"], r["delta"], r["rho"], r["precision"],
                   extrapolation=r["extrapolation"])
    pl.set_factors_dev(r["A0"])
    pl.set_observed(r["Y"], r["mask"])
    pl.sweep(r["sweeps"])
    X = pl.x()
    pl.close()
    return X


def _footprint(r):
    d = fctn.make_desc(r["dims"], r["ranks"], r["lam"], r["delta"], r["rho"], r["precision"],
                       extrapolation=r["extrapolation"])
    return (fctn.fctn_workspace_bytes(d) + 255) // 256 * 256


def test_mix_equals_alone_bitwise_and_f64_matches_oracle():
    reqs = [_request(i, *m) for i, m in enumerate(MIX)]
    srv = fctn.Server(arena_bytes=256 << 20, nstreams=3, max_active=4, depth=2)
    try:
        res = serve.run(srv, [r for _, r in reqs])
    finally:
        srv.close()
    for p, r in reqs:
        c, X = res["done"][r["tag"]]
        assert c["status"] == 0 and c["sweeps_done"] == r["sweeps"], c
        assert torch.equal(X, _alone(r)), r["tag"]
        if r["precision"] == "f64":
            Xo, _, _ = pam.complete(p.Y, p.mask != 0, p.ranks, p.lam, p.delta, p.rho,
                                    r["sweeps"], p.A0, reuse=True, order_policy=1,
                                    extrapolation=r["extrapolation"])
            Xg = X.cpu().numpy()
            assert np.linalg.norm(Xg - Xo) <= 1e-9 * np.linalg.norm(Xo)
            np.testing.assert_array_equal(Xg[p.mask != 0], p.Y[p.mask != 0])


def test_small_arena_admits_by_footprint():
    reqs = [_request(10 + i, *m, sweeps=4) for i, m in enumerate(MIX[:6])]
    sizes = [_footprint(r) for _, r in reqs]
    arena = max(sizes) + max(sizes) // 2   # room for one large request at a time
    srv = fctn.Server(arena_bytes=arena, nstreams=2, max_active=8, depth=2)
    done, max_used, max_active = {}, 0, 0
    try:
        for _, r in reqs:
            srv.submit(**r)
        while len(done) < len(reqs):
            for c, X in srv.step():
                done[c["tag"]] = (c, X)
            q, a, used = srv.query()
            max_used, max_active = max(max_used, used), max(max_active, a)
    finally:
        srv.close()
    assert max_used <= srv.arena_bytes
    assert 1 <= max_active < len(reqs)
    # some request had to wait for another to finish before it was admitted
    t_admit = sorted(c["t_admit"] for c, _ in done.values())
    t_done = sorted(c["t_done"] for c, _ in done.values())
    assert t_admit[-1] >= t_done[0]
    for _, r in reqs:
        assert torch.equal(done[r["tag"]][1], _alone(r))


def test_request_larger_than_arena_is_rejected():
    _, r = _request(50, "c3", (24, 28, 3, 6), (8, 3, 8, 3, 8, 3), "f32")
    srv = fctn.Server(arena_bytes=1 << 20, nstreams=1, max_active=2, depth=1)
    try:
        with pytest.raises(fctn.FctnError) as e:
            srv.submit(**r)
        assert e.value.status == fctn.E_NOMEM
    finally:
        srv.close()


def test_nonfinite_observed_value_is_flagged():
    p, r = _request(60, "c2", (16, 12, 3), None, "f32", sweeps=2)
    Y = r["Y"].clone()
    idx = np.argwhere(p.mask != 0)[0]
    Y[tuple(int(v) for v in idx)] = float("nan")
    r["Y"] = Y
    srv = fctn.Server(arena_bytes=64 << 20, nstreams=1, max_active=1, depth=1)
    try:
        res = serve.run(srv, [r])
    finally:
        srv.close()
    assert res["done"][r["tag"]][0]["status"] == fctn.E_NUMERIC


def test_cancel_queued_and_resident_requests():
    reqs = [_request(70 + i, "c3", (12, 10, 3, 5), (4, 2, 3, 2, 3, 2), "f32", sweeps=8)[1]
            for i in range(3)]
    srv = fctn.Server(arena_bytes=64 << 20, nstreams=1, max_active=1, depth=1)
    done = {}
    try:
        for r in reqs:
            srv.submit(**r)
        for c, X in srv.step():          # the first request is admitted
            done[c["tag"]] = (c, X)
        q, a, _ = srv.query()
        assert (q, a) == (2, 1)
        srv.cancel(reqs[1]["tag"])       # queued
        srv.cancel(reqs[0]["tag"])       # resident, sweeps already queued
        with pytest.raises(fctn.FctnError) as e:
            srv.cancel(12345)
        assert e.value.status == fctn.E_INVALID
        while len(done) < len(reqs):
            for c, X in srv.step():
                done[c["tag"]] = (c, X)
    finally:
        srv.close()
    c1, _ = done[reqs[1]["tag"]]
    assert c1["status"] == fctn.E_CANCELLED and c1["sweeps_done"] == 0
    c0, X0 = done[reqs[0]["tag"]]
    assert c0["status"] == fctn.E_CANCELLED and 1 <= c0["sweeps_done"] < 8
    r0 = dict(reqs[0], sweeps=c0["sweeps_done"])
    assert torch.equal(X0, _alone(r0))
    c2, X2 = done[reqs[2]["tag"]]
    assert c2["status"] == fctn.OK and c2["sweeps_done"] == 8
    assert torch.equal(X2, _alone(reqs[2]))
