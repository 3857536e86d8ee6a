"""Benchmark: PAM sweeps/s of trace-regularized FCTN completion on one MI355X.

One step = one full PAM sweep (every factor update: sub-network generation,
Gram + right-hand side, reduction, factor solve; then the reconstruction, the
X/mask pass and the per-sweep scalars) over the whole synthetic tensor, with
all inputs resident in HBM before the timed region.

Default workload: the order-4 video-shaped tensor 144 x 176 x 3 x 50 with
FCTN ranks R12 = R14 = R24 = 8, R13 = R23 = R34 = 3, sampling rate 0.05,
float32 with float64 reductions and solves, reuse on (Algorithm 2 with the
alternating factor order).

Prints ONE JSON line.  `value` is K sweeps timed as a caller runs them.
`roofline` is for the kernel with the largest summed time, from the same K
sweeps run again with HIP events around every launch on the plan's stream
(the events serialize the queue, so this pass is not the one `value` comes
from; `ms_per_step_with_events` is its rate): algorithmic flops (or bytes)
per launch / average launch time, against MI355X's published peak for that
kernel's bound.  `serving` is the request-serving
workload through the continuous-batching server (completions/s, p50/p99
latency, split bf16 against float32 at saturation).  `rank_schedule` runs
the rank-increasing schedule on the same workload (rank ones up to its ranks)
and times one growth.  `roofline_xpass_large` is the X/mask pass on a 1 GiB
tensor (larger than the Infinity Cache).  `other_workloads` times other
configurations the same way (by default the 256x256x3 image, which is
launch-bound).  `cpu_baseline` is the float64
oracle on the host cores over a bounded number of sweeps of the same
workload.

Other workloads (--workload): c1 low-rank 32x32x8 (float64), c2 color image
256x256x3, c4 multispectral 512x512x31, c5 new-video 500x550x3x24, c6
multi-temporal 300x300x4x5 (with the asymmetric extrapolation, as the paper
runs its multi-temporal images), c7 low-rank order-5 32x32x32x32x8.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PAM sweeps/s + % MFMA peak; served completions/s with p50/p99 latency"
PEAK = {  # MI355X published dense peaks
    "f32": 157.3e12, "f64": 78.6e12, "bf16": 2.5e15, "bf16x3": 2.5e15, "hbm": 8.0e12,
}
WORKLOADS = {
    "c3": ("c3", None, "video-shaped order-4 144x176x3x50, ranks (8,3,8,3,8,3), SR 0.05"),
    "c2": ("c2", None, "color-image order-3 256x256x3, ranks (12,3,3), SR 0.1"),
    "c4": ("c4", None, "multispectral order-3 512x512x31, ranks (16,8,8), SR 0.05"),
    "c1": ("c1", None, "low-rank order-3 32x32x8, ranks (3,3,3), SR 0.3"),
    "c5": ("c5", None, "new-video-shaped order-4 500x550x3x24, ranks (8,3,8,3,8,3), SR 0.05"),
    "c6": ("c6", None, "multi-temporal order-4 300x300x4x5, ranks (8,3,4,3,4,3), SR 0.05"),
    "c7": ("c7", None, "low-rank order-5 32x32x32x32x8, all ten ranks 3, SR 0.1"),
}
DEFAULT_PREC = {"c1": "f64", "c2": "f32", "c3": "f32", "c4": "f32", "c5": "f32", "c6": "f32",
                "c7": "f32"}
# the paper runs its multi-temporal images with the asymmetric extrapolation
# (alpha = beta = 0.5, Section 4.2) and its videos without
DEFAULT_EXTRAP = {"c6": (0.5, 0.5)}
# contraction stages: their algorithmic flops make up tflops_contractions;
# gram_rhs and reconstruct run on MFMA, pair on the vector ALUs writing the
# pair tensor (HBM-bound)
CONTRACTION_STAGES = ("gram_rhs", "reconstruct", "pair")
MFMA_STAGES = ("gram_rhs", "reconstruct")
# bound of every other stage: float64 MFMA products, float64 ALU-latency
# solves, HBM-bound passes
F64_MFMA_STAGES = ("transform",)
ALU_STAGES = ("solve",)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_22506_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision, stage):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if it is missing or was taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get(f"{workload}/{precision}/{stage}")
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def stage_roofline(stage, rec, prec):
    """Achieved rate of one stage's average launch against the bound of its
    kernel: algorithmic flops or bytes per launch / average launch time."""
    n = max(rec["launches"], 1)
    avg_s = rec["ms"] / 1e3 / n
    r = {"kernel": stage, "avg_launch_us": avg_s * 1e6, "launches": rec["launches"]}
    if avg_s <= 0:
        return r
    if stage in MFMA_STAGES or stage in F64_MFMA_STAGES or stage in ALU_STAGES:
        if stage == "gram_rhs":
            peak = PEAK[prec]          # bf16 forms run their Gram / RHS on bf16 MFMA
        elif stage in MFMA_STAGES:
            peak = PEAK["f64"] if prec == "f64" else PEAK["f32"]   # float32 MFMA otherwise
        else:
            peak = PEAK["f64"]
        a = rec["flops"] / n / avg_s
        r.update({"bound": "alu" if stage in ALU_STAGES else "mfma", "achieved": a / 1e12,
                  "peak": peak / 1e12, "unit": "TFLOP/s", "frac": a / peak})
    else:
        a = rec["bytes"] / n / avg_s
        r.update({"bound": "hbm", "achieved": a / 1e9, "peak": PEAK["hbm"] / 1e9,
                  "unit": "GB/s", "frac": a / PEAK["hbm"]})
    return r


def psnr(truth, X):
    """Mean over the trailing slices of 10 log10(1 / MSE) over the first two
    modes (pixel values in [0, 1])."""
    import numpy as np
    t = truth.reshape(truth.shape[0] * truth.shape[1], -1).astype(np.float64)
    x = X.reshape(t.shape).astype(np.float64)
    mse = np.mean((t - x) ** 2, axis=0)
    return float(np.mean(10.0 * np.log10(1.0 / np.maximum(mse, 1e-30))))


def serving(args):
    """The serving workload: a mix of independent completions (order-3
    image-shaped {64,128,256}^2 x 3 and order-4 video-shaped 72 x 88 x 3 x
    {10,25,50}, sampling rates {0.05,0.1,0.2}) through the continuous-batching
    server.  Poisson arrivals at `serve_rate` in the bf16 served form (split
    bf16), then saturation runs (every request at t = 0) of the same mix in
    split bf16, plain bf16 and float32, with per-request PSNR against float32
    (plain bf16 misses the 1e-3 bound against the oracle, so it is reported
    beside the served form, not as it)."""
    import numpy as np
    import torch
    from paper_2510_22506_amd import Server, serve
    from workloads import make_problem, serving_requests

    spec = serving_requests(seed=0, n=args.serve_n, rate=args.serve_rate,
                            sweeps=args.serve_sweeps)
    probs = [make_problem(q["config"], seed=q["seed"], dims=q["dims"], sr=q["sr"],
                          sweeps=q["sweeps"], precision="f32") for q in spec]
    dev = []
    for p in probs:
        dev.append((torch.from_numpy(np.ascontiguousarray(p.Y)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(p.mask.astype(np.uint8))).cuda(),
                    torch.from_numpy(np.concatenate([a.ravel() for a in p.A0])).cuda()))
    torch.cuda.synchronize()

    # the completed X of every request in every form, allocated up front: a
    # device allocation inside the timed loop can synchronize the device
    outs = {prec: [torch.empty(p.dims, dtype=torch.float32, device="cuda") for p in probs]
            for prec in ("bf16x3", "bf16", "f32")}

    def requests(prec, idx):
        return [dict(tag=i, dims=probs[i].dims, ranks=probs[i].ranks, Y=dev[i][0],
                     mask=dev[i][1], A0=dev[i][2], sweeps=spec[i]["sweeps"], lam=probs[i].lam,
                     delta=probs[i].delta, rho=probs[i].rho, precision=prec,
                     X_out=outs[prec][i]) for i in idx]

    arena = int(min(args.serve_budget, 16 << 30))
    srv = Server(arena, nstreams=args.serve_streams, max_active=args.serve_active,
                 depth=args.serve_depth)
    try:
        serve.run(srv, requests("bf16x3", range(min(8, len(spec)))))  # warm-up
        poisson = serve.run(srv, requests("bf16x3", range(len(spec))),
                            [q["arrival"] for q in spec])
        sat = {prec: serve.run(srv, requests(prec, range(len(spec))))
               for prec in ("bf16x3", "bf16", "f32")}
    finally:
        srv.close()

    def dpsnr_of(form):
        d = [psnr(p.truth, sat[form]["done"][i][1].cpu().numpy()) -
             psnr(p.truth, sat["f32"]["done"][i][1].cpu().numpy()) for i, p in enumerate(probs)]
        return np.abs(np.array(d))
    dpsnr = dpsnr_of("bf16x3")
    dpsnr1 = dpsnr_of("bf16")
    out = {"requests": len(spec), "sweeps_per_request": args.serve_sweeps,
           "arrival_rate_per_s": args.serve_rate, "form": "bf16x3",
           "poisson": serve.summarize(poisson),
           "saturation": {k: serve.summarize(v) for k, v in sat.items()},
           "psnr_bf16x3_vs_f32_abs_db": {"mean": float(dpsnr.mean()),
                                         "max": float(dpsnr.max())},
           "psnr_bf16_vs_f32_abs_db": {"mean": float(dpsnr1.mean()),
                                       "max": float(dpsnr1.max())},
           "server": {"arena_bytes": arena, "budget_bytes": int(args.serve_budget),
                      "streams": args.serve_streams, "max_active": args.serve_active,
                      "depth": args.serve_depth}}
    for form in ("bf16x3", "bf16"):
        out[f"saturation_speedup_{form}_over_f32"] = (
            out["saturation"][form]["completions_per_s"] /
            out["saturation"]["f32"]["completions_per_s"])
    return out


def xpass_large(dims=(1024, 1024, 256), launches=10):
    """The X/mask pass (eq. 10, x_update_k) on a float32 tensor of 1 GiB per
    operand, larger than the 256 MB Infinity Cache, so that its rate is HBM's:
    reads X, Z and the mask bits, writes X (12.125 bytes per element)."""
    import torch
    from paper_2510_22506_amd import Plan
    plan = Plan(dims, (2, 2, 2), precision="f32")
    g = torch.Generator(device="cuda:0")
    g.manual_seed(7)
    Y = torch.rand(dims, device="cuda:0", generator=g)
    mask = (torch.rand(dims, device="cuda:0", generator=g) < 0.05).to(torch.uint8)
    Z = torch.rand(dims, device="cuda:0", generator=g)
    plan.set_observed(Y, mask)
    del Y, mask
    plan.step_x_update(Z)
    plan.profile_enable(True)
    plan.profile_read(reset=True)
    for _ in range(launches):
        plan.step_x_update(Z)
    rec = plan.profile_read(reset=True)["x_update"]
    plan.close()
    r = stage_roofline("x_update", rec, "f32")
    r.update({"dims": list(dims), "bytes_per_launch": rec["bytes"] / max(rec["launches"], 1)})
    return r


def rank_schedule(prob, prec, ext, sweeps=20):
    """The rank-increasing schedule on the same workload: from rank ones to the
    workload's ranks, growing after every sweep (tau = inf) until the maximum,
    then fixed; wall time of the whole run (plans, growth, per-sweep stats) and
    of one growth (plan creation and fctn_regrow) at the last step."""
    import numpy as np
    import torch
    from paper_2510_22506_amd import Plan, complete_rank_increasing
    from workloads import init_factors, rank_growth_draws
    dims, rmax = prob.dims, prob.ranks
    A0 = init_factors(np.random.default_rng(31), dims, (1,) * len(rmax))
    fill = rank_growth_draws(32, dims)
    kw = dict(lam=prob.lam, delta=prob.delta, rho=prob.rho, precision=prec, extrapolation=ext)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p, hist = complete_rank_increasing(dims, rmax, prob.Y, prob.mask, A0, fill, sweeps,
                                       tau=float("inf"), **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    p.close()
    # one growth to the maximal ranks, timed alone
    below = tuple(max(r - 1, 1) for r in rmax)
    src = Plan(dims, below, **kw)
    src.set_factors(init_factors(np.random.default_rng(33), dims, below))
    src.set_observed(prob.Y, prob.mask)
    src.sweep(1)
    draws = fill(0, tuple(rmax))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dst = Plan(dims, rmax, **kw)
    t2 = time.perf_counter()
    dst.regrow_from(src, draws)
    t3 = time.perf_counter()
    src.close()
    dst.close()
    return {"sweeps": sweeps, "growths": len(set(h["ranks"] for h in hist)) - 1,
            "wall_s": wall, "sweeps_per_s": sweeps / wall,
            "ranks_first_last": [list(hist[0]["ranks"]), list(hist[-1]["ranks"])],
            "growth_ms": {"plan": (t2 - t1) * 1e3, "regrow": (t3 - t2) * 1e3,
                          "from": list(below), "to": list(rmax)}}


def other_workload(spec, steps=40, warmup=3):
    """Sweeps/s of another configuration, `name` or `name:precision` (default
    precision otherwise; reuse on), timed like the main one, with its
    dominant kernel's roofline from an event-bracketed pass."""
    import torch
    from paper_2510_22506_amd import Plan
    from workloads import make_problem
    name, _, prec = spec.partition(":")
    prec = prec or DEFAULT_PREC[name]
    prob = make_problem(name, seed=0, precision=("f64" if prec == "f64" else "f32"))
    plan = Plan(prob.dims, prob.ranks, prob.lam, prob.delta, prob.rho, precision=prec,
                device="cuda:0", extrapolation=DEFAULT_EXTRAP.get(name))
    plan.set_factors(prob.A0)
    plan.set_observed(torch.from_numpy(prob.Y), torch.from_numpy(prob.mask))
    plan.sweep(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.sweep(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.profile_enable(True)
    plan.profile_read(reset=True)
    plan.sweep(steps)
    torch.cuda.synchronize()
    prof = plan.profile_read(reset=True)
    plan.close()
    roofs = {k: stage_roofline(k, v, prec) for k, v in prof.items() if v["launches"]}
    dom = max(roofs, key=lambda k: prof[k]["ms"])
    return {"workload": f"{name}: {WORKLOADS[name][2]}", "dtype": prec, "steps": steps,
            "value": steps / dt, "unit": "sweeps/s", "ms_per_step": dt / steps * 1e3,
            "roofline": roofs[dom]}


def time_variant(prob, prec, ext, steps, warmup, reuse=True):
    """Sweeps/s of the workload in another form (precision, reuse switch),
    timed like the main measurement (no events), with the pair-tensor
    launches per sweep from a second, event-bracketed pass."""
    import torch
    from paper_2510_22506_amd import Plan
    plan = Plan(prob.dims, prob.ranks, prob.lam, prob.delta, prob.rho, precision=prec,
                reuse=reuse, order_policy=1, device="cuda:0", extrapolation=ext)
    plan.set_factors(prob.A0)
    plan.set_observed(torch.from_numpy(prob.Y), torch.from_numpy(prob.mask))
    plan.sweep(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.sweep(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.profile_enable(True)
    plan.profile_read(reset=True)
    plan.sweep(steps)
    prof = plan.profile_read(reset=True)
    plan.close()
    return {"precision": prec, "reuse": reuse, "value": steps / dt, "unit": "sweeps/s",
            "ms_per_step": dt / steps * 1e3,
            "pair_launches_per_sweep": prof["pair"]["launches"] / steps,
            "contraction_gflop_per_sweep":
                sum(prof[k]["flops"] for k in CONTRACTION_STAGES) / steps / 1e9}


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(prob, sweeps, ext=None, runs=3):
    """The float64 oracle on the host cores: the median over `runs` runs of
    `sweeps` sweeps each from the same initial factors (rate in sweeps/s)."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import pam
    A0 = prob.A0
    if prob.precision != "f64":
        A0 = [a.astype(np.float32).astype(np.float64) for a in A0]
    Y = prob.Y.astype(np.float64)
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        pam.complete(Y, prob.mask != 0, prob.ranks, prob.lam, prob.delta, prob.rho, sweeps, A0,
                     reuse=True, order_policy=1, extrapolation=ext)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": sweeps / dt, "unit": "sweeps/s", "cores": int(threads), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"median of {runs} runs of {sweeps} sweeps of the same workload from the "
                      f"same initial factors (run times "
                      f"{', '.join(f'{t:.1f}' for t in times)} s; float64 NumPy; "
                      f"{os.cpu_count()} host CPUs visible)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None)
    ap.add_argument("--reuse", type=int, default=1)
    ap.add_argument("--extrapolation", default=None,
                    help="alpha,beta of the asymmetric extrapolation, or 'off' "
                         "(default: on at 0.5,0.5 for c6, off otherwise)")
    ap.add_argument("--order-policy", type=int, default=1)
    ap.add_argument("--cpu-sweeps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stages", action="store_true", help="add the per-stage breakdown")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the reuse-off and bf16-form rates of the same workload")
    ap.add_argument("--no-rank-schedule", action="store_true",
                    help="skip the rank-increasing schedule measurement")
    ap.add_argument("--also", default="c2,c4,c4:bf16x3",
                    help="comma-separated other workloads (name or name:precision) reported "
                         "under 'other_workloads' ('' for none; default: the 256x256x3 image "
                         "and the 512x512x31 multispectral tensor in float32 and split bf16)")
    ap.add_argument("--no-xpass-large", action="store_true",
                    help="skip the X/mask pass on a 1 GiB tensor")
    ap.add_argument("--serve-n", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-sweeps", type=int, default=30)
    ap.add_argument("--serve-budget", type=float, default=200e9,
                    help="HBM admission budget in bytes (the arena is min(budget, 16 GiB))")
    ap.add_argument("--serve-streams", type=int, default=3,
                    help="server streams (default: one per hardware queue the default "
                         "stream leaves free, GPU_MAX_HW_QUEUES = 4)")
    ap.add_argument("--serve-active", type=int, default=16)
    ap.add_argument("--serve-depth", type=int, default=2)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, copy 256 MiB device-to-device once (a "
                         "kernel of known traffic for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU (the library has no multi-GPU path); "
              "use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2510_22506_amd import Plan
    from workloads import make_problem

    name, dims, desc = WORKLOADS[args.workload]
    prec = args.precision or DEFAULT_PREC[name]
    if args.extrapolation is None:
        ext = DEFAULT_EXTRAP.get(name)
    elif args.extrapolation == "off":
        ext = None
    else:
        ext = tuple(float(v) for v in args.extrapolation.split(","))
    prob = make_problem(name, seed=0, precision=("f64" if prec == "f64" else "f32"))
    plan = Plan(prob.dims, prob.ranks, prob.lam, prob.delta, prob.rho, precision=prec,
                reuse=bool(args.reuse), order_policy=args.order_policy, device="cuda:0",
                extrapolation=ext)
    plan.set_factors(prob.A0)
    plan.set_observed(torch.from_numpy(prob.Y), torch.from_numpy(prob.mask))
    torch.cuda.synchronize()

    plan.sweep(args.warmup)
    torch.cuda.synchronize()
    # timed region: K sweeps as a caller runs them (no per-launch events, which
    # serialize the queue and cost 14 % of the video-shape sweep rate)
    t0 = time.perf_counter()
    plan.sweep(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    value = args.steps / dt
    # the same K sweeps again with HIP events around every launch on the plan's
    # stream: per-kernel durations for the roofline figures
    plan.profile_enable(True)
    plan.profile_read(reset=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    plan.sweep(args.steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = plan.profile_read(reset=True)
    plan.profile_enable(False)

    total_flops = sum(v["flops"] for k, v in prof.items() if k in CONTRACTION_STAGES)
    roofs = {k: stage_roofline(k, v, prec) for k, v in prof.items() if v["launches"]}
    dom = max(roofs, key=lambda k: prof[k]["ms"])
    roof = dict(roofs[dom])
    roof["traffic"] = measured_traffic(name, prec, dom)
    roof_x = dict(roofs["x_update"])
    roof_x["traffic"] = measured_traffic(name, prec, "x_update")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "ms_per_step_with_events": (t3 - t2) / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"{name}: {desc}", "dims": list(prob.dims),
                   "ranks": list(prob.ranks), "precision": prec, "reuse": bool(args.reuse),
                   "order_policy": args.order_policy, "lambda": prob.lam, "rho": prob.rho,
                   "delta": prob.delta,
                   "extrapolation": list(ext) if ext else None},
        "tflops_contractions": total_flops / dt / 1e12,
        "roofline": roof,
        "roofline_xpass": roof_x,
    }
    if args.stages:
        line["stages"] = {k: {"launches": v["launches"], "ms_total": v["ms"],
                              "us_per_launch": v["ms"] * 1e3 / max(v["launches"], 1),
                              "gflop": v["flops"] / 1e9, "roofline": roofs[k]}
                          for k, v in prof.items() if v["launches"]}
    if not args.no_variants:
        # Table 1's reuse mechanism measured: the same sweeps with reuse off
        # (every sub-network and FCTN(A) contracted from the factors); and the
        # other precision forms of the same workload
        line["reuse_off"] = time_variant(prob, prec, ext, args.steps, args.warmup, reuse=False)
        line["reuse_off"]["speedup_reuse_on"] = value / line["reuse_off"]["value"]
        if prec == "f32":
            line["forms"] = {f: time_variant(prob, f, ext, args.steps, args.warmup)
                             for f in ("bf16x3", "bf16")}
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = src.numel() * 4
    if not args.no_xpass_large:
        try:
            line["roofline_xpass_large"] = xpass_large()
        except Exception as e:  # reported, never hides the sweep measurement
            line["roofline_xpass_large"] = {"error": f"{type(e).__name__}: {e}"}
    others = [w for w in args.also.split(",") if w and w != name and w != f"{name}:{prec}"]
    if others:
        line["other_workloads"] = {}
        for w in others:
            try:
                line["other_workloads"][w] = other_workload(w)
            except Exception as e:  # reported, never hides the main measurement
                line["other_workloads"][w] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_rank_schedule:
        try:
            line["rank_schedule"] = rank_schedule(prob, prec, ext)
        except Exception as e:  # reported, never hides the sweep measurement
            line["rank_schedule"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_serve:
        try:
            line["serving"] = serving(args)
        except Exception as e:  # reported, never hides the sweep measurement
            line["serving"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_sweeps, ext)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
