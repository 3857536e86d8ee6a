"""Request loop over the continuous-batching server (fctn_server_* in
libfctn.so): each request is submitted at its arrival time, the server is
stepped until every request has completed, and per-request latency (arrival
to completion, host monotonic clock) is recorded.  Argument marshalling and
bookkeeping only: admission, scheduling and every sweep run in the library.
"""

import time

import numpy as np


def run(server, requests, arrivals=None):
    """Drive `server` (a fctn.Server) over `requests`.

    requests: list of dicts of Server.submit keyword arguments (each with a
    unique integer "tag"); arrivals: seconds after the start at which each
    request arrives (None: all at once).  Returns a dict with per-tag
    completions and X tensors, latencies (seconds) and the wall time from the
    first arrival to the last completion.
    """
    n = len(requests)
    arr = np.zeros(n) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    order = np.argsort(arr, kind="stable")
    t0 = time.monotonic()
    nxt = 0
    done = {}
    while len(done) < n:
        now = time.monotonic() - t0
        while nxt < n and arr[order[nxt]] <= now:
            server.submit(**requests[order[nxt]])
            nxt += 1
        fresh = server.step()
        for c, X in fresh:
            done[c["tag"]] = (c, X)
        if fresh:
            continue
        if server.query()[:2] == (0, 0):
            # nothing resident or queued: idle until the next arrival
            if nxt < n:
                wait = arr[order[nxt]] - (time.monotonic() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        else:
            # work in flight and nothing finished: yield the host core briefly
            # instead of polling the completion events in a tight loop
            time.sleep(5e-5)
    wall = max(c["t_done"] for c, _ in done.values()) - (t0 + float(arr.min()))
    lat = {}
    for i, r in enumerate(requests):
        c = done[r["tag"]][0]
        lat[r["tag"]] = c["t_done"] - (t0 + float(arr[i]))
    return {"done": done, "latency": lat, "wall": wall, "t0": t0}


def summarize(result):
    """completions/s, p50/p99 latency (ms) of a run() result."""
    lat = np.array(sorted(result["latency"].values()))
    n = len(lat)
    return {
        "completions": n,
        "wall_s": result["wall"],
        "completions_per_s": n / result["wall"] if result["wall"] > 0 else float("inf"),
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "max_ms": 1e3 * float(lat.max()),
    }
