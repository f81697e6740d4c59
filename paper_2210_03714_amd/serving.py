"""Open-loop load generator for the serving runtime (pfm.Server).

Submits a request stream at its scheduled arrival times, drains completions
while waiting, and reports throughput and latency percentiles.  Latency of a
request = the library's submit-to-completion time plus how late the submit
itself was against the scheduled arrival (so a generator that falls behind
cannot hide queueing)."""

import time

import numpy as np


def to_device(pool, vpool, device="cuda"):
    import torch
    dp = {k: [torch.from_numpy(a).to(device) for a in v] for k, v in pool.items()}
    dv = {k: torch.from_numpy(v).to(device) for k, v in vpool.items()}
    return dp, dv


def run_stream(srv, reqs, dpool, dvpool, keep=(), progress=None):
    """Returns a dict of per-request results: latency (s), status, ticket;
    tickets listed in ``keep`` (request indices) are not released."""
    keep = set(keep)
    n = len(reqs)
    tickets = [None] * n
    lag = np.zeros(n)
    by_ticket = {}
    lat = np.full(n, np.nan)
    parts = np.full((n, 4), np.nan)
    status = np.zeros(n, dtype=np.int64)
    done = 0

    def collect():
        nonlocal done
        for t, l, s in srv.drain():
            i = by_ticket.pop(t)
            lat[i] = l + lag[i]
            parts[i] = srv.timing(t)
            status[i] = s
            done += 1
            if i not in keep:
                srv.release(t)

    t0 = time.perf_counter()
    last_report = t0
    for i, r in enumerate(reqs):
        target = t0 + r["t"]
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            if target - now > 0.001:
                collect()
                now = time.perf_counter()
                if target - now > 0.0005:
                    time.sleep(min(0.0005, target - now))
        A = dpool[r["kind"]][r["idx"]]
        V = dvpool[r["kind"]][: r["n"], : r["p"]] if r["mode"] == "action" else None
        lag[i] = max(0.0, time.perf_counter() - target)
        tk = srv.submit(A, V, r["func"], 8, r["tol"])
        tickets[i] = tk
        by_ticket[tk] = i
        if progress and time.perf_counter() - last_report > 5.0:
            last_report = time.perf_counter()
            progress("submitted %d/%d done %d" % (i + 1, n, done))
    t_sub = time.perf_counter()
    while done < n:
        collect()
        time.sleep(0.001)
        if progress and time.perf_counter() - last_report > 5.0:
            last_report = time.perf_counter()
            progress("draining: done %d/%d" % (done, n))
    t_end = time.perf_counter()
    return {"latency": lat, "status": status, "tickets": tickets, "lag": lag, "parts": parts,
            "wall": t_end - t0, "submit_wall": t_sub - t0}


def summarize(res, reqs):
    lat = res["latency"]
    return {
        "requests": len(reqs),
        "throughput_req_s": len(reqs) / res["wall"],
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "max_submit_lag_ms": float(res["lag"].max() * 1e3),
        "failed": int((res["status"] != 0).sum()),
        "wall_s": res["wall"],
        # where the latency went (library stamps; the submit lag is apart)
        "breakdown_ms": {name: {"p50": round(float(np.percentile(res["parts"][:, j], 50) * 1e3), 3),
                                "p99": round(float(np.percentile(res["parts"][:, j], 99) * 1e3), 3),
                                "mean": round(float(res["parts"][:, j].mean() * 1e3), 3)}
                         for j, name in enumerate(("admission_wait", "lane_wait", "host_enqueue",
                                                   "device_to_completion_seen"))},
    }
