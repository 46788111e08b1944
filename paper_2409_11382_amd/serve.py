"""Serving loop: a Poisson stream of loaded-strip solve requests driven through
the library's continuous-batching server (bp_server_* in biotlbm.h).

Requests arrive in wall-clock time; the loop submits each one when its arrival
time has passed, advances the server one coupled step at a time (every
admitted request moves together), and records for each request the latency
from arrival to the moment its fields are back in host memory.

    python -m paper_2409_11382_amd.serve --rates 1,2,5,10 --count 32
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import lbm
from . import problem as P


def simulate(rate: float, count: int, seed=2, ws_gib=32.0, max_slots=512, nmin=128, nmax=1024,
             steps=(100, 1000), prec="fp32_shifted", K=4, ne_fixed=3, keep_results=False):
    """Serve `count` requests arriving at `rate` per second; returns a summary
    (solves/s, latency percentiles, throughput) and, if asked, the results."""
    reqs = P.serving_requests(rate, count, seed=seed, nmin=nmin, nmax=nmax, steps=steps)
    srv = lbm.Server(int(ws_gib * (1 << 30)), prec=prec, K=K, ne_fixed=ne_fixed, max_slots=max_slots)
    pending = list(reqs)
    live = {}
    lat, finish = [], []
    failures = []
    results = {}
    cell_steps = 0
    peak_active = 0
    t0 = time.perf_counter()
    while pending or live:
        now = time.perf_counter() - t0
        while pending and pending[0][0] <= now:
            arr, prob, nsteps = pending.pop(0)
            t = srv.submit(prob, nsteps)
            live[t] = (arr, prob.ncells, nsteps, count - len(pending) - 1)
        if not live:
            time.sleep(max(0.0, pending[0][0] - now))
            continue
        active, _queued = srv.advance(1)
        peak_active = max(peak_active, active)
        for t in list(live):
            st, _ = srv.poll(t)
            if st in (lbm.REQ_DONE, lbm.REQ_FAILED):
                arr, cells, nsteps, idx = live.pop(t)
                try:
                    out = srv.result(t)
                except lbm.BiotError as e:  # a failed request is reported, the others go on
                    failures.append({"request": idx, "error": str(e)})
                    out = None
                done = time.perf_counter() - t0
                finish.append(done)
                if out is not None:       # latency and throughput of completed solves only
                    lat.append(done - arr)
                    cell_steps += cells * nsteps
                if keep_results:
                    results[idx] = out
    srv.close()
    makespan = max(finish) - reqs[0][0]
    lat = np.array(lat) if lat else np.zeros(1)
    summary = {
        "rate_per_s": rate, "requests": count, "completed": count - len(failures),
        "solves_per_s": round((count - len(failures)) / makespan, 3),
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
        # a 99th percentile needs about 100 samples; below that only the maximum is reported
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4) if len(lat) >= 100 else None,
        "max_latency_s": round(float(lat.max()), 4),
        "mean_latency_s": round(float(lat.mean()), 4),
        "mlups": round(cell_steps / makespan / 1e6, 2),
        "peak_active": peak_active,
        "makespan_s": round(makespan, 3),
        "failed": failures,
    }
    return (summary, results) if keep_results else summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="1,2,5,10")
    ap.add_argument("--count", type=int, default=32)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--ws-gib", type=float, default=32.0)
    args = ap.parse_args()
    for r in (float(x) for x in args.rates.split(",")):
        print(json.dumps(simulate(r, args.count, seed=args.seed, ws_gib=args.ws_gib)), flush=True)


if __name__ == "__main__":
    main()
