"""Poisson load generator for the continuous-batching server.

Requests arrive as a Poisson process and mix the shapes of the paper's Gset
instances (Table I): toroidal +-1 spin glasses of 8,000, 10,000, 14,000 and
20,000 vertices and a sparse random unweighted graph of 10,000 vertices with
average degree 2.  Each request anneals 256 replicas for up to 1000 sweeps
(linear beta 0.1 -> 3.0) and stops early, checked every 50 of its sweeps,
once a replica reaches its target cut: a fixed fraction of a reference best
cut of that instance, found once by a longer anneal.  Reports latency
percentiles (completion minus arrival) and throughput.

    python -m paper_2311_09275_amd.serve_load --rate 50 --requests 1000
    python -m paper_2311_09275_amd.serve_load --rates inf,25,50,100,200 --budget-mb 96
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import binding as B
from . import instances as I

SHAPES = [("torus 100x80", lambda: I.torus(100, 80, seed=501)),
          ("torus 100x100", lambda: I.torus(100, 100, seed=502)),
          ("torus 100x140", lambda: I.torus(100, 140, seed=503)),
          ("torus 100x200", lambda: I.torus(100, 200, seed=504)),
          ("random 10000/10000", lambda: I.random_graph(10000, 10000, seed=505))]


def run(rate: float = 50.0, n_requests: int = 1000, seed: int = 7, budget: int = 256 << 20,
        slots: int = 16, chunk: int = 50, replicas: int = 256, sweeps: int = 1000,
        quality: float = 0.99, stream=None) -> dict:
    insts = [mk() for _, mk in SHAPES]
    probs = [B.Problem.from_instance(x) for x in insts]
    sched = B.Schedule.make(B.LINEAR, sweeps, 0.1, 3.0)
    # reference best of each instance: the stored calibration, else a
    # longer anneal (1024 replicas, 5x the request's sweeps)
    from . import reference_cuts as RC
    stored = RC.load()
    refs = []
    for (name, _), p in zip(SHAPES, probs):
        key = "serve_" + name.replace(" ", "").replace("/", "_")
        if key in stored:
            refs.append(stored[key])
            continue
        p.anneal(B.Schedule.make(B.LINEAR, 5 * sweeps, 0.1, 3.0), 1024, 99,
                 B.Tuning(B.PATH_FIELD, 1, 512, 2), stream=stream)
        refs.append(p.cut().best_cut)
    targets = [int(math.ceil(quality * r)) for r in refs]

    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = rng.integers(0, len(probs), size=n_requests)
    # an infinite rate submits every request at once: the server's capacity
    arrivals = (I.poisson_arrivals(rate, n_requests, seed) if math.isfinite(rate)
                else np.zeros(n_requests))

    srv = B.ising_server_create(budget, slots, chunk, backend=0, stream=stream)
    t0 = time.perf_counter()
    tickets = []
    for i in range(n_requests):
        delay = arrivals[i] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        k = int(kinds[i])
        tickets.append((k, B.ising_server_submit(srv, probs[k].handle, sched, replicas, 10_000 + i,
                                                 targets[k], 50)))
    results = [(k, B.ising_server_wait(srv, t, 600.0)) for k, t in tickets]
    wall = time.perf_counter() - t0
    steps, finished, peak = B.ising_server_stats(srv)
    B.ising_server_destroy(srv)

    lat = np.array([r.t_done - r.t_submit for _, r in results])
    wait = np.array([r.t_admit - r.t_submit for _, r in results])
    footprint = [B.ising_server_footprint(p.handle, sched, replicas) for p in probs]
    attempts = sum(insts[k].n * replicas * r.sweeps_done for k, r in results)
    # work the stream asks for: the arrival rate times the mean attempts a
    # request took (requests stop at their target, so this is below the
    # rate times the full 1000 sweeps)
    demand = rate * attempts / n_requests
    reached = np.mean([r.reached_target for _, r in results])
    for p in probs:
        p.close()
    return {
        "workload": f"Poisson {rate}/s, {n_requests} requests over {len(SHAPES)} shapes, "
                    f"{replicas} replicas, <= {sweeps} sweeps linear 0.1->3.0, stop at "
                    f"{quality:.0%} of a reference best (checked every 50 sweeps)",
        "requests": n_requests, "wall_s": wall,
        "requests_per_s": n_requests / wall, "attempts_per_s": attempts / wall,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()), "admission_wait_p50_s": float(np.percentile(wait, 50)),
        "admission_wait_p99_s": float(np.percentile(wait, 99)),
        "admitted_after_waiting_fraction": float(np.mean(wait > 1e-3)),
        "footprint_bytes": {"min": int(min(footprint)), "max": int(max(footprint))},
        "target_reached_fraction": float(reached), "mean_sweeps": float(np.mean([r.sweeps_done for _, r in results])),
        "hbm_budget_bytes": budget, "slots": slots, "chunk_sweeps": chunk,
        "server_steps": steps, "peak_resident": peak,
        "offered_attempts_per_s": rate * float(np.mean([x.n for x in insts])) * replicas * sweeps,
        "demand_attempts_per_s": demand,
        "references": refs,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--rates", default=None, help="comma-separated rates: one JSON line each")
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--budget-mb", type=int, default=256)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=50)
    args = ap.parse_args()
    import torch
    stream = torch.cuda.Stream()
    rates = [args.rate] if args.rates is None else [float(x) for x in args.rates.split(",")]
    for rate in rates:
        print(json.dumps(run(rate, args.requests, budget=args.budget_mb << 20, slots=args.slots,
                             chunk=args.chunk, stream=stream)), flush=True)


if __name__ == "__main__":
    main()
