"""Benchmark: spin-flip attempts/s and time-to-target cut on one MI355X.

One step = one whole anneal of the 100x80 toroidal +-1 spin glass (the
shape of the paper's G65, Table I): threshold table, initial draw and
fields, 4000 colour-class sweeps of 256 replicas under a geometric beta
schedule 0.1 -> 4.0, end-of-sweep best tracking, argmax, and the best cut
copied back to the host.  The persistent LDS-resident kernel is timed; the
plain one-launch-per-colour-pass form is timed beside it on the same seeds
(identical results, so the time-to-target ratio is the wall-time ratio),
and so is the batched form on 64 uneven tori.  The CPU oracle is timed on a
bounded sample of the same workload on the host cores.

Prints one JSON line.  `--gpus N` with N > 1 exits: the benchmark measures
one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/s + time-to-target cut, batched vs plain, 1 MI355X"
UNIT = "spin-flip attempts/s"

# MI355X figures used as roofline peaks.
HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ = 256, 2.4
# Integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations/s.
# On gfx950 the 32x32->64-bit products of the RNG issue at (nearly) this
# full rate too; ising_valu_rates measures the rates live.
VALU_PEAK_PER_S = CUS * 64 * CLOCK_GHZ * 1e9
# Algorithmic 32-bit integer operations: a Philox4x32-10 block is ten
# rounds of two products and four XORs; an attempt's accept test is k = s h,
# the row index and one compare; an accepted flip updates the spin, the
# energy and one field per neighbour.
OPS_PER_PHILOX = 60
OPS_PER_TEST = 3


def _profile_figure(name, pattern, cast):
    """A figure from a committed counter summary, or None when the kernel
    source has changed since the counters were taken (each summary records
    the SHA-256 of kernels.hip)."""
    import hashlib
    import re
    summary = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2311_09275_amd", "csrc", "kernels.hip")
    try:
        text = open(summary).read()
        want = re.search(r"kernels\.hip sha256: ([0-9a-f]{64})", text).group(1)
        have = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if want != have:
            return None
        return cast(re.search(pattern, text).group(1))
    except (OSError, AttributeError):
        return None


def measured_traffic():
    """HBM bytes per launch of the timed kernel (FETCH_SIZE + WRITE_SIZE)."""
    return _profile_figure("k_field_torus100x80_r256_counters.md", r"HBM bytes per launch: (\d+)", int)


def measured_valu_issue():
    """Fraction of the SIMDs' cycles spent issuing VALU instructions."""
    return _profile_figure("k_field_torus100x80_r256_valu.md", r"VALU issue fraction: [^=]*= ([0-9]+\.[0-9]+)", float)


def measured_lds():
    """LDS active and bank-conflict fractions of the timed kernel."""
    act = _profile_figure("k_field_torus100x80_r256_lds.md", r"LDS active fraction: ([0-9.]+)", float)
    conf = _profile_figure("k_field_torus100x80_r256_lds.md", r"LDS bank-conflict fraction: ([0-9.]+)", float)
    return None if act is None else {"active_frac": act, "bank_conflict_frac": conf}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-torus batch leg")
    ap.add_argument("--no-random", action="store_true", help="skip the sparse random graph leg")
    ap.add_argument("--no-temper", action="store_true", help="skip the parallel tempering leg")
    ap.add_argument("--no-msc", action="store_true", help="skip the multispin leg")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests of the Poisson serving leg (0 = skip)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparisons")
    ap.add_argument("--no-ttt", action="store_true", help="skip the reference run for targets")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 256 MiB device copy first (byte-counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_09275_amd import binding as B
    from paper_2311_09275_amd import instances as I
    from paper_2311_09275_amd import ttt

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)

    if args.calib_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # ------------------------------------------------------------ workload
    L_X, L_Y, R, S, B0, B1, SEED = 100, 80, 256, 4000, 0.1, 4.0, 1002
    inst = I.workload_c2()
    sched = B.Schedule.make(B.GEOMETRIC, S, B0, B1)
    attempts = inst.n * R * S

    t0 = time.perf_counter()
    prob = B.Problem.from_instance(inst)
    create_ms = (time.perf_counter() - t0) * 1e3

    def run_steps(tuning, steps, warmup, problem=prob):
        for _ in range(warmup):
            problem.anneal(sched, R, SEED, tuning, stream=stream)
            problem.cut()
        torch.cuda.synchronize()
        walls, kern = [], []
        for _ in range(steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            problem.anneal(sched, R, SEED, tuning, stream=stream)
            res = problem.cut()  # synchronises the stream
            walls.append(time.perf_counter() - t)
            kern.append(problem.last_anneal_ms())
        torch.cuda.synchronize()
        return res, walls, kern

    field = B.Tuning(B.PATH_FIELD, 1, 1024)
    res, walls, kern = run_steps(field, args.steps, args.warmup)
    wall_s = sum(walls)
    ms_per_step = wall_s / args.steps * 1e3
    value = attempts * args.steps / wall_s
    per_rep = res.per_replica.copy()
    best_field = res.best_cut
    kern_ms = float(np.mean(kern))

    # plain form: same seeds, so identical results
    plain_ms = None
    if not args.no_plain:
        res_p, walls_p, kern_p = run_steps(B.Tuning(B.PATH_PLAIN, 1, 256), max(1, args.steps // 2), 1)
        plain_ms = float(np.mean(walls_p)) * 1e3
        assert np.array_equal(res_p.per_replica, per_rep), "plain and persistent forms disagree"

    # multispin form (32 replicas per word) on the same seeds: identical
    # results; its time and, below, its ALU roofline fraction
    msc_leg = None
    if not args.no_msc:
        msc_leg = {"workload": "the benchmark anneal on the multispin path", "configs": {}}
        for name, tun in (("words1_threads256", B.Tuning(B.PATH_MSC, 1, 256, 0)),
                          ("words2_threads512", B.Tuning(B.PATH_MSC, 2, 512, 0))):
            res_m, walls_m, kern_m = run_steps(tun, 2, 1)
            assert np.array_equal(res_m.per_replica, per_rep), "multispin and field forms disagree"
            msc_leg["configs"][name] = {"ms_per_anneal": float(np.mean(walls_m)) * 1e3,
                                        "kernel_ms": float(np.mean(kern_m)),
                                        "attempts_per_s": attempts / float(np.mean(walls_m))}

    # ------------------------------------------------------------ time to target
    # Reference best cut of this instance: a longer anneal of 1024 replicas
    # (512-thread blocks, so that its dispatches are told apart in profiles).
    c_ref, ttt_rows = None, None
    if not args.no_ttt:
        ref = B.Problem.from_instance(inst)
        ref.anneal(B.Schedule.make(B.GEOMETRIC, 20000, B0, B1), 1024, 7,
                   B.Tuning(B.PATH_FIELD, 1, 512, 0), stream=stream)
        c_ref = ref.cut().best_cut
        ref.close()
        ttt_rows = {}
        for q in (0.995, 0.998, 1.0):
            target = ttt.target_cut(c_ref, q)
            tf = ttt.replica_ttt(per_rep, target, ms_per_step / 1e3, S)
            row = {"target": target, "ps": tf["ps"], "ttt_persistent_s": tf["ttt_s"],
                   "sweeps_to_target": tf["sweeps_to_target"]}
            if plain_ms is not None:
                row["ttt_plain_s"] = ttt.replica_ttt(per_rep, target, plain_ms / 1e3, S)["ttt_s"]
            ttt_rows[str(q)] = row

    # ------------------------------------------------------------ batch leg
    batch = None
    if not args.no_batch:
        insts = I.workload_c4()
        probs = [B.Problem.from_instance(x) for x in insts]
        handles = [p.handle for p in probs]
        seeds = np.array([2000 + i for i in range(len(insts))], np.uint64)
        Rb = 128
        bat_att = sum(x.n for x in insts) * Rb * S
        tun = B.ising_autotune(handles, sched, Rb, prefix_sweeps=200, stream=stream)
        B.ising_anneal_batch(handles, sched, Rb, seeds, tun, stream=stream)  # warm (captures)
        torch.cuda.synchronize()
        t = time.perf_counter()
        B.ising_anneal_batch(handles, sched, Rb, seeds, tun, stream=stream)
        cuts_b = [B.ising_cut(h)[0] for h in handles]
        bat_s = time.perf_counter() - t
        t = time.perf_counter()
        B.ising_anneal_batch(handles, sched, Rb, seeds, B.Tuning(B.PATH_PLAIN, 1, 256), stream=stream)
        cuts_p = [B.ising_cut(h)[0] for h in handles]
        plain_b_s = time.perf_counter() - t
        assert cuts_b == cuts_p, "batched and plain forms disagree"
        # the batch on the multispin path (one 32-replica word per unit)
        msc_b = B.Tuning(B.PATH_MSC, 1, 256, 0)
        B.ising_anneal_batch(handles, sched, Rb, seeds, msc_b, stream=stream)  # warm (captures)
        torch.cuda.synchronize()
        t = time.perf_counter()
        B.ising_anneal_batch(handles, sched, Rb, seeds, msc_b, stream=stream)
        cuts_m = [B.ising_cut(h)[0] for h in handles]
        msc_b_s = time.perf_counter() - t
        assert cuts_m == cuts_p, "batched multispin and plain forms disagree"
        per_b = [B.ising_cut(h, Rb)[2].copy() for h in handles]  # identical on every form
        batch = {"workload": "64 LxL +-1 tori, L~U{32..141}, 128 replicas, 4000 sweeps geometric 0.1->4.0",
                 "attempts": bat_att, "batched_s": bat_s, "plain_s": plain_b_s,
                 "batched_attempts_per_s": bat_att / bat_s, "plain_attempts_per_s": bat_att / plain_b_s,
                 "msc_s": msc_b_s, "msc_attempts_per_s": bat_att / msc_b_s,
                 "tuning": {"path": int(tun.path), "replicas_per_block": int(tun.replicas_per_block),
                            "block_threads": int(tun.block_threads),
                            "lds_adjacency": int(tun.lds_adjacency)}}
        if not args.no_ttt:
            # reference best of every problem: one batched anneal of 5x the
            # sweeps with other seeds; a replica of the timed batch is a trial
            # of its problem, and the batch's wall time runs R trials of every
            # problem (t_trial = wall / R), batched and plain alike
            B.ising_anneal_batch(handles, B.Schedule.make(B.GEOMETRIC, 5 * S, B0, B1), Rb,
                                 seeds + np.uint64(50_000), tun, stream=stream)
            refs = [B.ising_cut(h)[0] for h in handles]
            batch["ttt"] = {}
            for q in (0.995, 0.998):
                rows = [ttt.replica_ttt(per_b[i], ttt.target_cut(refs[i], q), bat_s, S)
                        for i in range(len(handles))]
                hit = [r_ for r_ in rows if r_["ps"] > 0]
                med = float(np.median([r_["ttt_s"] for r_ in hit])) if hit else float("inf")
                batch["ttt"][str(q)] = {"problems_with_ps_above_0": len(hit),
                                        "median_ttt_batched_s": med,
                                        "median_ttt_plain_s": med * plain_b_s / bat_s,
                                        "median_ps": float(np.median([r_["ps"] for r_ in rows]))}
        for p in probs:
            p.close()

    # ------------------------------------------------------------ random graph leg
    # The sparse random graph (N = 10,000, M = 9,999, 1024 replicas, 4000
    # sweeps linear 0.05 -> 3.0) under the library's automatic configuration,
    # the plain form on the same seeds, and time to target against a longer
    # reference anneal.
    random_leg = None
    if not args.no_random:
        inst3 = I.workload_c3()
        R3, S3, SEED3 = 1024, 4000, 1003
        sched3 = B.Schedule.make(B.LINEAR, S3, 0.05, 3.0)
        p3 = B.Problem.from_instance(inst3)
        auto = B.Tuning(B.PATH_AUTO, 0, 0, 0)
        p3.anneal(sched3, R3, SEED3, auto, stream=stream)
        p3.cut()
        walls3 = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            p3.anneal(sched3, R3, SEED3, auto, stream=stream)
            res3 = p3.cut()
            walls3.append(time.perf_counter() - t)
        path3 = B.ising_last_run_info(p3.handle)[2]
        kern3 = p3.last_anneal_ms()
        per3 = res3.per_replica.copy()
        ms3 = float(np.mean(walls3)) * 1e3
        att3 = inst3.n * R3 * S3
        random_leg = {"workload": "sparse random graph N=10000 M=9999 w=1, 1024 replicas, "
                                  "4000 sweeps linear 0.05->3.0",
                      "attempts_per_s": att3 / (ms3 / 1e3), "ms_per_anneal": ms3,
                      "kernel_ms": kern3, "best_cut": int(res3.best_cut),
                      "path": {1: "plain", 2: "field", 3: "msc"}.get(path3, str(path3)),
                      "tuning": "automatic"}
        if not args.no_plain:
            t = time.perf_counter()
            p3.anneal(sched3, R3, SEED3, B.Tuning(B.PATH_PLAIN, 1, 256, 0), stream=stream)
            res3p = p3.cut()
            plain3_s = time.perf_counter() - t
            assert np.array_equal(res3p.per_replica, per3), "plain and automatic forms disagree"
            random_leg["plain_ms"] = plain3_s * 1e3
            random_leg["speedup_vs_plain"] = plain3_s * 1e3 / ms3
        if not args.no_ttt:
            ref3 = B.Problem.from_instance(inst3)
            ref3.anneal(B.Schedule.make(B.LINEAR, 5 * S3, 0.05, 3.0), R3, 7, auto, stream=stream)
            c_ref3 = ref3.cut().best_cut
            ref3.close()
            random_leg["reference_best_cut"] = int(c_ref3)
            random_leg["ttt"] = {}
            for q in (0.995, 0.998, 1.0):
                target = ttt.target_cut(c_ref3, q)
                tf = ttt.replica_ttt(per3, target, ms3 / 1e3, S3)
                random_leg["ttt"][str(q)] = {
                    "target": target, "ps": tf["ps"], "ttt_persistent_s": tf["ttt_s"]}
                if not args.no_plain:
                    random_leg["ttt"][str(q)]["ttt_plain_s"] = \
                        ttt.replica_ttt(per3, target, plain3_s, S3)["ttt_s"]
        p3.close()

    # ------------------------------------------------------------ tempering leg
    # Parallel tempering on the benchmark torus: 8 sets of 32 temperatures
    # (geometric 0.2 -> 3.0, 256 replicas), 4000 sweeps, an exchange round
    # every 10 sweeps (and every 100, for the cost of the segment launches),
    # the plain form on the same seeds; trial = one set for time to target.
    temper_leg = None
    if not args.no_temper:
        K, n_sets, P = 32, 8, 10
        ladder = list(np.geomspace(0.2, 3.0, K))
        pt_att = inst.n * K * n_sets * S

        def temper_run(P_, tuning=None, reps=2, cluster_from=None):
            prob.temper(ladder, n_sets, S, P_, SEED, tuning, stream=stream,
                        cluster_from=cluster_from)  # warm (captures)
            prob.cut()
            walls_t = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                prob.temper(ladder, n_sets, S, P_, SEED, tuning, stream=stream,
                            cluster_from=cluster_from)
                r_ = prob.cut()
                walls_t.append(time.perf_counter() - t)
            return r_, float(np.mean(walls_t)) * 1e3, prob.last_anneal_ms()

        res_t, ms_t, kern_t = temper_run(P)
        temp_t, swaps_t = prob.temper_results()
        per_t = res_t.per_replica.copy()
        path_t = B.ising_last_run_info(prob.handle)[2]
        _, ms_t100, kern_t100 = temper_run(100)
        # Houdayer cluster moves at the colder half of the ladder
        res_c, ms_c, kern_c = temper_run(P, cluster_from=K // 2)
        _, _, cm_c, cs_c = prob.temper_results()
        t = time.perf_counter()
        prob.temper(ladder, n_sets, S, P, SEED, B.Tuning(B.PATH_PLAIN, 1, 256, 0), stream=stream)
        res_tp = prob.cut()
        plain_t_ms = (time.perf_counter() - t) * 1e3
        assert np.array_equal(res_tp.per_replica, per_t), "plain and persistent tempering disagree"
        tries = np.array([len(range(k % 2, S // P, 2)) for k in range(K - 1)], np.float64)
        rate = swaps_t.sum(axis=0) / (tries * n_sets)
        temper_leg = {"workload": f"torus 100x80, {n_sets} sets x {K} temperatures geometric 0.2->3.0, "
                                  f"{S} sweeps, exchange every {P}",
                      "attempts_per_s": pt_att / (ms_t / 1e3), "ms_per_run": ms_t, "kernel_ms": kern_t,
                      "ms_per_run_exchange_every_100": ms_t100, "kernel_ms_exchange_every_100": kern_t100,
                      "plain_ms": plain_t_ms, "speedup_vs_plain": plain_t_ms / ms_t,
                      "path": {1: "plain", 2: "field", 3: "msc"}.get(path_t, str(path_t)),
                      "best_cut": int(res_t.best_cut),
                      "exchange_rate": {"min": float(rate.min()), "mean": float(rate.mean()),
                                        "max": float(rate.max())},
                      "cluster_moves": {"from_temperature": K // 2, "ms_per_run": ms_c, "kernel_ms": kern_c,
                                        "moves": int(cm_c.sum()),
                                        "mean_cluster_sites": float(cs_c.sum() / max(cm_c.sum(), 1)),
                                        "best_cut": int(res_c.best_cut)}}
        if c_ref is not None:
            temper_leg["ttt"] = {}
            temper_leg["cluster_moves"]["ttt"] = {}
            for q in (0.995, 0.998, 1.0):
                target = ttt.target_cut(c_ref, q)
                for per_, ms_, dst in ((per_t, ms_t, temper_leg["ttt"]),
                                       (res_c.per_replica, ms_c, temper_leg["cluster_moves"]["ttt"])):
                    tf = ttt.replica_ttt(per_.reshape(n_sets, K).max(axis=1), target, ms_ / 1e3, S)
                    dst[str(q)] = {"target": target, "ps_sets": tf["ps"], "ttt_s": tf["ttt_s"]}

    # ------------------------------------------------------------ serving leg
    serving = None
    if args.serve_requests > 0:
        from paper_2311_09275_amd import serve_load
        serving = serve_load.run(rate=50.0, n_requests=args.serve_requests, stream=stream)

    # ------------------------------------------------------------ CPU oracle
    cpu = None
    draws_per_attempt = accepts_per_attempt = None
    if not args.no_cpu:
        from oracle import oracle as O
        O.build(force=False)
        threads = max(1, min(os.cpu_count() or 1, 16))
        sample = min(R, 16 * threads)
        t = time.perf_counter()
        o = O.anneal(inst, S, R, SEED, kind=O.GEOMETRIC, beta0=B0, beta1=B1, r_begin=0,
                     r_end=sample, n_threads=threads, want_states=False)
        cpu_s = time.perf_counter() - t
        assert np.array_equal(o.best_cut, per_rep[:sample]), "oracle and GPU disagree"
        # one thread on two replicas, for the per-core rate
        t = time.perf_counter()
        O.anneal(inst, S, R, SEED, kind=O.GEOMETRIC, beta0=B0, beta1=B1, r_begin=0, r_end=2,
                 n_threads=1, want_states=False)
        one_s = time.perf_counter() - t
        cpu = {"value": inst.n * sample * S / cpu_s, "unit": UNIT, "cores": threads, "kind": "oracle",
               "sample": f"replicas 0..{sample - 1} of 256, all {S} sweeps, {threads} threads, {cpu_s:.1f} s",
               "one_thread_value": inst.n * 2 * S / one_s, "cpu_model": cpu_model()}
        draws_per_attempt = float(o.draws.sum()) / (inst.n * sample * S)
        accepts_per_attempt = float(o.accepts.sum()) / (inst.n * sample * S)
        if ttt_rows is not None:
            # the oracle's wall time for all R replicas at its measured rate
            oracle_wall = attempts / cpu["value"]
            for row in ttt_rows.values():
                row["ttt_oracle_s"] = ttt.replica_ttt(per_rep, row["target"], oracle_wall, S)["ttt_s"]

    # ------------------------------------------------------------ roofline
    # Algorithmic integer work per launch, from the exact counts of the
    # oracle's sample (Philox blocks drawn, moves accepted).
    if draws_per_attempt is None:
        draws_per_attempt, accepts_per_attempt = 0.24, 0.36
    mean_degree = 2.0 * inst.m / inst.n
    ops_per_attempt = (OPS_PER_PHILOX * draws_per_attempt + OPS_PER_TEST +
                       accepts_per_attempt * (2.0 + mean_degree))
    achieved = ops_per_attempt * attempts / (kern_ms / 1e3)
    rates = B.ising_valu_rates()
    if msc_leg is not None:
        for cfg_ in msc_leg["configs"].values():
            cfg_["alu_frac"] = ops_per_attempt * attempts / (cfg_["kernel_ms"] / 1e3) / VALU_PEAK_PER_S
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_PER_S / 1e12,
                "unit": "T int32 ops/s", "frac": achieved / VALU_PEAK_PER_S,
                "traffic": measured_traffic(), "valu_issue_frac": measured_valu_issue(),
                "lds": measured_lds(),
                "ops_per_attempt": ops_per_attempt,
                "measured_lane_ops_per_s": {k: v for k, v in rates.items()}}

    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"torus {L_X}x{L_Y} +-1 spin glass (N=8000, M=16000), {R} replicas, "
                               f"{S} sweeps geometric beta {B0}->{B1}",
                   "replicas": R, "sweeps": S, "seed": SEED, "path": "field (persistent, LDS)",
                   "block_threads": 1024, "replicas_per_block": 1},
        "kernel_ms": kern_ms,
        "plain_ms_per_step": plain_ms,
        "batched_vs_plain_speedup": None if plain_ms is None else plain_ms / ms_per_step,
        "create_ms": create_ms,
        "value_incl_create": attempts / (ms_per_step / 1e3 + create_ms / 1e3),
        "best_cut": best_field,
        "reference_best_cut": c_ref,
        "ttt": ttt_rows,
        "batch": batch,
        "random_graph": random_leg,
        "tempering": temper_leg,
        "multispin": msc_leg,
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    prob.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
