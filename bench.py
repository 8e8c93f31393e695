"""Benchmark: spin-flip attempts/s and time-to-target cut, batched vs plain, on one MI355X.

One step = one batched anneal of the 64-torus workload: 64 toroidal +-1 spin
glasses L x L with L uniform in 32..141 (the sizes of the paper's torus
instances and beyond, Table I), 128 replicas each, 4000 sweeps of a
geometric beta schedule 0.1 -> 4.0, all in one persistent launch captured
into a hipGraph, with the launch configuration chosen by the library's
autotuner; the step ends when every problem's best cut is back on the host.
Beside it, on the same seeds (identical results, so time-to-target ratios
are wall-time ratios):
  - the same 64 anneals as 64 separate persistent launches (batching's own gain);
  - the plain one-launch-per-colour-pass form;
  - the FIELD path's best batched form.
Time to target uses stored reference cuts (reference_cuts.json).  Further
legs: the 100x80 torus (256 replicas, 4000 sweeps), the sparse random graph
(N = 10,000, M = 9,999, 1024 replicas), parallel tempering, Poisson serving,
and the CPU oracle on a bounded sample of the headline workload.

Each leg carries a roofline object: the ALU work the method needs per attempt
(Philox blocks and draw-decided compares, counted by the oracle on a sample),
its HBM bytes per attempt, the LDS bytes its kernel moves, and measured
figures from the committed rocprofv3 summaries while the kernel source is the
one they were taken with.

Prints one JSON line.  `--gpus N` with N > 1 exits: the benchmark measures
one GPU.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/s + time-to-target cut, batched vs plain, 1 MI355X"
UNIT = "spin-flip attempts/s"

# MI355X figures used as roofline peaks.
HBM_PEAK_BPS = 8.0e12
CUS, CLOCK_HZ = 256, 2.4e9
# VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-instructions/s.
VALU_PEAK = CUS * 64 * CLOCK_HZ
# LDS: 128 bytes per clock per CU (the ds_read_b128 rate of the CDNA
# generations); ising_lds_rate measures it live.
LDS_PEAK_THEORY = CUS * 128 * CLOCK_HZ
# Minimum VALU instructions of the method: a Philox4x32-10 block is ten
# rounds of two 32x32->64 products (one v_mad_u64_u32 each) and two
# three-input XORs (one v_bitop3_b32 each); every attempt whose acceptance a
# draw decides needs one 32-bit compare.  Everything else the method does
# (the spin and field bookkeeping) is done 32 replicas per instruction by
# the multispin kernels, so it is not a per-attempt floor.
OPS_PER_BLOCK = 40
SCHED_C4 = dict(S=4000, b0=0.1, b1=4.0)


def kernels_sha():
    src = os.path.join(ROOT, "paper_2311_09275_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def profile_figure(name, key, cast=float):
    """`key: value` from a committed profile summary, or None when the
    summary is missing or was taken with another kernels.hip."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        text = open(path).read()
        want = re.search(r"kernels\.hip sha256: ([0-9a-f]{64})", text).group(1)
        if want != kernels_sha():
            return None
        m = re.search(re.escape(key) + r": ([-0-9.e+]+)", text)
        return cast(m.group(1)) if m else None
    except (OSError, AttributeError):
        return None


def cpu_info():
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["affinity"] = os.cpu_count()
    try:
        fields = {}
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = line.split(":", 1)
                k = k.strip()
                if k in ("model name", "cpu family", "model", "stepping", "cpu MHz") and k not in fields:
                    fields[k] = v.strip()
        info.update(fields)
    except OSError:
        pass
    return info


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline and tallies")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparisons")
    ap.add_argument("--no-separate", action="store_true", help="skip the 64 separate launches")
    ap.add_argument("--no-c2", action="store_true", help="skip the 100x80 torus leg")
    ap.add_argument("--no-random", action="store_true", help="skip the sparse random graph leg")
    ap.add_argument("--no-fields", action="store_true", help="skip the local-fields leg")
    ap.add_argument("--no-temper", action="store_true", help="skip the parallel tempering leg")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the Poisson serving leg (0 = skip)")
    ap.add_argument("--serve-budget-mb", type=int, default=96)
    ap.add_argument("--tuning", default=None,
                    help="path,replicas_per_block,threads,adjacency for the headline (default: autotune)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 256 MiB device copy first (byte-counter calibration)")
    return ap.parse_args()


# ---------------------------------------------------------------- oracle tallies
def oracle_tally(jobs, threads):
    """Sum of the oracle's per-attempt tallies over jobs (inst, S, R, seed,
    sched kwargs, replica range), run concurrently over `threads` host
    threads.  Returns the counts and the attempts they cover."""
    from oracle import oracle as O

    def one(job):
        inst, S, R, seed, kw, r0, r1 = job
        o = O.anneal(inst, S, R, seed, r_begin=r0, r_end=r1, n_threads=1, want_states=False,
                     want_tally=True, **kw)
        return {"attempts": inst.n * S * (r1 - r0), "blocks": int(o.draws.sum()),
                "tests": int(o.tests.sum()), "accepts": int(o.accepts.sum()),
                "touched": int(o.touched.sum()), "improvements": int(o.improvements.sum()),
                "improve_bytes": int(o.improvements.sum()) * inst.n,
                "degree_sum": 2 * inst.m, "n": inst.n}

    tot = {}
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for r in ex.map(one, jobs):
            for k, v in r.items():
                tot[k] = tot.get(k, 0) + v
    return tot


def per_attempt(t):
    a = float(t["attempts"])
    return {"blocks": t["blocks"] / a, "tests": t["tests"] / a, "flips": t["accepts"] / a,
            "touched": t["touched"] / a, "improve": t["improve_bytes"] / a,
            "mean_degree": t["degree_sum"] / float(t["n"])}


# ---------------------------------------------------------------- rooflines
def lds_bytes_per_attempt(form, pa, width=8):
    """LDS bytes a kernel form moves per attempt (its own reads and writes,
    from the access pattern of the source):
      msc4   per lane step of 32/W groups x W replicas (128 attempts): reads of
             4 own and 16 neighbour W-bit elements per group, writes of 4
             element pairs per group -> 112 bytes;
      deg4   FIELD degree-4 bond words: a group's 4 words, its 32-byte
             adjacency block and 4 threshold words per 4 attempts; per flip
             its word and 4 neighbour XORs (read and write);
      keys   FIELD key form with HBM adjacency: a group's 4 words, degree and
             base words and 4 thresholds per 4 attempts; per flip one word
             store and an atomic add (read and write) per neighbour;
      csr    the key form with its CSR adjacency staged in LDS: as keys, plus
             a 2-byte entry read per neighbour of a flip."""
    if form == "msc4":
        return 112.0 / 128.0
    if form == "deg4":
        return 64.0 / 4.0 + pa["flips"] * (4 + 4 * 8)
    if form == "csr":
        return 40.0 / 4.0 + pa["flips"] * (4 + 10 * pa["mean_degree"])
    return 40.0 / 4.0 + pa["flips"] * (4 + 8 * pa["mean_degree"])


def roofline(attempts, kernel_s, pa, form, lds_peak, profile=None):
    """ALU, HBM and LDS fractions of one launch of attempts in kernel_s."""
    ops = OPS_PER_BLOCK * pa["blocks"] + pa["tests"]
    achieved = ops * attempts / kernel_s
    hbm_b = 5.0 + pa["flips"] + 8.0 * pa["touched"] + pa["improve"]
    lds_b = lds_bytes_per_attempt(form, pa)
    out = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
           "unit": "T VALU lane-instructions/s", "frac": achieved / VALU_PEAK,
           "traffic": None,
           "alu_ops_per_attempt": ops,
           "per_attempt": {k: round(v, 6) for k, v in pa.items()},
           "kernel_ms": kernel_s * 1e3, "attempts": attempts,
           "hbm_algorithmic": {"bytes_per_attempt": hbm_b,
                               "achieved_GBps": hbm_b * attempts / kernel_s / 1e9,
                               "frac": hbm_b * attempts / kernel_s / HBM_PEAK_BPS},
           "lds": {"form": form, "bytes_per_attempt": lds_b,
                   "achieved_GBps": lds_b * attempts / kernel_s / 1e9,
                   "peak_GBps": lds_peak / 1e9, "peak_theory_GBps": LDS_PEAK_THEORY / 1e9,
                   "frac": lds_b * attempts / kernel_s / lds_peak}}
    if profile:
        traffic = profile_figure(profile, "HBM bytes per launch", int)
        out["traffic"] = traffic
        if traffic is not None:
            out["hbm_measured"] = {"bytes_per_launch": traffic, "GBps": traffic / kernel_s / 1e9,
                                   "frac": traffic / kernel_s / HBM_PEAK_BPS}
        vi = profile_figure(profile, "VALU instructions per attempt")
        if vi is not None:
            out["valu_instructions_per_attempt"] = vi
            out["valu_issue_frac"] = profile_figure(profile, "VALU issue fraction")
        la = profile_figure(profile, "LDS active fraction")
        if la is not None:
            out["lds"]["active_frac"] = la
            out["lds"]["bank_conflict_frac"] = profile_figure(profile, "LDS bank-conflict fraction")
    return out


def ttt_rows(per_replica, ref, wall_s, S, qs=(0.99, 0.995, 0.998, 1.0), **extra_walls):
    """Time to target at quality q of the reference: trial = replica."""
    from paper_2311_09275_amd import ttt
    rows = {}
    for q in qs:
        target = ttt.target_cut(ref, q)
        r = ttt.replica_ttt(per_replica, target, wall_s, S)
        row = {"target": target, "ps": r["ps"], "ttt_s": r["ttt_s"], "sweeps_to_target": r["sweeps_to_target"]}
        for name, w in extra_walls.items():
            row[f"ttt_{name}_s"] = ttt.replica_ttt(per_replica, target, w, S)["ttt_s"]
        rows[str(q)] = row
    return rows


# ---------------------------------------------------------------- main
def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_09275_amd import binding as B
    from paper_2311_09275_amd import instances as I
    from paper_2311_09275_amd import reference_cuts as RC
    from paper_2311_09275_amd import ttt

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    # a stream of its own: the library captures its launch sequences into
    # hipGraphs on streams other than the null stream
    stream = torch.cuda.Stream(device=dev)
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    log = lambda msg: print(msg, file=sys.stderr, flush=True)  # noqa: E731

    if args.calib_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    rates = B.ising_valu_rates()
    lds_peak = B.ising_lds_rate()
    refs = RC.load()
    above_reference = []

    # ------------------------------------------------------------ headline: 64-torus batch
    S, B0, B1 = SCHED_C4["S"], SCHED_C4["b0"], SCHED_C4["b1"]
    sched = B.Schedule.make(B.GEOMETRIC, S, B0, B1)
    insts = I.workload_c4()
    names = [f"batch{i:02d}_" + x.name for i, x in enumerate(insts)]
    probs = [B.Problem.from_instance(x) for x in insts]
    handles = [p.handle for p in probs]
    seeds = np.array([2000 + i for i in range(len(insts))], np.uint64)
    R = 128
    attempts = sum(x.n for x in insts) * R * S
    if args.tuning:
        tun = B.Tuning(*[int(v) for v in args.tuning.split(",")])
    else:
        tun = B.ising_autotune(handles, sched, R, prefix_sweeps=200, stream=stream)
    log(f"headline tuning: path {tun.path}, {tun.replicas_per_block} per block, "
        f"{tun.block_threads} threads, adjacency {tun.lds_adjacency}")

    def batch_once(tuning):
        B.ising_anneal_batch(handles, sched, R, seeds, tuning, stream=stream)
        return [B.ising_cut(h)[0] for h in handles]  # synchronises the stream

    for _ in range(args.warmup):
        batch_once(tun)
    torch.cuda.synchronize()
    kern = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cuts = batch_once(tun)
        kern.append(B.ising_last_batch_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = attempts * args.steps / wall
    kern_ms = float(np.mean(kern))
    per_b = [B.ising_cut(h, R)[2].copy() for h in handles]
    path_b = B.ising_last_run_info(handles[0])[2]
    log(f"headline {ms_per_step:.1f} ms/step, kernel {kern_ms:.1f} ms")

    # end to end, counting pre-processing as the paper's trial time does:
    # compile and upload all 64 problems, build their threshold tables,
    # anneal them in one batch and read the cuts back
    torch.cuda.synchronize()
    t = time.perf_counter()
    probs_e = [B.Problem.from_instance(x) for x in insts]
    create_s = time.perf_counter() - t
    B.ising_anneal_batch([q.handle for q in probs_e], sched, R, seeds, tun, stream=stream)
    cuts_e = [B.ising_cut(q.handle)[0] for q in probs_e]
    e2e_s = time.perf_counter() - t
    assert cuts_e == cuts, "end-to-end and resident batches disagree"
    for q in probs_e:
        q.close()
    end_to_end = {"create_ms": create_s * 1e3, "wall_ms": e2e_s * 1e3, "attempts_per_s": attempts / e2e_s,
                  "note": "ising_create of the 64 problems, threshold tables, one batched anneal and "
                          "the cuts read back, from host-side edge lists"}
    log(f"end to end {e2e_s * 1e3:.1f} ms (create {create_s * 1e3:.1f} ms)")

    def same(cs):
        return all(a == b for a, b in zip(cs, cuts))

    batch_forms = {"tuned": {"tuning": [int(tun.path), int(tun.replicas_per_block), int(tun.block_threads),
                                        int(tun.lds_adjacency)],
                             "ms_per_step": ms_per_step, "kernel_ms": kern_ms,
                             "kernel_ms_min": float(np.min(kern)), "kernel_ms_max": float(np.max(kern))}}
    # FIELD path's best batched form, same seeds
    field_tun = B.Tuning(B.PATH_FIELD, 1, 1024, 0)
    fw, fk = [], []
    for _ in range(3):
        t = time.perf_counter()
        c = batch_once(field_tun)
        fw.append(time.perf_counter() - t)
        fk.append(B.ising_last_batch_ms())
    assert same(c), "FIELD and tuned batches disagree"
    batch_forms["field_batched"] = {"tuning": [2, 1, 1024, 0], "wall_ms": float(np.mean(fw[1:]) * 1e3),
                                    "kernel_ms": float(np.mean(fk[1:]))}
    # the same anneals as separate persistent launches (tuned configuration)
    sep_s = None
    if not args.no_separate:
        walls = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for p, sd in zip(probs, seeds):
                p.anneal(sched, R, int(sd), tun, stream=stream)
            c = [p.cut().best_cut for p in probs]
            walls.append(time.perf_counter() - t)
        assert same(c), "separate and batched anneals disagree"
        sep_s = float(np.min(walls))
        batch_forms["separate_launches"] = {"wall_ms": sep_s * 1e3, "wall_ms_samples": [w * 1e3 for w in walls]}
        log(f"separate {sep_s * 1e3:.1f} ms")
    plain_s = None
    if not args.no_plain:
        t = time.perf_counter()
        c = batch_once(B.Tuning(B.PATH_PLAIN, 1, 256, 0))
        plain_s = time.perf_counter() - t
        assert same(c), "plain and batched forms disagree"
        batch_forms["plain"] = {"wall_ms": plain_s * 1e3}
        log(f"plain {plain_s:.1f} s")
    # time to target of every problem against its stored reference
    c4_ttt = None
    if all(n in refs for n in names):
        c4_ttt = {}
        for i, n in enumerate(names):
            if per_b[i].max() > refs[n]:
                above_reference.append({"instance": n, "reference": refs[n], "found": int(per_b[i].max())})
        for q in (0.99, 0.995, 0.998, 1.0):
            rows = [ttt.replica_ttt(per_b[i], ttt.target_cut(refs[n], q), wall / args.steps, S)
                    for i, n in enumerate(names)]
            hit = [r_ for r_ in rows if r_["ps"] > 0]
            med = float(np.median([r_["ttt_s"] for r_ in hit])) if hit else math.inf
            scale = lambda s_: None if s_ is None else med * s_ / (wall / args.steps)  # noqa: E731
            c4_ttt[str(q)] = {"problems_reached": len(hit), "median_ps": float(np.median([r_["ps"] for r_ in rows])),
                              "median_ttt_batched_s": med, "median_ttt_separate_s": scale(sep_s),
                              "median_ttt_plain_s": scale(plain_s)}

    # ------------------------------------------------------------ 100x80 torus
    c2 = None
    inst2 = I.workload_c2()
    R2, SEED2 = 256, 1002
    att2 = inst2.n * R2 * S
    if not args.no_c2:
        p2 = B.Problem.from_instance(inst2)

        def c2_run(tuning, steps, warm):
            for _ in range(warm):
                p2.anneal(sched, R2, SEED2, tuning, stream=stream)
                p2.cut()
            torch.cuda.synchronize()
            ws, ks = [], []
            for _ in range(steps):
                t = time.perf_counter()
                p2.anneal(sched, R2, SEED2, tuning, stream=stream)
                res = p2.cut()
                ws.append(time.perf_counter() - t)
                ks.append(p2.last_anneal_ms())
            return res, float(np.mean(ws)), float(np.mean(ks))

        res2, w2, k2 = c2_run(B.Tuning(B.PATH_FIELD, 1, 1024, 0), 5, 2)
        per2 = res2.per_replica.copy()
        c2 = {"workload": "torus 100x80 +-1 (N=8000, M=16000), 256 replicas, 4000 sweeps geometric 0.1->4.0",
              "field": {"ms_per_anneal": w2 * 1e3, "kernel_ms": k2, "attempts_per_s": att2 / w2},
              "best_cut": int(res2.best_cut)}
        best_m = None
        for w_, th in ((8, 256), (16, 256), (32, 256), (8, 512)):
            rm, wm, km = c2_run(B.Tuning(B.PATH_MSC, w_, th, 0), 2, 1)
            assert np.array_equal(rm.per_replica, per2), "multispin and field forms disagree"
            c2[f"multispin_w{w_}_b{th}"] = {"ms_per_anneal": wm * 1e3, "kernel_ms": km}
            if best_m is None or km < best_m[1]:
                best_m = (f"w{w_}_b{th}", km)
        c2["multispin_best"] = best_m[0]
        if not args.no_plain:
            rp, wp, kp = c2_run(B.Tuning(B.PATH_PLAIN, 1, 256, 0), 1, 0)
            assert np.array_equal(rp.per_replica, per2), "plain and persistent forms disagree"
            c2["plain"] = {"ms_per_anneal": wp * 1e3}
            c2["persistent_vs_plain_speedup"] = wp / w2
        ref2 = refs.get("torus100x80_s2")
        if ref2 is not None:
            if per2.max() > ref2:
                above_reference.append({"instance": "torus100x80_s2", "reference": ref2, "found": int(per2.max())})
            c2["reference_cut"] = ref2
            c2["ttt"] = ttt_rows(per2, ref2, w2, S, **({"plain": c2["plain"]["ms_per_anneal"] / 1e3}
                                                       if "plain" in c2 else {}))
        c2["_kernel_ms_msc"] = best_m[1]
        p2.close()
        log("c2 done")

    # ------------------------------------------------------------ sparse random graph
    c3 = None
    inst3 = I.workload_c3()
    R3, S3, SEED3 = 1024, 4000, 1003
    sched3 = B.Schedule.make(B.LINEAR, S3, 0.05, 3.0)
    att3 = inst3.n * R3 * S3
    if not args.no_random:
        p3 = B.Problem.from_instance(inst3)
        auto = B.Tuning(B.PATH_AUTO, 0, 0, 0)
        p3.anneal(sched3, R3, SEED3, auto, stream=stream)
        p3.cut()
        ws, ks = [], []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            p3.anneal(sched3, R3, SEED3, auto, stream=stream)
            res3 = p3.cut()
            ws.append(time.perf_counter() - t)
            ks.append(p3.last_anneal_ms())
        per3 = res3.per_replica.copy()
        w3, k3 = float(np.mean(ws)), float(np.mean(ks))
        c3 = {"workload": "sparse random graph N=10000 M=9999 w=1, 1024 replicas, 4000 sweeps linear 0.05->3.0",
              "ms_per_anneal": w3 * 1e3, "kernel_ms": k3, "attempts_per_s": att3 / w3,
              "best_cut": int(res3.best_cut), "path": B.ising_last_run_info(p3.handle)[2]}
        if not args.no_plain:
            t = time.perf_counter()
            p3.anneal(sched3, R3, SEED3, B.Tuning(B.PATH_PLAIN, 1, 256, 0), stream=stream)
            rp = p3.cut()
            wp = time.perf_counter() - t
            assert np.array_equal(rp.per_replica, per3), "plain and automatic forms disagree"
            c3["plain_ms"] = wp * 1e3
            c3["persistent_vs_plain_speedup"] = wp / w3
        ref3 = refs.get("random10000_9999_s3")
        if ref3 is not None:
            if per3.max() > ref3:
                above_reference.append({"instance": "random10000_9999_s3", "reference": ref3,
                                        "found": int(per3.max())})
            c3["reference_cut"] = ref3
            c3["ttt"] = ttt_rows(per3, ref3, w3, S3, **({"plain": c3["plain_ms"] / 1e3}
                                                         if "plain_ms" in c3 else {}))
        p3.close()
        log("c3 done")

    # ------------------------------------------------------------ local fields
    # The 100x80 torus with integer fields b in [-2, 2] on every vertex: the
    # field term enters the flip key, so the degree-4 bond-word forms do not
    # apply and the automatic configuration takes a key form.
    fields = None
    instf = I.with_fields(inst2, seed=2, bmax=2)
    attf = instf.n * R2 * S
    if not args.no_fields:
        pf = B.Problem.from_instance(instf)
        auto = B.Tuning(B.PATH_AUTO, 0, 0, 0)
        pf.anneal(sched, R2, SEED2, auto, stream=stream)
        pf.cut()
        ws, ks = [], []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            pf.anneal(sched, R2, SEED2, auto, stream=stream)
            resf = pf.cut()
            ws.append(time.perf_counter() - t)
            ks.append(pf.last_anneal_ms())
        perf_ = resf.per_replica.copy()
        wf, kf = float(np.mean(ws)), float(np.mean(ks))
        info_f = B.ising_last_run_info(pf.handle)
        fields = {"workload": "torus 100x80 +-1 with local fields b~U{-2..2} on every vertex, "
                              "256 replicas, 4000 sweeps geometric 0.1->4.0",
                  "ms_per_anneal": wf * 1e3, "kernel_ms": kf, "kernel_ms_samples": ks,
                  "attempts_per_s": attf / wf, "best_objective": int(resf.best_cut),
                  "path": info_f[2]}
        if not args.no_plain:
            t = time.perf_counter()
            pf.anneal(sched, R2, SEED2, B.Tuning(B.PATH_PLAIN, 1, 256, 0), stream=stream)
            rp = pf.cut()
            wp = time.perf_counter() - t
            assert np.array_equal(rp.per_replica, perf_), "plain and automatic forms disagree (fields)"
            fields["plain_ms"] = wp * 1e3
            fields["persistent_vs_plain_speedup"] = wp / wf
        pf.close()
        log("fields done")

    # ------------------------------------------------------------ parallel tempering
    temper = None
    if not args.no_temper:
        K, n_sets, P = 32, 8, 10
        ladder = list(np.geomspace(0.2, 3.0, K))
        pt_att = inst2.n * K * n_sets * S
        pt = B.Problem.from_instance(inst2)

        def temper_run(P_, tuning=None, cluster_from=None, reps=2):
            pt.temper(ladder, n_sets, S, P_, SEED2, tuning, stream=stream, cluster_from=cluster_from)
            pt.cut()
            ws = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                pt.temper(ladder, n_sets, S, P_, SEED2, tuning, stream=stream, cluster_from=cluster_from)
                r_ = pt.cut()
                ws.append(time.perf_counter() - t)
            return r_, float(np.mean(ws)) * 1e3, pt.last_anneal_ms()

        res_t, ms_t, k_t = temper_run(P)
        _, swaps_t = pt.temper_results()
        _, ms_100, k_100 = temper_run(100)
        res_c, ms_c, k_c = temper_run(P, cluster_from=K // 2)
        _, _, cm_c, cs_c = pt.temper_results()
        temper = {"workload": f"torus 100x80, {n_sets} sets x {K} temperatures geometric 0.2->3.0, "
                              f"{S} sweeps, exchange every {P}",
                  "attempts_per_s": pt_att / (ms_t / 1e3), "ms_per_run": ms_t, "kernel_ms": k_t,
                  "ms_per_run_exchange_every_100": ms_100, "kernel_ms_exchange_every_100": k_100,
                  "best_cut": int(res_t.best_cut),
                  "cluster_moves": {"ms_per_run": ms_c, "kernel_ms": k_c, "moves": int(cm_c.sum()),
                                    "mean_cluster_sites": float(cs_c.sum() / max(cm_c.sum(), 1)),
                                    "best_cut": int(res_c.best_cut)}}
        if not args.no_plain:
            t = time.perf_counter()
            pt.temper(ladder, n_sets, S, P, SEED2, B.Tuning(B.PATH_PLAIN, 1, 256, 0), stream=stream)
            r_p = pt.cut()
            temper["plain_ms"] = (time.perf_counter() - t) * 1e3
            assert np.array_equal(r_p.per_replica, res_t.per_replica), "plain and persistent tempering disagree"
        ref2 = refs.get("torus100x80_s2")
        if ref2 is not None:
            for key, res_, ms_ in (("ttt", res_t, ms_t), ("cluster_ttt", res_c, ms_c)):
                sets_best = res_.per_replica.reshape(n_sets, K).max(axis=1)
                if sets_best.max() > ref2:
                    above_reference.append({"instance": "torus100x80_s2 (tempering)", "reference": ref2,
                                            "found": int(sets_best.max())})
                temper[key] = {str(q): {"target": ttt.target_cut(ref2, q),
                                        "ps_sets": ttt.success_probability(sets_best, ttt.target_cut(ref2, q)),
                                        "ttt_s": ttt.replica_ttt(sets_best, ttt.target_cut(ref2, q), ms_ / 1e3,
                                                                 S)["ttt_s"]}
                               for q in (0.99, 0.995, 0.998, 1.0)}
        pt.close()
        log("tempering done")

    # ------------------------------------------------------------ serving
    serving = None
    if args.serve_requests > 0:
        from paper_2311_09275_amd import serve_load
        serving = serve_load.run(rate=50.0, n_requests=args.serve_requests,
                                 budget=args.serve_budget_mb << 20, stream=stream)
        log("serving done")

    # ------------------------------------------------------------ oracle: tallies and CPU baseline
    cpu = None
    rooflines = {}
    pa4 = pa2 = pa3 = paf = None
    if not args.no_cpu:
        from oracle import oracle as O
        O.build(force=False)
        geo = dict(kind=O.GEOMETRIC, beta0=B0, beta1=B1)
        # tallies: every 8th batch problem, four replicas each; the 100x80
        # torus and the random graph, sixteen replicas each
        pa4 = per_attempt(oracle_tally([(insts[i], S, R, int(seeds[i]), geo, 0, 4)
                                        for i in range(0, len(insts), 8)], threads))
        pa2 = per_attempt(oracle_tally([(inst2, S, R2, SEED2, geo, r, r + 1) for r in range(16)], threads))
        pa3 = per_attempt(oracle_tally([(inst3, S3, R3, SEED3, dict(kind=O.LINEAR, beta0=0.05, beta1=3.0),
                                         r, r + 1) for r in range(16)], threads))
        if fields is not None:
            paf = per_attempt(oracle_tally([(instf, S, R2, SEED2, geo, r, r + 1) for r in range(16)], threads))
        # CPU baseline: the oracle on replicas 0..7 of every batch problem
        jobs = [(i, r) for i in range(len(insts)) for r in range(8)]

        def run_one(job):
            i, r = job
            o = O.anneal(insts[i], S, R, int(seeds[i]), r_begin=r, r_end=r + 1, n_threads=1,
                         want_states=False, **geo)
            return i, r, int(o.best_cut[0])

        t = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            got = list(ex.map(run_one, jobs))
        cpu_s = time.perf_counter() - t
        for i, r, bc in got:
            assert bc == per_b[i][r], f"oracle and GPU disagree on problem {i} replica {r}"
        sample_att = sum(insts[i].n for i, _ in jobs) * S
        info = cpu_info()
        cpu = {"value": sample_att / cpu_s, "unit": UNIT, "cores": threads, "kind": "oracle",
               "sample": f"replicas 0..7 of each of the 64 batch problems, all {S} sweeps "
                         f"({sample_att:.3e} attempts), {threads} host threads, {cpu_s:.1f} s",
               "host": info,
               "cores_note": "threads used = this process's CPU share (the one-GPU share of the "
                             "measurement host, at most 16) of its affinity mask"}
        log("oracle done")

    # ------------------------------------------------------------ rooflines
    if pa4 is not None:
        form4 = "msc4" if path_b == 3 and tun.replicas_per_block >= 8 else "deg4"
        ktag = (f"k_msc4_b{tun.block_threads}_w{tun.replicas_per_block}" if form4 == "msc4"
                else f"k_field_b{tun.block_threads}")
        rooflines["c4_batch"] = roofline(attempts, kern_ms / 1e3, pa4, form4, lds_peak,
                                         f"{ktag}_batch64tori_r128_counters.md")
        rooflines["c4_batch"]["kernel"] = ktag
        rooflines["c4_field_batched"] = roofline(attempts, batch_forms["field_batched"]["kernel_ms"] / 1e3,
                                                 pa4, "deg4", lds_peak)
    if pa2 is not None and c2 is not None:
        rooflines["c2_field"] = roofline(att2, c2["field"]["kernel_ms"] / 1e3, pa2, "deg4", lds_peak,
                                         "k_field_torus100x80_r256_counters.md")
        rooflines["c2_multispin"] = roofline(att2, c2.pop("_kernel_ms_msc") / 1e3, pa2, "msc4", lds_peak)
    elif c2 is not None:
        c2.pop("_kernel_ms_msc", None)
    if pa3 is not None and c3 is not None:
        rooflines["c3"] = roofline(att3, c3["kernel_ms"] / 1e3, pa3, "keys", lds_peak,
                                   "k_field_random10000_r1024_counters.md")
    if paf is not None and fields is not None:
        rooflines["c2_fields"] = roofline(attf, fields["kernel_ms"] / 1e3, paf, "csr", lds_peak,
                                          "k_field_torus100x80_fields_r256_counters.md")
    roof = rooflines.get("c4_batch")
    if roof is not None:
        roof = dict(roof)
        roof["measured_rates"] = {**{k: v for k, v in rates.items()}, "lds_bytes_per_s": lds_peak}

    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "64 LxL +-1 toroidal spin glasses, L~U{32..141} (seed 100; torus i seed "
                               "101+i), 128 replicas each, 4000 sweeps geometric beta 0.1->4.0, one "
                               "persistent launch per step (hipGraph), autotuned",
                   "problems": len(insts), "vertices": int(sum(x.n for x in insts)), "replicas": R,
                   "sweeps": S, "attempts_per_step": attempts,
                   "path": {1: "plain", 2: "field", 3: "msc"}.get(path_b, str(path_b)),
                   "replicas_per_block": int(tun.replicas_per_block),
                   "block_threads": int(tun.block_threads)},
        "kernel_ms": kern_ms,
        "end_to_end": end_to_end,
        "batched_vs_plain_speedup": None if plain_s is None else plain_s / (wall / args.steps),
        "batched_vs_separate_speedup": None if sep_s is None else sep_s / (wall / args.steps),
        "batch_forms": batch_forms,
        "ttt": c4_ttt,
        "above_reference": above_reference,
        "torus100x80": c2,
        "random_graph": c3,
        "local_fields": fields,
        "tempering": temper,
        "serving": serving,
        "rooflines": rooflines,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    for p in probs:
        p.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
