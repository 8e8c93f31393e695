"""Gset ingestion and solution bitstrings (paper Sec. II.A, App. II-III).

Gset text format: a first line "n m", then m lines "i j w" with 1-based
vertex ids and integer MaxCut weights.  Solutions are printed in the paper
as hexadecimal strings: expanded to binary (most significant bit of each
digit first) they give the values of variables 1..n from left to right;
whitespace is ignored, and the bits past n in the last digit are zero.
A binary value x maps to the spin s = 2x - 1; the cut is the same for s and
-s.

    python -m paper_2311_09275_amd.gset solve GRAPH.txt --sweeps 4000 --replicas 256 \\
        --beta0 0.1 --beta1 4.0 --target 14030 [--hex-out best.txt]
    python -m paper_2311_09275_amd.gset solve GRAPH.txt --temps 32 --sets 8 --swap-every 10 \\
        --beta0 0.2 --beta1 3.0 [--cluster-from 16]   (parallel tempering, geometric ladder)
    python -m paper_2311_09275_amd.gset verify GRAPH.txt SOLUTION_HEX.txt

`solve` anneals (or, with --temps, runs parallel tempering) on the GPU
through the C ABI and reports the best cut, the success probability of the
target and the time to target (Eq. 1-2; one replica per trial, one set per
trial for tempering); `verify` evaluates a bitstring's cut on the host.
"""
from __future__ import annotations

import argparse
import io
import json
import os
import sys
import time

import numpy as np

from .instances import Instance


def read_gset(src, name: str | None = None) -> Instance:
    """Parse a Gset file (a path, or a text stream)."""
    if isinstance(src, (str, os.PathLike)):
        with open(src) as f:
            text = f.read()
        name = name or os.path.basename(str(src))
    else:
        text = src.read()
    rows = [l.split() for l in text.splitlines() if l.strip() and not l.lstrip().startswith("#")]
    if not rows or len(rows[0]) != 2:
        raise ValueError("the first line must be 'n m'")
    n, m = int(rows[0][0]), int(rows[0][1])
    if n <= 0 or m < 0:
        raise ValueError("bad header")
    body = rows[1:]
    if len(body) != m:
        raise ValueError(f"header says {m} edges, file has {len(body)}")
    a = np.array([[int(x) for x in r] for r in body], dtype=np.int64).reshape(m, -1) if m else \
        np.zeros((0, 3), np.int64)
    if a.shape[1] != 3:
        raise ValueError("edge lines must be 'i j w'")
    if m and (a[:, :2].min() < 1 or a[:, :2].max() > n):
        raise ValueError("vertex id outside 1..n")
    return Instance(name or "gset", n, (a[:, 0] - 1).astype(np.int32), (a[:, 1] - 1).astype(np.int32),
                    a[:, 2].astype(np.int32))


def write_gset(inst: Instance, dst) -> None:
    """Write inst in Gset format (1-based ids) to a path or a text stream."""
    out = io.StringIO()
    out.write(f"{inst.n} {inst.m}\n")
    for i, j, w in zip(inst.u, inst.v, inst.w):
        out.write(f"{int(i) + 1} {int(j) + 1} {int(w)}\n")
    if isinstance(dst, (str, os.PathLike)):
        with open(dst, "w") as f:
            f.write(out.getvalue())
    else:
        dst.write(out.getvalue())


def bits_from_hex(text: str, n: int) -> np.ndarray:
    """Binary values of variables 1..n (uint8 [n]) from a hexadecimal string."""
    digits = "".join(text.split())
    if len(digits) != (n + 3) // 4:
        raise ValueError(f"{len(digits)} hex digits for {n} variables (need {(n + 3) // 4})")
    try:
        vals = np.array([int(c, 16) for c in digits], dtype=np.uint8)
    except ValueError:
        raise ValueError("not a hexadecimal string") from None
    bits = ((vals[:, None] >> np.array([3, 2, 1, 0], np.uint8)) & 1).reshape(-1)
    if bits[n:].any():
        raise ValueError("bits past the last variable must be zero")
    return bits[:n].astype(np.uint8)


def hex_from_bits(bits) -> str:
    """Hexadecimal string of binary values (variables 1..n left to right)."""
    b = np.asarray(bits, dtype=np.uint8)
    pad = (-b.size) % 4
    b = np.concatenate([b, np.zeros(pad, np.uint8)]).reshape(-1, 4)
    vals = (b[:, 0] << 3) | (b[:, 1] << 2) | (b[:, 2] << 1) | b[:, 3]
    return "".join("0123456789ABCDEF"[v] for v in vals)


def spins_from_bits(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.int8) * 2 - 1).astype(np.int8)


def bits_from_spins(spins) -> np.ndarray:
    return (np.asarray(spins) > 0).astype(np.uint8)


def cut_value(inst: Instance, bits) -> int:
    """Weighted MaxCut objective of binary values: the sum of w over edges
    whose ends differ."""
    b = np.asarray(bits)
    return int(inst.w[b[inst.u] != b[inst.v]].astype(np.int64).sum())


def _solve(args) -> int:
    import torch

    from . import binding as B
    from . import ttt

    inst = read_gset(args.graph)
    stream = torch.cuda.current_stream()
    sched = B.Schedule.make(B.GEOMETRIC if args.geometric else B.LINEAR, args.sweeps, args.beta0,
                            args.beta1)
    t = time.perf_counter()  # the paper's t_trial counts pre-processing (Sec. III.A)
    p = B.Problem.from_instance(inst)
    if args.temps:
        ladder = np.geomspace(args.beta0, args.beta1, args.temps) if args.temps > 1 else [args.beta1]
        p.temper(list(ladder), args.sets, args.sweeps, args.swap_every, args.seed, stream=stream,
                 cluster_from=args.cluster_from)
    else:
        p.anneal(sched, args.replicas, args.seed, stream=stream)
    res = p.cut()
    wall = time.perf_counter() - t
    spins = p.best_state()
    p.close()
    bits = bits_from_spins(spins)
    assert cut_value(inst, bits) == res.best_cut
    out = {"graph": inst.name, "n": inst.n, "m": inst.m, "best_cut": int(res.best_cut),
           "replicas": int(res.per_replica.size), "sweeps": args.sweeps, "wall_s": wall}
    if args.target is not None:
        trials = res.per_replica.reshape(args.sets, args.temps).max(axis=1) if args.temps \
            else res.per_replica
        out.update(ttt.replica_ttt(trials, args.target, wall, args.sweeps))
    if args.hex_out:
        with open(args.hex_out, "w") as f:
            f.write(hex_from_bits(bits) + "\n")
    print(json.dumps(out))
    return 0


def _verify(args) -> int:
    inst = read_gset(args.graph)
    with open(args.solution) as f:
        text = "".join(l for l in f if not l.lstrip().startswith("#"))
    print(cut_value(inst, bits_from_hex(text, inst.n)))
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2311_09275_amd.gset")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("solve", help="anneal a Gset graph on the GPU")
    s.add_argument("graph")
    s.add_argument("--sweeps", type=int, default=4000)
    s.add_argument("--replicas", type=int, default=256)
    s.add_argument("--beta0", type=float, default=0.1)
    s.add_argument("--beta1", type=float, default=4.0)
    s.add_argument("--geometric", action="store_true", help="geometric schedule (default linear)")
    s.add_argument("--seed", type=int, default=1)
    s.add_argument("--target", type=int, default=None)
    s.add_argument("--hex-out", default=None)
    s.add_argument("--temps", type=int, default=0, help="parallel tempering: temperatures per set")
    s.add_argument("--sets", type=int, default=8)
    s.add_argument("--swap-every", type=int, default=10)
    s.add_argument("--cluster-from", type=int, default=None,
                   help="Houdayer cluster moves at temperatures >= this index")
    v = sub.add_parser("verify", help="cut of a hexadecimal solution string")
    v.add_argument("graph")
    v.add_argument("solution")
    args = ap.parse_args(argv)
    return _solve(args) if args.cmd == "solve" else _verify(args)


if __name__ == "__main__":
    sys.exit(main())
