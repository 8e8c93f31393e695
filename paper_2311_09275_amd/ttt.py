"""Time-to-target and related metrics (paper Sec. II.B, Eq. 1-2; Sec. III.A).

r   = max(1, log(1 - 0.99) / log(1 - P_s))      (Eq. 1)
TTT = t_trial * r                              (Eq. 2)
sweeps-to-target = sweeps per run * r          (Sec. III.A)
quality = value / best-known value             (Sec. II.B)

Edge cases: P_s = 0 gives r = infinity; P_s = 1 gives r = 1.
For a many-replica anneal, one replica is one trial, P_s is the fraction of
replicas whose best cut reaches the target, and t_trial is the wall time of
the whole anneal divided by the number of replicas (the paper measures
elapsed time over the outer loop of trials and divides, Sec. III.A).
"""
from __future__ import annotations

import math

import numpy as np


def repetitions(ps: float, confidence: float = 0.99) -> float:
    """Eq. 1: repetitions needed for success with the given confidence."""
    if not 0.0 <= ps <= 1.0:
        raise ValueError("P_s must lie in [0, 1]")
    if ps == 0.0:
        return math.inf
    if ps == 1.0:
        return 1.0
    return max(1.0, math.log(1.0 - confidence) / math.log(1.0 - ps))


def time_to_target(t_trial: float, ps: float) -> float:
    """Eq. 2."""
    r = repetitions(ps)
    return math.inf if math.isinf(r) else t_trial * r


def sweeps_to_target(sweeps_per_run: float, ps: float) -> float:
    r = repetitions(ps)
    return math.inf if math.isinf(r) else sweeps_per_run * r


def quality(value: float, best: float) -> float:
    return value / best


def success_probability(best_cuts, target: int) -> float:
    a = np.asarray(best_cuts)
    return float(np.count_nonzero(a >= target)) / float(a.size)


def target_cut(reference_best: int, q: float) -> int:
    """Target value at quality q of a reference best cut (rounded up)."""
    return int(math.ceil(q * reference_best - 1e-9))


def replica_ttt(best_cuts, target: int, wall_s: float, sweeps: int) -> dict:
    """TTT of a many-replica anneal: trial = replica, t_trial = wall / R."""
    r_count = len(best_cuts)
    ps = success_probability(best_cuts, target)
    t_trial = wall_s / r_count
    return {"target": int(target), "ps": ps, "t_trial_s": t_trial,
            "ttt_s": time_to_target(t_trial, ps),
            "sweeps_to_target": sweeps_to_target(sweeps, ps)}
