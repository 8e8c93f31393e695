"""Seeded synthetic problem instances (numpy only).

This module is the one piece shared by the HIP path, the oracle and the
benchmark: it only produces inputs (edge lists, initial states, arrival
times) and holds none of the annealing arithmetic.

The paper benchmarks on the seven largest Gset MaxCut instances (Sec. II.A,
Table I): six toroidal square-grid spin glasses with random +-1 weights
(2D Edwards-Anderson, M = 2N) and one sparse random unweighted graph
(G70: N = 10,000, M = 9,999).  Those files are not available here, so these
generators build stand-ins of the same shape and structure from a seed.

All instances are MaxCut weight lists (u, v, w) with 0-based vertex ids; the
Ising couplings are J = -w (the MaxCut <-> Ising sign reading used
throughout this package).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Instance:
    """An undirected weighted graph given as an edge list."""

    name: str
    n: int
    u: np.ndarray  # int32 [m]
    v: np.ndarray  # int32 [m]
    w: np.ndarray  # int32 [m]
    field: np.ndarray | None = None  # int32 [n] local fields b, or None

    @property
    def m(self) -> int:
        return int(self.u.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def torus(lx: int, ly: int, seed: int, weights: str = "pm1") -> Instance:
    """Toroidal square grid lx * ly (Sec. II.A, Table I: G65..G81 shape).

    Vertex id v = y*lx + x (x is the fast index).  Edges are listed for v in
    ascending order as (v, right neighbour), (v, down neighbour), so M = 2N.
    ``weights``: "pm1" = uniform +-1 from ``seed``; "one" = all +1.
    Both sides must be >= 3 so that no edge is listed twice.
    """
    if lx < 3 or ly < 3:
        raise ValueError("torus sides must be >= 3")
    n = lx * ly
    vid = np.arange(n, dtype=np.int64)
    x = vid % lx
    y = vid // lx
    right = y * lx + (x + 1) % lx
    down = ((y + 1) % ly) * lx + x
    u = np.repeat(vid, 2)
    v = np.empty(2 * n, dtype=np.int64)
    v[0::2] = right
    v[1::2] = down
    if weights == "pm1":
        w = _rng(seed).integers(0, 2, size=2 * n, dtype=np.int64) * 2 - 1
    elif weights == "one":
        w = np.ones(2 * n, dtype=np.int64)
    else:
        raise ValueError(weights)
    return Instance(f"torus{lx}x{ly}_s{seed}", n, u.astype(np.int32),
                    v.astype(np.int32), w.astype(np.int32))


def random_graph(n: int, m: int, seed: int, weight: int = 1) -> Instance:
    """Sparse random graph with m distinct edges, no self loops (G70 shape).

    Pairs (i, j) are drawn uniformly; a self loop or an already-present
    undirected pair is rejected and redrawn.  Draw order is kept.
    """
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    rng = _rng(seed)
    seen: set[tuple[int, int]] = set()
    us: list[int] = []
    vs: list[int] = []
    while len(us) < m:
        need = m - len(us)
        cand = rng.integers(0, n, size=(max(2 * need, 16), 2), dtype=np.int64)
        for a, b in cand:
            a = int(a)
            b = int(b)
            if a == b:
                continue
            key = (a, b) if a < b else (b, a)
            if key in seen:
                continue
            seen.add(key)
            us.append(a)
            vs.append(b)
            if len(us) == m:
                break
    w = np.full(m, weight, dtype=np.int32)
    return Instance(f"random{n}_{m}_s{seed}", n, np.asarray(us, np.int32),
                    np.asarray(vs, np.int32), w)


def random_regular4(n: int, seed: int, weights: str = "pm1") -> Instance:
    """Simple random 4-regular graph on n >= 5 vertices, +-1 (or all +1)
    weights.  Pairing model: the 4n vertex stubs are shuffled and paired;
    a pairing with a self loop or a repeated pair is drawn again.  Edges
    are listed as (min, max) in ascending order, so the listing itself is
    in general no orientation with two out-edges per vertex."""
    if n < 5:
        raise ValueError("a simple 4-regular graph needs n >= 5")
    rng = _rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), 4)
    for _ in range(10000):
        rng.shuffle(stubs)
        a, b = stubs[0::2], stubs[1::2]
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        if np.any(lo == hi):
            continue
        key = lo * n + hi
        if np.unique(key).size != key.size:
            continue
        order = np.argsort(key)
        lo, hi = lo[order], hi[order]
        if weights == "pm1":
            w = rng.integers(0, 2, size=lo.size, dtype=np.int64) * 2 - 1
        else:
            w = np.ones(lo.size, dtype=np.int64)
        return Instance(f"regular4_{n}_s{seed}", n, lo.astype(np.int32), hi.astype(np.int32),
                        w.astype(np.int32))
    raise RuntimeError("no simple pairing found")


def random_weighted(n: int, m: int, seed: int, wmax: int) -> Instance:
    """Random graph with nonzero integer weights uniform in [-wmax, wmax]."""
    base = random_graph(n, m, seed)
    rng = _rng(seed + 0x5EED)
    mag = rng.integers(1, wmax + 1, size=m)
    sign = rng.integers(0, 2, size=m) * 2 - 1
    return Instance(f"rw{n}_{m}_{wmax}_s{seed}", n, base.u, base.v,
                    (mag * sign).astype(np.int32))


def gauge(seed: int, n: int) -> np.ndarray:
    """A random +-1 gauge vector g (int8)."""
    return (_rng(seed).integers(0, 2, size=n) * 2 - 1).astype(np.int8)


def gauge_transform(inst: Instance, g: np.ndarray) -> Instance:
    """w'_ij = g_i g_j w_ij: the same energy landscape under s -> g*s."""
    g = g.astype(np.int32)
    w2 = (g[inst.u] * g[inst.v] * inst.w).astype(np.int32)
    return Instance(inst.name + "_gauged", inst.n, inst.u, inst.v, w2)


def planted(inst: Instance, g: np.ndarray) -> Instance:
    """Replace the weights by w_ij = -g_i g_j on the same graph.

    Every bond is then satisfied by s = +-g, so the maximum cut is known
    exactly: (W + M) / 2 with W = sum(w).
    """
    g = g.astype(np.int32)
    w2 = (-g[inst.u] * g[inst.v]).astype(np.int32)
    return Instance(inst.name + "_planted", inst.n, inst.u, inst.v, w2)


def random_spins(seed: int, r: int, n: int) -> np.ndarray:
    """int8 +-1 array [r][n] (initial states supplied by the caller)."""
    return (_rng(seed).integers(0, 2, size=(r, n)) * 2 - 1).astype(np.int8)


def torus_batch_sides(count: int, seed: int, lo: int = 32, hi: int = 141) -> list[int]:
    """Side lengths L ~ U{lo..hi} for a batch of L x L tori."""
    return [int(x) for x in _rng(seed).integers(lo, hi + 1, size=count)]


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    gaps = _rng(seed).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)


# Named workloads (the shapes of the paper's Table I instances and the
# configurations measured by the benchmark).
def workload_c1() -> Instance:
    return torus(16, 16, seed=1)


def workload_c2() -> Instance:
    return torus(100, 80, seed=2)


def workload_c3() -> Instance:
    return random_graph(10000, 9999, seed=3)


def workload_c4(count: int = 64) -> list[Instance]:
    sides = torus_batch_sides(count, seed=100)
    return [torus(L, L, seed=100 + i + 1) for i, L in enumerate(sides)]


def with_fields(inst: Instance, seed: int, bmax: int, density: float = 1.0) -> Instance:
    """inst with integer local fields b uniform in [-bmax, bmax] on a
    `density` fraction of the vertices (zero elsewhere)."""
    rng = _rng(seed + 0xF1E1D)
    b = rng.integers(-bmax, bmax + 1, size=inst.n)
    b[rng.random(inst.n) >= density] = 0
    return Instance(inst.name + f"_b{bmax}", inst.n, inst.u, inst.v, inst.w, b.astype(np.int32))
