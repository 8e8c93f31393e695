"""ctypes wrapper of the plain C oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path (the HIP library and
its Python binding) never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ising_oracle.c")
# ISING_ORACLE_LIB names another build of ising_oracle.c (the sanitizer run)
LIB = os.environ.get("ISING_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

LINEAR, GEOMETRIC, EXPLICIT = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 into oracle/liboracle.so."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-ffp-contract=off", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _GraphIn(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int64), ("u", C.c_void_p),
                ("v", C.c_void_p), ("w", C.c_void_p), ("colour", C.c_void_p),
                ("field", C.c_void_p)]


class _RunIn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_sweeps", C.c_int32),
                ("beta0", C.c_double), ("beta1", C.c_double),
                ("betas", C.c_void_p), ("n_replicas", C.c_int32),
                ("seed", C.c_uint64), ("init_spins", C.c_void_p),
                ("r_begin", C.c_int32), ("r_end", C.c_int32),
                ("n_threads", C.c_int32), ("check_every_sweep", C.c_int32),
                ("shuffle_seed", C.c_uint64)]


class _TemperIn(C.Structure):
    _fields_ = [("n_temps", C.c_int32), ("betas", C.c_void_p), ("n_sets", C.c_int32),
                ("n_sweeps", C.c_int32), ("swap_every", C.c_int32), ("seed", C.c_uint64),
                ("init_spins", C.c_void_p), ("n_threads", C.c_int32),
                ("set_begin", C.c_int32), ("set_end", C.c_int32),
                ("cluster_moves", C.c_int32), ("cluster_from", C.c_int32)]


class _TemperOut(C.Structure):
    _fields_ = [("best_cut", C.c_void_p), ("best_sweep", C.c_void_p),
                ("accepts", C.c_void_p), ("final_energy", C.c_void_p),
                ("final_temp", C.c_void_p), ("swaps", C.c_void_p),
                ("best_state", C.c_void_p), ("final_state", C.c_void_p),
                ("temp_energy", C.c_void_p), ("cluster_moves", C.c_void_p),
                ("cluster_sites", C.c_void_p), ("check_failures", C.c_int64)]


class _RunOut(C.Structure):
    _fields_ = [("best_cut", C.c_void_p), ("best_sweep", C.c_void_p),
                ("accepts", C.c_void_p), ("final_energy", C.c_void_p),
                ("best_state", C.c_void_p), ("final_state", C.c_void_p),
                ("final_field", C.c_void_p), ("energy_trace", C.c_void_p),
                ("check_failures", C.c_int64), ("draws", C.c_void_p),
                ("improvements", C.c_void_p), ("tests", C.c_void_p),
                ("touched", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.oracle_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_schedule.argtypes = [C.c_int32, C.c_int32, C.c_double,
                                      C.c_double, C.c_void_p, C.c_void_p]
        L.oracle_threshold.argtypes = [C.c_double, C.c_int64]
        L.oracle_threshold.restype = C.c_uint64
        L.oracle_colouring.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_colouring.restype = C.c_int32
        L.oracle_cut.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]
        L.oracle_cut.restype = C.c_int64
        L.oracle_validate.argtypes = [C.c_void_p]
        L.oracle_anneal.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_temper.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_cluster.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
        L.oracle_cluster.restype = C.c_int64
        L.oracle_stream_map.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_draws.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32,
                                   C.c_uint32, C.c_void_p]
        L.oracle_swap_accept.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                         C.c_int64, C.c_int64, C.c_double, C.c_double]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def schedule(kind, n_sweeps, beta0=0.0, beta1=0.0, betas=None) -> np.ndarray:
    b = None if betas is None else np.ascontiguousarray(betas, np.float64)
    out = np.zeros(max(n_sweeps, 1), np.float64)
    rc = lib().oracle_schedule(kind, n_sweeps, beta0, beta1, _p(b), _p(out))
    if rc != 0:
        raise ValueError("invalid schedule")
    return out[:n_sweeps]


def threshold(beta: float, k: int) -> int:
    return int(lib().oracle_threshold(float(beta), int(k)))


def colouring(n, u, v) -> tuple[int, np.ndarray]:
    u = np.ascontiguousarray(u, np.int32)
    v = np.ascontiguousarray(v, np.int32)
    col = np.zeros(n, np.int32)
    C_ = lib().oracle_colouring(n, u.shape[0], _p(u), _p(v), _p(col))
    if C_ < 0:
        raise ValueError("invalid graph")
    return int(C_), col


def cut(inst, spins) -> int:
    s = np.ascontiguousarray(spins, np.int8)
    return int(lib().oracle_cut(inst.n, inst.m, _p(inst.u), _p(inst.v), _p(inst.w), _p(s)))


def _graph(inst, colour=None):
    """The graph of an instance; its local fields (``inst.field``, when the
    instance has that attribute and it is not None) go along."""
    u = np.ascontiguousarray(inst.u, np.int32)
    v = np.ascontiguousarray(inst.v, np.int32)
    w = np.ascontiguousarray(inst.w, np.int32)
    col = None if colour is None else np.ascontiguousarray(colour, np.int32)
    f = getattr(inst, "field", None)
    f = None if f is None else np.ascontiguousarray(f, np.int32)
    g = _GraphIn(inst.n, inst.m, _p(u), _p(v), _p(w), _p(col), _p(f))
    return g, (u, v, w, col, f)


def stream_map(inst, colour=None) -> tuple[np.ndarray, np.ndarray]:
    """(run, rank) of every vertex: its draws are word rank[v] of the
    Philox block with counter (t, run[v], r, tag)."""
    g, keep = _graph(inst, colour)
    run = np.zeros(inst.n, np.int32)
    rank = np.zeros(inst.n, np.int32)
    if lib().oracle_stream_map(C.byref(g), _p(run), _p(rank)) != 0:
        raise ValueError("invalid graph")
    return run, rank


def draws(inst, seed, t, r, tag, colour=None) -> np.ndarray:
    """The u32 draw of every vertex for sweep t, replica r, purpose tag."""
    g, keep = _graph(inst, colour)
    out = np.zeros(inst.n, np.uint32)
    if lib().oracle_draws(C.byref(g), int(seed) & 0xFFFFFFFFFFFFFFFF, int(t), int(r), int(tag),
                          _p(out)) != 0:
        raise ValueError("invalid graph")
    return out


def validate(inst, colour=None) -> bool:
    g, keep = _graph(inst, colour)
    return lib().oracle_validate(C.byref(g)) == 0


@dataclass
class Result:
    best_cut: np.ndarray      # int64 [nr]
    best_sweep: np.ndarray    # int32 [nr]
    accepts: np.ndarray       # int64 [nr]
    final_energy: np.ndarray  # int64 [nr]
    best_state: np.ndarray | None
    final_state: np.ndarray | None
    final_field: np.ndarray | None
    energy_trace: np.ndarray | None
    check_failures: int
    r_begin: int
    draws: np.ndarray         # int64 [nr] Philox blocks needed by the sweeps
    improvements: np.ndarray  # int64 [nr] sweeps that raised the best cut
    tests: np.ndarray | None = None    # int64 [nr] attempts a draw decided
    touched: np.ndarray | None = None  # int64 [nr] distinct fields changed per pass, summed

    def argmax(self) -> int:
        """Replica with the largest best cut, lowest index on ties."""
        return int(np.argmax(self.best_cut)) + self.r_begin


def anneal(inst, n_sweeps, n_replicas, seed, kind=LINEAR, beta0=0.1,
           beta1=3.0, betas=None, colour=None, init_spins=None,
           r_begin=0, r_end=None, n_threads=1, check=False,
           shuffle_seed=0, want_states=True, want_trace=False,
           want_field=False, want_tally=False) -> Result:
    """The anneal of replicas [r_begin, r_end).  want_tally adds the
    measurement tallies (attempts decided by a draw, distinct fields
    changed per colour pass); they do not change the run."""
    r_end = n_replicas if r_end is None else r_end
    nr = r_end - r_begin
    n = inst.n
    g, keep = _graph(inst, colour)
    b = None if betas is None else np.ascontiguousarray(betas, np.float64)
    init = None if init_spins is None else np.ascontiguousarray(init_spins, np.int8)
    run = _RunIn(kind, n_sweeps, float(beta0), float(beta1), _p(b), n_replicas,
                 int(seed) & 0xFFFFFFFFFFFFFFFF, _p(init), r_begin, r_end,
                 n_threads, 1 if check else 0, int(shuffle_seed))
    best_cut = np.zeros(nr, np.int64)
    best_sweep = np.zeros(nr, np.int32)
    accepts = np.zeros(nr, np.int64)
    energy = np.zeros(nr, np.int64)
    best_state = np.zeros((nr, n), np.int8) if want_states else None
    final_state = np.zeros((nr, n), np.int8) if want_states else None
    final_field = np.zeros((nr, n), np.int32) if want_field else None
    trace = np.zeros((nr, n_sweeps), np.int64) if want_trace else None
    draws = np.zeros(nr, np.int64)
    impr = np.zeros(nr, np.int64)
    tests = np.zeros(nr, np.int64) if want_tally else None
    touched = np.zeros(nr, np.int64) if want_tally else None
    out = _RunOut(_p(best_cut), _p(best_sweep), _p(accepts), _p(energy),
                  _p(best_state), _p(final_state), _p(final_field), _p(trace), 0,
                  _p(draws), _p(impr), _p(tests), _p(touched))
    rc = lib().oracle_anneal(C.byref(g), C.byref(run), C.byref(out))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return Result(best_cut, best_sweep, accepts, energy, best_state,
                  final_state, final_field, trace, int(out.check_failures),
                  r_begin, draws, impr, tests, touched)


@dataclass
class TemperResult:
    best_cut: np.ndarray      # int64 [R]
    best_sweep: np.ndarray    # int32 [R]
    accepts: np.ndarray       # int64 [R]
    final_energy: np.ndarray  # int64 [R]
    final_temp: np.ndarray    # int32 [R] temperature index at the end
    swaps: np.ndarray         # int64 [n_sets, K-1] accepted exchanges
    best_state: np.ndarray | None
    final_state: np.ndarray | None
    temp_energy: np.ndarray | None  # int64 [n_sets, S, K]
    cluster_moves: np.ndarray | None  # int64 [n_sets // 2, K]
    cluster_sites: np.ndarray | None  # int64 [n_sets // 2, K]
    check_failures: int = 0           # cluster moves that changed E_a + E_b

    def argmax(self) -> int:
        return int(np.argmax(self.best_cut))


def temper(inst, betas, n_sets, n_sweeps, swap_every, seed, colour=None,
           init_spins=None, n_threads=1, want_states=True,
           want_temp_energy=False, sets=None, cluster_from=None) -> TemperResult:
    """Parallel tempering over the ladder ``betas`` (see oracle_temper).
    ``sets`` = (begin, end) simulates only those sets (the others' entries
    stay zero).  ``cluster_from`` = k enables Houdayer cluster moves at
    temperatures k and above."""
    b = np.ascontiguousarray(betas, np.float64)
    K = int(b.shape[0])
    R = K * n_sets
    n = inst.n
    g, keep = _graph(inst, colour)
    init = None if init_spins is None else np.ascontiguousarray(init_spins, np.int8)
    cm = cluster_from is not None
    pin = _TemperIn(K, _p(b), n_sets, n_sweeps, swap_every,
                    int(seed) & 0xFFFFFFFFFFFFFFFF, _p(init), n_threads,
                    *((0, 0) if sets is None else sets), 1 if cm else 0,
                    int(cluster_from) if cm else 0)
    best_cut = np.zeros(R, np.int64)
    best_sweep = np.zeros(R, np.int32)
    accepts = np.zeros(R, np.int64)
    energy = np.zeros(R, np.int64)
    temp = np.zeros(R, np.int32)
    swaps = np.zeros((n_sets, max(K - 1, 1)), np.int64)
    best_state = np.zeros((R, n), np.int8) if want_states else None
    final_state = np.zeros((R, n), np.int8) if want_states else None
    te = np.zeros((n_sets, n_sweeps, K), np.int64) if want_temp_energy else None
    cmoves = np.zeros((max(n_sets // 2, 1), K), np.int64) if cm else None
    csites = np.zeros((max(n_sets // 2, 1), K), np.int64) if cm else None
    out = _TemperOut(_p(best_cut), _p(best_sweep), _p(accepts), _p(energy), _p(temp),
                     _p(swaps), _p(best_state), _p(final_state), _p(te), _p(cmoves), _p(csites), 0)
    rc = lib().oracle_temper(C.byref(g), C.byref(pin), C.byref(out))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return TemperResult(best_cut, best_sweep, accepts, energy, temp,
                        swaps[:, :K - 1], best_state, final_state, te,
                        None if cmoves is None else cmoves[:n_sets // 2],
                        None if csites is None else csites[:n_sets // 2], int(out.check_failures))


def cluster(inst, sa, sb, i0):
    """Houdayer cluster of seed i0 between states sa and sb: a uint8 mask."""
    g, keep = _graph(inst)
    a = np.ascontiguousarray(sa, np.int8)
    b = np.ascontiguousarray(sb, np.int8)
    mask = np.zeros(inst.n, np.uint8)
    size = lib().oracle_cluster(C.byref(g), _p(a), _p(b), int(i0), _p(mask))
    if size < 0:
        raise ValueError("invalid input")
    assert size == int(mask.sum())
    return mask


def swap_accept(seed, m, k, set_, Ea, Eb, beta_k, beta_k1) -> bool:
    return bool(lib().oracle_swap_accept(int(seed) & 0xFFFFFFFFFFFFFFFF, m, k, set_,
                                         int(Ea), int(Eb), float(beta_k), float(beta_k1)))
