"""ctypes binding of libising (include/ising.h): argument marshalling only.

Every function named ``ising_*`` here calls the C function of the same name;
all computation happens in the HIP library.  PyTorch is used only to hand a
HIP stream to the library (``stream=`` accepts a ``torch.cuda.Stream``, a raw
handle, or ``None`` for the null stream).  Importing this module raises when
the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ISING_LIB names another build of the same sources (the host-sanitizer run)
LIB_PATH = os.environ.get("ISING_LIB") or os.path.join(HERE, "libising.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2311_09275_amd.build` "
        "(the annealer has no non-HIP implementation)")

# The library links libamdhip64.so.7.  PyTorch ships its own copy under the
# same soname; loading torch first makes the process use a single HIP
# runtime, so torch streams and memory can be handed to the library.
try:
    import torch  # noqa: F401
except ImportError:  # torch is optional for the C ABI itself
    torch = None

_L = C.CDLL(LIB_PATH)

OK, ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_STATE, ERR_UNSUPPORTED, ERR_TIMEOUT = 0, -1, -2, -3, -4, -5, -6
# server backend 2 fails every step in which a request with this seed is resident
NULL_FAIL_SEED = 0xFA11FA11FA11FA11
LINEAR, GEOMETRIC, EXPLICIT = 0, 1, 2
PATH_AUTO, PATH_PLAIN, PATH_FIELD, PATH_MSC = 0, 1, 2, 3


class IsingError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = _L.ising_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_L.ising_status_string(status).decode()} ({status}): {detail}")


class Schedule(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_sweeps", C.c_int32), ("beta0", C.c_double),
                ("beta1", C.c_double), ("betas", C.c_void_p)]

    @staticmethod
    def make(kind=LINEAR, n_sweeps=1000, beta0=0.1, beta1=3.0, betas=None) -> "Schedule":
        s = Schedule(kind, n_sweeps, beta0, beta1, None)
        if betas is not None:
            arr = np.ascontiguousarray(betas, np.float64)
            s._keep = arr
            s.betas = arr.ctypes.data
            s.kind = EXPLICIT
            s.n_sweeps = arr.shape[0]
        return s


class Tuning(C.Structure):
    _fields_ = [("path", C.c_int32), ("replicas_per_block", C.c_int32),
                ("block_threads", C.c_int32), ("lds_adjacency", C.c_int32)]


class Tempering(C.Structure):
    _fields_ = [("n_temps", C.c_int32), ("betas", C.c_void_p), ("n_sets", C.c_int32),
                ("n_sweeps", C.c_int32), ("swap_every", C.c_int32),
                ("cluster_moves", C.c_int32), ("cluster_from", C.c_int32)]

    @staticmethod
    def make(betas, n_sets, n_sweeps, swap_every, cluster_from=None) -> "Tempering":
        b = np.ascontiguousarray(betas, np.float64)
        cm = cluster_from is not None
        t = Tempering(int(b.shape[0]), b.ctypes.data, int(n_sets), int(n_sweeps), int(swap_every),
                      1 if cm else 0, int(cluster_from) if cm else 0)
        t._keep = b  # the struct points into this array
        return t


class DeviceResults(C.Structure):
    """Device pointers for ising_anneal_noalloc's results."""
    _fields_ = [("best_cut", C.c_void_p), ("best_sweep", C.c_void_p), ("final_energy", C.c_void_p),
                ("accepts", C.c_void_p), ("argmax", C.c_void_p), ("best_states", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_colours", C.c_int32), ("m", C.c_int64),
                ("total_weight", C.c_int64), ("kmax", C.c_int32), ("max_degree", C.c_int32),
                ("unit_weights", C.c_int32), ("n_padded", C.c_int32), ("fields", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("reached_target", C.c_int32),
                ("sweeps_done", C.c_int32), ("best_replica", C.c_int32),
                ("best_cut", C.c_int64), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


P = C.c_void_p
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
_sig = {
    "ising_status_string": ([C.c_int], C.c_char_p),
    "ising_last_error": ([], C.c_char_p),
    "ising_set_allocator": ([ALLOC_FN, FREE_FN, P], C.c_int),
    "ising_create": ([C.c_int32, C.c_int64, P, P, P, P, C.POINTER(C.c_void_p)], C.c_int),
    "ising_destroy": ([P], C.c_int),
    "ising_problem_info": ([P, C.POINTER(Info)], C.c_int),
    "ising_colouring": ([P, P], C.c_int),
    "ising_neighbour_labels": ([P, P], C.c_int),
    "ising_eval_cut": ([P, P, C.POINTER(C.c_int64)], C.c_int),
    "ising_set_fields": ([P, P], C.c_int),
    "ising_threshold_table": ([C.POINTER(Schedule), C.c_int32, P], C.c_int),
    "ising_anneal": ([P, C.POINTER(Schedule), C.c_int32, C.c_uint64, P], C.c_int),
    "ising_anneal_tuned": ([P, C.POINTER(Schedule), C.c_int32, C.c_uint64, C.POINTER(Tuning), P], C.c_int),
    "ising_anneal_range": ([P, C.POINTER(Schedule), C.c_int32, C.c_uint64, C.POINTER(Tuning), C.c_int32,
                            C.c_int32, P], C.c_int),
    "ising_checkpoint_size": ([P, C.POINTER(C.c_uint64)], C.c_int),
    "ising_checkpoint_save": ([P, P], C.c_int),
    "ising_checkpoint_load": ([P, C.POINTER(Schedule), P, C.c_uint64, P], C.c_int),
    "ising_set_initial_state": ([P, P, C.c_int32], C.c_int),
    "ising_set_trace": ([P, C.c_int32], C.c_int),
    "ising_cut": ([P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), P], C.c_int),
    "ising_best_state": ([P, P], C.c_int),
    "ising_replica_results": ([P, P, P, P], C.c_int),
    "ising_replica_state": ([P, C.c_int32, P, P], C.c_int),
    "ising_replica_field": ([P, C.c_int32, P], C.c_int),
    "ising_energy_trace": ([P, P], C.c_int),
    "ising_last_anneal_ms": ([P, C.POINTER(C.c_double)], C.c_int),
    "ising_last_run_info": ([P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "ising_anneal_noalloc": ([P, C.POINTER(Schedule), C.c_int32, C.c_uint64, C.POINTER(Tuning),
                              C.POINTER(DeviceResults), P], C.c_int),
    "ising_temper": ([P, C.POINTER(Tempering), C.c_uint64, C.POINTER(Tuning), P], C.c_int),
    "ising_temper_results": ([P, P, P, P, P], C.c_int),
    "ising_anneal_batch": ([P, C.c_int32, C.POINTER(Schedule), C.c_int32, P, C.POINTER(Tuning), P], C.c_int),
    "ising_last_batch_ms": ([C.POINTER(C.c_double)], C.c_int),
    "ising_autotune": ([P, C.c_int32, C.POINTER(Schedule), C.c_int32, C.c_int32, C.POINTER(Tuning), P], C.c_int),
    "ising_server_create": ([C.c_uint64, C.c_int32, C.c_int32, C.c_int32, P, C.POINTER(C.c_void_p)], C.c_int),
    "ising_server_submit": ([P, P, C.POINTER(Schedule), C.c_int32, C.c_uint64, C.c_int64, C.c_int32,
                             C.POINTER(C.c_uint64)], C.c_int),
    "ising_server_wait": ([P, C.c_uint64, C.c_double, C.POINTER(Result)], C.c_int),
    "ising_server_best_state": ([P, C.c_uint64, P], C.c_int),
    "ising_server_footprint": ([P, C.POINTER(Schedule), C.c_int32, C.POINTER(C.c_uint64)], C.c_int),
    "ising_server_stats": ([P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)], C.c_int),
    "ising_server_destroy": ([P], C.c_int),
    "ising_valu_rates": ([P], C.c_int),
    "ising_lds_rate": ([C.POINTER(C.c_double)], C.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_L, _name)
    _f.argtypes = _args
    _f.restype = _res
EXPORTED = tuple(_sig)


_allocator = None  # the ctypes callbacks in use (kept alive here)


def set_allocator(alloc=None, free=None) -> None:
    """Route the library's device memory through alloc(bytes, device) ->
    int address and free(address, bytes, device); no arguments restores
    hipMalloc/hipFree (see ising_set_allocator)."""
    global _allocator
    if alloc is None and free is None:
        _check(_L.ising_set_allocator(ALLOC_FN(), FREE_FN(), None), "ising_set_allocator")
        _allocator = None
        return
    a = ALLOC_FN(lambda n, dev, ctx: int(alloc(int(n), int(dev)) or 0))
    f = FREE_FN(lambda p, n, dev, ctx: free(int(p), int(n), int(dev)))
    _check(_L.ising_set_allocator(a, f, None), "ising_set_allocator")
    _allocator = (a, f)


def use_torch_allocator() -> None:
    """Take the library's device memory from PyTorch's caching allocator."""
    import torch

    set_allocator(lambda n, dev: torch.cuda.caching_allocator_alloc(n, device=dev),
                  lambda p, n, dev: torch.cuda.caching_allocator_delete(p))


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise IsingError(rc, where)


def _stream(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def _ptr(a):
    return None if a is None else a.ctypes.data


# ------------------------------------------------------------------ problem
def ising_create(n, u, v, w, colour=None) -> int:
    u = np.ascontiguousarray(u, np.int32)
    v = np.ascontiguousarray(v, np.int32)
    w = np.ascontiguousarray(w, np.int32)
    col = None if colour is None else np.ascontiguousarray(colour, np.int32)
    h = C.c_void_p()
    _check(_L.ising_create(int(n), int(u.shape[0]), _ptr(u), _ptr(v), _ptr(w), _ptr(col),
                           C.byref(h)), "ising_create")
    return h.value


def ising_destroy(h) -> None:
    _check(_L.ising_destroy(h), "ising_destroy")


def ising_problem_info(h) -> Info:
    out = Info()
    _check(_L.ising_problem_info(h, C.byref(out)), "ising_problem_info")
    return out


def ising_colouring(h, n) -> np.ndarray:
    out = np.zeros(n, np.int32)
    _check(_L.ising_colouring(h, _ptr(out)), "ising_colouring")
    return out


def ising_neighbour_labels(h, n) -> np.ndarray:
    out = np.zeros(4 * n, np.int32)
    _check(_L.ising_neighbour_labels(h, _ptr(out)), "ising_neighbour_labels")
    return out


def ising_eval_cut(h, spins) -> int:
    s = np.ascontiguousarray(spins, np.int8)
    out = C.c_int64()
    _check(_L.ising_eval_cut(h, _ptr(s), C.byref(out)), "ising_eval_cut")
    return out.value


def ising_threshold_table(sched: Schedule, kmax: int) -> np.ndarray:
    out = np.zeros((sched.n_sweeps, kmax), np.uint64)
    _check(_L.ising_threshold_table(C.byref(sched), kmax, _ptr(out)), "ising_threshold_table")
    return out


# ------------------------------------------------------------------ anneal
def ising_anneal(h, sched: Schedule, n_replicas: int, seed: int, stream=None) -> None:
    _check(_L.ising_anneal(h, C.byref(sched), n_replicas, seed & (2**64 - 1), _stream(stream)),
           "ising_anneal")


def ising_anneal_tuned(h, sched: Schedule, n_replicas: int, seed: int, tuning: Tuning | None,
                       stream=None) -> None:
    _check(_L.ising_anneal_tuned(h, C.byref(sched), n_replicas, seed & (2**64 - 1),
                                 None if tuning is None else C.byref(tuning), _stream(stream)),
           "ising_anneal_tuned")


def ising_set_initial_state(h, spins, n_replicas) -> None:
    s = None if spins is None else np.ascontiguousarray(spins, np.int8)
    _check(_L.ising_set_initial_state(h, _ptr(s), n_replicas), "ising_set_initial_state")


def ising_set_trace(h, enable: bool) -> None:
    _check(_L.ising_set_trace(h, 1 if enable else 0), "ising_set_trace")


def ising_cut(h, n_replicas: int | None = None):
    best = C.c_int64()
    rep = C.c_int32()
    per = None if n_replicas is None else np.zeros(n_replicas, np.int64)
    _check(_L.ising_cut(h, C.byref(best), C.byref(rep), _ptr(per)), "ising_cut")
    return best.value, rep.value, per


def ising_best_state(h, n) -> np.ndarray:
    out = np.zeros(n, np.int8)
    _check(_L.ising_best_state(h, _ptr(out)), "ising_best_state")
    return out


def ising_replica_results(h, n_replicas):
    bs = np.zeros(n_replicas, np.int32)
    acc = np.zeros(n_replicas, np.int64)
    en = np.zeros(n_replicas, np.int64)
    _check(_L.ising_replica_results(h, _ptr(bs), _ptr(acc), _ptr(en)), "ising_replica_results")
    return bs, acc, en


def ising_replica_state(h, r, n):
    best = np.zeros(n, np.int8)
    fin = np.zeros(n, np.int8)
    _check(_L.ising_replica_state(h, r, _ptr(best), _ptr(fin)), "ising_replica_state")
    return best, fin


def ising_replica_field(h, r, n) -> np.ndarray:
    out = np.zeros(n, np.int32)
    _check(_L.ising_replica_field(h, r, _ptr(out)), "ising_replica_field")
    return out


def ising_energy_trace(h, n_replicas, n_sweeps) -> np.ndarray:
    out = np.zeros((n_replicas, n_sweeps), np.int64)
    _check(_L.ising_energy_trace(h, _ptr(out)), "ising_energy_trace")
    return out


def ising_last_run_info(h):
    r, s_, p = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_L.ising_last_run_info(h, C.byref(r), C.byref(s_), C.byref(p)), "ising_last_run_info")
    return r.value, s_.value, p.value


def ising_last_anneal_ms(h) -> float:
    out = C.c_double()
    _check(_L.ising_last_anneal_ms(h, C.byref(out)), "ising_last_anneal_ms")
    return out.value


# ------------------------------------------------------------------ tempering
def ising_anneal_noalloc(h, sched: Schedule, n_replicas: int, seed: int, tuning: Tuning | None,
                         best_cut, best_sweep, final_energy, accepts, argmax, best_states,
                         stream=None) -> None:
    """The allocation-free anneal; the six result arguments are device
    addresses (ints), e.g. torch tensors' data_ptr()."""
    out = DeviceResults(best_cut, best_sweep, final_energy, accepts, argmax, best_states)
    _check(_L.ising_anneal_noalloc(h, C.byref(sched), int(n_replicas), int(seed),
                                   None if tuning is None else C.byref(tuning), C.byref(out),
                                   _stream(stream)), "ising_anneal_noalloc")


def ising_temper(h, pt: Tempering, seed: int, tuning: Tuning | None = None, stream=None) -> None:
    _check(_L.ising_temper(h, C.byref(pt), seed & (2**64 - 1),
                           None if tuning is None else C.byref(tuning), _stream(stream)),
           "ising_temper")


def ising_temper_results(h, n_temps: int, n_sets: int, clusters: bool = False):
    """(final temperatures, exchanges) or, with clusters, also the cluster
    move and flipped-site counts [n_sets // 2, K]."""
    temp = np.zeros(n_temps * n_sets, np.int32)
    swaps = np.zeros((n_sets, max(n_temps - 1, 1)), np.int64)
    cm = np.zeros((max(n_sets // 2, 1), n_temps), np.int64) if clusters else None
    cs = np.zeros((max(n_sets // 2, 1), n_temps), np.int64) if clusters else None
    _check(_L.ising_temper_results(h, _ptr(temp), _ptr(swaps), _ptr(cm), _ptr(cs)),
           "ising_temper_results")
    if clusters:
        return temp, swaps[:, :n_temps - 1], cm[:n_sets // 2], cs[:n_sets // 2]
    return temp, swaps[:, :n_temps - 1]


# ------------------------------------------------------------------ batching
def ising_anneal_batch(handles, sched: Schedule, n_replicas, seeds, tuning: Tuning | None = None,
                       stream=None) -> None:
    hs = (C.c_void_p * len(handles))(*handles)
    sd = np.ascontiguousarray(seeds, np.uint64)
    _check(_L.ising_anneal_batch(C.cast(hs, C.c_void_p), len(handles), C.byref(sched), n_replicas,
                                 _ptr(sd), None if tuning is None else C.byref(tuning),
                                 _stream(stream)), "ising_anneal_batch")


def ising_last_batch_ms() -> float:
    out = C.c_double()
    _check(_L.ising_last_batch_ms(C.byref(out)), "ising_last_batch_ms")
    return out.value


VALU_RATE_NAMES = ("v_mad_u64_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_xor_b32")


def ising_valu_rates() -> dict:
    """Measured lane-operations per second of the integer VALU instructions
    the kernels use (a roofline measurement helper)."""
    out = np.zeros(4, np.float64)
    _check(_L.ising_valu_rates(_ptr(out)), "ising_valu_rates")
    return dict(zip(VALU_RATE_NAMES, (float(x) for x in out)))



def ising_lds_rate() -> float:
    """LDS read bandwidth of the current device, bytes/s (ising_lds_rate)."""
    out = C.c_double()
    _check(_L.ising_lds_rate(C.byref(out)), "ising_lds_rate")
    return out.value

def ising_autotune(handles, sched: Schedule, n_replicas, prefix_sweeps=0, stream=None) -> Tuning:
    hs = (C.c_void_p * len(handles))(*handles)
    out = Tuning()
    _check(_L.ising_autotune(C.cast(hs, C.c_void_p), len(handles), C.byref(sched), n_replicas,
                             prefix_sweeps, C.byref(out), _stream(stream)), "ising_autotune")
    return out


# ------------------------------------------------------------------ serving
def ising_server_create(hbm_budget, max_slots, chunk_sweeps, backend=0, stream=None) -> int:
    h = C.c_void_p()
    _check(_L.ising_server_create(int(hbm_budget), max_slots, chunk_sweeps, backend,
                                  _stream(stream), C.byref(h)), "ising_server_create")
    return h.value


def ising_server_submit(srv, problem, sched: Schedule, n_replicas, seed, target_cut, check_every) -> int:
    t = C.c_uint64()
    _check(_L.ising_server_submit(srv, problem, C.byref(sched), n_replicas, seed & (2**64 - 1),
                                  int(target_cut), check_every, C.byref(t)), "ising_server_submit")
    return t.value


def ising_server_wait(srv, ticket, timeout_s=-1.0) -> Result:
    out = Result()
    _check(_L.ising_server_wait(srv, ticket, float(timeout_s), C.byref(out)), "ising_server_wait")
    return out


def ising_server_best_state(srv, ticket, n) -> np.ndarray:
    out = np.zeros(n, np.int8)
    _check(_L.ising_server_best_state(srv, ticket, _ptr(out)), "ising_server_best_state")
    return out


def ising_server_footprint(problem, sched: Schedule, n_replicas) -> int:
    out = C.c_uint64()
    _check(_L.ising_server_footprint(problem, C.byref(sched), n_replicas, C.byref(out)),
           "ising_server_footprint")
    return out.value


def ising_server_stats(srv):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int32()
    _check(_L.ising_server_stats(srv, C.byref(a), C.byref(b), C.byref(c)), "ising_server_stats")
    return a.value, b.value, c.value


def ising_server_destroy(srv) -> None:
    _check(_L.ising_server_destroy(srv), "ising_server_destroy")


# ------------------------------------------------------------------ object API
@dataclass
class AnnealResult:
    best_cut: int
    best_replica: int
    per_replica: np.ndarray


class Problem:
    """Owning wrapper of an ``ising_problem`` handle."""

    def __init__(self, n, u, v, w, colour=None):
        self.n = int(n)
        self.handle = ising_create(n, u, v, w, colour)

    @classmethod
    def from_instance(cls, inst, colour=None) -> "Problem":
        """The problem of an instance, with its local fields when it has any."""
        p = cls(inst.n, inst.u, inst.v, inst.w, colour)
        f = getattr(inst, "field", None)
        if f is not None:
            p.set_fields(f)
        return p

    def set_fields(self, b) -> None:
        """Local fields b [n] (None removes them); see ``ising_set_fields``."""
        arr = None if b is None else np.ascontiguousarray(b, np.int32)
        _check(_L.ising_set_fields(self.handle, _ptr(arr)), "ising_set_fields")

    def close(self) -> None:
        if self.handle:
            ising_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> Info:
        return ising_problem_info(self.handle)

    def colouring(self) -> np.ndarray:
        return ising_colouring(self.handle, self.n)

    def neighbour_labels(self) -> np.ndarray:
        return ising_neighbour_labels(self.handle, self.n)

    def anneal(self, sched: Schedule, n_replicas: int, seed: int, tuning: Tuning | None = None,
               stream=None) -> None:
        ising_anneal_tuned(self.handle, sched, n_replicas, seed, tuning, stream)

    def anneal_range(self, sched: Schedule, n_replicas: int, seed: int, t_begin: int, t_end: int,
                     tuning: Tuning | None = None, stream=None) -> None:
        """Sweeps [t_begin, t_end) of an anneal (see ``ising_anneal_range``)."""
        _check(_L.ising_anneal_range(self.handle, C.byref(sched), n_replicas, seed & (2**64 - 1),
                                     None if tuning is None else C.byref(tuning), t_begin, t_end,
                                     _stream(stream)), "ising_anneal_range")

    def checkpoint(self) -> bytes:
        """The device state of the last anneal (see ``ising_checkpoint_save``)."""
        n = C.c_uint64()
        _check(_L.ising_checkpoint_size(self.handle, C.byref(n)), "ising_checkpoint_size")
        buf = (C.c_char * n.value)()
        _check(_L.ising_checkpoint_save(self.handle, buf), "ising_checkpoint_save")
        return bytes(buf)

    def restore(self, sched: Schedule, data: bytes, stream=None) -> None:
        """Put a checkpoint back (see ``ising_checkpoint_load``)."""
        buf = C.create_string_buffer(data, len(data))
        _check(_L.ising_checkpoint_load(self.handle, C.byref(sched), buf, len(data), _stream(stream)),
               "ising_checkpoint_load")

    def temper(self, betas, n_sets: int, n_sweeps: int, swap_every: int, seed: int,
               tuning: Tuning | None = None, stream=None, cluster_from=None) -> None:
        """Parallel tempering over the ladder ``betas`` (see ``ising_temper``);
        ``cluster_from`` = k adds Houdayer cluster moves at temperatures >= k."""
        self._ladder = (len(betas), int(n_sets), cluster_from is not None)
        ising_temper(self.handle, Tempering.make(betas, n_sets, n_sweeps, swap_every, cluster_from),
                     seed, tuning, stream)

    def temper_results(self):
        """(final temperature index [R], accepted exchanges [n_sets, K-1]),
        plus the cluster move and site counts after a run with cluster moves."""
        K, n_sets, cl = getattr(self, "_ladder", (1, 1, False))
        return ising_temper_results(self.handle, K, n_sets, cl)

    @property
    def R(self) -> int:
        return ising_last_run_info(self.handle)[0]

    @property
    def S(self) -> int:
        return ising_last_run_info(self.handle)[1]

    def cut(self) -> AnnealResult:
        b, r, per = ising_cut(self.handle, self.R)
        return AnnealResult(b, r, per)

    def best_state(self) -> np.ndarray:
        return ising_best_state(self.handle, self.n)

    def replica_results(self):
        return ising_replica_results(self.handle, self.R)

    def replica_state(self, r):
        return ising_replica_state(self.handle, r, self.n)

    def replica_field(self, r):
        return ising_replica_field(self.handle, r, self.n)

    def energy_trace(self):
        return ising_energy_trace(self.handle, self.R, self.S)

    def set_trace(self, on=True):
        ising_set_trace(self.handle, on)

    def set_initial_state(self, spins, n_replicas):
        ising_set_initial_state(self.handle, spins, n_replicas)

    def eval_cut(self, spins) -> int:
        return ising_eval_cut(self.handle, spins)

    def last_anneal_ms(self) -> float:
        return ising_last_anneal_ms(self.handle)
