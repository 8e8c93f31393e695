"""HIP path vs the CPU oracle, element by element, through the C ABI.

Every integer the method produces is compared exactly: per-sweep energy of
every replica, accepted-flip counts, best cut and best sweep, best and final
states, final local fields and the argmax replica.  Runs on an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_09275_amd import instances as I

pytestmark = pytest.mark.gpu

from tests.conftest import load_binding

B = load_binding()

PATHS = {
    "plain": B.Tuning(B.PATH_PLAIN, 1, 256, 0),
    "field_g1_b256_hbmadj": B.Tuning(B.PATH_FIELD, 1, 256, 2),
    "field_g1_b1024_ldsadj": B.Tuning(B.PATH_FIELD, 1, 1024, 1),
    "field_g1_b1024_csradj": B.Tuning(B.PATH_FIELD, 1, 1024, 3),
    "field_g4_b256_csradj": B.Tuning(B.PATH_FIELD, 4, 256, 3),
    "field_g1_b512_hbmdeg4": B.Tuning(B.PATH_FIELD, 1, 512, 4),
    "field_g2_b512_ldsadj": B.Tuning(B.PATH_FIELD, 2, 512, 1),
    "field_g4_b256_hbmadj": B.Tuning(B.PATH_FIELD, 4, 256, 2),
    "field_g1_b512_auto": B.Tuning(B.PATH_FIELD, 1, 512, 0),
    "msc_g1_b256": B.Tuning(B.PATH_MSC, 1, 256, 0),
    "msc_g2_b512": B.Tuning(B.PATH_MSC, 2, 512, 0),
    # the multispin degree-4 form: 8, 16 or 32 replicas per unit
    "msc4_w8_b256": B.Tuning(B.PATH_MSC, 8, 256, 0),
    "msc4_w16_b512": B.Tuning(B.PATH_MSC, 16, 512, 0),
    "msc4_w32_b1024": B.Tuning(B.PATH_MSC, 32, 1024, 0),
    "msc4_w8_b1024": B.Tuning(B.PATH_MSC, 8, 1024, 0),
}
DEG4_ONLY = {"field_g1_b512_hbmdeg4", "msc4_w8_b256", "msc4_w16_b512", "msc4_w32_b1024",
             "msc4_w8_b1024"}


def _needs_deg4(tuning):
    return tuning is not None and (tuning.lds_adjacency == 4 or
                                   (tuning.path == B.PATH_MSC and tuning.replicas_per_block >= 8))


def _sched(kind, S, b0, b1, betas=None):
    if betas is not None:
        return B.Schedule.make(betas=betas), dict(kind=O.EXPLICIT, betas=betas)
    return B.Schedule.make(kind, S, b0, b1), dict(kind=kind, beta0=b0, beta1=b1)


def compare(inst, S, R, seed, kind=O.LINEAR, b0=0.1, b1=3.0, betas=None, tuning=None,
            init=None, replicas=None, trace=True, colour=None):
    """Run the GPU path and check it against the oracle on `replicas`."""
    n = inst.n
    if _needs_deg4(tuning):
        deg = np.bincount(np.concatenate([inst.u, inst.v]), minlength=n)
        if n == 0 or not (deg == 4).all() or not (np.abs(inst.w) == 1).all():
            pytest.skip("the degree-4 forms need a 4-regular unit-weight graph")
    sched, okw = _sched(kind, S, b0, b1, betas)
    p = B.Problem.from_instance(inst, colour)
    if init is not None:
        p.set_initial_state(init, R)
    p.set_trace(trace)
    p.anneal(sched, R, seed, tuning)
    best, arg, per = B.ising_cut(p.handle, R)
    bs, acc, en = p.replica_results()
    reps = list(range(R)) if replicas is None else list(replicas)
    full = replicas is None
    tr = p.energy_trace() if trace else None
    for r in reps:
        o = O.anneal(inst, S, R, seed, init_spins=init, r_begin=r, r_end=r + 1,
                     want_trace=trace, want_field=True, colour=colour, **okw)
        assert per[r] == o.best_cut[0], (r, per[r], o.best_cut[0])
        assert bs[r] == o.best_sweep[0], r
        assert acc[r] == o.accepts[0], r
        assert en[r] == o.final_energy[0], r
        if trace:
            np.testing.assert_array_equal(tr[r], o.energy_trace[0], err_msg=f"replica {r}")
        gb, gf = p.replica_state(r)
        np.testing.assert_array_equal(gb, o.best_state[0], err_msg=f"best state r={r}")
        np.testing.assert_array_equal(gf, o.final_state[0], err_msg=f"final state r={r}")
        if tuning is None or tuning.path != B.PATH_MSC:
            np.testing.assert_array_equal(p.replica_field(r), o.final_field[0])
    if full:
        assert best == per.max()
        assert arg == int(np.argmax(per))
        bstate = p.best_state()
        # with local fields the reported value is cut + sum b s
        f = getattr(inst, "field", None)
        lin = 0 if f is None else int((f.astype(np.int64) * bstate).sum())
        assert p.eval_cut(bstate) + lin == best
    p.close()
    return per


# ------------------------------------------------------------------ small cases
@pytest.mark.parametrize("path", list(PATHS))
def test_c1_torus16(path):
    """16x16 +-1 torus, 8 replicas, 1000 sweeps, beta linear 0.1 -> 3.0."""
    compare(I.workload_c1(), 1000, 8, 1001, tuning=PATHS[path])


@pytest.mark.parametrize("path", list(PATHS))
def test_odd_torus_ragged_classes(path):
    """7x9 torus: three colour classes whose sizes are not multiples of 4;
    40 replicas (not a multiple of 32 or of the block size)."""
    compare(I.torus(7, 9, 5), 150, 40, 77, kind=O.GEOMETRIC, b0=0.2, b1=4.0, tuning=PATHS[path])


NOT_DEG4 = [p for p in PATHS if p not in DEG4_ONLY]


@pytest.mark.parametrize("path", NOT_DEG4)
def test_random_graph_with_isolated_vertices(path):
    """G70-shaped (m = n - 1) sparse random graph: isolated vertices, varied
    degrees, greedy colouring with several classes."""
    compare(I.random_graph(700, 699, 11), 200, 33, 5, kind=O.LINEAR, b0=0.05, b1=3.0,
            tuning=PATHS[path])


def circulant4(n, a, b, seed):
    """4-regular circulant graph, i ~ i+a and i ~ i+b (mod n), +-1 weights:
    every vertex of degree 4 but, unlike a torus, not 2-colourable."""
    i = np.arange(n, dtype=np.int32)
    u = np.concatenate([i, i])
    v = np.concatenate([(i + a) % n, (i + b) % n]).astype(np.int32)
    w = (np.random.Generator(np.random.PCG64(seed)).integers(0, 2, 2 * n) * 2 - 1).astype(np.int32)
    return I.Instance(f"circulant{n}_{a}_{b}", n, u, v, w)


@pytest.mark.parametrize("path", list(PATHS))
def test_degree4_non_bipartite(path):
    """Degree-4 graph with several colour classes of ragged sizes, so the
    degree-4 adjacency form meets padding slots in many groups."""
    compare(circulant4(331, 1, 17, 4), 150, 20, 12, kind=O.GEOMETRIC, b0=0.1, b1=3.0,
            tuning=PATHS[path])


@pytest.mark.parametrize("path", list(PATHS))
def test_degree4_random_regular(path):
    """Random 4-regular graph listed as sorted (min, max) pairs: its degree-4
    labels come from the closed-walk construction, not the listing."""
    compare(I.random_regular4(403, 21), 130, 20, 13, kind=O.GEOMETRIC, b0=0.1, b1=3.0,
            tuning=PATHS[path])


@pytest.mark.parametrize("path", ["plain", "field_g1_b256_hbmadj", "field_g4_b256_hbmadj",
                                  "field_g1_b512_auto"])
def test_weighted_graph(path):
    compare(I.random_weighted(500, 1400, 12, 7), 120, 20, 9, kind=O.GEOMETRIC, b0=0.05, b1=1.5,
            tuning=PATHS[path])


def weight_limit_instance():
    """Weights at the largest allowed magnitude: |w| uniform in [1, 2^15] on a
    random graph, every seventh edge at exactly +-2^15 (k reaches 250,226)."""
    inst = I.random_weighted(120, 300, 31, 32768)
    w = inst.w.copy()
    w[::7] = np.where(w[::7] > 0, 32768, -32768)
    return I.Instance("wlimit", inst.n, inst.u, inst.v, w)


@pytest.mark.parametrize("path", ["plain", "field_g1_b256_hbmadj", "field_g4_b256_hbmadj",
                                  "field_g1_b512_auto"])
def test_weights_at_the_limit_long_rows(path):
    """From beta 0.011 the threshold rows hold about 1008 keys, near the LDS
    paths' 1024-key limit (2018 words: the FIELD path stages one sweep's row
    at a time)."""
    compare(weight_limit_instance(), 40, 12, 3, kind=O.LINEAR, b0=0.011, b1=0.05,
            tuning=PATHS[path])


@pytest.mark.parametrize("b0", [0.0008, 1e-5])
def test_weights_at_the_limit_rows_beyond_lds_paths(b0):
    """At beta 0.0008 a row covers k up to ~13,900, at 1e-5 every k up to
    250,226: the FIELD path refuses the schedule, and the automatic
    configuration runs the plain path with oracle-equal results."""
    inst = weight_limit_instance()
    p = B.Problem.from_instance(inst)
    with pytest.raises(B.IsingError) as e:
        p.anneal(B.Schedule.make(B.LINEAR, 40, b0, 10 * b0), 12, 3, PATHS["field_g1_b256_hbmadj"])
    assert e.value.status == B.ERR_UNSUPPORTED
    p.close()
    compare(inst, 40, 12, 3, kind=O.LINEAR, b0=b0, b1=10 * b0,
            tuning=B.Tuning(B.PATH_AUTO, 0, 0, 0))


def hub_graph(n_leaves, seed):
    """A hub joined to n_leaves leaves, the leaves joined in a ring, +-1
    weights: one vertex of degree n_leaves, the rest of degree 3."""
    leaves = np.arange(1, n_leaves + 1, dtype=np.int32)
    u = np.concatenate([np.zeros(n_leaves, np.int32), leaves])
    v = np.concatenate([leaves, np.roll(leaves, -1)]).astype(np.int32)
    w = (np.random.Generator(np.random.PCG64(seed)).integers(0, 2, 2 * n_leaves) * 2 - 1)
    return I.Instance(f"hub{n_leaves}", n_leaves + 1, u, v, w.astype(np.int32))


_DEG_PATHS = ["plain", "field_g1_b256_hbmadj", "field_g1_b1024_ldsadj", "field_g2_b512_ldsadj",
              "field_g1_b1024_csradj"]


@pytest.mark.parametrize("hub,path", [(31, p) for p in _DEG_PATHS + ["msc_g1_b256"]] +
                         [(255, p) for p in _DEG_PATHS])
def test_degree_at_the_limits(hub, path):
    """Degree 31 (the multispin path's limit) and 255 (the LDS paths' 8-bit
    degree field)."""
    compare(hub_graph(hub, 5), 60, 40, 7, kind=O.GEOMETRIC, b0=0.1, b1=3.0, tuning=PATHS[path])


def test_degree_beyond_the_limits():
    """Degree 32 is refused by the multispin path and 256 by the FIELD
    path; the automatic configuration runs them with oracle-equal results."""
    sched = B.Schedule.make(B.LINEAR, 10, 0.1, 1.0)
    for hub, refused in ((32, ["msc_g1_b256"]), (256, ["field_g1_b256_hbmadj", "field_g1_b1024_ldsadj"])):
        inst = hub_graph(hub, 6)
        p = B.Problem.from_instance(inst)
        for path in refused:
            with pytest.raises(B.IsingError) as e:
                p.anneal(sched, 8, 1, PATHS[path])
            assert e.value.status == B.ERR_UNSUPPORTED, (hub, path)
        p.close()
        compare(inst, 60, 40, 7, kind=O.GEOMETRIC, b0=0.1, b1=3.0,
                tuning=B.Tuning(B.PATH_AUTO, 0, 0, 0))


def test_field_path_colour_limit():
    """The FIELD path keeps class bounds in two registers (at most 64
    classes): a supplied 70-colouring is refused there, and the automatic
    configuration falls back to the plain path with oracle-equal results."""
    n = 140
    inst = I.Instance("cycle140", n, np.arange(n, dtype=np.int32),
                      ((np.arange(n) + 1) % n).astype(np.int32), np.ones(n, np.int32))
    colour = (np.arange(n) % 70).astype(np.int32)
    p = B.Problem.from_instance(inst, colour)
    with pytest.raises(B.IsingError) as e:
        p.anneal(B.Schedule.make(B.LINEAR, 10, 0.1, 1.0), 8, 1, PATHS["field_g1_b256_hbmadj"])
    assert e.value.status == B.ERR_UNSUPPORTED
    compare(inst, 60, 8, 3, tuning=B.Tuning(B.PATH_AUTO, 0, 0, 0), colour=colour)


def test_unit_weight_paths_reject_weighted():
    p = B.Problem.from_instance(I.random_weighted(50, 100, 1, 3))
    for path in ("msc_g1_b256", "field_g1_b1024_ldsadj", "field_g1_b1024_csradj",
                 "field_g1_b512_hbmdeg4"):
        with pytest.raises(B.IsingError) as e:
            p.anneal(B.Schedule.make(B.LINEAR, 10, 0.1, 1.0), 32, 1, PATHS[path])
        assert e.value.status == B.ERR_UNSUPPORTED


@pytest.mark.parametrize("path", list(PATHS))
def test_beta_zero_and_infinite(path):
    inst = I.torus(6, 5, 3)
    compare(inst, 9, 12, 3, betas=np.zeros(9), tuning=PATHS[path])
    compare(inst, 30, 12, 3, betas=np.full(30, 1e300), tuning=PATHS[path])


@pytest.mark.parametrize("path", list(PATHS))
def test_given_initial_state(path):
    inst = I.torus(10, 6, 2)
    init = I.random_spins(5, 35, inst.n)
    compare(inst, 60, 35, 8, tuning=PATHS[path], init=init)


@pytest.mark.parametrize("path", NOT_DEG4)
def test_degenerate_sizes(path):
    # one vertex, no edges; a single edge; one sweep; one replica
    compare(I.Instance("one", 1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32)),
            5, 3, 1, tuning=PATHS[path])
    compare(I.Instance("edge", 2, np.array([0], np.int32), np.array([1], np.int32),
                       np.array([1], np.int32)), 1, 1, 2, tuning=PATHS[path])
    compare(I.torus(3, 3, 1), 1, 1, 3, tuning=PATHS[path])


def test_supplied_colouring():
    inst = I.torus(8, 8, 4)
    v = np.arange(inst.n)
    colour = ((v % 8 + v // 8) % 2 + 2 * ((v % 8) >= 4)).astype(np.int32)  # 4 classes
    for path in ("plain", "field_g1_b256_hbmadj", "field_g1_b1024_ldsadj", "msc_g1_b256"):
        compare(inst, 80, 16, 6, tuning=PATHS[path], colour=colour)


def test_argmax_ties_lowest_replica():
    inst = I.torus(6, 6, 1, weights="one")
    for path in ("plain", "field_g1_b256_hbmadj", "field_g1_b1024_ldsadj", "msc_g1_b256"):
        p = B.Problem.from_instance(inst)
        p.anneal(B.Schedule.make(B.GEOMETRIC, 300, 0.5, 8.0), 6, 2, PATHS[path])
        best, arg, per = B.ising_cut(p.handle, 6)
        assert best == inst.m and np.all(per == inst.m) and arg == 0
        p.close()


def test_repeatable_and_stream():
    import torch
    inst = I.torus(12, 12, 7)
    s = torch.cuda.Stream()
    outs = []
    for _ in range(3):
        p = B.Problem.from_instance(inst)
        p.set_trace(True)
        p.anneal(B.Schedule.make(B.LINEAR, 200, 0.1, 3.0), 64, 99, PATHS["field_g1_b1024_ldsadj"], stream=s)
        outs.append(p.energy_trace())
        p.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


# ------------------------------------------------------------------ full sizes
def test_c2_full_size_sampled_replicas():
    """100x80 torus, 256 replicas, 4000 sweeps geometric 0.1 -> 4.0 (the
    benchmarked configuration, in the launch configuration the benchmark
    times), four replicas recomputed by the oracle."""
    compare(I.workload_c2(), 4000, 256, 1002, kind=O.GEOMETRIC, b0=0.1, b1=4.0,
            tuning=B.Tuning(B.PATH_FIELD, 1, 1024), replicas=[0, 1, 130, 255], trace=True)


def test_c2_full_size_automatic_configuration():
    """The same workload with the library choosing the configuration."""
    compare(I.workload_c2(), 4000, 256, 1002, kind=O.GEOMETRIC, b0=0.1, b1=4.0,
            tuning=None, replicas=[7, 200], trace=False)


def test_c3_full_size_sampled_replicas():
    """Random graph n=10,000, m=9,999, 1024 replicas, 4000 sweeps linear
    0.05 -> 3.0, three replicas recomputed by the oracle."""
    compare(I.workload_c3(), 4000, 1024, 1003, kind=O.LINEAR, b0=0.05, b1=3.0,
            tuning=None, replicas=[0, 513, 1023], trace=False)


def test_schedule_and_table_reuse_across_anneals():
    """One problem annealed with alternating schedules and replica counts:
    cached threshold tables and skipped uploads must never leave a stale
    table behind (each result equals a fresh problem's)."""
    inst = I.torus(20, 18, 21)
    a = B.Schedule.make(B.GEOMETRIC, 300, 0.1, 4.0)
    b = B.Schedule.make(B.LINEAR, 300, 0.2, 2.0)
    c = B.Schedule.make(betas=np.linspace(0.3, 3.3, 300))
    p = B.Problem.from_instance(inst)
    for sched, R, tun in [(a, 24, None), (b, 24, None), (a, 24, None), (a, 40, None),
                          (c, 40, None), (c, 40, B.Tuning(B.PATH_PLAIN, 1, 256, 0)), (a, 24, None)]:
        p.anneal(sched, R, 5, tun)
        got = B.ising_cut(p.handle, R)[2]
        q = B.Problem.from_instance(inst)
        q.anneal(sched, R, 5, B.Tuning(B.PATH_PLAIN, 1, 256, 0))
        np.testing.assert_array_equal(got, B.ising_cut(q.handle, R)[2])
        q.close()
    p.close()


@pytest.mark.parametrize("width", [8, 16])
def test_msc4_at_its_size_limit(width):
    """The largest torus the multispin degree-4 form takes: 180x180 pads to
    32,512 tiled words, just under its 2^15 limit (8-bit elements: 65 KB of
    LDS pairs; 16-bit: 130 KB, one unit per CU).  Every replica against the
    oracle."""
    compare(I.torus(180, 180, 7), 30, width, 11, kind=O.GEOMETRIC, b0=0.1, b1=4.0,
            tuning=B.Tuning(B.PATH_MSC, width, 256, 0))


def test_msc4_beyond_its_size_limit_is_refused():
    """One size up (182x182, 33,124 vertices) the form is refused with
    ISING_ERR_UNSUPPORTED, as is 32-bit elements at 180x180 (260 KB of
    pairs), and the automatic configuration still runs both."""
    sched = B.Schedule.make(B.GEOMETRIC, 5, 0.1, 4.0)
    for side, width in ((182, 8), (180, 32)):
        p = B.Problem.from_instance(I.torus(side, side, 8))
        with pytest.raises(B.IsingError) as e:
            p.anneal(sched, width, 3, B.Tuning(B.PATH_MSC, width, 256, 0))
        assert e.value.status == B.ERR_UNSUPPORTED
        p.anneal(sched, width, 3, None)
        assert p.cut().best_cut > 0
        p.close()


@pytest.mark.parametrize("path", sorted(DEG4_ONLY - {"field_g1_b512_hbmdeg4"}))
def test_msc4_small_shapes(path):
    """The multispin degree-4 form on the smallest torus (3 classes of
    3 vertices, one sweep, one replica), on replica counts that leave the
    last unit partly empty, and on a torus whose groups span two tiles."""
    compare(I.torus(3, 3, 1), 1, 1, 3, tuning=PATHS[path])
    compare(I.torus(3, 5, 2), 20, 5, 4, tuning=PATHS[path])
    compare(I.torus(4, 4, 3), 30, 33, 5, kind=O.GEOMETRIC, b0=0.1, b1=4.0, tuning=PATHS[path])
    compare(I.torus(34, 30, 4), 40, 9, 6, kind=O.GEOMETRIC, b0=0.1, b1=4.0, tuning=PATHS[path])
