"""Batching and serving on the GPU: results must equal separate anneals
exactly, whatever the batch composition, chunking or graph replay."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_09275_amd import instances as I
from tests.conftest import load_binding

pytestmark = pytest.mark.gpu
B = load_binding()


def _batch_instances():
    # uneven sizes, odd and even tori (2 and 3 colours), a random graph
    return [I.torus(33, 33, 101), I.torus(16, 20, 102), I.torus(41, 37, 103),
            I.random_graph(900, 899, 104), I.torus(64, 64, 105), I.torus(7, 5, 106)]


def _single(inst, sched, R, seed, tuning):
    p = B.Problem.from_instance(inst)
    p.anneal(sched, R, seed, tuning)
    best, arg, per = B.ising_cut(p.handle, R)
    bs, acc, en = p.replica_results()
    state = p.best_state()
    p.close()
    return per, bs, acc, en, state


@pytest.mark.parametrize("tun", [B.Tuning(B.PATH_FIELD, 1, 512, 0), B.Tuning(B.PATH_FIELD, 2, 1024, 2),
                                 B.Tuning(B.PATH_MSC, 1, 256, 0), None],
                         ids=["field_auto", "field_g2_hbm", "msc", "autotuned"])
def test_batch_equals_separate_anneals(tun):
    insts = _batch_instances()
    sched = B.Schedule.make(B.GEOMETRIC, 300, 0.1, 4.0)
    R = 40
    seeds = np.array([7000 + i for i in range(len(insts))], np.uint64)
    probs = [B.Problem.from_instance(x) for x in insts]
    hs = [p.handle for p in probs]
    if tun is None:
        tun = B.ising_autotune(hs, sched, R, prefix_sweeps=50)
    B.ising_anneal_batch(hs, sched, R, seeds, tun)
    for i, (inst, p) in enumerate(zip(insts, probs)):
        per, bs, acc, en, state = _single(inst, sched, R, int(seeds[i]), B.Tuning(B.PATH_PLAIN, 1, 256, 0))
        best, arg, per_b = B.ising_cut(p.handle, R)
        bs_b, acc_b, en_b = p.replica_results()
        np.testing.assert_array_equal(per_b, per)
        np.testing.assert_array_equal(bs_b, bs)
        np.testing.assert_array_equal(acc_b, acc)
        np.testing.assert_array_equal(en_b, en)
        np.testing.assert_array_equal(p.best_state(), state)
    # one problem also against the oracle
    o = O.anneal(insts[1], 300, R, int(seeds[1]), kind=O.GEOMETRIC, beta0=0.1, beta1=4.0)
    np.testing.assert_array_equal(B.ising_cut(probs[1].handle, R)[2], o.best_cut)
    for p in probs:
        p.close()


@pytest.mark.parametrize("tun", [B.Tuning(B.PATH_FIELD, 1, 1024, 0), B.Tuning(B.PATH_FIELD, 2, 512, 0)],
                         ids=["g1_b1024", "g2_b512"])
def test_batch_mixed_adjacency_forms(tun):
    """One launch whose problems use different adjacency forms: a small
    torus (degree-4 form in LDS), a random graph (CSR form in LDS), a torus
    too large to stage (degree-4 form read from HBM) and a weighted graph
    ({position, w} pairs from HBM)."""
    insts = [I.torus(24, 24, 111), I.random_graph(700, 699, 112), I.torus(110, 110, 113),
             I.torus(9, 11, 114), I.random_weighted(300, 800, 115, 5)]
    sched = B.Schedule.make(B.GEOMETRIC, 120, 0.1, 4.0)
    R = 40
    seeds = np.array([7100 + i for i in range(len(insts))], np.uint64)
    probs = [B.Problem.from_instance(x) for x in insts]
    B.ising_anneal_batch([p.handle for p in probs], sched, R, seeds, tun)
    for i, (inst, p) in enumerate(zip(insts, probs)):
        per, bs, acc, en, state = _single(inst, sched, R, int(seeds[i]), B.Tuning(B.PATH_PLAIN, 1, 256, 0))
        best, arg, per_b = B.ising_cut(p.handle, R)
        bs_b, acc_b, en_b = p.replica_results()
        np.testing.assert_array_equal(per_b, per, err_msg=inst.name)
        np.testing.assert_array_equal(bs_b, bs, err_msg=inst.name)
        np.testing.assert_array_equal(acc_b, acc, err_msg=inst.name)
        np.testing.assert_array_equal(en_b, en, err_msg=inst.name)
        np.testing.assert_array_equal(p.best_state(), state, err_msg=inst.name)
    for p in probs:
        p.close()


def test_graph_replays_match_eager():
    import torch
    insts = _batch_instances()[:4]
    sched = B.Schedule.make(B.LINEAR, 200, 0.1, 3.0)
    R = 32
    seeds = np.arange(4, dtype=np.uint64) + 11
    probs = [B.Problem.from_instance(x) for x in insts]
    hs = [p.handle for p in probs]
    tun = B.Tuning(B.PATH_FIELD, 1, 512, 0)
    B.ising_anneal_batch(hs, sched, R, seeds, tun, stream=None)  # eager (null stream)
    eager = [B.ising_cut(h, R)[2].copy() for h in hs]
    states = [p.best_state() for p in probs]
    s = torch.cuda.Stream()
    x = torch.ones(1 << 20, device="cuda")
    for rep in range(4):  # first call captures, the rest replay
        B.ising_anneal_batch(hs, sched, R, seeds, tun, stream=s)
        for i, h in enumerate(hs):
            np.testing.assert_array_equal(B.ising_cut(h, R)[2], eager[i])
            np.testing.assert_array_equal(probs[i].best_state(), states[i])
        x = x * 2 - 1  # unrelated eager work between replays
        torch.cuda.synchronize()
    for p in probs:
        p.close()


def test_batch_timing_api():
    insts = _batch_instances()[:2]
    probs = [B.Problem.from_instance(x) for x in insts]
    B.ising_anneal_batch([p.handle for p in probs], B.Schedule.make(B.LINEAR, 50, 0.1, 3.0), 8,
                         np.array([1, 2], np.uint64), B.Tuning(B.PATH_FIELD, 1, 256, 0))
    assert B.ising_last_batch_ms() > 0
    for p in probs:
        p.close()


# ------------------------------------------------------------------ serving
def _serve(requests, chunk, budget=1 << 28, slots=8):
    srv = B.ising_server_create(budget, slots, chunk, backend=0)
    tickets = [B.ising_server_submit(srv, p.handle, s, R, seed, target, ce)
               for (p, s, R, seed, target, ce) in requests]
    out = []
    for (p, *_), t in zip(requests, tickets):
        r = B.ising_server_wait(srv, t, 120.0)
        assert r.status == 0
        out.append((r.best_cut, r.best_replica, r.sweeps_done, r.reached_target,
                    B.ising_server_best_state(srv, t, p.n)))
    stats = B.ising_server_stats(srv)
    B.ising_server_destroy(srv)
    return out, stats


def test_serving_results_same_alone_and_in_mix():
    insts = [I.torus(30, 30, 201), I.torus(25, 31, 202), I.random_graph(1200, 1200, 203),
             I.torus(48, 40, 204), I.torus(15, 15, 205)]
    probs = [B.Problem.from_instance(x) for x in insts]
    S = 400
    sched = B.Schedule.make(B.LINEAR, S, 0.1, 3.0)
    reqs = []
    for i, p in enumerate(probs):
        R, seed = 64 + 32 * (i % 3), 300 + i
        # even requests run the full schedule; odd ones stop at a target
        # slightly below what their full schedule reaches
        target = 10 ** 9
        if i % 2 == 1:
            p.anneal(sched, R, seed, B.Tuning(B.PATH_FIELD, 1, 256, 2))
            target = int(0.97 * B.ising_cut(p.handle, R)[0])
        reqs.append((p, sched, R, seed, target, 50))
    mixed, stats = _serve(reqs, chunk=37, slots=3)
    assert stats[2] <= 3
    for req, res in zip(reqs, mixed):
        alone, _ = _serve([req], chunk=64)
        assert alone[0][:4] == res[:4]
        np.testing.assert_array_equal(alone[0][4], res[4])
        # and equal to a one-shot anneal of the sweeps it ran
        p, s, R, seed, target, ce = req
        done = res[2]
        betas = O.schedule(O.LINEAR, S, 0.1, 3.0)[:done]
        p.anneal(B.Schedule.make(betas=betas), R, seed, B.Tuning(B.PATH_FIELD, 1, 256, 2))
        best, arg, per = B.ising_cut(p.handle, R)
        assert (best, arg) == (res[0], res[1])
        np.testing.assert_array_equal(p.best_state(), res[4])
        if target < 10 ** 9:
            assert res[3] == 1 and res[0] >= target and done % 50 == 0
    for p in probs:
        p.close()


def test_serving_admission_under_memory_pressure():
    insts = [I.torus(40, 40, 300 + i) for i in range(6)]
    probs = [B.Problem.from_instance(x) for x in insts]
    sched = B.Schedule.make(B.LINEAR, 200, 0.1, 3.0)
    fp = B.ising_server_footprint(probs[0].handle, sched, 128)
    reqs = [(p, sched, 128, 500 + i, 10 ** 9, 0) for i, p in enumerate(probs)]
    out, stats = _serve(reqs, chunk=25, budget=int(2.5 * fp), slots=6)
    assert 1 <= stats[2] <= 2
    for (p, s, R, seed, *_), res in zip(reqs, out):
        p.anneal(s, R, seed, B.Tuning(B.PATH_PLAIN, 1, 256, 0))
        assert B.ising_cut(p.handle, R)[0] == res[0]
    for p in probs:
        p.close()


def test_serving_with_local_fields():
    """Served requests on problems with local fields equal one-shot anneals
    and the oracle (the objective cut + sum b s)."""
    insts = [I.with_fields(I.torus(20, 18, 211), 1, 3), I.torus(16, 16, 212),
             I.with_fields(I.random_graph(600, 700, 213), 2, 2, 0.5)]
    probs = [B.Problem.from_instance(x) for x in insts]
    S = 200
    sched = B.Schedule.make(B.LINEAR, S, 0.1, 3.0)
    reqs = [(p, sched, 32, 400 + i, 10 ** 9, 50) for i, p in enumerate(probs)]
    mixed, _ = _serve(reqs, chunk=37, slots=2)
    for x, req, res in zip(insts, reqs, mixed):
        p, s, R, seed, target, ce = req
        o = O.anneal(x, S, R, seed, kind=O.LINEAR, beta0=0.1, beta1=3.0)
        assert res[0] == int(o.best_cut.max()) and res[1] == o.argmax()
        np.testing.assert_array_equal(res[4], o.best_state[o.argmax()])
    for p in probs:
        p.close()


@pytest.mark.parametrize("form", ["msc4_w8_b256", "autotuned", "msc"])
def test_c4_full_size_batch_sampled(form):
    """The 64-torus batch at full size (sides uniform in 32..141, 128
    replicas, 4000 sweeps geometric 0.1 -> 4.0) in the launch configuration
    the benchmark's headline runs (the degree-4 multispin form, 8 replicas
    per 256-thread unit, which the autotuner picks there), in whatever the
    autotuner picks here, and in the general multispin form (one 32-replica
    word per unit).  The oracle recomputes two replicas each of the
    smallest, a middle and the largest problem."""
    insts = I.workload_c4()
    S, R = 4000, 128
    sched = B.Schedule.make(B.GEOMETRIC, S, 0.1, 4.0)
    probs = [B.Problem.from_instance(x) for x in insts]
    hs = [p.handle for p in probs]
    seeds = np.array([2000 + i for i in range(len(insts))], np.uint64)
    tun = {"autotuned": lambda: B.ising_autotune(hs, sched, R, prefix_sweeps=200),
           "msc4_w8_b256": lambda: B.Tuning(B.PATH_MSC, 8, 256, 0),
           "msc": lambda: B.Tuning(B.PATH_MSC, 1, 256, 0)}[form]()
    B.ising_anneal_batch(hs, sched, R, seeds, tun)
    order = np.argsort([x.n for x in insts], kind="stable")
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        p = probs[i]
        _, _, per = B.ising_cut(p.handle, R)
        bs, acc, en = p.replica_results()
        for r in (i % R, R - 1 - i % 7):
            o = O.anneal(insts[i], S, R, int(seeds[i]), kind=O.GEOMETRIC, beta0=0.1, beta1=4.0,
                         r_begin=r, r_end=r + 1)
            assert (per[r], bs[r], acc[r], en[r]) == (o.best_cut[0], o.best_sweep[0], o.accepts[0],
                                                      o.final_energy[0]), (insts[i].name, r)
            gb, gf = p.replica_state(r)
            np.testing.assert_array_equal(gb, o.best_state[0], err_msg=f"{insts[i].name} r={r}")
            np.testing.assert_array_equal(gf, o.final_state[0], err_msg=f"{insts[i].name} r={r}")
    for p in probs:
        p.close()


def test_c5_full_size_serving_sampled():
    """Serving at full size, in the benchmark's server configuration (96 MiB
    budget, 16 slots, chunks of 50 sweeps): two requests of each of the five
    shapes (tori of 8,000 to 20,000 vertices, the random 10,000-vertex
    graph), 256 replicas, up to 1000 sweeps linear 0.1 -> 3.0, submitted at
    once.  Odd requests stop at a target (checked every 50 sweeps).  Each
    result equals a one-shot anneal of the sweeps it ran, and the oracle
    recomputes the served best replica and one other replica of each."""
    from paper_2311_09275_amd import serve_load
    insts = [mk() for _, mk in serve_load.SHAPES]
    probs = [B.Problem.from_instance(x) for x in insts]
    S, R = 1000, 256
    sched = B.Schedule.make(B.LINEAR, S, 0.1, 3.0)
    reqs = []
    for i in range(2 * len(insts)):
        k = i % len(insts)
        target = 10 ** 9
        if i % 2 == 1:
            probs[k].anneal(B.Schedule.make(B.LINEAR, S, 0.1, 3.0), R, 900 + i,
                            B.Tuning(B.PATH_FIELD, 1, 512, 2))
            target = int(0.98 * B.ising_cut(probs[k].handle, R)[0])
        reqs.append((probs[k], sched, R, 900 + i, target, 50))
    served, stats = _serve(reqs, chunk=50, budget=96 << 20, slots=16)
    betas_all = O.schedule(O.LINEAR, S, 0.1, 3.0)
    for i, (req, res) in enumerate(zip(reqs, served)):
        p, _, _, seed, target, _ = req
        k = i % len(insts)
        best, arg, done, reached, state = res
        if target < 10 ** 9:
            assert reached == 1 and best >= target and done % 50 == 0 and done <= S
        else:
            assert done == S
        # one-shot anneal of the sweeps the request ran
        p.anneal(B.Schedule.make(betas=betas_all[:done]), R, seed, B.Tuning(B.PATH_FIELD, 1, 512, 2))
        b1, a1, per = B.ising_cut(p.handle, R)
        assert (b1, a1) == (best, arg)
        np.testing.assert_array_equal(p.best_state(), state)
        for r in (arg, (arg + 101) % R):
            o = O.anneal(insts[k], done, R, seed, betas=betas_all[:done], kind=O.EXPLICIT,
                         r_begin=r, r_end=r + 1)
            assert per[r] == o.best_cut[0], (insts[k].name, i, r)
            if r == arg:
                np.testing.assert_array_equal(state, o.best_state[0])
    for p in probs:
        p.close()


def test_back_to_back_batches_on_two_streams():
    """Two batches of disjoint problems enqueued back to back on two streams
    (no host wait between them) share the batch launch structures; each
    must still equal separate anneals."""
    import torch
    sA, sB = torch.cuda.Stream(), torch.cuda.Stream()
    sched = B.Schedule.make(B.GEOMETRIC, 400, 0.1, 4.0)
    R = 32
    insts_a = [I.torus(40, 40, 121), I.torus(17, 23, 122), I.random_graph(800, 799, 123)]
    insts_b = [I.torus(12, 12, 124), I.torus(30, 31, 125)]
    seeds_a = np.array([7200 + i for i in range(len(insts_a))], np.uint64)
    seeds_b = np.array([7300 + i for i in range(len(insts_b))], np.uint64)
    pa = [B.Problem.from_instance(x) for x in insts_a]
    pb = [B.Problem.from_instance(x) for x in insts_b]
    tun = B.Tuning(B.PATH_FIELD, 1, 512, 0)
    for _ in range(2):
        B.ising_anneal_batch([p.handle for p in pa], sched, R, seeds_a, tun, stream=sA)
        B.ising_anneal_batch([p.handle for p in pb], sched, R, seeds_b, tun, stream=sB)
    torch.cuda.synchronize()
    for insts, probs, seeds in ((insts_a, pa, seeds_a), (insts_b, pb, seeds_b)):
        for i, (inst, p) in enumerate(zip(insts, probs)):
            per, bs, acc, en, state = _single(inst, sched, R, int(seeds[i]),
                                              B.Tuning(B.PATH_PLAIN, 1, 256, 0))
            np.testing.assert_array_equal(B.ising_cut(p.handle, R)[2], per, err_msg=inst.name)
            bs_b, acc_b, en_b = p.replica_results()
            np.testing.assert_array_equal(acc_b, acc, err_msg=inst.name)
            np.testing.assert_array_equal(en_b, en, err_msg=inst.name)
            np.testing.assert_array_equal(p.best_state(), state, err_msg=inst.name)
    for p in pa + pb:
        p.close()


def test_batch_schedule_changes_between_calls():
    """Each problem keeps its threshold table while its schedule repeats; a
    batch with another schedule (and then the first one again, and a single
    anneal of one member in between) must use the right table every time.
    Twenty problems, so that the whole-problem unit lists are used too."""
    insts = [I.torus(12 + i, 14 + (i % 5), 800 + i) for i in range(20)]
    probs = [B.Problem.from_instance(x) for x in insts]
    hs = [p.handle for p in probs]
    R = 16
    seeds = np.array([8100 + i for i in range(len(insts))], np.uint64)
    sa = B.Schedule.make(B.GEOMETRIC, 120, 0.1, 4.0)
    sb = B.Schedule.make(B.LINEAR, 90, 0.05, 2.0)
    tun = B.Tuning(B.PATH_MSC, 8, 256, 0)
    checks = [(sa, O.GEOMETRIC, 120, 0.1, 4.0), (sb, O.LINEAR, 90, 0.05, 2.0),
              (sa, O.GEOMETRIC, 120, 0.1, 4.0)]
    for step, (sched, kind, S, b0, b1) in enumerate(checks):
        B.ising_anneal_batch(hs, sched, R, seeds, tun)
        for i in (0, 7, 19):
            o = O.anneal(insts[i], S, R, int(seeds[i]), kind=kind, beta0=b0, beta1=b1)
            np.testing.assert_array_equal(B.ising_cut(hs[i], R)[2], o.best_cut, err_msg=f"step {step} problem {i}")
        if step == 0:
            # a single anneal of a member with the other schedule
            probs[7].anneal(sb, R, int(seeds[7]), B.Tuning(B.PATH_FIELD, 1, 256, 0))
            o = O.anneal(insts[7], 90, R, int(seeds[7]), kind=O.LINEAR, beta0=0.05, beta1=2.0)
            np.testing.assert_array_equal(B.ising_cut(hs[7], R)[2], o.best_cut)
    for p in probs:
        p.close()
