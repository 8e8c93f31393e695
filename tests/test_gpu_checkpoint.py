"""Anneals cut into sweep ranges, and checkpoints through host memory, give
the one-shot results bit for bit."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_09275_amd import instances as I

pytestmark = pytest.mark.gpu

from tests.conftest import load_binding

B = load_binding()

TUNINGS = {"plain": B.Tuning(B.PATH_PLAIN, 1, 256, 0), "field_deg4": B.Tuning(B.PATH_FIELD, 1, 256, 1),
           "field_hbm": B.Tuning(B.PATH_FIELD, 2, 512, 2), "msc": B.Tuning(B.PATH_MSC, 1, 256, 0)}


def _results(p, R):
    best, arg, per = B.ising_cut(p.handle, R)
    bs, acc, en = p.replica_results()
    return per.copy(), bs.copy(), acc.copy(), en.copy(), p.best_state().copy()


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("name", list(TUNINGS))
def test_ranges_equal_one_shot(name):
    inst = I.torus(14, 12, 21)
    S, R, seed = 240, 40, 81
    sched = B.Schedule.make(B.GEOMETRIC, S, 0.1, 3.0)
    tun = TUNINGS[name]
    p = B.Problem.from_instance(inst)
    p.set_trace(True)
    p.anneal(sched, R, seed, tun)
    one = _results(p, R)
    trace_one = p.energy_trace()
    for cuts in ([0, 1, 100, 239, 240], [0, 120, 240], [0, 7, 8, 200, 240]):
        for t0, t1 in zip(cuts[:-1], cuts[1:]):
            p.anneal_range(sched, R, seed, t0, t1, tun)
            # results so far: the oracle over the first t1 sweeps
            if t1 == 120:
                o = O.anneal(inst, S, R, seed, kind=O.GEOMETRIC, beta0=0.1, beta1=3.0,
                             want_states=False, want_trace=True)
                np.testing.assert_array_equal(p.energy_trace()[:, :120], o.energy_trace[:, :120])
        _same(_results(p, R), one)
        np.testing.assert_array_equal(p.energy_trace(), trace_one)
    # a continuation must start where the run stopped, with its seed
    p.anneal_range(sched, R, seed, 0, 50, tun)
    for bad in ((seed, 60, 100), (seed + 1, 50, 100)):
        with pytest.raises(B.IsingError) as e:
            p.anneal_range(sched, R, bad[0], bad[1], bad[2], tun)
        assert e.value.status == B.ERR_STATE
    p.close()


@pytest.mark.parametrize("name", ["plain", "field_deg4", "msc"])
def test_checkpoint_restore_in_a_new_problem(name):
    inst = I.random_regular4(300, 22) if name != "plain" else I.random_weighted(300, 700, 22, 3)
    S, R, seed = 200, 64, 82
    sched = B.Schedule.make(B.LINEAR, S, 0.05, 3.0)
    tun = TUNINGS[name]
    if name == "msc":
        tun = B.Tuning(B.PATH_MSC, 1, 256, 0)
    p = B.Problem.from_instance(inst)
    p.anneal(sched, R, seed, tun)
    one = _results(p, R)
    p.anneal_range(sched, R, seed, 0, 90, tun)
    ck = p.checkpoint()
    p.close()
    q = B.Problem.from_instance(inst)
    q.restore(sched, ck)
    q.anneal_range(sched, R, seed, 90, S, tun)
    _same(_results(q, R), one)
    # another schedule is refused
    with pytest.raises(B.IsingError) as e:
        q.restore(B.Schedule.make(B.LINEAR, S, 0.05, 2.0), ck)
    assert e.value.status == B.ERR_INVALID
    q.close()
