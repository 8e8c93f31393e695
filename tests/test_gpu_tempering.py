"""Parallel tempering on the HIP path vs the CPU oracle, through the C ABI.

Compared exactly: every replica's best cut, best sweep, accepted flips and
final energy, the final temperature of every replica, every pair's
accepted exchanges, and best and final states.  Runs on an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_09275_amd import instances as I

pytestmark = pytest.mark.gpu

from tests.conftest import load_binding

B = load_binding()

PATHS = {
    "auto": None,
    "plain": B.Tuning(B.PATH_PLAIN, 1, 256, 0),
    "field_g1_b256_hbmadj": B.Tuning(B.PATH_FIELD, 1, 256, 2),
    "field_g1_b1024_ldsadj": B.Tuning(B.PATH_FIELD, 1, 1024, 1),
    "field_g1_b512_csradj": B.Tuning(B.PATH_FIELD, 1, 512, 3),
    "field_g4_b256_ldsadj": B.Tuning(B.PATH_FIELD, 4, 256, 1),
    "field_g2_b512_hbmadj": B.Tuning(B.PATH_FIELD, 2, 512, 2),
    "field_g1_b512_hbmdeg4": B.Tuning(B.PATH_FIELD, 1, 512, 4),
}


def compare(inst, betas, n_sets, S, P, seed, tuning=None, sets=None, states=True, init=None,
            cluster_from=None):
    """Run tempering on the GPU and check it against the oracle (on the
    sets (begin, end) when given, else on all)."""
    if tuning is not None and tuning.lds_adjacency == 4:
        deg = np.bincount(np.concatenate([inst.u, inst.v]), minlength=inst.n)
        if not (deg == 4).all() or not (np.abs(inst.w) == 1).all():
            pytest.skip("the degree-4 form needs a 4-regular unit-weight graph")
    if tuning is not None and tuning.lds_adjacency in (1, 3) and not (np.abs(inst.w) == 1).all():
        pytest.skip("the adjacency staged in LDS needs unit weights")
    K = len(betas)
    R = K * n_sets
    p = B.Problem.from_instance(inst)
    if init is not None:
        p.set_initial_state(init, R)
    p.temper(betas, n_sets, S, P, seed, tuning, cluster_from=cluster_from)
    best, arg, per = B.ising_cut(p.handle, R)
    bs, acc, en = p.replica_results()
    if cluster_from is None:
        temp, swaps = p.temper_results()
    else:
        temp, swaps, cmoves, csites = p.temper_results()
    assert p.R == R and p.S == S
    s0, s1 = (0, n_sets) if sets is None else sets
    o = O.temper(inst, betas, n_sets, S, P, seed, init_spins=init, n_threads=4,
                 want_states=states, sets=None if sets is None else sets,
                 cluster_from=cluster_from)
    if cluster_from is not None:
        assert o.check_failures == 0
        ps = slice(s0 // 2, s1 // 2)  # the pairs inside the checked sets
    rs = slice(s0 * K, s1 * K)
    np.testing.assert_array_equal(per[rs], o.best_cut[rs])
    np.testing.assert_array_equal(bs[rs], o.best_sweep[rs])
    np.testing.assert_array_equal(acc[rs], o.accepts[rs])
    np.testing.assert_array_equal(en[rs], o.final_energy[rs])
    np.testing.assert_array_equal(temp[rs], o.final_temp[rs])
    np.testing.assert_array_equal(swaps[s0:s1], o.swaps[s0:s1])
    if cluster_from is not None:
        np.testing.assert_array_equal(cmoves[ps], o.cluster_moves[ps])
        np.testing.assert_array_equal(csites[ps], o.cluster_sites[ps])
    if states:
        for r in list(range(s0 * K, s1 * K))[:: max(1, (s1 - s0) * K // 12)]:
            gb, gf = p.replica_state(r)
            np.testing.assert_array_equal(gb, o.best_state[r], err_msg=f"best state r={r}")
            np.testing.assert_array_equal(gf, o.final_state[r], err_msg=f"final state r={r}")
    if sets is None:
        assert best == per.max() and arg == int(np.argmax(per))
        assert p.eval_cut(p.best_state()) == best
    p.close()
    return o


@pytest.mark.parametrize("path", list(PATHS))
def test_torus16(path):
    """16x16 +-1 torus, 8 temperatures geometric 0.2 -> 2.0, 4 sets, a round
    every 5 sweeps."""
    compare(I.workload_c1(), list(np.geomspace(0.2, 2.0, 8)), 4, 200, 5, 31, PATHS[path])


@pytest.mark.parametrize("path", list(PATHS))
def test_odd_torus_partial_last_segment(path):
    """7x9 torus (three ragged classes); S = 120 is not a multiple of P = 7,
    so the last segment has no exchange round after it."""
    o = compare(I.torus(7, 9, 5), [0.1, 0.4, 0.8, 1.5, 3.0], 3, 120, 7, 32, PATHS[path])
    assert o.swaps.sum() > 0


@pytest.mark.parametrize("path", [p for p in PATHS if p != "field_g1_b512_hbmdeg4"])
def test_random_graph_every_sweep(path):
    """Sparse random graph with isolated vertices, a round after every sweep."""
    compare(I.random_graph(300, 299, 8), list(np.linspace(0.1, 2.5, 6)), 3, 150, 1, 33,
            PATHS[path])


@pytest.mark.parametrize("path", ["auto", "plain", "field_g1_b256_hbmadj", "field_g2_b512_hbmadj"])
def test_weighted_graph(path):
    """|w| up to 5: exchange thresholds over cut differences above 1."""
    compare(I.random_weighted(400, 1000, 12, 5), [0.05, 0.1, 0.2, 0.35, 0.6], 4, 100, 3, 34,
            PATHS[path])


@pytest.mark.parametrize("path", ["auto", "plain", "field_g4_b256_ldsadj"])
def test_equal_betas_and_single_temperature(path):
    """Equal betas: every exchange is accepted (the ladders reverse after K
    rounds).  One temperature: no exchange kernel runs at all."""
    o = compare(I.torus(10, 8, 2), [0.7] * 4, 3, 41, 10, 35, PATHS[path])
    assert (o.swaps == 2).all()
    compare(I.torus(10, 8, 2), [0.7], 5, 30, 4, 36, PATHS[path])


def test_zero_beta_rung_and_given_initial_states():
    """A beta = 0 rung accepts every flip; initial states given by the caller."""
    inst = I.torus(12, 12, 6)
    K, n_sets = 4, 3
    init = I.random_spins(17, K * n_sets, inst.n)
    compare(inst, [0.0, 0.5, 1.0, 2.0], n_sets, 80, 2, 37, None, init=init)


def test_repeated_runs_reuse_the_graph():
    """Two runs with different seeds and one with a different ladder on one
    problem: the captured graph must carry each run's exchange arguments."""
    inst = I.torus(16, 12, 7)
    for seed, betas in [(41, [0.3, 0.6, 1.2]), (42, [0.3, 0.6, 1.2]), (42, [0.2, 0.9, 1.0])]:
        compare(inst, betas, 4, 60, 4, seed, None)


def test_full_size_torus_sampled_sets():
    """The benchmark shape: 100x80 torus, 32 temperatures geometric
    0.2 -> 3.0, 8 sets (256 replicas), a round every 10 sweeps; the oracle
    checks two of the sets over 1000 sweeps."""
    compare(I.workload_c2(), list(np.geomspace(0.2, 3.0, 32)), 8, 1000, 10, 1002, None,
            sets=(3, 5), states=False)


def test_full_size_torus_whole_run_one_set():
    """The benchmark's tempering run at its full length (100x80 torus, 32
    temperatures, 8 sets, a round every 10 sweeps, 4000 sweeps, the
    automatic configuration): the oracle checks the last set."""
    compare(I.workload_c2(), list(np.geomspace(0.2, 3.0, 32)), 8, 4000, 10, 1002, None,
            sets=(7, 8), states=False)


def test_errors_and_state():
    inst = I.torus(8, 8, 1)
    p = B.Problem.from_instance(inst)
    with pytest.raises(B.IsingError) as e:
        p.temper([0.1, 0.5], 2, 10, 1, 1, B.Tuning(B.PATH_MSC, 1, 256, 0))
    assert e.value.status == B.ERR_UNSUPPORTED
    p.set_trace(True)
    with pytest.raises(B.IsingError) as e:
        p.temper([0.1, 0.5], 2, 10, 1, 1)
    assert e.value.status == B.ERR_UNSUPPORTED
    p.set_trace(False)
    p.temper([0.1, 0.5], 2, 10, 1, 1)
    p.temper_results()
    p.anneal(B.Schedule.make(B.LINEAR, 10, 0.1, 1.0), 4, 1)
    with pytest.raises(B.IsingError) as e:
        p.temper_results()
    assert e.value.status == B.ERR_STATE
    p.close()


# ---------------------------------------------------------------- cluster moves
CLUSTER_PATHS = ["auto", "plain", "field_g1_b256_hbmadj", "field_g1_b1024_ldsadj",
                 "field_g1_b512_csradj", "field_g4_b256_ldsadj", "field_g2_b512_hbmadj"]


@pytest.mark.parametrize("path", CLUSTER_PATHS)
def test_cluster_moves_torus(path):
    """Houdayer moves at the four coldest of 8 temperatures, 6 sets (3
    pairs), a round every 4 sweeps (the moves change the replicas' states,
    fields and energies between launches)."""
    o = compare(I.torus(14, 10, 41), list(np.geomspace(0.2, 2.5, 8)), 6, 120, 4, 51, PATHS[path],
                cluster_from=4)
    assert (o.cluster_moves[:, 4:] > 0).all()


@pytest.mark.parametrize("path", [p for p in CLUSTER_PATHS if PATHS.get(p) is None or
                                  PATHS[p].lds_adjacency not in (1, 3)])
def test_cluster_moves_every_temperature_odd_sets(path):
    """Moves at every temperature and after every sweep, on a weighted
    random graph with isolated vertices (the LDS adjacency forms need unit
    weights); 5 sets, the last without a partner."""
    compare(I.random_weighted(300, 330, 17, 4), [0.1, 0.3, 0.7, 1.4], 5, 60, 1, 52, PATHS[path],
            cluster_from=0)


@pytest.mark.parametrize("path", CLUSTER_PATHS)
def test_cluster_moves_unit_random_graph(path):
    compare(I.random_graph(300, 330, 18), [0.1, 0.3, 0.7, 1.4], 5, 60, 1, 53, PATHS[path],
            cluster_from=1)


def test_cluster_moves_full_size_sampled_pairs():
    """The benchmark torus shape with moves at the 16 coldest of 32
    temperatures: the oracle checks one pair of sets over 400 sweeps."""
    compare(I.workload_c2(), list(np.geomspace(0.2, 3.0, 32)), 8, 400, 10, 1002, None,
            sets=(2, 4), states=False, cluster_from=16)


def test_cluster_moves_full_size_whole_run_one_pair():
    """The benchmark's run with cluster moves at its full length (moves at
    the 16 coldest of 32 temperatures, a round every 10 sweeps, 4000
    sweeps): the oracle checks one pair of sets."""
    compare(I.workload_c2(), list(np.geomspace(0.2, 3.0, 32)), 8, 4000, 10, 1002, None,
            sets=(6, 8), states=False, cluster_from=16)


@pytest.mark.parametrize("path", ["plain", "field_g1_b256_hbmadj"])
def test_interval_longer_than_run(path):
    """P > S: no exchange round at all; every replica anneals at its
    starting temperature."""
    o = compare(I.torus(9, 8, 4), [0.3, 0.9, 1.8], 2, 25, 40, 54, PATHS[path])
    assert (o.swaps == 0).all()
    np.testing.assert_array_equal(o.final_temp, np.tile(np.arange(3), 2))
