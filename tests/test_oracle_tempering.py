"""Pins of the parallel-tempering oracle (replica exchange, paper Sec. II.C)
against facts that do not come from the oracle: reductions to the pinned
annealing oracle, the closed form of an exchange pattern that always
accepts, exact enumeration of the stationary energies at every temperature
and of the exchange acceptance rates, and the acceptance frequency of the
exchange test itself.  CPU only."""
import math

import numpy as np
import pytest

from paper_2311_09275_amd import instances as I


def _anneal_const(O, inst, beta, R, S, seed):
    return O.anneal(inst, S, R, seed, kind=O.EXPLICIT, betas=np.full(S, beta))


def test_single_temperature_is_constant_beta_anneal(oracle_lib):
    """K = 1: no exchanges exist, so each set is one replica annealed at a
    constant beta, with the same Philox streams (replica r = set r)."""
    O = oracle_lib
    inst = I.torus(8, 6, 3)
    R, S = 6, 40
    pt = O.temper(inst, [0.6], n_sets=R, n_sweeps=S, swap_every=3, seed=11)
    an = _anneal_const(O, inst, 0.6, R, S, 11)
    np.testing.assert_array_equal(pt.best_cut, an.best_cut)
    np.testing.assert_array_equal(pt.best_sweep, an.best_sweep)
    np.testing.assert_array_equal(pt.accepts, an.accepts)
    np.testing.assert_array_equal(pt.final_energy, an.final_energy)
    np.testing.assert_array_equal(pt.best_state, an.best_state)
    np.testing.assert_array_equal(pt.final_state, an.final_state)
    assert (pt.final_temp == 0).all()
    assert pt.swaps.shape == (R, 0)


@pytest.mark.parametrize("K,rounds_in_units_of_K", [(5, 1), (5, 2), (4, 1), (4, 3), (2, 1)])
def test_equal_betas_always_exchange(oracle_lib, K, rounds_in_units_of_K):
    """All betas equal: every exchange has ratio 1 and is accepted.  The
    spin dynamics then cannot depend on the labels, so every replica equals
    a constant-beta anneal; and alternating even/odd transpositions that
    always swap reverse a sequence of K items after K rounds (the classical
    odd-even transposition network), restoring it after 2K."""
    O = oracle_lib
    inst = I.random_weighted(40, 70, 5, 2)
    n_sets, P = 3, 2
    rounds = rounds_in_units_of_K * K
    S = rounds * P + 1  # one more sweep after the last round
    pt = O.temper(inst, [0.8] * K, n_sets=n_sets, n_sweeps=S, swap_every=P, seed=21)
    an = _anneal_const(O, inst, 0.8, n_sets * K, S, 21)
    np.testing.assert_array_equal(pt.best_cut, an.best_cut)
    np.testing.assert_array_equal(pt.final_energy, an.final_energy)
    np.testing.assert_array_equal(pt.final_state, an.final_state)
    j = np.arange(K)
    want = K - 1 - j if rounds_in_units_of_K % 2 else j
    for s in range(n_sets):
        np.testing.assert_array_equal(pt.final_temp[s * K:(s + 1) * K], want)
    # pair k is tried in the rounds m < rounds with m = k (mod 2)
    tries = np.array([len(range(k % 2, rounds, 2)) for k in range(K - 1)])
    for s in range(n_sets):
        np.testing.assert_array_equal(pt.swaps[s], tries)


def test_exchange_test_frequencies(oracle_lib):
    """The exchange of a pair whose colder replica has the better cut by q
    is accepted with probability exp(-2 q dbeta) (the Metropolis ratio of
    the product of Boltzmann weights); q <= 0 and dbeta = 0 always accept."""
    O = oracle_lib
    n = 20000
    for q, b0, b1 in [(1, 0.3, 0.5), (3, 1.0, 1.1), (2, 0.05, 0.4)]:
        Ea, Eb = 2 * q, 0  # q = (Ea - Eb) / 2
        acc = sum(O.swap_accept(77, m, 1, 2, Ea, Eb, b0, b1) for m in range(n))
        p = math.exp(-2 * q * (b1 - b0))
        se = math.sqrt(p * (1 - p) / n)
        assert abs(acc / n - p) < 5 * se + 1e-9, (q, acc / n, p)
        # the sign matters: the opposite exponent would be > 1 and accept all
        assert acc < n
    for m in range(50):
        assert O.swap_accept(3, m, 0, 0, -6, 10, 0.2, 3.0)   # colder already worse
        assert O.swap_accept(3, m, 0, 0, 4, 4, 0.2, 3.0)     # equal energies
        assert O.swap_accept(3, m, 0, 0, 400, 0, 0.7, 0.7)   # equal betas
        assert not O.swap_accept(3, m, 0, 0, 400, 0, 0.0, 1.0)  # exp(-400) -> Tq = 0


def _levels(inst):
    n = inst.n
    states = ((np.arange(1 << n)[:, None] >> np.arange(n)) & 1).astype(np.int64) * 2 - 1
    E = np.zeros(1 << n, np.int64)
    for a, b, w in zip(inst.u, inst.v, inst.w):
        E += w * states[:, a] * states[:, b]
    return E


def test_stationary_energies_and_exchange_rates(oracle_lib):
    """Each sweep and each exchange leave the product of the K Boltzmann
    distributions invariant, so in the long run the replica found at
    temperature k has energies distributed as exp(-beta_k E)/Z, and pair
    (k, k+1) exchanges at the rate sum_ab pi_k(a) pi_k+1(b) min(1, ratio),
    both computed here by enumerating all 2^n states."""
    O = oracle_lib
    inst = I.random_weighted(9, 16, 51, 3)
    betas = np.array([0.1, 0.3, 0.6])
    K, n_sets, S, P, burn = len(betas), 8, 40000, 1, 500
    pt = O.temper(inst, betas, n_sets=n_sets, n_sweeps=S, swap_every=P, seed=99,
                  n_threads=4, want_states=False, want_temp_energy=True)
    E = _levels(inst)
    x = pt.temp_energy[:, burn:, :].astype(np.float64)  # [sets, t, K]
    nb = 50
    for k, b in enumerate(betas):
        wgt = np.exp(-b * (E - E.min()))
        exact = float((wgt * E).sum() / wgt.sum())
        per_batch = x[:, :, k].reshape(n_sets, nb, -1).mean(axis=2).ravel()
        mean = per_batch.mean()
        se = per_batch.std(ddof=1) / math.sqrt(per_batch.size)
        assert abs(mean - exact) < 5 * se, (k, mean, exact, se)
        # a temperature mix-up must be detectable: the neighbours' means
        for b2 in set(betas) - {b}:
            w2 = np.exp(-b2 * (E - E.min()))
            other = float((w2 * E).sum() / w2.sum())
            assert abs(mean - other) > 8 * se
    rounds = S // P
    for k in range(K - 1):
        pa = np.exp(-betas[k] * (E - E.min()))
        pa /= pa.sum()
        pb = np.exp(-betas[k + 1] * (E - E.min()))
        pb /= pb.sum()
        ratio = np.minimum(1.0, np.exp(-(betas[k + 1] - betas[k]) * (E[:, None] - E[None, :])))
        rate = float(pa @ ratio @ pb)
        tries = len(range(k % 2, rounds, 2)) * n_sets
        got = pt.swaps[:, k].sum() / tries
        se = math.sqrt(rate * (1 - rate) / tries)
        assert abs(got - rate) < 6 * se, (k, got, rate)


def test_threads_agree(oracle_lib):
    O = oracle_lib
    inst = I.torus(6, 6, 8)
    a = O.temper(inst, [0.2, 0.5, 1.0, 1.6], n_sets=5, n_sweeps=60, swap_every=4, seed=5)
    b = O.temper(inst, [0.2, 0.5, 1.0, 1.6], n_sets=5, n_sweeps=60, swap_every=4, seed=5,
                 n_threads=3)
    for f in ("best_cut", "best_sweep", "accepts", "final_energy", "final_temp", "swaps",
              "best_state", "final_state"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))


def test_best_cut_matches_state(oracle_lib):
    O = oracle_lib
    inst = I.random_weighted(50, 90, 9, 4)
    pt = O.temper(inst, [0.1, 0.4, 0.9, 2.0], n_sets=3, n_sweeps=80, swap_every=5, seed=6)
    for r in range(12):
        assert O.cut(inst, pt.best_state[r]) == pt.best_cut[r]
        assert O.cut(inst, pt.final_state[r]) == (inst.w.sum() - pt.final_energy[r]) // 2
    # every set's temperatures remain a permutation
    for s in range(3):
        assert sorted(pt.final_temp[4 * s:4 * s + 4]) == [0, 1, 2, 3]


@pytest.mark.parametrize("betas,n_sets,S,P", [([0.5, 0.4], 1, 10, 1), ([], 1, 10, 1),
                                               ([0.1, -0.2], 1, 10, 1), ([0.1], 0, 10, 1),
                                               ([0.1], 1, 0, 1), ([0.1], 1, 10, 0),
                                               ([0.1, float("inf")], 1, 10, 1)])
def test_rejects(oracle_lib, betas, n_sets, S, P):
    O = oracle_lib
    with pytest.raises(ValueError):
        O.temper(I.torus(4, 4, 1), np.array(betas, np.float64), n_sets=n_sets, n_sweeps=S,
                 swap_every=P, seed=1)


# ---------------------------------------------------------------- cluster moves
def _component(inst, sa, sb, i0):
    """The component of i0 in the subgraph induced by the disagreeing sites,
    by scipy's connected components."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    d = sa != sb
    keep = d[inst.u] & d[inst.v]
    n = inst.n
    A = coo_matrix((np.ones(int(keep.sum())), (inst.u[keep], inst.v[keep])), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    if not d[i0]:
        return np.zeros(n, np.uint8)
    return ((lab == lab[i0]) & d).astype(np.uint8)


@pytest.mark.parametrize("seed", range(6))
def test_cluster_is_the_induced_component(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.Generator(np.random.PCG64(seed))
    inst = [I.torus(12, 9, seed), I.random_graph(200, 260, seed), I.random_weighted(150, 300, seed, 3)][seed % 3]
    for trial in range(8):
        sa = (rng.integers(0, 2, inst.n) * 2 - 1).astype(np.int8)
        sb = sa.copy()
        flip = rng.random(inst.n) < [0.2, 0.5, 0.8, 1.0][trial % 4]
        sb[flip] = -sb[flip]
        i0 = int(rng.integers(0, inst.n))
        np.testing.assert_array_equal(O.cluster(inst, sa, sb, i0), _component(inst, sa, sb, i0))
    # opposite states on a connected graph: the cluster is every site
    sa = np.ones(inst.n, np.int8) if seed % 3 == 0 else None
    if sa is not None:
        assert O.cluster(inst, sa, -sa, 5).all()


def test_cluster_moves_keep_pair_energy_and_count(oracle_lib):
    """Every move keeps E_a + E_b (checked by the oracle after each move);
    moves happen at temperatures >= cluster_from only, at most one per
    pair, temperature and round."""
    O = oracle_lib
    inst = I.random_weighted(80, 160, 4, 3)
    betas = [0.1, 0.3, 0.7, 1.5]
    S, P, n_sets = 90, 3, 5  # an odd last set has no partner
    pt = O.temper(inst, betas, n_sets, S, P, seed=9, cluster_from=1)
    assert pt.check_failures == 0
    assert pt.cluster_moves.shape == (2, 4)
    assert (pt.cluster_moves[:, 0] == 0).all()
    assert (pt.cluster_moves[:, 1:] > 0).all() and (pt.cluster_moves <= S // P).all()
    assert (pt.cluster_sites >= pt.cluster_moves).all()
    assert (pt.cluster_sites <= inst.n * pt.cluster_moves).all()
    for s in range(n_sets):
        assert sorted(pt.final_temp[4 * s:4 * s + 4]) == [0, 1, 2, 3]
    for r in range(n_sets * 4):
        assert O.cut(inst, pt.best_state[r]) == pt.best_cut[r]
        assert O.cut(inst, pt.final_state[r]) == (inst.w.sum() - pt.final_energy[r]) // 2
    # the unpaired last set runs exactly as without cluster moves
    plain = O.temper(inst, betas, n_sets, S, P, seed=9)
    np.testing.assert_array_equal(pt.best_cut[16:], plain.best_cut[16:])
    np.testing.assert_array_equal(pt.swaps[4], plain.swaps[4])
    assert (pt.best_cut[:16] != plain.best_cut[:16]).any() or \
           (pt.final_energy[:16] != plain.final_energy[:16]).any()


def test_stationary_energies_with_cluster_moves(oracle_lib):
    """Cluster moves keep the product of the Boltzmann distributions at each
    temperature invariant (a symmetric proposal that keeps E_a + E_b): the
    long-run mean energy at every temperature still equals exact
    enumeration."""
    O = oracle_lib
    inst = I.random_weighted(9, 16, 51, 3)
    betas = np.array([0.1, 0.3, 0.6])
    K, n_sets, S, burn = len(betas), 8, 40000, 500
    pt = O.temper(inst, betas, n_sets=n_sets, n_sweeps=S, swap_every=1, seed=98, n_threads=4,
                  want_states=False, want_temp_energy=True, cluster_from=0)
    assert pt.check_failures == 0 and (pt.cluster_moves > 0).all()
    E = _levels(inst)
    x = pt.temp_energy[:, burn:, :].astype(np.float64)
    for k, b in enumerate(betas):
        wgt = np.exp(-b * (E - E.min()))
        exact = float((wgt * E).sum() / wgt.sum())
        per_batch = x[:, :, k].reshape(n_sets, 50, -1).mean(axis=2).ravel()
        se = per_batch.std(ddof=1) / math.sqrt(per_batch.size)
        assert abs(per_batch.mean() - exact) < 5 * se, (k, per_batch.mean(), exact, se)


def test_cluster_moves_need_whole_pairs(oracle_lib):
    O = oracle_lib
    with pytest.raises(ValueError):
        O.temper(I.torus(6, 6, 1), [0.2, 0.5], 4, 10, 2, 1, sets=(1, 3), cluster_from=0)
    with pytest.raises(ValueError):
        O.temper(I.torus(6, 6, 1), [0.2, 0.5], 4, 10, 2, 1, cluster_from=3)
