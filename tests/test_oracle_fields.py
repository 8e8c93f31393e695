"""Pins of the oracle's local fields (E = sum w s s - 2 sum b s; the paper
notes that some sparse Ising problems have local fields, Sec. II.C):
brute force, the Boltzmann distribution, an isolated spin's closed form,
gauge invariance, and the reduction to no fields.  CPU only."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from paper_2311_09275_amd import instances as I


def _objective(inst, s):
    """cut(s) + sum_v b_v s_v."""
    s = np.asarray(s, np.int64)
    cut = int(inst.w[s[inst.u] != s[inst.v]].astype(np.int64).sum())
    return cut + int((inst.field.astype(np.int64) * s).sum())


def _energies(inst):
    n = inst.n
    states = ((np.arange(1 << n)[:, None] >> np.arange(n)) & 1).astype(np.int64) * 2 - 1
    E = np.zeros(1 << n, np.int64)
    for a, b, w in zip(inst.u, inst.v, inst.w):
        E += w * states[:, a] * states[:, b]
    E -= 2 * states @ inst.field.astype(np.int64)
    return states, E


@pytest.mark.parametrize("inst", [I.with_fields(I.torus(4, 4, 21), 1, 2),
                                  I.with_fields(I.random_weighted(12, 20, 3, 4), 2, 5),
                                  I.with_fields(I.random_graph(14, 16, 5), 3, 1, 0.5)])
def test_brute_force_objective(oracle_lib, inst):
    """The best cut reported is cut + sum b s of the best state, never above
    the brute-force maximum, and reaches it on these small instances."""
    O = oracle_lib
    best = max(_objective(inst, s) for s in itertools.product([-1, 1], repeat=inst.n))
    res = O.anneal(inst, 3000, 16, 7, kind=O.LINEAR, beta0=0.05, beta1=4.0, check=True)
    assert res.check_failures == 0
    for r in range(16):
        assert res.best_cut[r] == _objective(inst, res.best_state[r])
        assert res.best_cut[r] <= best
    assert res.best_cut.max() == best
    # E and the objective: (W - E) / 2 = cut + sum b s for the final state
    W = int(inst.w.sum())
    for r in range(16):
        assert (W - res.final_energy[r]) // 2 == _objective(inst, res.final_state[r])


def test_boltzmann_with_fields(oracle_lib):
    """At fixed beta the end-of-sweep energies follow exp(-beta E)/Z with the
    field term; the same data reject a field of the opposite sign."""
    O = oracle_lib
    inst = I.with_fields(I.random_weighted(9, 14, 52, 3), 4, 3)
    beta = 0.3
    states, E = _energies(inst)
    levels, inv = np.unique(E, return_inverse=True)
    p = np.bincount(inv, weights=np.exp(-beta * (E - E.min())))
    p /= p.sum()
    R, S = 40000, 24
    res = O.anneal(inst, S, R, seed=53, kind=O.EXPLICIT, betas=np.full(S, beta), n_threads=4,
                   want_states=False)
    idx = np.searchsorted(levels, res.final_energy)
    assert (levels[idx] == res.final_energy).all()
    obs = np.bincount(idx, minlength=len(levels)).astype(float)
    exp_ = p * R
    keep = exp_ >= 5
    obs_k = np.append(obs[keep], obs[~keep].sum())
    exp_k = np.append(exp_[keep], exp_[~keep].sum())
    chi2, pval = stats.chisquare(obs_k, exp_k)
    assert pval > 1e-4, (chi2, pval)
    # the states' distribution: the mean magnetisation per vertex
    flipped = I.Instance(inst.name, inst.n, inst.u, inst.v, inst.w, -inst.field)
    _, E2 = _energies(flipped)
    p2 = np.exp(-beta * (E2 - E2.min()))
    p2 /= p2.sum()
    res_s = O.anneal(inst, S, 4000, seed=54, kind=O.EXPLICIT, betas=np.full(S, beta), n_threads=4)
    w_exact = np.exp(-beta * (E - E.min()))
    mag = (w_exact[:, None] * states).sum(0) / w_exact.sum()
    mag_wrong = (p2[:, None] * states).sum(0)
    got = res_s.final_state.mean(axis=0)
    se = 1.0 / math.sqrt(4000)
    assert np.all(np.abs(got - mag) < 5 * se), (got, mag)
    assert np.any(np.abs(got - mag_wrong) > 8 * se)


def test_isolated_spins_closed_form(oracle_lib):
    """No edges: each spin sees only its field, E = -2 b s, so at inverse
    temperature beta P(s = +1) = e^(2 beta b) / (e^(2 beta b) + e^(-2 beta b))."""
    O = oracle_lib
    b = np.array([-3, -1, 0, 1, 2, 5], np.int32)
    inst = I.Instance("fields_only", len(b), np.zeros(0, np.int32), np.zeros(0, np.int32),
                      np.zeros(0, np.int32), b)
    beta, R = 0.2, 20000
    res = O.anneal(inst, 5, R, seed=8, kind=O.EXPLICIT, betas=np.full(5, beta), n_threads=4)
    up = (res.final_state > 0).mean(axis=0)
    p = np.exp(2 * beta * b) / (np.exp(2 * beta * b) + np.exp(-2 * beta * b))
    se = np.sqrt(p * (1 - p) / R) + 1e-12
    assert np.all(np.abs(up - p) < 5 * se), (up, p)
    # beta = infinity: every spin ends along its field (b = 0: accepted, keeps flipping)
    res = O.anneal(inst, 4, 8, seed=9, kind=O.EXPLICIT, betas=np.full(4, 1e6))
    nz = b != 0
    assert (res.final_state[:, nz] == np.sign(b[nz])).all()


def test_gauge_with_fields(oracle_lib):
    """s -> g s with w' = g_i g_j w and b' = g b gives the same energies
    sweep by sweep when the initial states are gauged too."""
    O = oracle_lib
    inst = I.with_fields(I.random_weighted(60, 150, 6, 3), 5, 4)
    g = I.gauge(7, inst.n)
    gi = I.gauge_transform(inst, g)
    gi = I.Instance(gi.name, gi.n, gi.u, gi.v, gi.w, (g.astype(np.int32) * inst.field).astype(np.int32))
    init = I.random_spins(3, 6, inst.n)
    a = O.anneal(inst, 60, 6, 4, kind=O.LINEAR, init_spins=init, want_trace=True)
    b = O.anneal(gi, 60, 6, 4, kind=O.LINEAR, init_spins=(init * g).astype(np.int8), want_trace=True)
    np.testing.assert_array_equal(a.energy_trace, b.energy_trace)
    np.testing.assert_array_equal(a.accepts, b.accepts)
    np.testing.assert_array_equal(b.best_state, a.best_state * g)


def test_zero_fields_are_no_fields(oracle_lib):
    O = oracle_lib
    inst = I.torus(8, 8, 3)
    z = I.Instance(inst.name, inst.n, inst.u, inst.v, inst.w, np.zeros(inst.n, np.int32))
    a = O.anneal(inst, 50, 4, 2, want_trace=True)
    b = O.anneal(z, 50, 4, 2, want_trace=True)
    np.testing.assert_array_equal(a.energy_trace, b.energy_trace)
    np.testing.assert_array_equal(a.best_state, b.best_state)


def test_field_validation(oracle_lib):
    O = oracle_lib
    inst = I.torus(4, 4, 1)
    big = I.Instance(inst.name, inst.n, inst.u, inst.v, inst.w, np.full(inst.n, 40000, np.int32))
    assert not O.validate(big)
    ok = I.Instance(inst.name, inst.n, inst.u, inst.v, inst.w, np.full(inst.n, 32768, np.int32))
    assert O.validate(ok)
    with pytest.raises(ValueError):
        O.temper(I.with_fields(inst, 1, 2), [0.2, 0.5], 2, 10, 2, 1, cluster_from=0)
