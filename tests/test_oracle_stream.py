"""Pins of the oracle's random-number stream (CPU only).

The paper fixes no random stream.  The reading adopted: a vertex's draw for
sweep t, replica r and purpose tag is word rank(v) of Philox4x32-10 with
counter (t, run(v), r, tag) and key = the 64-bit seed, where the runs are
consecutive fours of a colour class taken in ascending id, numbered in
class order and then in id order inside a class.  The stream therefore
depends on the colouring.

These tests fix that layout from outside the oracle:
- hand-written tables of run and rank for small graphs (typed in, not
  computed), including a class longer than four and a supplied colouring;
- the draws, the initial state and a two-sweep trajectory rebuilt from those
  tables and the Philox block function (pinned by its published
  known-answer vectors) and the threshold function (pinned against 50-digit
  arithmetic);
- injectivity of (counter, word) over vertices, sweeps, replicas and tags;
- uniformity and independence of the words by chi-square tests.
"""
import numpy as np
import pytest
from scipy import stats

from paper_2311_09275_amd import instances as I


def _graph(name, n, edges, w=None):
    u = np.array([a for a, _ in edges], np.int32).reshape(-1)
    v = np.array([b for _, b in edges], np.int32).reshape(-1)
    ww = np.ones(len(edges), np.int32) if w is None else np.array(w, np.int32)
    return I.Instance(name, n, u, v, ww)


PATH5 = _graph("path5", 5, [(0, 1), (1, 2), (2, 3), (3, 4)])
STAR12 = _graph("star12", 12, [(0, j) for j in range(1, 12)])

# Written out by hand from the definition (greedy first-fit colouring in id
# order, runs of four inside each class in ascending id, runs numbered
# across classes in class order).
#
# Path 0-1-2-3-4: colours 0 1 0 1 0; class 0 = {0, 2, 4} is run 0,
# class 1 = {1, 3} is run 1.
PATH5_RUN = [0, 1, 0, 1, 0]
PATH5_RANK = [0, 0, 1, 1, 2]
# 3x3 torus (v = 3y + x): first fit gives colours 0 1 2 1 0 3 2 3 0, so the
# classes are {0, 4, 8}, {1, 3}, {2, 6}, {5, 7}, runs 0..3.
TORUS3_RUN = [0, 1, 2, 1, 0, 3, 2, 3, 0]
TORUS3_RANK = [0, 0, 0, 1, 1, 0, 1, 1, 2]
# Star, centre 0, leaves 1..11: colour 0 = {0} (run 0), colour 1 = the 11
# leaves, runs 1, 2, 3 of 4, 4 and 3 leaves.
STAR12_RUN = [0, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3]
STAR12_RANK = [0, 0, 1, 2, 3, 0, 1, 2, 3, 0, 1, 2]
# The same star with a supplied colouring: the centre colour 1, leaf 5
# colour 2, the other leaves colour 0.  Class 0 = {1,2,3,4,6,7,8,9,10,11}
# (runs 0, 1, 2), class 1 = {0} (run 3), class 2 = {5} (run 4).
STAR12_SUPPLIED = [1, 0, 0, 0, 0, 2, 0, 0, 0, 0, 0, 0]
STAR12_SUPPLIED_RUN = [3, 0, 0, 0, 0, 4, 1, 1, 1, 1, 2, 2]
STAR12_SUPPLIED_RANK = [0, 0, 1, 2, 3, 0, 0, 1, 2, 3, 0, 1]

CASES = [
    ("path5", lambda: PATH5, None, PATH5_RUN, PATH5_RANK),
    ("torus3x3", lambda: I.torus(3, 3, seed=5), None, TORUS3_RUN, TORUS3_RANK),
    ("star12", lambda: STAR12, None, STAR12_RUN, STAR12_RANK),
    ("star12_supplied", lambda: STAR12, STAR12_SUPPLIED, STAR12_SUPPLIED_RUN,
     STAR12_SUPPLIED_RANK),
]


def _key(seed):
    return [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]


@pytest.mark.parametrize("name,make,colour,run,rank", CASES, ids=[c[0] for c in CASES])
def test_stream_map_literal_tables(oracle_lib, name, make, colour, run, rank):
    got_run, got_rank = oracle_lib.stream_map(make(), colour)
    assert got_run.tolist() == run
    assert got_rank.tolist() == rank


@pytest.mark.parametrize("name,make,colour,run,rank", CASES, ids=[c[0] for c in CASES])
def test_draws_from_literal_tables(oracle_lib, name, make, colour, run, rank):
    """Every draw is word rank(v) of the block (t, run(v), r, tag)."""
    O = oracle_lib
    inst = make()
    seed = 0x0123456789ABCDEF
    for t, r, tag in [(0, 0, 0), (0, 0, 1), (7, 3, 0), (3999, 255, 0), (0, 1023, 1), (2, 5, 3)]:
        got = O.draws(inst, seed, t, r, tag, colour)
        want = [int(O.philox([t, run[v], r, tag], _key(seed))[rank[v]]) for v in range(inst.n)]
        assert got.tolist() == want, (t, r, tag)


def test_initial_state_uses_init_draws(oracle_lib):
    """At beta = 0 every spin flips in the one sweep, so the final state is
    minus the initial one, whose spin v is +1 exactly when bit 31 of the
    tag-1 draw of sweep 0 is set."""
    O = oracle_lib
    inst = I.torus(3, 3, seed=5)
    R, seed = 6, 99
    o = O.anneal(inst, 1, R, seed, kind=O.EXPLICIT, betas=[0.0])
    for r in range(R):
        init = [1 if int(O.philox([0, TORUS3_RUN[v], r, 1], _key(seed))[TORUS3_RANK[v]]) >> 31 else -1
                for v in range(inst.n)]
        assert o.final_state[r].tolist() == [-s for s in init]


def test_two_sweeps_rebuilt_from_the_tables(oracle_lib):
    """Two sweeps on the 3x3 torus from a given state, recomputed here from
    the literal run/rank table, the Philox block and the threshold: classes
    0..3 in order, vertices of a class in ascending id, k = s h, accept iff
    k <= 0 or draw < Tq(beta_t, k)."""
    O = oracle_lib
    inst = I.torus(3, 3, seed=5)
    classes = [[0, 4, 8], [1, 3], [2, 6], [5, 7]]
    nbr = {v: [] for v in range(inst.n)}
    for a, b, w in zip(inst.u.tolist(), inst.v.tolist(), inst.w.tolist()):
        nbr[a].append((b, w))
        nbr[b].append((a, w))
    betas = [0.4, 0.9]
    R, seed = 5, 0xFEEDFACE12345
    init = I.random_spins(11, R, inst.n)
    o = O.anneal(inst, 2, R, seed, kind=O.EXPLICIT, betas=betas, init_spins=init,
                 want_trace=True)
    for r in range(R):
        s = init[r].astype(int).tolist()
        for t, beta in enumerate(betas):
            for cls in classes:
                for v in cls:
                    h = -sum(w * s[j] for j, w in nbr[v])
                    k = s[v] * h
                    if k <= 0:
                        acc = True
                    else:
                        u = int(O.philox([t, TORUS3_RUN[v], r, 0], _key(seed))[TORUS3_RANK[v]])
                        acc = u < O.threshold(beta, k)
                    if acc:
                        s[v] = -s[v]
            E = sum(w * s[a] * s[b] for a, b, w in zip(inst.u.tolist(), inst.v.tolist(),
                                                      inst.w.tolist()))
            assert o.energy_trace[r][t] == E, (r, t)
        assert o.final_state[r].tolist() == s


def _four_colouring():
    """A proper 4-colouring of the 6x4 torus other than first fit's."""
    return np.array([(x + y) % 2 + 2 * ((x // 2) % 2) for y in range(4) for x in range(6)],
                    np.int32)


def _stream_graphs():
    return [
        ("torus6x4", I.torus(6, 4, seed=1), None),
        ("torus5x7", I.torus(5, 7, seed=2), None),           # odd: 3 colours, ragged classes
        ("random", I.random_graph(200, 150, seed=3), None),  # isolated vertices, 4+ classes
        ("supplied", I.torus(6, 4, seed=1), _four_colouring()),
    ]


@pytest.mark.parametrize("idx", range(4))
def test_stream_is_injective(oracle_lib, idx):
    """(counter, word) never repeats over (vertex, sweep, replica, tag); runs
    of a class are consecutive ordinals, each run holds ranks 0..len-1, and
    the number of runs is the sum over classes of ceil(size / 4)."""
    O = oracle_lib
    name, inst, colour = _stream_graphs()[idx]
    if colour is not None:
        # the supplied colouring must be proper for this graph
        assert np.all(colour[inst.u] != colour[inst.v])
        col = colour
    else:
        _, col = O.colouring(inst.n, inst.u, inst.v)
    run, rank = O.stream_map(inst, colour)
    pairs = set(zip(run.tolist(), rank.tolist()))
    assert len(pairs) == inst.n
    assert rank.min() >= 0 and rank.max() <= 3
    sizes = np.bincount(col)
    assert run.max() + 1 == int(sum((s + 3) // 4 for s in sizes))
    first = 0
    for c, size in enumerate(sizes):
        members = np.sort(np.nonzero(col == c)[0])
        assert run[members].tolist() == [first + i // 4 for i in range(size)]
        assert rank[members].tolist() == [i % 4 for i in range(size)]
        first += (size + 3) // 4
    seen = set()
    for t in range(3):
        for r in range(3):
            for tag in (0, 1):
                for v in range(inst.n):
                    key = (t, int(run[v]), r, tag, int(rank[v]))
                    assert key not in seen
                    seen.add(key)


def test_stream_depends_on_the_colouring(oracle_lib):
    """The same graph under two proper colourings gets different streams."""
    O = oracle_lib
    inst = I.torus(6, 4, seed=1)
    other = _four_colouring()
    a = O.draws(inst, 5, 0, 0, 0)
    b = O.draws(inst, 5, 0, 0, 0, other)
    assert not np.array_equal(a, b)


def test_words_uniform_and_independent(oracle_lib):
    """Chi-square tests on 160,000 draws of a 10,000-vertex random graph:
    the top four bits are uniform; the four words of a run, and one
    vertex's words at consecutive sweeps and consecutive replicas, are
    pairwise independent (top two bits, 16 cells)."""
    O = oracle_lib
    inst = I.random_graph(10000, 9999, seed=3)
    run, rank = O.stream_map(inst)
    seed = 1003
    D = np.stack([O.draws(inst, seed, t, r, 0) for t in range(4) for r in range(4)])  # [16, n]
    alpha = 1e-6
    top4 = (D >> np.uint32(28)).astype(np.int64).ravel()
    assert stats.chisquare(np.bincount(top4, minlength=16)).pvalue > alpha

    def indep(a, b):
        tab = np.zeros((4, 4), np.int64)
        np.add.at(tab, ((a >> np.uint32(30)).astype(np.int64), (b >> np.uint32(30)).astype(np.int64)), 1)
        return stats.chisquare(tab.ravel(), np.full(16, tab.sum() / 16.0)).pvalue

    # the words of full runs: vertex of rank j in run q
    full = np.bincount(run, minlength=run.max() + 1) == 4
    byrank = np.full((4, run.max() + 1), -1, np.int64)
    byrank[rank, run] = np.arange(inst.n)
    cols = byrank[:, full]
    for i in range(4):
        for j in range(i + 1, 4):
            assert indep(D[:, cols[i]].ravel(), D[:, cols[j]].ravel()) > alpha, (i, j)
    # consecutive sweeps (same replica), consecutive replicas (same sweep)
    Dt = D.reshape(4, 4, -1)  # [t][r][v]
    assert indep(Dt[:-1].ravel(), Dt[1:].ravel()) > alpha
    assert indep(Dt[:, :-1].ravel(), Dt[:, 1:].ravel()) > alpha
