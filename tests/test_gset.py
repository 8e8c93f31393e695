"""Gset ingestion and the solution bitstrings of the paper's appendices
(Sec. II.A; App. II and III).  CPU only."""
import io
import os

import numpy as np
import pytest

from paper_2311_09275_amd import gset
from paper_2311_09275_amd import instances as I
from tests.conftest import load_binding

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _hex(name):
    with open(os.path.join(GOLD, name)) as f:
        return "".join(l for l in f if not l.startswith("#"))


@pytest.mark.parametrize("name,n", [("g72_solution_hex.txt", 10000), ("g77_solution_hex.txt", 14000)])
def test_paper_bitstrings_give_one_bit_per_variable(name, n):
    """App. II and III: the strings expand to the values of variables 1..n
    (G72: n = 10,000; G77: n = 14,000), four per hexadecimal digit."""
    text = _hex(name)
    digits = "".join(text.split())
    assert len(digits) == n // 4
    bits = gset.bits_from_hex(text, n)
    assert bits.shape == (n,) and set(np.unique(bits)) <= {0, 1}
    assert gset.hex_from_bits(bits) == digits
    # one variable fewer or more cannot be read from the same string
    with pytest.raises(ValueError):
        gset.bits_from_hex(text, n + 4)


def test_hex_convention():
    """Most significant bit of a digit first; bits past n must be zero."""
    np.testing.assert_array_equal(gset.bits_from_hex("A", 4), [1, 0, 1, 0])
    np.testing.assert_array_equal(gset.bits_from_hex("3 8", 5), [0, 0, 1, 1, 1])
    np.testing.assert_array_equal(gset.bits_from_hex("a", 3), [1, 0, 1])
    with pytest.raises(ValueError):
        gset.bits_from_hex("B", 3)   # the fourth bit is set
    with pytest.raises(ValueError):
        gset.bits_from_hex("G", 4)
    assert gset.hex_from_bits([1, 0, 1]) == "A"
    np.testing.assert_array_equal(gset.spins_from_bits([1, 0]), [1, -1])


def test_read_write_round_trip(tmp_path):
    inst = I.random_weighted(60, 140, 3, 4)
    path = tmp_path / "g.txt"
    gset.write_gset(inst, path)
    back = gset.read_gset(path)
    assert back.n == inst.n and back.m == inst.m
    for f in ("u", "v", "w"):
        np.testing.assert_array_equal(getattr(back, f), getattr(inst, f))
    first = open(path).readline().split()
    assert first == [str(inst.n), str(inst.m)]
    # 1-based ids in the file
    second = open(path).readlines()[1].split()
    assert int(second[0]) == inst.u[0] + 1


def test_hand_written_file_and_cut():
    """A 4-cycle with one negative edge: the cut of x = (1, 0, 1, 0) takes
    every edge."""
    text = "4 4\n1 2 1\n2 3 1\n3 4 -1\n4 1 1\n"
    inst = gset.read_gset(io.StringIO(text))
    assert gset.cut_value(inst, [1, 0, 1, 0]) == 1 + 1 - 1 + 1
    assert gset.cut_value(inst, [1, 1, 1, 1]) == 0
    assert gset.cut_value(inst, gset.bits_from_hex("A", 4)) == 2


def test_cut_matches_oracle_and_library(oracle_lib):
    B = load_binding()
    inst = I.random_weighted(300, 900, 8, 5)
    bits = np.random.Generator(np.random.PCG64(4)).integers(0, 2, inst.n).astype(np.uint8)
    s = gset.spins_from_bits(bits)
    want = oracle_lib.cut(inst, s)
    assert gset.cut_value(inst, bits) == want
    p = B.Problem.from_instance(inst)
    assert p.eval_cut(s) == want
    p.close()
    # the cut is invariant under a global flip
    assert gset.cut_value(inst, 1 - bits) == want


@pytest.mark.parametrize("text", ["", "4\n", "4 2\n1 2 1\n", "4 1\n1 5 1\n", "4 1\n0 2 1\n",
                                  "4 1\n1 2\n"])
def test_rejects(text):
    with pytest.raises(ValueError):
        gset.read_gset(io.StringIO(text))


def test_stored_reference_cuts_cover_every_benchmark_instance():
    """Every instance the benchmark measures has a stored reference cut, and
    each lies above half the total weight (a uniformly random cut's
    expectation) and at most the sum of the positive weights (no cut does
    better than cutting every positive edge and no negative one)."""
    from paper_2311_09275_amd import reference_cuts as RC
    cuts = RC.load()
    insts = RC.named_instances()
    assert set(cuts) == set(insts)
    for name, inst in insts.items():
        w = inst.w.astype(np.int64)
        assert w.sum() / 2 < cuts[name] <= w[w > 0].sum(), (name, cuts[name])
