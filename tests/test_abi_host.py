"""The C ABI library on the host: it loads, exports every declared symbol,
and its host-side logic (validation, colouring, layout, schedules,
thresholds, cut evaluation) agrees with the oracle.  No device compute."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_09275_amd import instances as I
from tests.conftest import ROOT, load_binding

B = load_binding()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ising.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ising_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    syms = declared_symbols()
    assert len(syms) >= 25
    for s in syms:
        assert hasattr(B._L, s), s
    assert set(syms) == set(B.EXPORTED)


def test_status_strings():
    for code in range(-6, 1):
        assert B._L.ising_status_string(code)


BAD = [
    ("selfloop", 3, [0], [0], [1]),
    ("dup", 3, [0, 1], [1, 0], [1, 1]),
    ("zero", 3, [0], [1], [0]),
    ("range", 3, [0], [3], [1]),
    ("neg", 3, [-1], [1], [1]),
    ("big", 3, [0], [1], [40000]),
    ("bigsum", 40000, list(range(0, 39999)), list(range(1, 40000)), [32768] * 39999),
]


@pytest.mark.parametrize("case", BAD, ids=[c[0] for c in BAD])
def test_validation_matches_oracle(case):
    name, n, u, v, w = case
    inst = I.Instance(name, n, np.array(u, np.int32), np.array(v, np.int32), np.array(w, np.int32))
    assert not O.validate(inst)
    with pytest.raises(B.IsingError) as e:
        B.Problem.from_instance(inst)
    assert e.value.status == B.ERR_INVALID


def test_bad_colourings_rejected():
    inst = I.torus(4, 4, 1)
    for col in (np.zeros(16, np.int32), np.full(16, 2000, np.int32)):
        assert not O.validate(inst, colour=col)
        with pytest.raises(B.IsingError):
            B.Problem.from_instance(inst, colour=col)
    with pytest.raises(B.IsingError):
        B.ising_create(0, [], [], [])


GRAPHS = {
    "c1": lambda: I.workload_c1(),
    "odd": lambda: I.torus(7, 9, 5),
    "c2": lambda: I.workload_c2(),
    "c3": lambda: I.workload_c3(),
    "weighted": lambda: I.random_weighted(800, 2000, 2, 50),
    "L141": lambda: I.torus(141, 141, 3),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_colouring_and_info_match_oracle(name):
    inst = GRAPHS[name]()
    p = B.Problem.from_instance(inst)
    C, col = O.colouring(inst.n, inst.u, inst.v)
    np.testing.assert_array_equal(p.colouring(), col)
    info = p.info()
    assert info.n_colours == C and info.n == inst.n and info.m == inst.m
    assert info.total_weight == int(inst.w.sum())
    deg = np.bincount(np.concatenate([inst.u, inst.v]), minlength=inst.n)
    assert info.max_degree == deg.max()
    absw = np.zeros(inst.n, np.int64)
    np.add.at(absw, inst.u, np.abs(inst.w))
    np.add.at(absw, inst.v, np.abs(inst.w))
    assert info.kmax == absw.max()
    assert info.unit_weights == int(np.all(np.abs(inst.w) == 1))
    sizes = np.bincount(col, minlength=C)
    assert info.n_padded == int(np.sum((sizes + 3) // 4 * 4))
    s = I.random_spins(3, 1, inst.n)[0]
    assert p.eval_cut(s) == O.cut(inst, s)
    p.close()


SCHEDULES = [
    (O.LINEAR, 1000, 0.1, 3.0, 4),        # 16x16 torus
    (O.GEOMETRIC, 4000, 0.1, 4.0, 4),     # 100x80 torus and the batch
    (O.LINEAR, 4000, 0.05, 3.0, 12),      # random graph
    (O.LINEAR, 1000, 0.1, 3.0, 12),       # serving requests
    (O.GEOMETRIC, 300, 0.001, 0.01, 200),  # long rows
    (O.LINEAR, 1, 0.7, 3.0, 5),
]


@pytest.mark.parametrize("sch", SCHEDULES)
def test_threshold_table_bitwise_equal_to_oracle(sch):
    kind, S, b0, b1, kmax = sch
    lib = B.ising_threshold_table(B.Schedule.make(kind, S, b0, b1), kmax)
    betas = O.schedule(kind, S, b0, b1)
    ref = np.array([[O.threshold(b, k) for k in range(1, kmax + 1)] for b in betas], np.uint64)
    np.testing.assert_array_equal(lib, ref)


def test_threshold_table_explicit_with_zero_and_infinity():
    betas = np.array([0.0, 0.25, 1e300, 3.0])
    lib = B.ising_threshold_table(B.Schedule.make(betas=betas), 6)
    ref = np.array([[O.threshold(b, k) for k in range(1, 7)] for b in betas], np.uint64)
    np.testing.assert_array_equal(lib, ref)
    assert np.all(lib[0] == 2 ** 32) and np.all(lib[2] == 0)


def test_bad_schedules_rejected():
    inst = I.torus(4, 4, 1)
    p = B.Problem.from_instance(inst)
    for s in (B.Schedule.make(B.LINEAR, 0, 0.1, 1.0), B.Schedule.make(B.GEOMETRIC, 10, 0.0, 1.0),
              B.Schedule.make(B.LINEAR, 10, -1.0, 1.0), B.Schedule.make(betas=np.array([0.1, np.nan]))):
        with pytest.raises(B.IsingError) as e:
            B.ising_threshold_table(s, 4)
        assert e.value.status == B.ERR_INVALID
    p.close()


def test_initial_state_validation():
    p = B.Problem.from_instance(I.torus(4, 4, 1))
    with pytest.raises(B.IsingError):
        p.set_initial_state(np.zeros((2, 16), np.int8), 2)
    p.set_initial_state(np.ones((2, 16), np.int8), 2)
    p.set_initial_state(None, 0)
    p.close()


LABEL_GRAPHS = {
    "torus3x3": lambda: I.torus(3, 3, 1),
    "torus7x9": lambda: I.torus(7, 9, 5),
    "c2": lambda: I.workload_c2(),
    "regular4_5": lambda: I.random_regular4(5, 1),
    "regular4_101": lambda: I.random_regular4(101, 2),
    "regular4_5000": lambda: I.random_regular4(5000, 3),
    "two_k5": lambda: I.Instance("two_k5", 10,
                                 np.array([5 * c + a for c in range(2) for a in range(5) for b in range(a + 1, 5)], np.int32),
                                 np.array([5 * c + b for c in range(2) for a in range(5) for b in range(a + 1, 5)], np.int32),
                                 np.ones(20, np.int32)),
}


@pytest.mark.parametrize("name", list(LABEL_GRAPHS))
def test_degree4_labels_pair_up(name):
    """Every edge carries labels 2f and 2f+1 at its two ends: the degree-4
    form's pushes rely on it (a flip of v toggles bit e XOR 1 of the
    neighbour with label e).  Tori keep their listed orientation; random
    graphs go through the closed-walk construction."""
    inst = LABEL_GRAPHS[name]()
    if inst.name.startswith("torus"):
        inst = I.Instance(inst.name, inst.n, inst.u, inst.v, np.ones_like(inst.w))
    p = B.Problem.from_instance(inst)
    lab = p.neighbour_labels().reshape(inst.n, 4)
    nbrs = [set() for _ in range(inst.n)]
    for a, b in zip(inst.u.tolist(), inst.v.tolist()):
        nbrs[a].add(b)
        nbrs[b].add(a)
    for v in range(inst.n):
        assert set(lab[v].tolist()) == nbrs[v]
        for e in range(4):
            assert lab[lab[v, e], e ^ 1] == v
    if inst.name.startswith("torus"):
        x = np.arange(inst.n) % int(inst.name[5:].split("x")[0])
        lx = int(inst.name[5:].split("x")[0])
        right = (np.arange(inst.n) // lx) * lx + (x + 1) % lx
        np.testing.assert_array_equal(lab[:, 0], right)


def test_degree4_labels_need_degree4_unit_weights():
    for inst in (I.workload_c3(), I.torus(5, 5, 1, weights="pm1"),
                 I.Instance("w2", 5, I.random_regular4(5, 1).u, I.random_regular4(5, 1).v,
                            np.full(10, 2, np.int32))):
        p = B.Problem.from_instance(inst)
        if inst.name.startswith("torus"):
            lab = p.neighbour_labels()  # +-1 weights are unit weights
            assert lab.shape == (4 * inst.n,)
            continue
        with pytest.raises(B.IsingError) as e:
            p.neighbour_labels()
        assert e.value.status == B.ERR_UNSUPPORTED


@pytest.mark.parametrize("betas,n_sets,S,P", [([], 1, 10, 1), ([0.5, 0.4], 1, 10, 1),
                                               ([0.1, float("nan")], 1, 10, 1), ([-0.1], 1, 10, 1),
                                               ([0.1], 0, 10, 1), ([0.1], 1, 0, 1), ([0.1], 1, 10, 0)])
def test_temper_rejects_bad_ladders(betas, n_sets, S, P):
    """Tempering arguments are checked before any device work."""
    p = B.Problem.from_instance(I.torus(6, 6, 1))
    with pytest.raises(B.IsingError) as e:
        p.temper(betas, n_sets, S, P, 1)
    assert e.value.status == B.ERR_INVALID
    with pytest.raises(B.IsingError) as e:
        p.temper_results()
    assert e.value.status == B.ERR_STATE
    p.close()


def test_local_fields_host():
    """ising_set_fields: kmax becomes max_v (sum |w| + 2 |b|), the info flag
    follows, bad fields are refused, NULL removes them."""
    inst = I.with_fields(I.random_weighted(50, 120, 3, 4), 2, 6)
    p = B.Problem.from_instance(inst)
    info = p.info()
    wsum = np.zeros(inst.n, np.int64)
    np.add.at(wsum, inst.u, np.abs(inst.w))
    np.add.at(wsum, inst.v, np.abs(inst.w))
    assert info.fields == 1
    assert info.kmax == int((wsum + 2 * np.abs(inst.field)).max())
    with pytest.raises(B.IsingError) as e:
        p.set_fields(np.full(inst.n, 40000, np.int32))
    assert e.value.status == B.ERR_INVALID
    assert p.info().kmax == info.kmax  # a refused call changes nothing
    p.set_fields(None)
    assert p.info().fields == 0 and p.info().kmax == int(wsum.max())
    p.set_fields(np.zeros(inst.n, np.int32))
    assert p.info().fields == 0
    p.close()
    big = I.torus(200, 200, 1)
    q = B.Problem.from_instance(big)
    with pytest.raises(B.IsingError):
        q.set_fields(np.full(big.n, 32768, np.int32))  # total above 2^30
    q.close()


def test_allocator_needs_both_functions():
    a = B.ALLOC_FN(lambda n, dev, ctx: 0)
    assert B._L.ising_set_allocator(a, B.FREE_FN(), None) == B.ERR_INVALID
    assert B._L.ising_set_allocator(B.ALLOC_FN(), B.FREE_FN(), None) == B.OK


def test_c_program_uses_the_header(tmp_path):
    """A plain C99 program compiled against include/ising.h (-Wall -Wextra
    -Werror -pedantic) and linked to the library runs the host-only entry
    points: problem compile and info, colouring, cut evaluation on all 32
    states of a small weighted graph, rejected inputs and thresholds."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    root = ROOT
    pkg = os.path.join(root, "paper_2311_09275_amd")
    exe = str(tmp_path / "host_abi")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(root, "include"), os.path.join(root, "tests", "c", "host_abi.c"),
                    "-L", pkg, "-lising", f"-Wl,-rpath,{pkg}", "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "ok"
