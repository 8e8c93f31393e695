"""Local fields on the HIP path vs the oracle (exact): every path that can
carry a field term, tempering with fields, a batch mixing problems with
and without fields, and the refusals."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_09275_amd import instances as I
from tests.test_gpu_parity import PATHS, compare

pytestmark = pytest.mark.gpu

from tests.conftest import load_binding

B = load_binding()

FIELD_PATHS = ["plain", "field_g1_b256_hbmadj", "field_g1_b1024_ldsadj", "field_g1_b1024_csradj",
               "field_g4_b256_csradj", "field_g2_b512_ldsadj", "field_g4_b256_hbmadj",
               "field_g1_b512_auto"]


@pytest.mark.parametrize("path", FIELD_PATHS)
def test_fields_torus(path):
    """A torus with fields: the degree-4 forms are not used, the CSR and
    HBM forms carry the field in h."""
    compare(I.with_fields(I.torus(16, 12, 3), 4, 2), 300, 12, 61, tuning=PATHS[path])


@pytest.mark.parametrize("path", ["plain", "field_g1_b256_hbmadj", "field_g4_b256_hbmadj",
                                  "field_g1_b512_auto"])
def test_fields_weighted_sparse(path):
    """Weighted random graph with fields on half the vertices (isolated
    vertices with a field flip toward it)."""
    compare(I.with_fields(I.random_weighted(400, 500, 12, 5), 5, 7, 0.5), 200, 20, 62,
            kind=O.GEOMETRIC, b0=0.05, b1=2.0, tuning=PATHS[path])


def test_fields_automatic_configuration():
    compare(I.with_fields(I.workload_c1(), 6, 3), 400, 8, 63, tuning=None)


def test_fields_full_size_sampled_replicas():
    """The benchmark's local-fields workload at full size, in the launch it
    times (the automatic configuration): the 100x80 torus with b in [-2, 2]
    on every vertex, 256 replicas, 4000 sweeps geometric 0.1 -> 4.0; three
    replicas recomputed by the oracle."""
    compare(I.with_fields(I.workload_c2(), seed=2, bmax=2), 4000, 256, 1002, kind=O.GEOMETRIC,
            b0=0.1, b1=4.0, tuning=None, replicas=[0, 129, 255], trace=False)


def test_fields_refusals():
    inst = I.with_fields(I.torus(8, 8, 1), 1, 2)
    p = B.Problem.from_instance(inst)
    sched = B.Schedule.make(B.LINEAR, 10, 0.1, 1.0)
    for t in (B.Tuning(B.PATH_MSC, 1, 256, 0), B.Tuning(B.PATH_FIELD, 1, 256, 4)):
        with pytest.raises(B.IsingError) as e:
            p.anneal(sched, 4, 1, t)
        assert e.value.status == B.ERR_UNSUPPORTED
    with pytest.raises(B.IsingError) as e:
        p.temper([0.2, 0.5], 2, 10, 2, 1, cluster_from=0)
    assert e.value.status == B.ERR_UNSUPPORTED
    # removing the fields brings the degree-4 form back
    p.set_fields(None)
    p.anneal(sched, 4, 1, B.Tuning(B.PATH_FIELD, 1, 256, 4))
    p.cut()
    p.close()


@pytest.mark.parametrize("tuning", [None, B.Tuning(B.PATH_PLAIN, 1, 256, 0)])
def test_fields_tempering(tuning):
    inst = I.with_fields(I.torus(12, 10, 9), 7, 3)
    betas = [0.2, 0.5, 1.0, 2.0]
    p = B.Problem.from_instance(inst)
    p.temper(betas, 3, 80, 4, 64, tuning)
    best, arg, per = B.ising_cut(p.handle, 12)
    temp, swaps = p.temper_results()
    bs, acc, en = p.replica_results()
    p.close()
    o = O.temper(inst, betas, 3, 80, 4, 64)
    np.testing.assert_array_equal(per, o.best_cut)
    np.testing.assert_array_equal(en, o.final_energy)
    np.testing.assert_array_equal(temp, o.final_temp)
    np.testing.assert_array_equal(swaps, o.swaps)


def test_fields_batch_mixed():
    """A batch of problems with and without fields equals separate anneals."""
    insts = [I.with_fields(I.torus(10, 10, 11), 8, 2), I.torus(12, 8, 12),
             I.with_fields(I.random_graph(90, 120, 13), 9, 4)]
    probs = [B.Problem.from_instance(x) for x in insts]
    sched = B.Schedule.make(B.GEOMETRIC, 150, 0.1, 3.0)
    seeds = np.array([71, 72, 73], np.uint64)
    B.ising_anneal_batch([p.handle for p in probs], sched, 16, seeds, None)
    got = [B.ising_cut(p.handle, 16)[2] for p in probs]
    for x, p, g, sd in zip(insts, probs, got, seeds):
        o = O.anneal(x, 150, 16, int(sd), kind=O.GEOMETRIC, beta0=0.1, beta1=3.0, want_states=False)
        np.testing.assert_array_equal(g, o.best_cut)
        p.close()
