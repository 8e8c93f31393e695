"""The allocation-free anneal (ising_anneal_noalloc) against the allocating
one (ising_anneal_tuned), through the C ABI, element by element.

Two calls in a row share the library's one scratch array: a 24 x 20 torus
with 64 replicas, then a smaller random graph with isolated vertices and 16
replicas.  Every result buffer is filled with a sentinel first, so a stale
or unwritten value fails."""
import numpy as np
import pytest
import torch

from paper_2311_09275_amd import instances as I
from tests.conftest import load_binding

pytestmark = pytest.mark.gpu

B = load_binding()


def _expected(p, R):
    best, arg, per = B.ising_cut(p.handle, R)
    bs, acc, en = p.replica_results()
    states = np.stack([p.replica_state(r)[0] for r in range(R)])
    key = (((int(best) + (1 << 31)) % (1 << 32)) << 32) | ((1 << 32) - 1 - int(arg))
    return per.astype(np.int64), bs, acc, en, states, key


def _noalloc(p, sched, R, seed, tuning, n, stream):
    dev = torch.device("cuda", 0)
    bc = torch.full((R,), -7, dtype=torch.int32, device=dev)
    bsw = torch.full((R,), -7, dtype=torch.int32, device=dev)
    en = torch.full((R,), -7, dtype=torch.int32, device=dev)
    acc = torch.full((R,), -7, dtype=torch.int64, device=dev)
    am = torch.full((1,), -7, dtype=torch.int64, device=dev)
    st = torch.zeros((R, n), dtype=torch.int8, device=dev)
    B.ising_anneal_noalloc(p.handle, sched, R, seed, tuning, bc.data_ptr(), bsw.data_ptr(),
                           en.data_ptr(), acc.data_ptr(), am.data_ptr(), st.data_ptr(), stream=stream)
    stream.synchronize()
    return (bc.cpu().numpy().astype(np.int64), bsw.cpu().numpy(), acc.cpu().numpy(),
            en.cpu().numpy(), st.cpu().numpy(), int(am.cpu().numpy().view(np.uint64)[0]))


CASES = [
    # (instance, replicas, sweeps, schedule, seed): the second is smaller
    (lambda: I.torus(24, 20, seed=5), 64, 300, (B.GEOMETRIC, 0.1, 4.0), 41),
    (lambda: I.random_graph(150, 120, seed=6), 16, 200, (B.LINEAR, 0.05, 3.0), 42),
]


@pytest.mark.parametrize("tuning", [None, B.Tuning(B.PATH_FIELD, 2, 512, 2)],
                         ids=["auto", "field_g2_b512_hbmadj"])
def test_noalloc_equals_allocating_anneal_twice(tuning):
    stream = torch.cuda.Stream(device=0)
    for make, R, S, (kind, b0, b1), seed in CASES:
        inst = make()
        print(f"noalloc case n={inst.n} R={R} S={S} seed={seed}", flush=True)
        sched = B.Schedule.make(kind, S, b0, b1)
        p = B.Problem.from_instance(inst)
        p.anneal(sched, R, seed, tuning if tuning is not None else B.Tuning(B.PATH_FIELD, 1, 1024, 0),
                 stream=stream)
        per, bs, acc, en, states, key = _expected(p, R)
        got = _noalloc(p, sched, R, seed, tuning, inst.n, stream)
        assert np.array_equal(got[0], per)
        assert np.array_equal(got[1], bs)
        assert np.array_equal(got[2], acc)
        assert np.array_equal(got[3], en)
        assert np.array_equal(got[4], states)
        assert got[5] == key
        p.close()


def test_noalloc_refusals():
    stream = torch.cuda.Stream(device=0)
    inst = I.torus(100, 80, seed=2)
    sched = B.Schedule.make(B.GEOMETRIC, 50, 0.1, 4.0)
    p = B.Problem.from_instance(inst)
    dev = torch.device("cuda", 0)
    bufs = [torch.zeros(8, dtype=torch.int64, device=dev) for _ in range(5)]
    st = torch.zeros((4, inst.n), dtype=torch.int8, device=dev)
    args = [b.data_ptr() for b in bufs] + [st.data_ptr()]
    # the graph is not on the device before the problem's first anneal
    with pytest.raises(B.IsingError) as e:
        B.ising_anneal_noalloc(p.handle, sched, 4, 1, None, *args, stream=stream)
    assert e.value.status == B.ERR_STATE
    p.anneal(sched, 4, 1, B.Tuning(B.PATH_FIELD, 1, 1024, 0), stream=stream)
    p.cut()
    # 4096 replicas x 8000 positions of snapshots exceed the fixed array
    with pytest.raises(B.IsingError) as e:
        B.ising_anneal_noalloc(p.handle, sched, 4096, 1, None, *args, stream=stream)
    assert e.value.status == B.ERR_UNSUPPORTED and "fixed maximum" in str(e.value)
    # a path other than FIELD
    with pytest.raises(B.IsingError) as e:
        B.ising_anneal_noalloc(p.handle, sched, 4, 1, B.Tuning(B.PATH_PLAIN, 1, 256, 0), *args,
                               stream=stream)
    assert e.value.status == B.ERR_UNSUPPORTED
    p.close()
