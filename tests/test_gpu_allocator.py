"""The caller's allocator (ising_set_allocator) backs every device
allocation of the library, and results do not change."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_09275_amd import instances as I

pytestmark = pytest.mark.gpu

from tests.conftest import load_binding

B = load_binding()


def test_torch_caching_allocator_backs_the_library():
    import torch
    calls = {"alloc": 0, "free": 0}
    live = {}

    def alloc(n, dev):
        calls["alloc"] += 1
        p = torch.cuda.caching_allocator_alloc(n, device=dev)
        live[p] = n
        return p

    def free(p, n, dev):
        calls["free"] += 1
        assert live.pop(p) == n
        torch.cuda.caching_allocator_delete(p)

    inst = I.torus(20, 18, 31)
    B.set_allocator(alloc, free)
    try:
        p = B.Problem.from_instance(inst)
        p.anneal(B.Schedule.make(B.LINEAR, 200, 0.1, 3.0), 16, 5, B.Tuning(B.PATH_FIELD, 1, 256, 0))
        per = p.cut().per_replica
        assert torch.cuda.memory_allocated() > 0 and live
        p.temper([0.2, 0.6, 1.5], 2, 60, 5, 6, cluster_from=1)
        temp, swaps, cm, cs = p.temper_results()
        p.close()
        srv = B.ising_server_create(1 << 24, 2, 25, backend=0)
        q = B.Problem.from_instance(inst)
        t = B.ising_server_submit(srv, q.handle, B.Schedule.make(B.LINEAR, 100, 0.1, 3.0), 16, 7,
                                  10 ** 9, 50)
        r = B.ising_server_wait(srv, t, 60.0)
        assert r.status == 0
        B.ising_server_destroy(srv)
        q.close()
    finally:
        B.set_allocator()
    assert calls["alloc"] > 0 and calls["free"] == calls["alloc"] and not live
    o = O.anneal(inst, 200, 16, 5, kind=O.LINEAR, beta0=0.1, beta1=3.0, want_states=False)
    np.testing.assert_array_equal(per, o.best_cut)
    ot = O.temper(inst, [0.2, 0.6, 1.5], 2, 60, 5, 6, cluster_from=1)
    np.testing.assert_array_equal(temp, ot.final_temp)
    np.testing.assert_array_equal(cs, ot.cluster_sites)
    # back on hipMalloc: the library still works
    p = B.Problem.from_instance(inst)
    p.anneal(B.Schedule.make(B.LINEAR, 200, 0.1, 3.0), 16, 5, B.Tuning(B.PATH_FIELD, 1, 256, 0))
    np.testing.assert_array_equal(p.cut().per_replica, o.best_cut)
    p.close()
