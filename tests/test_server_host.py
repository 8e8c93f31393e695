"""Scheduling logic of the continuous-batching server, exercised on the host
with its null backend (no device work: sweep counters advance and the
reported best cut equals the sweeps done, so target checks are visible)."""
import numpy as np
import pytest

from paper_2311_09275_amd import instances as I
from tests.conftest import load_binding

B = load_binding()


def _problem(side=10, seed=1):
    return B.Problem.from_instance(I.torus(side, side, seed))


def test_footprint_grows_with_replicas_and_size():
    p = _problem(10)
    q = _problem(20)
    s = B.Schedule.make(B.LINEAR, 1000, 0.1, 3.0)
    f1 = B.ising_server_footprint(p.handle, s, 64)
    f2 = B.ising_server_footprint(p.handle, s, 128)
    f3 = B.ising_server_footprint(q.handle, s, 64)
    assert 0 < f1 < f2 and f1 < f3
    # state words of every replica are part of it
    assert f2 - f1 >= 64 * p.info().n_padded * 4


def test_oversized_request_rejected_at_submit():
    p = _problem(10)
    s = B.Schedule.make(B.LINEAR, 100, 0.1, 3.0)
    need = B.ising_server_footprint(p.handle, s, 256)
    srv = B.ising_server_create(need // 2, 4, 50, backend=1)
    with pytest.raises(B.IsingError) as e:
        B.ising_server_submit(srv, p.handle, s, 256, 1, 10 ** 9, 50)
    assert e.value.status == B.ERR_NOMEM
    B.ising_server_destroy(srv)


def test_runs_to_completion_and_early_stop():
    p = _problem(10)
    s = B.Schedule.make(B.LINEAR, 1000, 0.1, 3.0)
    srv = B.ising_server_create(1 << 30, 8, 64, backend=1)
    full = B.ising_server_submit(srv, p.handle, s, 32, 1, 10 ** 9, 50)
    early = B.ising_server_submit(srv, p.handle, s, 32, 2, 120, 50)   # cut = sweeps done
    never = B.ising_server_submit(srv, p.handle, s, 32, 3, 120, 0)    # no checks: full run
    rf = B.ising_server_wait(srv, full, 10.0)
    re = B.ising_server_wait(srv, early, 10.0)
    rn = B.ising_server_wait(srv, never, 10.0)
    assert rf.status == 0 and rf.sweeps_done == 1000 and rf.reached_target == 0
    # the target is checked only after multiples of 50 sweeps: 150 >= 120
    assert re.status == 0 and re.sweeps_done == 150 and re.reached_target == 1
    assert rn.sweeps_done == 1000 and rn.reached_target == 1
    for r in (rf, re, rn):
        assert 0 <= r.t_submit <= r.t_admit <= r.t_done
    st = B.ising_server_best_state(srv, full, p.n)
    assert st.shape == (p.n,)
    B.ising_server_destroy(srv)


def test_admission_respects_budget_slots_and_order():
    p = _problem(12)
    s = B.Schedule.make(B.LINEAR, 2000, 0.1, 3.0)
    fp = B.ising_server_footprint(p.handle, s, 64)
    budget = int(2.5 * fp)  # at most two resident by memory
    srv = B.ising_server_create(budget, 3, 10, backend=1)
    tickets = [B.ising_server_submit(srv, p.handle, s, 64, i, 10 ** 9, 0) for i in range(12)]
    res = [B.ising_server_wait(srv, t, 30.0) for t in tickets]
    steps, finished, peak = B.ising_server_stats(srv)
    assert finished == 12 and 1 <= peak <= 2
    admits = [r.t_admit for r in res]
    assert admits == sorted(admits)                  # arrival order is kept
    assert all(r.sweeps_done == 2000 and r.status == 0 for r in res)
    assert steps >= 2000 // 10 * 12 // 2
    B.ising_server_destroy(srv)


def test_slot_limit():
    p = _problem(8)
    s = B.Schedule.make(B.LINEAR, 500, 0.1, 3.0)
    srv = B.ising_server_create(1 << 30, 2, 5, backend=1)
    tickets = [B.ising_server_submit(srv, p.handle, s, 16, i, 10 ** 9, 0) for i in range(8)]
    for t in tickets:
        assert B.ising_server_wait(srv, t, 30.0).status == 0
    assert B.ising_server_stats(srv)[2] <= 2
    B.ising_server_destroy(srv)


def test_bad_arguments_and_unknown_ticket():
    p = _problem(8)
    s = B.Schedule.make(B.LINEAR, 10, 0.1, 3.0)
    with pytest.raises(B.IsingError):
        B.ising_server_create(1 << 20, 0, 5, backend=1)
    srv = B.ising_server_create(1 << 20, 1, 5, backend=1)
    with pytest.raises(B.IsingError):
        B.ising_server_wait(srv, 999, 0.1)
    with pytest.raises(B.IsingError):
        B.ising_server_submit(srv, p.handle, B.Schedule.make(B.LINEAR, 0, 0.1, 3.0), 8, 1, 5, 5)
    B.ising_server_destroy(srv)


def test_destroy_with_pending_requests_cancels_them():
    p = _problem(8)
    s = B.Schedule.make(B.LINEAR, 10 ** 6, 0.1, 3.0)
    srv = B.ising_server_create(1 << 30, 1, 1, backend=1)
    for i in range(4):
        B.ising_server_submit(srv, p.handle, s, 8, i, 10 ** 9, 0)
    B.ising_server_destroy(srv)  # must return promptly


def test_results_are_published_whole_while_polled():
    """Two threads poll wait(ticket, 0) and best_state on every request while
    the scheduler runs them one sweep per step: a request seen as done
    always carries its final sweep count, a finish time not before its
    admission, and its whole best state."""
    import threading
    p = _problem(10)
    S = 300
    s = B.Schedule.make(B.LINEAR, S, 0.1, 3.0)
    srv = B.ising_server_create(1 << 30, 4, 1, backend=1)
    tickets = [B.ising_server_submit(srv, p.handle, s, 16, i, 10 ** 9, 0) for i in range(24)]
    problems = []

    def poll():
        seen = set()
        while len(seen) < len(tickets) and not problems:
            for t in tickets:
                if t in seen:
                    continue
                try:
                    r = B.ising_server_wait(srv, t, 0.0)
                except B.IsingError as e:
                    if e.status != B.ERR_TIMEOUT:
                        problems.append(("wait", t, e.status))
                    continue
                if not (r.status == 0 and r.sweeps_done == S and 0 <= r.t_admit <= r.t_done):
                    problems.append(("result", t, r.status, r.sweeps_done, r.t_admit, r.t_done))
                st = B.ising_server_best_state(srv, t, p.n)
                if st.shape != (p.n,) or not (st == 1).all():
                    problems.append(("state", t))
                seen.add(t)

    threads = [threading.Thread(target=poll) for _ in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(60)
    assert not any(th.is_alive() for th in threads)
    assert problems == []
    B.ising_server_destroy(srv)


def test_failed_step_ends_the_request_and_frees_its_slot():
    """Backend 2 fails every step in which the marked request is resident
    (as a device error would).  With one slot, the marked request fails
    alone with ISING_ERR_DEVICE; its memory and slot are freed and the
    requests queued behind it run to completion."""
    p = _problem(10)
    s = B.Schedule.make(B.LINEAR, 200, 0.1, 3.0)
    need = B.ising_server_footprint(p.handle, s, 32)
    srv = B.ising_server_create(need + need // 2, 1, 50, backend=2)
    bad = B.ising_server_submit(srv, p.handle, s, 32, B.NULL_FAIL_SEED, 10 ** 9, 50)
    good = [B.ising_server_submit(srv, p.handle, s, 32, 10 + i, 10 ** 9, 50) for i in range(3)]
    rb = B.ising_server_wait(srv, bad, 10.0)
    assert rb.status == B.ERR_DEVICE and rb.sweeps_done == 0
    with pytest.raises(B.IsingError) as e:
        B.ising_server_best_state(srv, bad, p.n)
    assert e.value.status == B.ERR_STATE
    for t in good:
        r = B.ising_server_wait(srv, t, 10.0)
        assert r.status == 0 and r.sweeps_done == 200
    steps, finished, peak = B.ising_server_stats(srv)
    assert finished == 4 and peak == 1
    B.ising_server_destroy(srv)


def test_failed_step_ends_every_request_resident_in_it():
    """A long request is resident when the marked one joins it: the step
    they share fails, and both end with ISING_ERR_DEVICE part-way; a
    request submitted afterwards is served normally."""
    p = _problem(10)
    s_long = B.Schedule.make(B.LINEAR, 1_000_000, 0.1, 3.0)
    s = B.Schedule.make(B.LINEAR, 100, 0.1, 3.0)
    srv = B.ising_server_create(1 << 30, 4, 1, backend=2)
    long_t = B.ising_server_submit(srv, p.handle, s_long, 16, 1, 10 ** 9, 0)
    import time
    t0 = time.monotonic()
    while B.ising_server_stats(srv)[0] < 3:  # the long request alone has run a few steps
        assert time.monotonic() - t0 < 10.0
        time.sleep(0.001)
    bad = B.ising_server_submit(srv, p.handle, s, 16, B.NULL_FAIL_SEED, 10 ** 9, 0)
    rl = B.ising_server_wait(srv, long_t, 30.0)
    rb = B.ising_server_wait(srv, bad, 30.0)
    assert rl.status == B.ERR_DEVICE and 0 < rl.sweeps_done < 1_000_000
    assert rb.status == B.ERR_DEVICE
    after = B.ising_server_submit(srv, p.handle, s, 16, 2, 10 ** 9, 0)
    ra = B.ising_server_wait(srv, after, 10.0)
    assert ra.status == 0 and ra.sweeps_done == 100
    B.ising_server_destroy(srv)
