"""Future-graph semantics of the runtime on a host-only context (no GPU):
when_all, wait/query/timeouts, user events, host continuations (the paper's
then/dataflow, Sec. III-A), failure propagation, fault injection and stale
handles."""
import threading
import time

import pytest

import paper_1810_11482_amd as hx


@pytest.fixture
def ctx():
    c = hx.hx_ctx_create(-1, check=True)
    yield c
    hx.hx_ctx_destroy(c)


def test_when_all_of_zero_one_many(ctx):
    e0 = hx.hx_when_all(ctx, [])
    assert hx.hx_event_query(ctx, e0) == hx.HX_OK
    u = [hx.hx_user_event_create(ctx) for _ in range(5)]
    one = hx.hx_when_all(ctx, u[:1])
    many = hx.hx_when_all(ctx, u)
    assert hx.hx_event_query(ctx, one) == hx.HX_PENDING
    hx.hx_user_event_set(ctx, u[0])
    assert hx.hx_event_query(ctx, one) == hx.HX_OK
    assert hx.hx_event_query(ctx, many) == hx.HX_PENDING
    for e in u[1:]:
        hx.hx_user_event_set(ctx, e)
    assert hx.hx_wait(ctx, many) == hx.HX_OK
    nested = hx.hx_when_all(ctx, [one, many, 0])
    assert hx.hx_wait(ctx, nested) == hx.HX_OK


def test_wait_timeout_then_completion(ctx):
    u = hx.hx_user_event_create(ctx)
    t0 = time.perf_counter()
    assert hx.hx_wait(ctx, u, 20_000_000) == hx.HX_ERR_TIMEOUT
    assert time.perf_counter() - t0 >= 0.015
    threading.Timer(0.05, lambda: hx.hx_user_event_set(ctx, u)).start()
    assert hx.hx_wait(ctx, u) == hx.HX_OK


def test_host_tasks_run_in_dependency_order(ctx):
    log = []
    gate = hx.hx_user_event_create(ctx)
    a = hx.hx_host_task(ctx, lambda: log.append("a"), [gate])
    b = hx.hx_host_task(ctx, lambda: log.append("b"), [a])
    c = hx.hx_host_task(ctx, lambda: log.append("c"), [a])
    d = hx.hx_host_task(ctx, lambda: log.append("d"), [b, c])
    time.sleep(0.05)
    assert log == []  # held by the gate
    hx.hx_user_event_set(ctx, gate)
    assert hx.hx_wait(ctx, d) == hx.HX_OK
    assert log[0] == "a" and log[-1] == "d" and sorted(log[1:3]) == ["b", "c"]


def test_failure_propagates_and_skips_dependents(ctx):
    ran = []
    bad = hx.hx_host_task(ctx, lambda: hx.HX_ERR_HIP)
    after = hx.hx_host_task(ctx, lambda: ran.append(1), [bad])
    join = hx.hx_when_all(ctx, [after, hx.hx_when_all(ctx, [])])
    assert hx.hx_wait(ctx, bad) == hx.HX_ERR_HIP
    assert hx.hx_wait(ctx, after) == hx.HX_ERR_DEP_FAILED
    assert hx.hx_wait(ctx, join) == hx.HX_ERR_DEP_FAILED
    assert ran == []
    u = hx.hx_user_event_create(ctx)
    chain = hx.hx_host_task(ctx, lambda: ran.append(2), [u])
    hx.hx_user_event_set(ctx, u, hx.HX_ERR_TIMEOUT)
    assert hx.hx_wait(ctx, chain) == hx.HX_ERR_DEP_FAILED and ran == []


def test_exception_in_task_fails_event(ctx):
    e = hx.hx_host_task(ctx, lambda: 1 / 0)
    assert hx.hx_wait(ctx, e) == hx.HX_ERR_ARG


def test_fault_injection(ctx):
    ran = []
    seq = hx.hx_debug_next_seq(ctx)
    hx.hx_debug_inject(ctx, seq + 1)
    a = hx.hx_host_task(ctx, lambda: ran.append("a"))          # seq
    b = hx.hx_host_task(ctx, lambda: ran.append("b"), [a])     # seq + 1: injected
    c = hx.hx_host_task(ctx, lambda: ran.append("c"), [b])
    assert hx.hx_wait(ctx, b) == hx.HX_ERR_INJECTED
    assert hx.hx_wait(ctx, c) == hx.HX_ERR_DEP_FAILED
    assert hx.hx_wait(ctx, a) == hx.HX_OK and ran == ["a"]
    assert "injected" in hx.hx_last_error(ctx)


def test_stale_and_foreign_handles(ctx):
    e = hx.hx_user_event_create(ctx)
    hx.hx_event_release(ctx, e)
    for call in (lambda: hx.hx_event_query(ctx, e), lambda: hx.hx_user_event_set(ctx, e),
                 lambda: hx.hx_when_all(ctx, [e]), lambda: hx.hx_host_task(ctx, lambda: 0, [e])):
        with pytest.raises(hx.HxError) as ex:
            call()
        assert ex.value.status == hx.HX_ERR_INVALID
    e2 = hx.hx_user_event_create(ctx)  # reuses the slot with a new generation
    assert e2 != e
    with pytest.raises(hx.HxError) as ex:
        hx.hx_wait(ctx, 12345, 0)
    assert ex.value.status == hx.HX_ERR_INVALID
    with pytest.raises(hx.HxError):
        hx.hx_user_event_set(ctx, hx.hx_when_all(ctx, []))  # not a user event
    hx.hx_user_event_set(ctx, e2)
    with pytest.raises(hx.HxError):
        hx.hx_user_event_set(ctx, e2)  # already set


def test_released_dependency_still_orders(ctx):
    """Releasing an event drops only the caller's reference: operations that
    already depend on it still wait for it and still run after it."""
    log = []
    u = hx.hx_user_event_create(ctx)
    a = hx.hx_host_task(ctx, lambda: log.append("a"), [u])
    b = hx.hx_host_task(ctx, lambda: log.append("b"), [a])
    hx.hx_event_release(ctx, a)
    time.sleep(0.02)
    assert log == []
    hx.hx_user_event_set(ctx, u)
    assert hx.hx_wait(ctx, b) == hx.HX_OK
    assert log == ["a", "b"]


def test_concurrent_submission(ctx):
    count = []
    lock = threading.Lock()

    def worker(k):
        evs = []
        for i in range(50):
            evs.append(hx.hx_host_task(ctx, lambda: (lock.acquire(), count.append(1),
                                                     lock.release()) and None))
        j = hx.hx_when_all(ctx, evs)
        assert hx.hx_wait(ctx, j) == hx.HX_OK

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert len(count) == 200


def test_gpu_operations_refused(ctx):
    with pytest.raises(hx.HxError) as e:
        hx.hx_buffer_create(ctx, 64)
    assert e.value.status == hx.HX_ERR_NO_DEVICE
    with pytest.raises(hx.HxError) as e:
        hx.hx_host_alloc(ctx, 64)
    assert e.value.status == hx.HX_ERR_NO_DEVICE
    assert hx.hx_hazard_count(ctx) == 0
