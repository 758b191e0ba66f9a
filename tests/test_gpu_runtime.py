"""Runtime semantics with real GPU work: dependency gating, failure
propagation, the hazard checker, deferred frees, host continuations mixed with
GPU operations, and foreign-stream interop."""
import time

import numpy as np
import pytest

import oracle
import workloads
from conftest import rel_l2

pytestmark = pytest.mark.gpu
hx = pytest.importorskip("paper_1810_11482_amd")
from hxutil import download, upload  # noqa: E402


@pytest.fixture
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0, check=True)
    yield c
    hx.hx_ctx_destroy(c)


def chain(ctx, src, dst, n, deps):
    """H2D src -> stencil (10 steps) -> D2H dst; returns (events, buffers)."""
    a = hx.hx_buffer_create(ctx, n * 4)
    b = hx.hx_buffer_create(ctx, n * 4)
    e1 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, src.ctypes.data, a, 0, 0, 0, n * 4), deps)
    e2 = hx.hx_launch_stencil(ctx, hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=n, steps=10, r=0.25,
                                                   inp=a, out=b), [e1])
    e3 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, dst.ctypes.data, b, 0, 0, 0, n * 4), [e2])
    return (e1, e2, e3), (a, b)


def test_user_event_gates_the_chain(ctx):
    n = 1 << 16
    src = workloads.uniform(n, 700, 0, 0, 1, np.float32)
    dst = np.full(n, -1.0, np.float32)
    gate = hx.hx_user_event_create(ctx)
    evs, bufs = chain(ctx, src, dst, n, [gate])
    assert hx.hx_wait(ctx, evs[2], 50_000_000) == hx.HX_ERR_TIMEOUT
    assert hx.hx_event_query(ctx, evs[0]) == hx.HX_PENDING
    assert np.all(dst == -1.0)  # nothing ran
    hx.hx_user_event_set(ctx, gate)
    assert hx.hx_wait(ctx, evs[2]) == hx.HX_OK
    ref = oracle.heat1d_periodic(src.astype(np.float64), 0.25, 10)
    assert rel_l2(dst, ref) <= 1e-5
    assert hx.hx_hazard_count(ctx) == 0


def test_failed_gate_skips_the_chain(ctx):
    n = 4096
    src = np.ones(n, np.float32)
    dst = np.full(n, -1.0, np.float32)
    gate = hx.hx_user_event_create(ctx)
    evs, bufs = chain(ctx, src, dst, n, [gate])
    hx.hx_user_event_set(ctx, gate, hx.HX_ERR_HIP)
    for e in evs:
        assert hx.hx_wait(ctx, e) == hx.HX_ERR_DEP_FAILED
    assert np.all(dst == -1.0)


def test_injected_failure_in_the_middle(ctx):
    n = 4096
    src = np.ones(n, np.float32)
    dst = np.full(n, -1.0, np.float32)
    seq = hx.hx_debug_next_seq(ctx)
    hx.hx_debug_inject(ctx, seq + 1)  # the stencil launch of the chain
    evs, bufs = chain(ctx, src, dst, n, [])
    assert hx.hx_wait(ctx, evs[0]) == hx.HX_OK
    assert hx.hx_wait(ctx, evs[1]) == hx.HX_ERR_INJECTED
    assert hx.hx_wait(ctx, evs[2]) == hx.HX_ERR_DEP_FAILED
    assert np.all(dst == -1.0)


def build_graph(ctx, bufs_a, bufs_b, sizes, steps, drop=None):
    """Per-partition graph by hand: node (p, b) reads its own and its
    neighbours' buffers; `drop` = (p, b, which) removes one dependency edge."""
    P = len(sizes)
    prev = [0] * P
    D = 5
    for b in range(steps // D):
        cur = []
        src, dst = (bufs_a, bufs_b) if b % 2 == 0 else (bufs_b, bufs_a)
        for p in range(P):
            lp, rp = (p - 1) % P, (p + 1) % P
            deps = {"own": prev[p], "left": prev[lp], "right": prev[rp]}
            if drop and drop[0] == p and drop[1] == b:
                deps.pop(drop[2])
            a = hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=sizes[p], steps=D, r=0.25, inp=src[p],
                                out=dst[p], bc_lo=hx.HX_BC_GHOST, bc_hi=hx.HX_BC_GHOST,
                                halo_lo=src[lp], halo_lo_offset=(sizes[lp] - D) * 4,
                                halo_hi=src[rp], halo_width=D)
            cur.append(hx.hx_launch_stencil(ctx, a, [e for e in deps.values() if e]))
        prev = cur
    return prev


@pytest.mark.parametrize("drop", [None, (3, 2, "right"), (0, 1, "left"), (5, 3, "own")])
def test_hazard_checker(ctx, drop):
    P, n = 8, 4096
    A = [upload(ctx, workloads.uniform(n, 701, p, 0, 1, np.float32)) for p in range(P)]
    B = [hx.hx_buffer_create(ctx, n * 4) for _ in range(P)]
    last = build_graph(ctx, A, B, [n] * P, 20, drop)
    assert hx.hx_wait(ctx, hx.hx_when_all(ctx, last)) == hx.HX_OK
    count = hx.hx_hazard_count(ctx)
    report = hx.hx_hazard_report(ctx)
    if drop is None:
        assert count == 0, report
    else:
        assert count > 0 and "unordered" in report


def test_partitioned_graph_is_hazard_free(ctx):
    P, n = 6, 5000
    A = [upload(ctx, workloads.uniform(n, 702, p, 0, 1, np.float32)) for p in range(P)]
    B = [hx.hx_buffer_create(ctx, n * 4) for _ in range(P)]
    for mode, tb in ((hx.HX_PART_GRAPH, 7), (hx.HX_PART_PLAIN, 1)):
        d = hx.partitioned_desc(hx.HX_F32, [n] * P, A, B, 21, 0.25, mode=mode, time_block=tb)
        ev, _, _ = hx.hx_run_partitioned(ctx, d)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK
    assert hx.hx_hazard_count(ctx) == 0, hx.hx_hazard_report(ctx)


def test_unordered_writer_is_flagged(ctx):
    n = 1 << 20
    a = upload(ctx, np.ones(n, np.float32))
    b = hx.hx_buffer_create(ctx, n * 4)
    args = hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=n, steps=3, r=0.25, inp=a, out=b)
    e1 = hx.hx_launch_stencil(ctx, args)
    e2 = hx.hx_launch_stencil(ctx, args)  # writes b again with no order to e1
    hx.hx_wait(ctx, hx.hx_when_all(ctx, [e1, e2]))
    assert hx.hx_hazard_count(ctx) >= 1
    # ordering through a host wait clears it for later operations
    n0 = hx.hx_hazard_count(ctx)
    e3 = hx.hx_launch_stencil(ctx, args)
    hx.hx_wait(ctx, e3)
    assert hx.hx_hazard_count(ctx) == n0


def test_destroy_is_deferred_until_use_completes(ctx):
    n = 1 << 24
    src = workloads.uniform(n, 703, 0, 0, 1, np.float32)
    dst = np.zeros(n, np.float32)
    a = upload(ctx, src)
    b = hx.hx_buffer_create(ctx, n * 4)
    e1 = hx.hx_launch_stencil(ctx, hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=n, steps=40,
                                                   r=0.25, inp=a, out=b, time_block=40))
    e2 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, dst.ctypes.data, b, 0, 0, 0, n * 4), [e1])
    hx.hx_buffer_destroy(ctx, a)  # still read by e1
    hx.hx_buffer_destroy(ctx, b)  # still written by e1, read by e2
    with pytest.raises(hx.HxError):
        hx.hx_buffer_ptr(ctx, a)
    assert hx.hx_wait(ctx, e2) == hx.HX_OK
    idx = np.arange(0, n, n // 37)
    ref = oracle.heat1d_periodic_at(src.astype(np.float64), 0.25, 40, idx)
    assert np.max(np.abs(dst[idx] - ref) / ref) <= 1e-5


def test_host_tasks_between_gpu_operations(ctx):
    n = 1 << 16
    host = hx.hx_host_alloc(ctx, n * 4)
    arr = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * n).from_address(host))
    arr[:] = 0.0
    src = workloads.uniform(n, 704, 0, 0, 1, np.float32)
    fill = hx.hx_host_task(ctx, lambda: arr.__setitem__(slice(None), src))
    a = hx.hx_buffer_create(ctx, n * 4)
    b = hx.hx_buffer_create(ctx, n * 4)
    e1 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, host, a, 0, 0, 0, n * 4), [fill])
    e2 = hx.hx_launch_stencil(ctx, hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=n, steps=5,
                                                   r=0.25, inp=a, out=b), [e1])
    e3 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, host, b, 0, 0, 0, n * 4), [e2])
    seen = {}

    def grab():
        seen["v"] = arr.copy()

    check = hx.hx_host_task(ctx, grab, [e3])
    assert hx.hx_wait(ctx, check) == hx.HX_OK
    ref = oracle.heat1d_periodic(src.astype(np.float64), 0.25, 5)
    assert rel_l2(seen["v"], ref) <= 1e-5


def test_foreign_stream_interop(ctx):
    import torch
    n = 1 << 20
    t = torch.rand(n, device="cuda", dtype=torch.float32)
    out = torch.empty_like(t)
    s = torch.cuda.current_stream()
    t.mul_(2.0)  # queued on torch's stream
    ev_t = hx.hx_event_record_stream(ctx, s.cuda_stream)
    bi = hx.hx_buffer_wrap(ctx, t.data_ptr(), n * 4)
    bo = hx.hx_buffer_wrap(ctx, out.data_ptr(), n * 4)
    e = hx.hx_launch_stencil(ctx, hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=n, steps=3, r=0.25,
                                                  inp=bi, out=bo), [ev_t])
    hx.hx_stream_wait_event(ctx, s.cuda_stream, e)
    total = out.sum()  # torch reads out after the stencil, on its own stream
    ref = oracle.heat1d_periodic(t.cpu().double().numpy(), 0.25, 3)
    assert abs(total.item() - ref.sum()) <= 1e-4 * abs(ref.sum())
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-5


def test_band_batches_are_hazard_free(ctx):
    """2D bands in one launch per pass (two groups: 20 bands) and one launch
    per band: every halo read is ordered after its write, every overwrite
    after its reads."""
    nx, bands = 512, 20
    sizes = [9 + (p % 3) for p in range(bands)]
    A = [upload(ctx, workloads.uniform(s * nx, 705, p, 0, 1, np.float32)) for p, s in
         enumerate(sizes)]
    B = [hx.hx_buffer_create(ctx, s * nx * 4) for s in sizes]
    for mode in (hx.HX_PART_BATCHED, hx.HX_PART_GRAPH):
        d = hx.partitioned_desc(hx.HX_F32, sizes, A, B, 20, 0.2, periodic=False, mode=mode,
                                time_block=6, dims=2, nx=nx, rows_per_block=8)
        ev, _, _ = hx.hx_run_partitioned(ctx, d)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
        hx.hx_event_release(ctx, ev)
    assert hx.hx_hazard_count(ctx) == 0, hx.hx_hazard_report(ctx)
    d1 = hx.partitioned_desc(hx.HX_F32, [64, 64], A[:2], B[:2], 4, 0.2, mode=hx.HX_PART_BATCHED)
    with pytest.raises(hx.HxError) as e:
        hx.hx_run_partitioned(ctx, d1)
    assert e.value.status == hx.HX_ERR_ARG
