"""GPU parity of the partitioned future graph (Sec. V-A.2 / Algorithm 1 with
the Sec. V-A.1 stencil) and of the host-to-host pipeline, against the oracle's
whole-array loop.  Every time-block split agrees with the oracle; the plain
one-step-per-launch form is bit-identical to the graph at time block 1."""
import numpy as np
import pytest

import oracle
import workloads
from conftest import rel_l2, rel_max

pytestmark = pytest.mark.gpu
hx = pytest.importorskip("paper_1810_11482_amd")
from hxutil import download, upload  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0, compute_streams=4)
    yield c
    hx.hx_ctx_destroy(c)


def run_graph(ctx, u0, parts, steps, r, periodic=True, mode=hx.HX_PART_GRAPH, tb=0, cpl=0):
    dt = u0.dtype.type
    code = hx.HX_F64 if dt == np.float64 else hx.HX_F32
    bounds = workloads.partition_bounds(u0.size, parts)
    A = [upload(ctx, u0[o:o + s]) for o, s in bounds]
    B = [hx.hx_buffer_create(ctx, s * u0.itemsize) for _, s in bounds]
    d = hx.partitioned_desc(code, [s for _, s in bounds], A, B, steps, r, periodic=periodic,
                            mode=mode, time_block=tb, cells_per_lane=cpl)
    ev, in_b, _ = hx.hx_run_partitioned(ctx, d)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, ev)
    res = np.concatenate([download(ctx, b, s, dt) for b, (_, s) in zip(B if in_b else A, bounds)])
    for b in A + B:
        hx.hx_buffer_destroy(ctx, b)
    return res


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
@pytest.mark.parametrize("periodic", [True, False])
def test_graph_matches_oracle_and_splits_agree(ctx, dtype, tol, periodic):
    n, parts, steps, r = 200003, 9, 50, 0.25
    u0 = workloads.uniform(n, 300, int(periodic), 0, 1, dtype)
    ref_fn = oracle.heat1d_periodic if periodic else oracle.heat1d_dirichlet
    ref = ref_fn(u0.astype(np.float64), r, steps)
    outs = []
    for tb, cpl in [(1, 8), (7, 16), (10, 32), (25, 32), (50, 64)]:
        got = run_graph(ctx, u0, parts, steps, r, periodic, tb=tb, cpl=cpl)
        e2, em = rel_l2(got, ref), rel_max(got, ref)
        print(f"{dtype.__name__} periodic={periodic} tb={tb}: rel_l2={e2:.2e} rel_max={em:.2e}")
        assert e2 <= tol and em <= 10 * tol
        outs.append(got)
    plain = run_graph(ctx, u0, parts, steps, r, periodic, mode=hx.HX_PART_PLAIN)
    # one-step passes: the graph at time block 1 and the plain form run the
    # same per-cell arithmetic, so they agree bit for bit
    assert np.array_equal(plain, outs[0])
    assert rel_l2(plain, ref) <= tol


def test_single_partition_graph_is_periodic_run(ctx):
    u0 = workloads.uniform(5000, 301, 0, 0, 1, np.float64)
    got = run_graph(ctx, u0, 1, 33, 0.3, tb=11)
    assert rel_l2(got, oracle.heat1d_periodic(u0, 0.3, 33)) <= 1e-12


@pytest.mark.parametrize("parts,steps", [(8, 50), (5, 13), (3, 0), (2, 7), (1, 5)])
def test_pipeline_host_to_host(ctx, parts, steps):
    """Host to host through hx_run_pipeline, on a context with the hazard
    checker and timing: the output against the oracle, no unordered access,
    every kernel after the copies in it reads, every copy out after its kernel."""
    ctx = hx.hx_ctx_create(0, compute_streams=4, check=True, timing=True)
    n = 100003
    u0 = workloads.uniform(n, 302, parts, 0, 1, np.float32)
    bounds = workloads.partition_bounds(n, parts)
    hin = hx.hx_host_alloc(ctx, n * 4)
    hout = hx.hx_host_alloc(ctx, n * 4)
    ain = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * n).from_address(hin))
    aout = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * n).from_address(hout))
    ain[:] = u0
    aout[:] = np.nan
    A = [hx.hx_buffer_create(ctx, s * 4) for _, s in bounds]
    B = [hx.hx_buffer_create(ctx, s * 4) for _, s in bounds]
    base = hx.partitioned_desc(hx.HX_F32, [s for _, s in bounds], A, B, steps, 0.25)
    pd = hx.hx_pipeline_desc(base, hin, hout)
    ev, h2d, ker, d2h = hx.hx_run_pipeline(ctx, pd, op_events=True)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    assert hx.hx_hazard_count(ctx) == 0, hx.hx_hazard_report(ctx)
    ref0 = h2d[0]
    for p in range(parts):
        ks, ke = hx.hx_event_span(ctx, ker[p], ref0)
        reads = {p} | ({(p - 1) % parts, (p + 1) % parts} if steps > 0 else set())
        for q in reads:
            assert hx.hx_event_span(ctx, h2d[q], ref0)[1] <= ks + 1e-6, (p, q)
        assert ke <= hx.hx_event_span(ctx, d2h[p], ref0)[0] + 1e-6, p
    for e in h2d + ker + d2h + [ev]:
        assert hx.hx_event_query(ctx, e) == hx.HX_OK
        hx.hx_event_release(ctx, e)
    ref = oracle.heat1d_periodic(u0.astype(np.float64), 0.25, steps)
    assert rel_l2(aout, ref) <= 1e-5
    for b in A + B:
        hx.hx_buffer_destroy(ctx, b)
    hx.hx_host_free(ctx, hin)
    hx.hx_host_free(ctx, hout)
    hx.hx_ctx_destroy(ctx)


def test_full_size_bench_configuration_sampled(ctx):
    """2^28 fp32 cells in 64 partitions, r = 0.25, 50 steps, in the graph form
    the bench times (time blocks 25 and 50): sampled outputs against the
    oracle's light cone, and the two splits agree on the samples."""
    n, parts, T, r = 1 << 28, 64, 50, 0.25
    spec = workloads.Partitioned1D()
    hin = hx.hx_host_alloc(ctx, n * 4)
    u0 = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * n).from_address(hin))
    workloads.partitioned1d_u0(spec, out=u0)
    bounds = workloads.partition_bounds(n, parts)
    A = [hx.hx_buffer_create(ctx, s * 4) for _, s in bounds]
    B = [hx.hx_buffer_create(ctx, s * 4) for _, s in bounds]
    rng = np.random.default_rng(5)
    idx = np.sort(np.concatenate([rng.choice(n, 40, replace=False),
                                  [0, 1, n - 1, (1 << 22) - 1, 1 << 22, 63 << 22]]))
    ref = oracle.heat1d_periodic_at(u0.astype(np.float64), r, T, idx)
    samples = []
    for tb, cpl in [(25, 32), (50, 64)]:
        evs = []
        for (o, s), a in zip(bounds, A):
            evs.append(hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, hin + o * 4, a, 0, 0, 0,
                                                             s * 4)))
        d = hx.partitioned_desc(hx.HX_F32, [s for _, s in bounds], A, B, T, r, time_block=tb,
                                cells_per_lane=cpl)
        ev, in_b, _ = hx.hx_run_partitioned(ctx, d, deps=evs)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK
        for e in evs + [ev]:
            hx.hx_event_release(ctx, e)
        res = []
        for i in idx:
            p = int(i) >> 22
            res.append(download(ctx, (B if in_b else A)[p], 1, np.float32,
                                offset=(int(i) - bounds[p][0]) * 4)[0])
        res = np.array(res, dtype=np.float64)
        err = np.max(np.abs(res - ref) / np.abs(ref))
        print(f"tb={tb}: sampled max rel err {err:.2e}")
        assert err <= 1e-5
        samples.append(res)
    assert np.max(np.abs(samples[0] - samples[1]) / np.abs(samples[1])) <= 2e-5
    for b in A + B:
        hx.hx_buffer_destroy(ctx, b)
    hx.hx_host_free(ctx, hin)


@pytest.mark.parametrize("cpl", [32, 16])
def test_full_size_batched_pass_arena_sampled(ctx, cpl):
    """The bench's headline form: 2^28 fp32 cells as 64 partition views of one
    HBM arena, r = 0.25, 50 steps as one batched launch over all partitions
    (halos from the neighbour views); sampled cells against the oracle's light
    cone, including every partition seam of a few partitions."""
    n, parts, T, r = 1 << 28, 64, 50, 0.25
    spec = workloads.Partitioned1D()
    hin = hx.hx_host_alloc(ctx, n * 4)
    u0 = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * n).from_address(hin))
    workloads.partitioned1d_u0(spec, out=u0)
    bounds = workloads.partition_bounds(n, parts)
    arena_a = hx.hx_buffer_create(ctx, n * 4)
    arena_b = hx.hx_buffer_create(ctx, n * 4)
    pa, pb = hx.hx_buffer_ptr(ctx, arena_a)[0], hx.hx_buffer_ptr(ctx, arena_b)[0]
    A = [hx.hx_buffer_wrap(ctx, pa + o * 4, s * 4) for o, s in bounds]
    B = [hx.hx_buffer_wrap(ctx, pb + o * 4, s * 4) for o, s in bounds]
    e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, hin, arena_a, 0, 0, 0, n * 4))
    assert hx.hx_wait(ctx, e) == hx.HX_OK
    hx.hx_event_release(ctx, e)
    segs = []
    for p in range(parts):
        lp, rp = (p - 1) % parts, (p + 1) % parts
        segs.append(hx.segment(inp=A[p], out=B[p], n=bounds[p][1], r=r, bc_lo=hx.HX_BC_GHOST,
                               bc_hi=hx.HX_BC_GHOST, halo_lo=A[lp],
                               halo_lo_offset=(bounds[lp][1] - T) * 4, halo_hi=A[rp],
                               halo_width=T))
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, T, segs, hx.HX_BATCH_PERSISTENT,
                                     cells_per_lane=cpl, grid_waves_per_cu=-1)
    ev = hx.hx_launch_batched(ctx, plan)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, ev)
    hx.hx_plan_destroy(ctx, plan)
    rng = np.random.default_rng(17)
    seams = [k << 22 for k in (1, 17, 63)]
    idx = np.sort(np.concatenate([rng.choice(n, 40, replace=False), [0, n - 1],
                                  [s + d for s in seams for d in (-2, -1, 0, 1)]]))
    ref = oracle.heat1d_periodic_at(u0.astype(np.float64), r, T, idx)
    got = np.array([download(ctx, arena_b, 1, np.float32, offset=int(i) * 4)[0] for i in idx],
                   dtype=np.float64)
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-5
    for b in A + B + [arena_a, arena_b]:
        hx.hx_buffer_destroy(ctx, b)
    hx.hx_host_free(ctx, hin)
