"""GPU parity of the batched driver: every problem of a batch equals the
oracle run on its own (n, r); persistent and graph modes (one pass of all
steps) are bit-identical, plain (one step per launch) agrees within the
tolerance; guard cells between problems are never written."""
import numpy as np
import pytest

import oracle
import workloads
from conftest import rel_l2, rel_max

pytestmark = pytest.mark.gpu
hx = pytest.importorskip("paper_1810_11482_amd")
from hxutil import download, upload  # noqa: E402

GUARD = 67  # guard cells between problems in the packed buffers


@pytest.fixture(scope="module")
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0)
    yield c
    hx.hx_ctx_destroy(c)


def pack(sizes):
    offs = []
    o = GUARD
    for n in sizes:
        offs.append(o)
        o += int(n) + GUARD
    return np.array(offs), o


def run_batch(ctx, sizes, rs, steps, dtype, mode, cpl=0, sentinel=-7.0, seed=0, grid=0):
    offs, total = pack(sizes)
    u = np.full(total, sentinel, dtype=dtype)
    for k, (o, n) in enumerate(zip(offs, sizes)):
        u[o:o + n] = workloads.uniform(int(n), 400 + seed, k, 0, 1, dtype)
    es = u.itemsize
    code = hx.HX_F64 if dtype == np.float64 else hx.HX_F32
    bin_ = upload(ctx, u)
    bout = upload(ctx, np.full(total, sentinel, dtype=dtype))
    btmp = upload(ctx, np.full(total, sentinel, dtype=dtype))
    segs = [hx.segment(inp=bin_, in_offset=int(o) * es, out=bout, out_offset=int(o) * es,
                       tmp=btmp, tmp_offset=int(o) * es, n=int(n), r=float(r),
                       bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
            for o, n, r in zip(offs, sizes, rs)]
    plan = hx.hx_plan_create_batched(ctx, code, steps, segs, mode, cells_per_lane=cpl,
                                     grid_waves_per_cu=grid)
    ev = hx.hx_launch_batched(ctx, plan)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, ev)
    out = download(ctx, bout, total, dtype)
    hx.hx_plan_destroy(ctx, plan)
    for b in (bin_, bout, btmp):
        hx.hx_buffer_destroy(ctx, b)
    return u, out, offs


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
def test_uneven_batch_matches_oracle_all_modes(ctx, dtype, tol):
    spec = workloads.Batched1D(count=60, nmin=1, nmax=70000)
    sizes, rs, _ = workloads.batched1d_problems(spec)
    sizes = np.concatenate([[1, 2, 3, 5, 63, 64, 100, 1023, 1024, 4096], sizes])
    rs = np.concatenate([np.full(10, 0.2), rs])
    results = []
    for mode in (hx.HX_BATCH_PERSISTENT, hx.HX_BATCH_GRAPH, hx.HX_BATCH_PLAIN):
        u, out, offs = run_batch(ctx, sizes, rs, 20, dtype, mode, cpl=16)
        results.append(out)
        # guards untouched
        mask = np.ones(out.size, bool)
        for o, n in zip(offs, sizes):
            mask[o:o + n] = False
        assert np.all(out[mask] == -7.0)
    for k, (o, n, r) in enumerate(zip(offs, sizes, rs)):
        ref = oracle.heat1d_periodic(u[o:o + n].astype(np.float64), float(r), 20)
        got = results[0][o:o + n]
        assert rel_l2(got, ref) <= tol and rel_max(got, ref) <= 10 * tol, (k, n)
    # persistent and graph run each problem as one 20-step pass: same arithmetic
    assert np.array_equal(results[0], results[1])
    for o, n in zip(offs, sizes):  # plain runs 20 one-step passes
        assert rel_l2(results[2][o:o + n], results[0][o:o + n]) <= 2 * tol


@pytest.mark.parametrize("cpl", [8, 32, 64])
@pytest.mark.parametrize("grid", [-1, 0, 1, 3])
def test_geometries_bitwise(ctx, cpl, grid):
    """Tile shapes and grid forms (one wave per tile, or persistent waves that
    prefetch their next tile, with 1 or 3 waves per CU so that every wave
    walks many tiles across segment boundaries) give identical bits."""
    sizes = [1000, 50000, 7, 300000, 2000000, 65]
    rs = [0.1, 0.25, 0.05, 0.2, 0.15, 0.45]
    base = run_batch(ctx, sizes, rs, 20, np.float32, hx.HX_BATCH_PERSISTENT, cpl=16, grid=-1)[1]
    got = run_batch(ctx, sizes, rs, 20, np.float32, hx.HX_BATCH_PERSISTENT, cpl=cpl, grid=grid)[1]
    assert np.array_equal(base, got)


def test_halo_coupled_batch_is_one_pass_of_partitions(ctx):
    """A batch whose segments are the partitions of one periodic array, halos
    read from the neighbours' input buffers: one pass of the partitioned graph."""
    n, parts, steps = 150001, 13, 25
    u0 = workloads.uniform(n, 410, 0, 0, 1, np.float32)
    bounds = workloads.partition_bounds(n, parts)
    A = [upload(ctx, u0[o:o + s]) for o, s in bounds]
    B = [hx.hx_buffer_create(ctx, s * 4) for _, s in bounds]
    segs = []
    for p, (o, s) in enumerate(bounds):
        lp, rp = (p - 1) % parts, (p + 1) % parts
        segs.append(hx.segment(inp=A[p], out=B[p], n=s, r=0.25, bc_lo=hx.HX_BC_GHOST,
                               bc_hi=hx.HX_BC_GHOST, halo_lo=A[lp],
                               halo_lo_offset=(bounds[lp][1] - steps) * 4, halo_hi=A[rp],
                               halo_width=steps))
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, steps, segs, hx.HX_BATCH_PERSISTENT)
    ev = hx.hx_launch_batched(ctx, plan)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    got = np.concatenate([download(ctx, b, s, np.float32) for b, (_, s) in zip(B, bounds)])
    ref = oracle.heat1d_periodic(u0.astype(np.float64), 0.25, steps)
    assert rel_l2(got, ref) <= 1e-5
    hx.hx_event_release(ctx, ev)
    hx.hx_plan_destroy(ctx, plan)
    for b in A + B:
        hx.hx_buffer_destroy(ctx, b)


@pytest.mark.parametrize("cpl,grid", [(0, 0), (16, -1), (32, -1), (16, 64)])
def test_full_size_batch_sampled(ctx, cpl, grid):
    """The full 4096-problem workload (sizes log-uniform in [1024, 2^20], r in
    [0.05, 0.25], 20 steps, fp32) as one launch, in the default geometry and in
    the ones the bench sweeps: the 64 smallest problems checked whole, cells of
    64 other problems checked through their light cones."""
    spec = workloads.Batched1D()
    sizes, rs, offs = workloads.batched1d_problems(spec)
    total = int(sizes.sum())
    u0 = workloads.batched1d_u0(spec)
    bin_ = upload(ctx, u0)
    bout = hx.hx_buffer_create(ctx, total * 4)
    segs = [hx.segment(inp=bin_, in_offset=int(o) * 4, out=bout, out_offset=int(o) * 4,
                       n=int(n), r=float(r), bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
            for o, n, r in zip(offs, sizes, rs)]
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, spec.steps, segs, hx.HX_BATCH_PERSISTENT,
                                     cells_per_lane=cpl, grid_waves_per_cu=grid)
    ev = hx.hx_launch_batched(ctx, plan)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    hx.hx_event_release(ctx, ev)
    hx.hx_plan_destroy(ctx, plan)
    small = np.argsort(sizes)[:64]
    for k in small:
        o, n = int(offs[k]), int(sizes[k])
        got = download(ctx, bout, n, np.float32, offset=o * 4)
        ref = oracle.heat1d_periodic(u0[o:o + n].astype(np.float64), float(rs[k]), spec.steps)
        assert rel_l2(got, ref) <= 1e-5
    rng = np.random.default_rng(3)
    for k in rng.choice(spec.count, 64, replace=False):
        o, n = int(offs[k]), int(sizes[k])
        i = int(rng.integers(0, n))
        got = download(ctx, bout, 1, np.float32, offset=(o + i) * 4)[0]
        ref = oracle.heat1d_periodic_at(u0[o:o + n].astype(np.float64), float(rs[k]), spec.steps,
                                        [i])[0]
        assert abs(got - ref) <= 1e-5 * abs(ref)
    hx.hx_buffer_destroy(ctx, bin_)
    hx.hx_buffer_destroy(ctx, bout)


def test_plan_errors(ctx):
    b = hx.hx_buffer_create(ctx, 4096)
    c = hx.hx_buffer_create(ctx, 4096)
    seg = hx.segment(inp=b, out=c, n=1024, r=0.2, bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
    with pytest.raises(hx.HxError):
        hx.hx_plan_create_batched(ctx, hx.HX_F32, 2, [seg], hx.HX_BATCH_PLAIN)  # no tmp
    with pytest.raises(hx.HxError) as e:
        hx.hx_plan_create_batched(ctx, hx.HX_F32, 1000, [seg], hx.HX_BATCH_PERSISTENT, cells_per_lane=8)
    assert e.value.status == hx.HX_ERR_ARG
    bad = hx.segment(inp=b, out=c, n=1025, r=0.2, bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
    with pytest.raises(hx.HxError) as e:
        hx.hx_plan_create_batched(ctx, hx.HX_F32, 1, [seg, bad])
    assert e.value.status == hx.HX_ERR_RANGE
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_batched(ctx, 12345)
    assert e.value.status == hx.HX_ERR_INVALID
    hx.hx_buffer_destroy(ctx, b)
    hx.hx_buffer_destroy(ctx, c)
