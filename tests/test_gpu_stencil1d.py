"""GPU parity of the 1D heat stencil against the FP64 oracle.

Bars: FP64 path <= 1e-12 relative (L2 and max) to the oracle; FP32 path
<= 1e-5 relative L2 to the FP64 oracle run on the same FP32-rounded input.
Launch geometries that differ only in tile shape (cells per lane, waves per
group) must give bit-identical results: a pass's arithmetic depends only on its
step count.  Different pass splits agree within the tolerance.
"""
import numpy as np
import pytest

import oracle
import workloads
from conftest import rel_l2, rel_max

pytestmark = pytest.mark.gpu

hx = pytest.importorskip("paper_1810_11482_amd")
from hxutil import download, run, upload  # noqa: E402

TOL = {np.float64: 1e-12, np.float32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0)
    yield c
    hx.hx_ctx_destroy(c)


def gpu_run(ctx, u0, r, steps, bc=hx.HX_BC_PERIODIC, **geom):
    dt = u0.dtype.type
    code = hx.HX_F64 if dt == np.float64 else hx.HX_F32
    n = u0.size
    bin_ = upload(ctx, u0)
    bout = hx.hx_buffer_create(ctx, u0.nbytes)
    btmp = hx.hx_buffer_create(ctx, u0.nbytes)
    args = hx.stencil_args(dims=1, dtype=code, nx=n, steps=steps, r=r, inp=bin_, out=bout,
                           tmp=btmp, bc_lo=bc, bc_hi=bc, **geom)
    run(ctx, args)
    res = download(ctx, bout, n, dt)
    for b in (bin_, bout, btmp):
        hx.hx_buffer_destroy(ctx, b)
    return res


def test_full_size_fp64_periodic_modes(ctx):
    """2^20 fp64 cells, r = 1/4, 100 steps, sine modes + noise: <= 1e-12."""
    spec = workloads.Periodic1D()
    u0 = workloads.periodic1d_u0(spec)
    ref = oracle.heat1d_periodic(u0, spec.r, spec.steps)
    for geom in [{}, dict(cells_per_lane=16, time_block=100), dict(time_block=1),
                 dict(cells_per_lane=64, time_block=25, waves_per_group=2)]:
        got = gpu_run(ctx, u0, spec.r, spec.steps, **geom)
        e2, em = rel_l2(got, ref), rel_max(got, ref)
        print(f"fp64 2^20 geom={geom}: rel_l2={e2:.3e} rel_max={em:.3e}")
        assert e2 <= 1e-12 and em <= 1e-12


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("bc", [hx.HX_BC_PERIODIC, hx.HX_BC_DIRICHLET0])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 255, 1000, 4099, 65537])
@pytest.mark.parametrize("steps", [0, 1, 5, 33])
def test_small_and_ragged(ctx, dtype, bc, n, steps):
    u0 = workloads.uniform(n, 200, n, -1, 1, dtype)
    ref_fn = oracle.heat1d_periodic if bc == hx.HX_BC_PERIODIC else oracle.heat1d_dirichlet
    ref = ref_fn(u0.astype(np.float64), 0.3, steps)
    got = gpu_run(ctx, u0, 0.3, steps, bc, cells_per_lane=8, time_block=4)
    e = rel_l2(got, ref)
    assert e <= TOL[dtype], e


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("r", [0.0, 0.05, 0.125, 0.25, 0.375, 0.4, 0.45, 0.5])
@pytest.mark.parametrize("tb", [1, 7, 40])
def test_rates_both_update_forms(ctx, dtype, r, tb):
    """Rates 0 <= r <= 3/8 run the rescaled update (with rescales every few
    steps and a remainder factor), larger rates the direct one; both against
    the oracle, across the rate range up to the stability limit 1/2."""
    u0 = workloads.uniform(70001, 204, int(r * 1000), 0, 1, dtype)
    ref = oracle.heat1d_periodic(u0.astype(np.float64), r, 40)
    got = gpu_run(ctx, u0, r, 40, cells_per_lane=16, time_block=tb)
    assert rel_l2(got, ref) <= TOL[dtype] and rel_max(got, ref) <= 10 * TOL[dtype]


@pytest.mark.parametrize("tb", [1, 13, 50])
@pytest.mark.parametrize("cpl,wpg", [(16, 2), (32, 4), (64, 4), (32, 1)])
def test_geometries_bitwise_equal(ctx, cpl, tb, wpg):
    u0 = workloads.uniform(300007, 201, 0, 0, 1, np.float32)
    base = gpu_run(ctx, u0, 0.25, 50, cells_per_lane=8, time_block=tb, waves_per_group=4)
    got = gpu_run(ctx, u0, 0.25, 50, cells_per_lane=cpl, time_block=tb, waves_per_group=wpg)
    assert np.array_equal(base, got)
    ref = oracle.heat1d_periodic(u0.astype(np.float64), 0.25, 50)
    assert rel_l2(got, ref) <= 1e-5


@pytest.mark.parametrize("dtype,r", [(np.float32, 0.25), (np.float32, 0.45), (np.float64, 0.3)])
def test_large_run_persistent_kernel(ctx, dtype, r):
    """A long single run against the same pass as a one-segment batch run by
    the persistent prefetching kernel (2 waves per CU, so every wave walks
    dozens of tiles): bit-identical, and sampled cells against the oracle's
    light cone."""
    n = (1 << 25) + 12345
    steps = 20
    u0 = workloads.uniform(n, 205, int(r * 100), 0, 1, dtype)
    code = hx.HX_F64 if dtype == np.float64 else hx.HX_F32
    es = u0.itemsize
    bin_ = upload(ctx, u0)
    bout = hx.hx_buffer_create(ctx, n * es)
    bref = hx.hx_buffer_create(ctx, n * es)
    run(ctx, hx.stencil_args(dims=1, dtype=code, nx=n, steps=steps, r=r, inp=bin_, out=bout,
                             cells_per_lane=8, time_block=steps))
    plan = hx.hx_plan_create_batched(ctx, code, steps,
                                     [hx.segment(inp=bin_, out=bref, n=n, r=r,
                                                 bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)],
                                     hx.HX_BATCH_PERSISTENT, cells_per_lane=8,
                                     grid_waves_per_cu=2)
    ev = hx.hx_launch_batched(ctx, plan)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    hx.hx_event_release(ctx, ev)
    hx.hx_plan_destroy(ctx, plan)
    got = download(ctx, bout, n, dtype)
    ref_flat = download(ctx, bref, n, dtype)
    assert np.array_equal(got, ref_flat)
    rng = np.random.default_rng(21)
    idx = np.sort(np.concatenate([rng.choice(n, 60, replace=False), [0, 1, n - 2, n - 1]]))
    ref = oracle.heat1d_periodic_at(u0.astype(np.float64), r, steps, idx)
    assert np.max(np.abs(got[idx] - ref) / np.abs(ref)) <= 10 * TOL[dtype]
    for b in (bin_, bout, bref):
        hx.hx_buffer_destroy(ctx, b)


def test_paper_kernel_identity_on_gpu(ctx):
    """Sec. V-A.1's s(x) = 0.5 x_{i-1} + x_i + 0.5 x_{i+1} is 2 x one heat step at r = 1/4."""
    x = workloads.uniform(100003, 202, 0, -1, 1, np.float64)
    got = gpu_run(ctx, x, 0.25, 1)
    assert rel_max(2 * got, oracle.prk_stencil(x)) <= 1e-15


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("parts,steps", [(4, 10), (7, 33), (16, 1)])
def test_partitions_with_neighbour_halos(ctx, dtype, parts, steps):
    """A periodic array split into uneven partitions; each partition's halos are
    read straight from its neighbours' buffers (GHOST), one fused pass."""
    n = 123457
    u0 = workloads.uniform(n, 203, parts, 0, 1, dtype)
    bounds = workloads.partition_bounds(n, parts)
    es = u0.itemsize
    code = hx.HX_F64 if dtype == np.float64 else hx.HX_F32
    bins = [upload(ctx, u0[o:o + s]) for o, s in bounds]
    bouts = [hx.hx_buffer_create(ctx, s * es) for _, s in bounds]
    evs = []
    for p, (o, s) in enumerate(bounds):
        lp, rp = (p - 1) % parts, (p + 1) % parts
        args = hx.stencil_args(dims=1, dtype=code, nx=s, steps=steps, r=0.25, inp=bins[p],
                               out=bouts[p], bc_lo=hx.HX_BC_GHOST, bc_hi=hx.HX_BC_GHOST,
                               halo_lo=bins[lp], halo_lo_offset=(bounds[lp][1] - steps) * es,
                               halo_hi=bins[rp], halo_hi_offset=0, halo_width=steps)
        evs.append(hx.hx_launch_stencil(ctx, args))
    all_ = hx.hx_when_all(ctx, evs)
    assert hx.hx_wait(ctx, all_) == hx.HX_OK
    got = np.concatenate([download(ctx, b, s, dtype) for b, (_, s) in zip(bouts, bounds)])
    ref = oracle.heat1d_periodic(u0.astype(np.float64), 0.25, steps)
    assert rel_l2(got, ref) <= TOL[dtype] and rel_max(got, ref) <= 10 * TOL[dtype]


def test_argument_errors(ctx):
    b = hx.hx_buffer_create(ctx, 4096)
    c = hx.hx_buffer_create(ctx, 4096)
    ok = dict(dims=1, dtype=hx.HX_F32, nx=1024, steps=1, r=0.25, inp=b, out=c)
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_stencil(ctx, hx.stencil_args(**{**ok, "nx": 1025}))
    assert e.value.status == hx.HX_ERR_RANGE
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_stencil(ctx, hx.stencil_args(**{**ok, "out": b}))
    assert e.value.status == hx.HX_ERR_ARG
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_stencil(ctx, hx.stencil_args(**{**ok, "steps": 70, "time_block": 8}))
    assert e.value.status == hx.HX_ERR_ARG  # more than one pass and no tmp
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_stencil(ctx, hx.stencil_args(**{**ok, "bc_lo": hx.HX_BC_GHOST,
                                                     "halo_width": 0}))
    assert e.value.status == hx.HX_ERR_ARG
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_stencil(ctx, hx.stencil_args(**{**ok, "cells_per_lane": 12}))
    assert e.value.status == hx.HX_ERR_ARG
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_stencil(ctx, hx.stencil_args(**ok), deps=[12345])
    assert e.value.status == hx.HX_ERR_INVALID
    hx.hx_buffer_destroy(ctx, b)
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_stencil(ctx, hx.stencil_args(**ok))
    assert e.value.status == hx.HX_ERR_INVALID
    hx.hx_buffer_destroy(ctx, c)
