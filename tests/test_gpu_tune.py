"""The autotuner picks a geometry that runs, stores it, and later default
launches use it; results never depend on the geometry."""
import json
import os

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
    c = hx.hx_ctx_create(0)
    yield c
    hx.hx_ctx_destroy(c)


def test_tune_1d_and_2d(ctx, tmp_path):
    hx.hx_tune_cache_clear()
    n = 1 << 22
    u0 = workloads.uniform(n, 900, 0, 0, 1, np.float32)
    a, b, t = upload(ctx, u0), hx.hx_buffer_create(ctx, n * 4), hx.hx_buffer_create(ctx, n * 4)
    args = hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=n, steps=50, r=0.25, inp=a, out=b, tmp=t)
    best = hx.hx_tune_stencil(ctx, args, 1500)
    assert best.cells_per_lane in (8, 16, 32, 64) and 1 <= best.time_block <= 50
    ev = hx.hx_launch_stencil(ctx, args)  # geometry from the cache
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    got = download(ctx, b, n, np.float32)
    idx = np.arange(0, n, n // 29)
    ref = oracle.heat1d_periodic_at(u0.astype(np.float64), 0.25, 50, idx)
    assert np.max(np.abs(got[idx] - ref) / ref) <= 1e-5

    ny, nx = 1024, 2048
    v0 = workloads.uniform((ny, nx), 901, 0, 0, 1, np.float32)
    c2, d2, t2 = upload(ctx, v0), hx.hx_buffer_create(ctx, v0.nbytes), \
        hx.hx_buffer_create(ctx, v0.nbytes)
    args2 = hx.stencil_args(dims=2, dtype=hx.HX_F32, nx=nx, ny=ny, steps=40, r=0.2, inp=c2,
                            out=d2, tmp=t2, bc_lo=hx.HX_BC_DIRICHLET0, bc_hi=hx.HX_BC_DIRICHLET0)
    best2 = hx.hx_tune_stencil(ctx, args2, 1500)
    assert best2.cells_per_lane in (4, 8) and best2.rows_per_block > 0
    ev = hx.hx_launch_stencil(ctx, args2)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    got2 = download(ctx, d2, (ny, nx), np.float32)
    pts = [(0, 0), (511, 1024), (1023, 2047), (7, 2000)]
    ref2 = oracle.heat2d_dirichlet_at(v0.astype(np.float64), 0.2, 40, pts)
    for p, r in zip(pts, ref2):
        assert abs(got2[p] - r) <= 1e-5 * max(abs(r), 1e-3)

    path = str(tmp_path / "tune.json")
    hx.hx_tune_cache_save(path)
    saved = json.load(open(path))
    assert any(k.startswith("stencil1d/f32") for k in saved)
    assert any(k.startswith("stencil2d/f32") for k in saved)


def test_tune_batched(ctx):
    spec = workloads.Batched1D(count=200, nmax=100000)
    sizes, rs, offs = workloads.batched1d_problems(spec)
    total = int(sizes.sum())
    u0 = workloads.batched1d_u0(spec)
    a, b = upload(ctx, u0), hx.hx_buffer_create(ctx, total * 4)
    segs = [hx.segment(inp=a, in_offset=int(o) * 4, out=b, out_offset=int(o) * 4, n=int(n),
                       r=float(r), bc_lo=0, bc_hi=0) for o, n, r in zip(offs, sizes, rs)]
    best = hx.hx_tune_batched(ctx, hx.HX_F32, spec.steps, segs, 1000)
    assert best.cells_per_lane in (8, 16, 32, 64)
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, spec.steps, segs)  # tuned defaults
    ev = hx.hx_launch_batched(ctx, plan)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    k = int(np.argmin(sizes))
    o, n = int(offs[k]), int(sizes[k])
    got = download(ctx, b, n, np.float32, offset=o * 4)
    ref = oracle.heat1d_periodic(u0[o:o + n].astype(np.float64), float(rs[k]), spec.steps)
    assert rel_l2(got, ref) <= 1e-5
    hx.hx_plan_destroy(ctx, plan)


def test_tune_batched_depth_runs_the_whole_run(ctx):
    """The batched tuner searches the pass depth: its answer divides the run's
    steps, and T / D passes of the tuned plan (ping-ponging between two
    buffers) equal the oracle's T steps.  In a timing context it times the
    candidates with HIP events."""
    tctx = hx.hx_ctx_create(0, timing=True)
    try:
        spec = workloads.Batched1D(count=64, nmax=200000, steps=20)
        sizes, rs, offs = workloads.batched1d_problems(spec)
        total = int(sizes.sum())
        u0 = workloads.batched1d_u0(spec)
        a, b = upload(tctx, u0), hx.hx_buffer_create(tctx, total * 4)
        fwd = [hx.segment(inp=a, in_offset=int(o) * 4, out=b, out_offset=int(o) * 4, n=int(n),
                          r=float(r), bc_lo=0, bc_hi=0) for o, n, r in zip(offs, sizes, rs)]
        back = [hx.segment(inp=b, in_offset=int(o) * 4, out=a, out_offset=int(o) * 4, n=int(n),
                           r=float(r), bc_lo=0, bc_hi=0) for o, n, r in zip(offs, sizes, rs)]
        best = hx.hx_tune_batched(tctx, hx.HX_F32, spec.steps, fwd, 1500)
        D = best.steps
        assert 1 <= D <= 64 and spec.steps % D == 0
        # the run, from the initial state again (the tuner wrote b only)
        kw = dict(cells_per_lane=best.cells_per_lane, waves_per_group=best.waves_per_group,
                  grid_waves_per_cu=best.grid_waves_per_cu, form=best.form,
                  span_blocks=best.span_blocks)
        plans = [hx.hx_plan_create_batched(tctx, hx.HX_F32, D, segs, hx.HX_BATCH_PERSISTENT, **kw)
                 for segs in (fwd, back)]
        last = []
        for k in range(spec.steps // D):
            e = hx.hx_launch_batched(tctx, plans[k % 2], deps=last)
            for x in last:
                hx.hx_event_release(tctx, x)
            last = [e]
        assert hx.hx_wait(tctx, last[0]) == hx.HX_OK, hx.hx_last_error(tctx)
        hx.hx_event_release(tctx, last[0])
        res = b if (spec.steps // D) % 2 == 1 else a
        got = download(tctx, res, total, np.float32)
        ref = oracle.heat1d_batched(sizes, rs, u0.astype(np.float64), spec.steps)
        assert rel_l2(got, ref) <= 1e-5
        for pl in plans:
            hx.hx_plan_destroy(tctx, pl)
        hx.hx_buffer_destroy(tctx, a)
        hx.hx_buffer_destroy(tctx, b)
    finally:
        hx.hx_ctx_destroy(tctx)
