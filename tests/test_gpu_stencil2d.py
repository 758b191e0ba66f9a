"""GPU parity of the 2D five-point stencil (zero-Dirichlet) against the FP64
oracle, bit-identity across launch geometries and pass splits, row bands
coupled by halo rows, and the full 16384^2 x 200-step workload on sampled
cells."""
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
    c = hx.hx_ctx_create(0, compute_streams=4)
    yield c
    hx.hx_ctx_destroy(c)


def gpu2d(ctx, u0, r, steps, **geom):
    dt = u0.dtype.type
    code = hx.HX_F64 if dt == np.float64 else hx.HX_F32
    ny, nx = u0.shape
    bi = upload(ctx, u0)
    bo = hx.hx_buffer_create(ctx, u0.nbytes)
    bt = hx.hx_buffer_create(ctx, u0.nbytes)
    args = hx.stencil_args(dims=2, dtype=code, nx=nx, ny=ny, steps=steps, r=r, inp=bi, out=bo,
                           tmp=bt, bc_lo=hx.HX_BC_DIRICHLET0, bc_hi=hx.HX_BC_DIRICHLET0, **geom)
    run(ctx, args)
    res = download(ctx, bo, (ny, nx), dt)
    for b in (bi, bo, bt):
        hx.hx_buffer_destroy(ctx, b)
    return res


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (17, 33), (100, 257), (300, 1030), (64, 1024)])
@pytest.mark.parametrize("steps", [0, 1, 5, 13])
def test_small_and_ragged(ctx, dtype, shape, steps):
    u0 = workloads.uniform(shape, 500, shape[0] * 1000 + shape[1], -1, 1, dtype)
    ref = oracle.heat2d_dirichlet(u0.astype(np.float64), 0.2, steps)
    got = gpu2d(ctx, u0, 0.2, steps, time_block=4, rows_per_block=32)
    assert rel_l2(got, ref) <= TOL[dtype], rel_l2(got, ref)


def test_geometries_bitwise(ctx):
    """r = 1/4 runs the direct update, whose arithmetic does not depend on the
    pass depth: every split and tile shape gives the same bits."""
    u0 = workloads.uniform((333, 1500), 501, 0, 0, 1, np.float32)
    base = gpu2d(ctx, u0, 0.25, 48, cells_per_lane=4, time_block=1, rows_per_block=64)
    ref = oracle.heat2d_dirichlet(u0.astype(np.float64), 0.25, 48)
    assert rel_l2(base, ref) <= 1e-5
    for geom in [dict(cells_per_lane=4, time_block=8, rows_per_block=256),
                 dict(cells_per_lane=8, time_block=6, rows_per_block=7),
                 dict(cells_per_lane=4, time_block=16, rows_per_block=100, waves_per_group=1),
                 dict(cells_per_lane=4, time_block=12, rows_per_block=1000),
                 dict(cells_per_lane=4, time_block=10, rows_per_block=33, waves_per_group=2)]:
        got = gpu2d(ctx, u0, 0.25, 48, **geom)
        assert np.array_equal(base, got), geom


@pytest.mark.parametrize("r", [0.2, 0.05, 0.21875, 0.22])
@pytest.mark.parametrize("tb", [4, 6, 8, 16])
def test_rescaled_update_geometries(ctx, r, tb):
    """Rates up to 7/32 run the rescaled update (rescales every few levels and
    a remainder factor at the end of a pass); 0.22 just above runs the direct
    one.  Tile shapes of one depth agree bit for bit; every run matches the
    oracle."""
    u0 = workloads.uniform((300, 1100), 503, int(r * 1000), 0, 1, np.float32)
    steps = 2 * tb + 3
    ref = oracle.heat2d_dirichlet(u0.astype(np.float64), r, steps)
    base = gpu2d(ctx, u0, r, steps, cells_per_lane=4, time_block=tb, rows_per_block=64)
    assert rel_l2(base, ref) <= 1e-5 and rel_max(base, ref) <= 2e-5
    for geom in [dict(cells_per_lane=4, time_block=tb, rows_per_block=13, waves_per_group=1),
                 dict(cells_per_lane=4, time_block=tb, rows_per_block=500, waves_per_group=2)]:
        assert np.array_equal(base, gpu2d(ctx, u0, r, steps, **geom)), geom


def test_fp64_multi_pass_closed_form_mode(ctx):
    ny, nx, k, l, r, steps = 70, 90, 3, 5, 0.2, 37
    i = np.arange(ny)[:, None]
    j = np.arange(nx)[None, :]
    phi = np.sin(np.pi * k * (i + 1) / (ny + 1)) * np.sin(np.pi * l * (j + 1) / (nx + 1))
    mu = 1 - 4 * r * (np.sin(np.pi * k / (2 * (ny + 1))) ** 2 +
                      np.sin(np.pi * l / (2 * (nx + 1))) ** 2)
    got = gpu2d(ctx, phi, r, steps, time_block=8)
    assert np.max(np.abs(got - mu ** steps * phi)) < 1e-13


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("bands,steps,tb", [(4, 20, 5), (7, 24, 8), (3, 16, 16), (20, 12, 4)])
def test_band_graph(ctx, dtype, bands, steps, tb):
    """A grid split into row bands; every band reads its halo rows from its
    neighbours' buffers; future graph over (band, pass)."""
    if dtype == np.float64 and tb > 8:
        pytest.skip("fp64 fused depth is at most 8")
    ny, nx = (211, 517) if bands < 16 else (260, 1024)
    u0 = workloads.uniform((ny, nx), 502, bands, 0, 1, dtype)
    bounds = workloads.band_bounds(ny, bands)
    code = hx.HX_F64 if dtype == np.float64 else hx.HX_F32
    A = [upload(ctx, u0[o:o + s]) for o, s in bounds]
    B = [hx.hx_buffer_create(ctx, s * nx * u0.itemsize) for _, s in bounds]
    outs = []
    for mode in (hx.HX_PART_GRAPH, hx.HX_PART_PLAIN, hx.HX_PART_BATCHED):
        d = hx.partitioned_desc(code, [s for _, s in bounds], A, B, steps, 0.2, periodic=False,
                                mode=mode, time_block=tb, dims=2, nx=nx, rows_per_block=64)
        ev, in_b, _ = hx.hx_run_partitioned(ctx, d)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
        hx.hx_event_release(ctx, ev)
        outs.append(np.concatenate([download(ctx, b, (s, nx), dtype)
                                    for b, (_, s) in zip(B if in_b else A, bounds)]))
        for buf, (o, s) in zip(A, bounds):  # restore the input for the next mode
            src = np.ascontiguousarray(u0[o:o + s])
            e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, src.ctypes.data, buf, 0, 0, 0,
                                                      src.nbytes))
            assert hx.hx_wait(ctx, e) == hx.HX_OK
            hx.hx_event_release(ctx, e)
    ref = oracle.heat2d_dirichlet(u0.astype(np.float64), 0.2, steps)
    for o in outs:  # graph (fused passes) and plain (one step per launch)
        assert rel_l2(o, ref) <= TOL[dtype] and rel_max(o, ref) <= 20 * TOL[dtype]
    if tb == 1:  # one-step passes in both forms: the same arithmetic
        assert np.array_equal(outs[0], outs[1])
    # one launch per band or one per group of bands: the same per-cell arithmetic
    assert np.array_equal(outs[0], outs[2])
    for b in A + B:
        hx.hx_buffer_destroy(ctx, b)


@pytest.mark.parametrize("mode,tb,rows", [(hx.HX_PART_GRAPH, 8, 0),
                                          (hx.HX_PART_BATCHED, 16, 128)])
def test_full_size_banded_sampled(ctx, mode, tb, rows):
    """16384^2 fp32, r = 0.2, 200 steps, 16 row bands with halo-row futures,
    Gaussian-bump initial field, in the per-band graph and in the batched form
    the bench times; 24 cells (corners, band edges, bump centres, random)
    checked against the oracle's light cone."""
    spec = workloads.Banded2D()
    u0 = workloads.banded2d_u0(spec)
    bounds = workloads.band_bounds(spec.ny, spec.bands)
    A = [upload(ctx, u0[o:o + s]) for o, s in bounds]
    B = [hx.hx_buffer_create(ctx, s * spec.nx * 4) for _, s in bounds]
    d = hx.partitioned_desc(hx.HX_F32, [s for _, s in bounds], A, B, spec.steps, spec.r,
                            periodic=False, time_block=tb, dims=2, nx=spec.nx, mode=mode,
                            rows_per_block=rows)
    ev, in_b, _ = hx.hx_run_partitioned(ctx, d)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, ev)
    res = B if in_b else A
    rng = np.random.default_rng(8)
    g = workloads.rng(4, 10)
    yc = g.uniform(0, spec.ny, spec.centres)
    xc = g.uniform(0, spec.nx, spec.centres)
    pts = [(0, 0), (spec.ny - 1, spec.nx - 1), (1023, 5000), (1024, 5000), (8191, 17)]
    pts += [(int(yc[c]), int(xc[c])) for c in range(8)]
    pts += [(int(rng.integers(0, spec.ny)), int(rng.integers(0, spec.nx))) for _ in range(11)]
    ref = oracle.heat2d_dirichlet_at(u0.astype(np.float64), spec.r, spec.steps, pts)
    for (y, x), rv in zip(pts, ref):
        band = next(k for k, (o, s) in enumerate(bounds) if o <= y < o + s)
        got = download(ctx, res[band], 1, np.float32,
                       offset=((y - bounds[band][0]) * spec.nx + x) * 4)[0]
        assert abs(got - rv) <= 1e-5 * max(abs(rv), 1e-3), ((y, x), got, rv)
    for b in A + B:
        hx.hx_buffer_destroy(ctx, b)


def test_2d_argument_errors(ctx):
    b = hx.hx_buffer_create(ctx, 64 * 64 * 4)
    c = hx.hx_buffer_create(ctx, 64 * 64 * 4)
    ok = dict(dims=2, dtype=hx.HX_F32, nx=64, ny=64, steps=4, r=0.2, inp=b, out=c,
              bc_lo=hx.HX_BC_DIRICHLET0, bc_hi=hx.HX_BC_DIRICHLET0)
    for bad, st in [({"bc_lo": hx.HX_BC_PERIODIC}, hx.HX_ERR_ARG),
                    ({"ny": 65}, hx.HX_ERR_RANGE),
                    ({"time_block": 9}, hx.HX_ERR_ARG),
                    ({"cells_per_lane": 16}, hx.HX_ERR_ARG),
                    ({"bc_lo": hx.HX_BC_GHOST, "halo_lo": b, "halo_width": 2}, hx.HX_ERR_ARG)]:
        with pytest.raises(hx.HxError) as e:
            hx.hx_launch_stencil(ctx, hx.stencil_args(**{**ok, **bad}))
        assert e.value.status == st, bad
    hx.hx_buffer_destroy(ctx, b)
    hx.hx_buffer_destroy(ctx, c)
