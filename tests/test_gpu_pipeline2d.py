"""GPU parity of the host-to-host 2D band pipeline (Pipeline2D): every band
copied in, advanced over several kernel passes on its extended rows (its own
plus the light cone's halo rows, filled by device copies from the
neighbours), and copied out, against the FP64 oracle on the whole grid; the
copies-only run returns its input; the composed graph is hazard-free under
the runtime's checker, and every band's kernel waits only for its own and its
neighbours' copies in."""
import numpy as np
import pytest

import oracle
import workloads
from conftest import rel_l2, rel_max

pytestmark = pytest.mark.gpu
hx = pytest.importorskip("paper_1810_11482_amd")
from paper_1810_11482_amd.pipeline2d import Pipeline2D  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0, check=True, timing=True)
    yield c
    hx.hx_ctx_destroy(c)


def host_grid(ctx, a):
    p = hx.hx_host_alloc(ctx, a.nbytes)
    v = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * a.size).from_address(p))
    v[:] = a.ravel()
    return p, v


@pytest.mark.parametrize("ny,nx,bands,steps,tb", [(390, 260, 4, 40, 16), (512, 256, 8, 64, 16),
                                                  (300, 100, 3, 17, 8), (128, 64, 1, 30, 12)])
def test_pipeline2d_matches_oracle(ctx, ny, nx, bands, steps, tb):
    r = 0.2
    u0 = workloads.uniform(ny * nx, 610, steps, 0, 1, np.float32).reshape(ny, nx)
    hin, _ = host_grid(ctx, u0)
    hout, out = host_grid(ctx, np.full((ny, nx), np.nan, np.float32))
    bounds = workloads.band_bounds(ny, bands)
    pl = Pipeline2D(ctx, ny, nx, bounds, steps, r, time_block=tb)
    n0 = hx.hx_hazard_count(ctx)
    ev, h2d, ker, d2h = pl.run(hin, hout)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    assert hx.hx_hazard_count(ctx) == n0, hx.hx_hazard_report(ctx)
    # every band's kernel starts after its own and its upper neighbour's
    # copies in have ended and after its lower neighbour's first rows (its
    # bottom halo) are in, and its copy out starts after it has ended
    assert len(pl.h2d_index) == bands and sum(map(len, pl.h2d_index)) == len(h2d)
    for p in range(bands):
        ks, ke = hx.hx_event_span(ctx, ker[p], h2d[0])
        need = [pl.h2d_index[q][-1] for q in range(max(0, p - 1), p + 1)]
        if p + 1 < bands:
            need.append(pl.h2d_index[p + 1][0])
        for i in need:
            assert hx.hx_event_span(ctx, h2d[i], h2d[0])[1] <= ks + 1e-6
        assert ke <= hx.hx_event_span(ctx, d2h[p], h2d[0])[0] + 1e-6
    # a band's copy in is split in two exactly where a neighbour reads its first rows
    assert all(len(pl.h2d_index[p]) == (2 if p >= 1 and pl.bot[p - 1] < bounds[p][1] else 1)
               for p in range(bands))
    for e in [ev] + h2d + ker + d2h:
        hx.hx_event_release(ctx, e)
    ref = oracle.heat2d_dirichlet(u0.astype(np.float64), r, steps)
    got = out.reshape(ny, nx)
    assert rel_l2(got, ref) <= 1e-5 and rel_max(got, ref) <= 1e-5
    # copies alone return the input
    ev, h2d, ker, d2h = pl.run(hin, hout, kernels=False)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    assert not ker
    for e in [ev] + h2d + d2h:
        hx.hx_event_release(ctx, e)
    assert np.array_equal(out.reshape(ny, nx), u0)
    pl.close()
    hx.hx_host_free(ctx, hin)
    hx.hx_host_free(ctx, hout)


def test_pipeline2d_rejects_thin_bands(ctx):
    with pytest.raises(ValueError):
        Pipeline2D(ctx, 100, 64, workloads.band_bounds(100, 4), 30, 0.2)


def test_pipeline2d_full_size_sampled(ctx):
    """The benchmark's configuration: 16384^2 fp32, 16 bands, r = 0.2, 200
    steps, Gaussian bumps, 64 rows per wave; sampled cells (band seams, grid
    edges, random points) against the oracle's light cones."""
    spec = workloads.Banded2D()
    u0 = workloads.banded2d_u0(spec)
    ny, nx, T, r = spec.ny, spec.nx, spec.steps, spec.r
    hin, _ = host_grid(ctx, u0)
    hout, out = host_grid(ctx, np.zeros(ny * nx, np.float32))
    pl = Pipeline2D(ctx, ny, nx, workloads.band_bounds(ny, spec.bands), T, r, time_block=16,
                    cells_per_lane=4, rows_per_block=64)
    ev, h2d, ker, d2h = pl.run(hin, hout)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    for e in [ev] + h2d + ker + d2h:
        hx.hx_event_release(ctx, e)
    rng = np.random.default_rng(23)
    pts = [(0, 0), (ny - 1, nx - 1), (1023, 7000), (1024, 7000), (8191, 100), (8192, 100)] + \
        [(int(a), int(b)) for a, b in zip(rng.integers(0, ny, 6), rng.integers(0, nx, 6))]
    ref = oracle.heat2d_dirichlet_at(u0, r, T, pts)
    got = np.array([out[y * nx + x] for y, x in pts], dtype=np.float64)
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)) <= 1e-5
    pl.close()
    hx.hx_host_free(ctx, hin)
    hx.hx_host_free(ctx, hout)
