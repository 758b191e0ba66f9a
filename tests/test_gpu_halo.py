"""Halo pack/unpack plans: bitwise against numpy slicing (contiguous row
halos and strided column halos), and a ghost-slot partitioned graph (one pack
launch per pass, stencils reading their halos from the ghost slots) against
the oracle, hazard-free."""
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


def run_plan(ctx, descs, deps=()):
    plan = hx.hx_plan_create_halo(ctx, descs)
    ev = hx.hx_launch_halo(ctx, plan, deps)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, ev)
    hx.hx_plan_destroy(ctx, plan)


@pytest.mark.parametrize("ny,nx,D", [(50, 77, 3), (64, 256, 8), (7, 5, 2)])
def test_pack_and_unpack(ctx, ny, nx, D):
    u = workloads.uniform((ny, nx), 800, nx, -1, 1, np.float32)
    bu = upload(ctx, u)
    nb = 4 * nx
    ghost_cells = 2 * D * nx + 2 * D * ny
    bg = upload(ctx, np.full(ghost_cells, np.nan, np.float32))
    off_bot = D * nx * 4
    off_left = 2 * D * nx * 4
    off_right = off_left + D * ny * 4
    pack = [hx.hx_halo_desc(bu, 0, bg, 0, 1, D * nb, 0, 0),                        # top rows
            hx.hx_halo_desc(bu, (ny - D) * nb, bg, off_bot, 1, D * nb, 0, 0),      # bottom rows
            hx.hx_halo_desc(bu, 0, bg, off_left, ny, D * 4, nb, D * 4),            # left cols
            hx.hx_halo_desc(bu, (nx - D) * 4, bg, off_right, ny, D * 4, nb, D * 4)]
    run_plan(ctx, pack)
    g = download(ctx, bg, ghost_cells, np.float32)
    assert np.array_equal(g[:D * nx], u[:D].ravel())
    assert np.array_equal(g[D * nx:2 * D * nx], u[ny - D:].ravel())
    assert np.array_equal(g[2 * D * nx:2 * D * nx + D * ny], u[:, :D].ravel())
    assert np.array_equal(g[2 * D * nx + D * ny:], u[:, nx - D:].ravel())
    # unpack into the ghost frame of a padded array
    P = np.zeros((ny + 2 * D, nx + 2 * D), np.float32)
    bp = upload(ctx, P)
    pn = (nx + 2 * D) * 4
    unpack = [hx.hx_halo_desc(bg, 0, bp, D * 4, D, nx * 4, nx * 4, pn),
              hx.hx_halo_desc(bg, off_bot, bp, (ny + D) * pn + D * 4, D, nx * 4, nx * 4, pn),
              hx.hx_halo_desc(bg, off_left, bp, D * pn, ny, D * 4, D * 4, pn),
              hx.hx_halo_desc(bg, off_right, bp, D * pn + (nx + D) * 4, ny, D * 4, D * 4, pn)]
    run_plan(ctx, unpack)
    got = download(ctx, bp, P.shape, np.float32)
    ref = P.copy()
    ref[:D, D:D + nx] = u[:D]
    ref[ny + D:, D:D + nx] = u[ny - D:]
    ref[D:D + ny, :D] = u[:, :D]
    ref[D:D + ny, nx + D:] = u[:, nx - D:]
    assert np.array_equal(got, ref)
    assert hx.hx_hazard_count(ctx) == 0


@pytest.mark.parametrize("parts,steps,D", [(5, 30, 6), (8, 20, 20), (3, 12, 4)])
def test_ghost_slot_graph(ctx, parts, steps, D):
    n = 30011
    u0 = workloads.uniform(n, 801, parts, 0, 1, np.float32)
    bounds = workloads.partition_bounds(n, parts)
    A = [upload(ctx, u0[o:o + s]) for o, s in bounds]
    B = [hx.hx_buffer_create(ctx, s * 4) for _, s in bounds]
    G = hx.hx_buffer_create(ctx, 2 * D * parts * 4)
    plans = []
    for src in (A, B):
        descs = []
        for p in range(parts):
            lp, rp = (p - 1) % parts, (p + 1) % parts
            descs.append(hx.hx_halo_desc(src[lp], (bounds[lp][1] - D) * 4, G, 2 * D * p * 4, 1,
                                         D * 4, 0, 0))
            descs.append(hx.hx_halo_desc(src[rp], 0, G, (2 * D * p + D) * 4, 1, D * 4, 0, 0))
        plans.append(hx.hx_plan_create_halo(ctx, descs))
    prev = []
    for b in range(steps // D):
        src, dst = (A, B) if b % 2 == 0 else (B, A)
        pk = hx.hx_launch_halo(ctx, plans[b % 2], prev)
        cur = []
        for p, (o, s) in enumerate(bounds):
            a = hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=s, steps=D, r=0.25, inp=src[p],
                                out=dst[p], bc_lo=hx.HX_BC_GHOST, bc_hi=hx.HX_BC_GHOST,
                                halo_lo=G, halo_lo_offset=2 * D * p * 4, halo_hi=G,
                                halo_hi_offset=(2 * D * p + D) * 4, halo_width=D)
            cur.append(hx.hx_launch_stencil(ctx, a, [pk]))
        prev = cur
    assert hx.hx_wait(ctx, hx.hx_when_all(ctx, prev)) == hx.HX_OK
    res = B if (steps // D) % 2 == 1 else A
    got = np.concatenate([download(ctx, b, s, np.float32) for b, (_, s) in zip(res, bounds)])
    ref = oracle.heat1d_periodic(u0.astype(np.float64), 0.25, steps)
    assert rel_l2(got, ref) <= 1e-5
    assert hx.hx_hazard_count(ctx) == 0, hx.hx_hazard_report(ctx)


def test_halo_plan_errors(ctx):
    b = hx.hx_buffer_create(ctx, 1024)
    c = hx.hx_buffer_create(ctx, 1024)
    for desc, st in [(hx.hx_halo_desc(b, 0, c, 0, 1, 6, 0, 0), hx.HX_ERR_ARG),       # not x4
                     (hx.hx_halo_desc(b, 0, c, 0, 3, 512, 512, 512), hx.HX_ERR_RANGE),
                     (hx.hx_halo_desc(b, 0, b, 64, 1, 128, 0, 0), hx.HX_ERR_ARG),     # overlap
                     (hx.hx_halo_desc(b, 0, c, 0, 2, 64, 32, 64), hx.HX_ERR_ARG)]:    # pitch
        with pytest.raises(hx.HxError) as e:
            hx.hx_plan_create_halo(ctx, [desc])
        assert e.value.status == st
