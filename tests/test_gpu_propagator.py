"""GPU parity of the propagator form of a batched 1D pass against the oracle's
stepping.  The form runs D steps as one convolution with the D-step propagator
on the matrix cores.

Covered:
- periodic segments and halo-coupled partitions, depths 1..64, ragged sizes
  and every span of blocks per wave;
- identical bits for every span;
- the interleaved walk (segments of one size and one rate, fp16 two-term
  split at a per-window scale): the oracle, the span walk within the
  tolerance, waves of one and of several blocks, halo-coupled partitions,
  extreme and mixed magnitudes, and the plan's rejections;
- the plan rejects segments the form cannot take, and AUTO falls back to the
  direct form for them;
- the full-size headline form (2^28 cells, 64 partition views of one arena,
  50 steps), every cell against the oracle;
- the accuracy check after the products: spikes up to 1e30 on U[0,1],
  windows spanning 20 orders of magnitude, zero crossings and NaN/inf input
  cells, each cell against the oracle (blocks that fail the check are
  stepped).

The FP32 bar is the suite's: 1e-5 relative (L2 and per cell) against FP64."""
import numpy as np
import pytest

import oracle
import workloads
from conftest import rel_l2, rel_max

pytestmark = pytest.mark.gpu
hx = pytest.importorskip("paper_1810_11482_amd")
from hxutil import download, upload  # noqa: E402

GUARD = 64  # guard cells between packed segments (a multiple of 4)


@pytest.fixture(scope="module")
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0)
    yield c
    hx.hx_ctx_destroy(c)


def periodic_batch(ctx, sizes, rs, steps, form, span=0, seed=0, sentinel=-7.0):
    """Segments packed at 16-byte-aligned offsets of one buffer, run once;
    returns (input, output, offsets)."""
    offs, o = [], GUARD
    for n in sizes:
        offs.append(o)
        o += -(-int(n) // 4) * 4 + GUARD
    total = o
    u = np.full(total, sentinel, dtype=np.float32)
    for k, (o, n) in enumerate(zip(offs, sizes)):
        u[o:o + n] = workloads.uniform(int(n), 500 + seed, k, 0, 1, np.float32)
    bin_ = upload(ctx, u)
    bout = upload(ctx, np.full(total, sentinel, dtype=np.float32))
    segs = [hx.segment(inp=bin_, in_offset=o * 4, out=bout, out_offset=o * 4, n=int(n),
                       r=float(r), bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
            for o, n, r in zip(offs, sizes, rs)]
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, steps, segs, hx.HX_BATCH_PERSISTENT,
                                     form=form, span_blocks=span)
    ev = hx.hx_launch_batched(ctx, plan)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, ev)
    hx.hx_plan_destroy(ctx, plan)
    out = download(ctx, bout, total, np.float32)
    hx.hx_buffer_destroy(ctx, bin_)
    hx.hx_buffer_destroy(ctx, bout)
    return u, out, offs


def sizes_for(D):
    """Ragged periodic sizes (multiples of 4, at least D) spanning the edge and
    interior wave paths: tiny, just under and over a 1024-cell block, several
    spans."""
    m = -(-D // 4) * 4
    return [m, max(m, 64), 1000, 1024, 1028, 4108, 30000, 262180]


@pytest.mark.parametrize("D", [1, 3, 8, 20, 33, 50, 64])
def test_periodic_segments_match_oracle(ctx, D):
    sizes = sizes_for(D)
    rs = [0.25, 0.05, 0.45, 0.2, 0.125, 0.3, 0.25, 0.1][:len(sizes)]
    u, out, offs = periodic_batch(ctx, sizes, rs, D, hx.HX_FORM_PROPAGATOR, seed=D)
    mask = np.ones(out.size, bool)
    for k, (o, n, r) in enumerate(zip(offs, sizes, rs)):
        mask[o:o + n] = False
        ref = oracle.heat1d_periodic(u[o:o + n].astype(np.float64), float(r), D)
        got = out[o:o + n]
        e2, em = rel_l2(got, ref), rel_max(got, ref)
        assert e2 <= 1e-5 and em <= 1e-5, (D, k, n, e2, em)
    assert np.all(out[mask] == -7.0)  # guards untouched


def test_spans_give_identical_bits(ctx):
    """Every cell's taps meet the same window values in the same order,
    whether its wave is an edge or an interior wave and however many blocks
    a wave walks."""
    sizes, rs = [4108, 30000, 262180, 64, 2052], [0.25, 0.1, 0.2, 0.3, 0.45]
    base = periodic_batch(ctx, sizes, rs, 50, hx.HX_FORM_PROPAGATOR, span=0)[1]
    for span in (1, 2, 3, 5, 6, 7, 13, 40):
        got = periodic_batch(ctx, sizes, rs, 50, hx.HX_FORM_PROPAGATOR, span=span)[1]
        assert np.array_equal(base, got), span


@pytest.mark.parametrize("D,hw_extra", [(50, 0), (50, 6), (17, 3), (64, 0)])
def test_halo_coupled_partitions(ctx, D, hw_extra):
    """Partitions of one periodic array laid back to back in one buffer, halos
    read from the neighbours' views: one pass equals the oracle on the whole
    array, and agrees with the direct form within the tolerance."""
    sizes = [4096, 1028, 70000, 8, 1024 * 37, 9000, 65536] if D <= 8 else \
        [4096, 1028, 70000, 68, 1024 * 37, 9000, 65536]
    n = sum(sizes)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    u0 = workloads.uniform(n, 510, D, 0, 1, np.float32)
    hw = 4 * (-(-D // 4)) + hw_extra
    a = upload(ctx, u0)
    results = []
    for form in (hx.HX_FORM_PROPAGATOR, hx.HX_FORM_DIRECT):
        b = hx.hx_buffer_create(ctx, n * 4)
        segs = []
        P = len(sizes)
        for p in range(P):
            lp, rp = (p - 1) % P, (p + 1) % P
            segs.append(hx.segment(inp=a, in_offset=int(offs[p]) * 4, out=b,
                                   out_offset=int(offs[p]) * 4, n=sizes[p], r=0.25,
                                   bc_lo=hx.HX_BC_GHOST, bc_hi=hx.HX_BC_GHOST, halo_lo=a,
                                   halo_lo_offset=int(offs[lp] + sizes[lp] - hw) * 4,
                                   halo_hi=a, halo_hi_offset=int(offs[rp]) * 4, halo_width=hw))
        plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, D, segs, hx.HX_BATCH_PERSISTENT,
                                         form=form)
        ev = hx.hx_launch_batched(ctx, plan)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
        hx.hx_event_release(ctx, ev)
        hx.hx_plan_destroy(ctx, plan)
        results.append(download(ctx, b, n, np.float32))
        hx.hx_buffer_destroy(ctx, b)
    hx.hx_buffer_destroy(ctx, a)
    ref = oracle.heat1d_periodic(u0.astype(np.float64), 0.25, D)
    prop, direct = results
    assert rel_l2(prop, ref) <= 1e-5 and rel_max(prop, ref) <= 1e-5
    assert rel_l2(prop, direct) <= 1e-5


def test_unfit_segments_rejected_and_auto_falls_back(ctx):
    b = hx.hx_buffer_create(ctx, 1 << 16)
    c = hx.hx_buffer_create(ctx, 1 << 16)
    per = dict(bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
    ok = hx.segment(inp=b, out=c, n=1024, r=0.2, **per)
    cases = [
        (hx.HX_F64, 20, [ok], hx.HX_BATCH_PERSISTENT),                        # f64
        (hx.HX_F32, 65, [ok], hx.HX_BATCH_PERSISTENT),                        # too deep
        (hx.HX_F32, 20, [ok], hx.HX_BATCH_GRAPH),                             # not persistent
        (hx.HX_F32, 20, [hx.segment(inp=b, out=c, n=1022, r=0.2, **per)],
         hx.HX_BATCH_PERSISTENT),                                             # n % 4
        (hx.HX_F32, 20, [hx.segment(inp=b, in_offset=4, out=c, n=1024, r=0.2, **per)],
         hx.HX_BATCH_PERSISTENT),                                             # misaligned
        (hx.HX_F32, 20, [hx.segment(inp=b, out=c, n=1024, r=0.2, bc_lo=hx.HX_BC_DIRICHLET0,
                                    bc_hi=hx.HX_BC_DIRICHLET0)],
         hx.HX_BATCH_PERSISTENT),                                             # Dirichlet
        (hx.HX_F32, 18, [hx.segment(inp=b, out=c, n=1024, r=0.2, bc_lo=hx.HX_BC_GHOST,
                                    bc_hi=hx.HX_BC_GHOST, halo_lo=b, halo_lo_offset=8192,
                                    halo_hi=b, halo_hi_offset=12288, halo_width=18)],
         hx.HX_BATCH_PERSISTENT),                                  # halo 18 < 4 ceil(18/4)
        (hx.HX_F32, 20, [hx.segment(inp=b, out=c, n=16, r=0.2, **per)],
         hx.HX_BATCH_PERSISTENT),                                             # n < steps
    ]
    for dt, steps, segs, mode in cases:
        with pytest.raises(hx.HxError) as e:
            hx.hx_plan_create_batched(ctx, dt, steps, segs, mode, form=hx.HX_FORM_PROPAGATOR)
        assert e.value.status == hx.HX_ERR_ARG
    with pytest.raises(hx.HxError) as e:
        hx.hx_plan_create_batched(ctx, hx.HX_F32, 20, [ok], form=7)
    assert e.value.status == hx.HX_ERR_ARG
    # AUTO over an unfit (Dirichlet) segment runs the direct form
    d = hx.segment(inp=b, out=c, n=1024, r=0.2, bc_lo=hx.HX_BC_DIRICHLET0,
                   bc_hi=hx.HX_BC_DIRICHLET0)
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, 20, [d], form=hx.HX_FORM_AUTO)
    hx.hx_plan_destroy(ctx, plan)
    hx.hx_buffer_destroy(ctx, b)
    hx.hx_buffer_destroy(ctx, c)


def test_auto_takes_the_propagator_where_every_segment_fits(ctx):
    sizes, rs = [4108, 30000, 64], [0.25, 0.1, 0.3]
    prop = periodic_batch(ctx, sizes, rs, 30, hx.HX_FORM_PROPAGATOR)[1]
    auto = periodic_batch(ctx, sizes, rs, 30, hx.HX_FORM_AUTO)[1]
    direct = periodic_batch(ctx, sizes, rs, 30, hx.HX_FORM_DIRECT)[1]
    assert np.array_equal(prop, auto)
    assert not np.array_equal(prop, direct)  # a different evaluation, same result to f32


def test_full_size_headline_form_every_cell(ctx):
    """2^28 fp32 cells as 64 partition views of one HBM arena, r = 0.25,
    50 steps as one propagator launch (halos of 52 cells from the neighbour
    views), in the plan's own walk and in the block walk: the whole array
    against the oracle's serial FP64 run (about 8 s on one core), 1e-5
    relative L2 and 1e-5 of itself in every cell, and the two walks bit for
    bit."""
    n, parts, T, r, hw = 1 << 28, 64, 50, 0.25, 52
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
                               halo_lo_offset=(bounds[lp][1] - hw) * 4, halo_hi=A[rp],
                               halo_width=hw))
    outs = []
    for span in (0, -2):
        plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, T, segs, hx.HX_BATCH_PERSISTENT,
                                         form=hx.HX_FORM_PROPAGATOR, span_blocks=span)
        ev = hx.hx_launch_batched(ctx, plan)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
        hx.hx_event_release(ctx, ev)
        hx.hx_plan_destroy(ctx, plan)
        outs.append(download(ctx, arena_b, n, np.float32))
    got = outs[0]
    assert np.array_equal(outs[1], got)
    ref = oracle.heat1d_periodic(u0.astype(np.float64), r, T)
    for b in A + B + [arena_a, arena_b]:
        hx.hx_buffer_destroy(ctx, b)
    hx.hx_host_free(ctx, hin)
    err2 = rel_l2(got, ref)
    errc = float(np.max(np.abs(got - ref) / np.abs(ref)))
    print(f"full 2^28 array vs oracle: rel L2 {err2:.3e}, max per cell {errc:.3e}")
    assert err2 <= 1e-5 and errc <= 1e-5


@pytest.mark.parametrize("D,n,count", [(1, 1028, 5), (20, 4108, 7), (50, 30000, 3),
                                       (64, 1000, 4), (50, 4000000, 3), (33, 64, 9)])
def test_interleaved_walk_matches_oracle_and_spans(ctx, D, n, count):
    """Segments of one size and one rate, walked interleaved (span_blocks = -1):
    the oracle on every segment, the span walk within the tolerance, and the
    same bits as the block walk (span_blocks = -2) and the plan's own choice
    (the block walk).  With
    1.2 x 10^7 cells the launch has about four times as many blocks as the
    persistent grid has waves, so waves take several blocks; n = 1000 and
    1028 leave a partial last block, n = 64 a segment of one partial block."""
    sizes, rs = [n] * count, [0.2] * count
    u, il, offs = periodic_batch(ctx, sizes, rs, D, hx.HX_FORM_PROPAGATOR, span=-1, seed=D + 7)
    span = periodic_batch(ctx, sizes, rs, D, hx.HX_FORM_PROPAGATOR, span=5, seed=D + 7)[1]
    auto = periodic_batch(ctx, sizes, rs, D, hx.HX_FORM_PROPAGATOR, span=0, seed=D + 7)[1]
    bw = periodic_batch(ctx, sizes, rs, D, hx.HX_FORM_PROPAGATOR, span=-2, seed=D + 7)[1]
    assert np.array_equal(il, auto)
    # the block walk runs the same arithmetic in the same order
    assert np.array_equal(bw, il)
    mask = np.ones(il.size, bool)
    for k, o in enumerate(offs):
        mask[o:o + n] = False
        ref = oracle.heat1d_periodic(u[o:o + n].astype(np.float64), 0.2, D)
        got = il[o:o + n]
        assert rel_l2(got, ref) <= 1e-5 and rel_max(got, ref) <= 1e-5, (D, n, k)
        assert rel_l2(got, span[o:o + n]) <= 1e-5
    assert np.all(il[mask] == -7.0)  # guards untouched


@pytest.mark.parametrize("D,hw", [(50, 52), (17, 23), (8, 8)])
def test_interleaved_halo_coupled_partitions(ctx, D, hw):
    """Equal partitions of one periodic array, halos from the neighbours'
    views, walked interleaved: the oracle on the whole array, and the span
    walk within the tolerance."""
    P, m = 9, 70004
    n = P * m
    u0 = workloads.uniform(n, 511, D, 0, 1, np.float32)
    a = upload(ctx, u0)
    results = []
    for span in (-1, 3, -2):
        b = hx.hx_buffer_create(ctx, n * 4)
        segs = []
        for p in range(P):
            lp, rp = (p - 1) % P, (p + 1) % P
            segs.append(hx.segment(inp=a, in_offset=p * m * 4, out=b, out_offset=p * m * 4,
                                   n=m, r=0.25, bc_lo=hx.HX_BC_GHOST, bc_hi=hx.HX_BC_GHOST,
                                   halo_lo=a, halo_lo_offset=(lp * m + m - hw) * 4, halo_hi=a,
                                   halo_hi_offset=rp * m * 4, halo_width=hw))
        plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, D, segs, hx.HX_BATCH_PERSISTENT,
                                         form=hx.HX_FORM_PROPAGATOR, span_blocks=span)
        ev = hx.hx_launch_batched(ctx, plan)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
        hx.hx_event_release(ctx, ev)
        hx.hx_plan_destroy(ctx, plan)
        results.append(download(ctx, b, n, np.float32))
        hx.hx_buffer_destroy(ctx, b)
    hx.hx_buffer_destroy(ctx, a)
    ref = oracle.heat1d_periodic(u0.astype(np.float64), 0.25, D)
    il, span, bw = results
    assert rel_l2(il, ref) <= 1e-5 and rel_max(il, ref) <= 1e-5
    assert rel_l2(il, span) <= 1e-5
    assert np.array_equal(bw, il)


def test_interleaved_walk_rejections(ctx):
    """span_blocks = -1 and -2 need segments of one size and one rate; below
    -2 and above 256 are invalid; unequal segments with span_blocks = 0 take
    the span walk."""
    b = hx.hx_buffer_create(ctx, 1 << 16)
    c = hx.hx_buffer_create(ctx, 1 << 16)
    per = dict(bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
    s1 = hx.segment(inp=b, out=c, n=1024, r=0.2, **per)
    s2 = hx.segment(inp=b, in_offset=4096, out=c, out_offset=4096, n=2048, r=0.2, **per)
    s3 = hx.segment(inp=b, in_offset=4096, out=c, out_offset=4096, n=1024, r=0.1, **per)
    for segs, span in (([s1, s2], -1), ([s1, s3], -1), ([s1, s2], -2), ([s1, s3], -2),
                       ([s1], -3), ([s1], 257)):
        with pytest.raises(hx.HxError) as e:
            hx.hx_plan_create_batched(ctx, hx.HX_F32, 20, segs, hx.HX_BATCH_PERSISTENT,
                                      form=hx.HX_FORM_PROPAGATOR, span_blocks=span)
        assert e.value.status == hx.HX_ERR_ARG
    for segs in ([s1, s2], [s1, s3]):
        plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, 20, segs, hx.HX_BATCH_PERSISTENT,
                                         form=hx.HX_FORM_PROPAGATOR, span_blocks=0)
        hx.hx_plan_destroy(ctx, plan)
    hx.hx_buffer_destroy(ctx, b)
    hx.hx_buffer_destroy(ctx, c)


def run_segments(ctx, vals, r, D, span, wpg=0):
    """Periodic segments holding `vals` (f32), one propagator pass walked
    interleaved (span = -1, segments of one size), one wave per block
    (span = -2, likewise) or in spans; returns the f32 inputs and outputs per
    segment."""
    n = len(vals[0])
    offs, o = [], GUARD
    for _ in vals:
        offs.append(o)
        o += n + GUARD
    u = np.full(o, -7.0, dtype=np.float32)
    for v, o in zip(vals, offs):
        u[o:o + n] = np.asarray(v).astype(np.float32)
    bin_ = upload(ctx, u)
    bout = upload(ctx, np.full(u.size, -7.0, dtype=np.float32))
    segs = [hx.segment(inp=bin_, in_offset=o * 4, out=bout, out_offset=o * 4, n=n, r=r,
                       bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC) for o in offs]
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, D, segs, hx.HX_BATCH_PERSISTENT,
                                     form=hx.HX_FORM_PROPAGATOR, span_blocks=span,
                                     waves_per_group=wpg)
    ev = hx.hx_launch_batched(ctx, plan)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, ev)
    hx.hx_plan_destroy(ctx, plan)
    out = download(ctx, bout, u.size, np.float32)
    hx.hx_buffer_destroy(ctx, bin_)
    hx.hx_buffer_destroy(ctx, bout)
    mask = np.ones(u.size, bool)
    for o in offs:
        mask[o:o + n] = False
    assert np.all(out[mask] == -7.0)  # guards untouched
    return [u[o:o + n] for o in offs], [out[o:o + n] for o in offs]


def envelope(u, r, D):
    """sum_j |p_j| |u_{i+j}| on a periodic segment: the scale of f32 rounding in
    an output, which stepping and the propagator form both keep to."""
    taps = np.asarray(hx.hx_propagator_coefficients(r, D), np.float64)
    a = np.abs(np.asarray(u, np.float64))
    env = np.zeros(a.size)
    for j in range(-D, D + 1):
        env += abs(taps[j + D]) * np.roll(a, -j)
    return env


def per_cell(got, ref):
    """Largest per-cell relative error |got - ref| / |ref| (cells with ref = 0
    must be exact)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    nz = ref != 0
    assert np.all(got[~nz] == 0.0)
    return float(np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz]))) if nz.any() else 0.0


@pytest.mark.parametrize("span", [-1, -2, 5])
@pytest.mark.parametrize("spike", [1e6, 1e8, 1e10, 1e30])
def test_spikes_keep_every_cell_to_f32(ctx, span, spike):
    """U[0,1] segments with spikes many orders of magnitude above the
    background: every cell, near the spike or not, matches the oracle to 1e-5
    of itself (of the magnitude envelope sum_j |p_j u_{i+j}| next to a negative
    spike, where the outputs cross zero and stepping in f32 is no closer).  The spikes sit inside a block, at a block boundary (so two
    windows hold them) and next to the periodic seam; without the accuracy
    check, cells more than D away from a 1e8 spike lost up to 1e-4 of
    themselves to the fp16 split's window scale, and 1e10 about 1e-2."""
    n, D, r = 8192, 50, 0.25
    vals = [workloads.uniform(n, 513, k, 0, 1, np.float64) for k in range(4)]
    vals[0][3000] = spike
    vals[1][1024] = spike
    vals[1][1023] = spike / 3
    vals[2][n - 2] = spike
    vals[3][5000] = -spike
    u, out = run_segments(ctx, vals, r, D, span)
    for k in range(4):
        ref = oracle.heat1d_periodic(u[k].astype(np.float64), r, D)
        if k < 3:
            err = per_cell(out[k], ref)
        else:  # a negative spike on positive data: outputs cross zero near it
            err = np.max(np.abs(out[k] - ref) / envelope(u[k], r, D))
        assert err <= 1e-5, (k, spike, span, err)


@pytest.mark.parametrize("span", [-1, -2, 5])
def test_wide_dynamic_range_and_mixed_signs(ctx, span):
    """A steep exponential (e^-i/24 down to about 1e-37, so each window spans
    about 20 orders of magnitude), U[0,1] times 1e-30, 1 and 1e30, zeros, and
    a sign-alternating field: every cell matches the oracle to 1e-5 of
    sum_j |p_j u_{i+j}| (of itself where the data are of one sign), and zeros
    stay exact zeros."""
    n, D, r = 2048, 50, 0.25
    i = np.arange(n, dtype=np.float64)
    base = [workloads.uniform(n, 514, k, 0, 1, np.float64) for k in range(6)]
    vals = [np.exp(-i / 24.0), base[0] * 1e-30, base[1], base[2] * 1e30, np.zeros(n),
            base[5] * np.where(i % 2 == 0, 1.0, -1.0)]
    u, out = run_segments(ctx, vals, r, D, span)
    for k in range(len(vals)):
        ref = oracle.heat1d_periodic(u[k].astype(np.float64), r, D)
        if k == 4:
            assert np.all(out[k] == 0.0)
            continue
        env = envelope(u[k], r, D)
        got = out[k].astype(np.float64)
        big = env > 1e-35  # clear of f32's subnormal range
        err = np.max(np.abs(got[big] - ref[big]) / env[big])
        assert err <= 1e-5, (k, span, err)
        if k < 4:
            assert per_cell(got[big], ref[big]) <= 1e-5, k


@pytest.mark.parametrize("span", [-1, -2, 5])
def test_non_finite_cells_reach_what_stepping_reaches(ctx, span):
    """NaN, +inf and -inf input cells: the outputs that are NaN, +inf or -inf
    are exactly those of the oracle's stepping (within D cells of each such
    cell), and every finite output matches the oracle to 1e-5 of itself,
    right up to the edge of that reach."""
    n, D, r = 16384, 50, 0.25
    vals = [workloads.uniform(n, 515, k, 0, 1, np.float64) for k in range(3)]
    vals[0][5000] = np.nan
    vals[1][1024] = np.inf
    vals[1][9000] = -np.inf
    vals[2][30] = np.nan
    vals[2][n - 1] = np.inf
    u, out = run_segments(ctx, vals, r, D, span)
    for k in range(3):
        ref = oracle.heat1d_periodic(u[k].astype(np.float64), r, D)
        got = out[k].astype(np.float64)
        assert np.array_equal(np.isnan(got), np.isnan(ref)), k
        assert np.array_equal(np.isposinf(got), np.isposinf(ref)), k
        assert np.array_equal(np.isneginf(got), np.isneginf(ref)), k
        fin = np.isfinite(ref)
        assert np.isfinite(ref).sum() < n  # the reach is not empty
        assert per_cell(got[fin], ref[fin]) <= 1e-5, k


@pytest.mark.parametrize("span", [-1, -2, 5])
def test_every_block_stepped(ctx, span):
    """3 x 2^20 cells of (-1)^i plus a smooth part of 1e-5: at r = 1/4 one step
    annihilates the alternating part, so every output is about 1e-5 of its
    window's largest value, every block fails the accuracy check and its wave
    steps it after its other blocks.  Against the oracle, to 1e-5 of the
    magnitude envelope (not of the outputs themselves: the cancellation of the
    alternating part leaves f32 stepping an error of a few 2^-24 of the
    envelope, i.e. about 1e-2 of the outputs, as stepping directly would)."""
    n, D, r = 1 << 20, 50, 0.25
    i = np.arange(n, dtype=np.float64)
    vals = [np.where(i % 2 == 0, 1.0, -1.0) + 1e-5 * (1.5 + np.sin(2 * np.pi * (k + 2) * i / n))
            for k in range(3)]
    u, out = run_segments(ctx, vals, r, D, span)
    for k in range(3):
        ref = oracle.heat1d_periodic(u[k].astype(np.float64), r, D)
        err = np.max(np.abs(out[k] - ref) / envelope(u[k], r, D))
        assert err <= 1e-5, (k, span, err)


@pytest.mark.parametrize("n,D", [(30000, 50), (8192, 50), (4100, 17), (1024, 64), (64, 20)])
def test_block_walk_four_waves_per_group_same_bits(ctx, n, D):
    """The block walk with four waves per workgroup (consecutive blocks, one
    staged tap table; segments whose block count is not a multiple of four
    leave waves with no block) gives the bits of one wave per workgroup and of
    the interleaved walk, on U[0,1] data with a spike, a NaN and a field whose
    every block fails the accuracy check and is stepped (by its wave alone)."""
    i = np.arange(n, dtype=np.float64)
    vals = [workloads.uniform(n, 516, k, 0, 1, np.float64) for k in range(3)]
    vals[0][n // 3] = 1e9
    vals[1][n // 2] = np.nan
    vals[2] = np.where(i % 2 == 0, 1.0, -1.0) + 1e-5 * (1.5 + np.sin(2 * np.pi * 3 * i / n))
    u, one = run_segments(ctx, vals, 0.25, D, -2, wpg=1)
    _, four = run_segments(ctx, vals, 0.25, D, -2, wpg=4)
    _, il = run_segments(ctx, vals, 0.25, D, -1)
    for k in range(3):
        assert np.array_equal(four[k], one[k], equal_nan=True), k
        assert np.array_equal(four[k], il[k], equal_nan=True), k
    ref = oracle.heat1d_periodic(u[0].astype(np.float64), 0.25, D)
    assert per_cell(four[0], ref) <= 1e-5


def test_block_walk_group_sizes(ctx):
    """Waves per group for the block walk: 1 or 4; 2 is rejected."""
    b = hx.hx_buffer_create(ctx, 1 << 16)
    c = hx.hx_buffer_create(ctx, 1 << 16)
    s1 = hx.segment(inp=b, out=c, n=4096, r=0.2, bc_lo=hx.HX_BC_PERIODIC,
                    bc_hi=hx.HX_BC_PERIODIC)
    for w in (1, 4):
        plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, 20, [s1], hx.HX_BATCH_PERSISTENT,
                                         form=hx.HX_FORM_PROPAGATOR, span_blocks=-2,
                                         waves_per_group=w)
        hx.hx_plan_destroy(ctx, plan)
    with pytest.raises(hx.HxError) as e:
        hx.hx_plan_create_batched(ctx, hx.HX_F32, 20, [s1], hx.HX_BATCH_PERSISTENT,
                                  form=hx.HX_FORM_PROPAGATOR, span_blocks=-2, waves_per_group=2)
    assert e.value.status == hx.HX_ERR_ARG
    hx.hx_buffer_destroy(ctx, b)
    hx.hx_buffer_destroy(ctx, c)
