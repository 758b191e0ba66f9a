"""The allocation-free loss (hx_launch_loss_noalloc) against hx_launch_loss:
the same kernels over the same inputs, so the FP64 loss and the residual are
bit for bit those of the entry point with a workspace; two calls in a row, the
second with a smaller input (the static scratch keeps the first call's
partials, which the second must not see)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
hx = pytest.importorskip("paper_1810_11482_amd")
from hxutil import download, upload  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0)
    yield c
    hx.hx_ctx_destroy(c)


def run_pair(ctx, dtype, n, seed):
    """Loss and residual of n cells by both entry points."""
    u = workloads.uniform(n, 620, seed, -1, 1, dtype)
    y = workloads.uniform(n, 620, seed + 1, -1, 1, dtype)
    bu, by = upload(ctx, u), upload(ctx, y)
    es = np.dtype(dtype).itemsize
    code = hx.HX_F64 if dtype == np.float64 else hx.HX_F32
    outs = []
    for noalloc in (False, True):
        br = hx.hx_buffer_create(ctx, n * es)
        bl = hx.hx_buffer_create(ctx, 8)
        if noalloc:
            ev = hx.hx_launch_loss_noalloc(ctx, code, n, bu, by, br, bl)
        else:
            work = hx.hx_buffer_create(ctx, 4096 * 8)
            ev = hx.hx_launch_loss(ctx, code, n, bu, by, br, bl, work)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
        hx.hx_event_release(ctx, ev)
        outs.append((download(ctx, bl, 1, np.float64)[0], download(ctx, br, n, dtype)))
        hx.hx_buffer_destroy(ctx, br)
        hx.hx_buffer_destroy(ctx, bl)
        if not noalloc:
            hx.hx_buffer_destroy(ctx, work)
    hx.hx_buffer_destroy(ctx, bu)
    hx.hx_buffer_destroy(ctx, by)
    ref = 0.5 * np.sum((u.astype(np.float64) - y.astype(np.float64)) ** 2)
    return outs, ref


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_loss_matches_the_workspace_form(ctx, dtype):
    for n, seed in ((5_000_000, 1), (3001, 3)):  # the second call smaller
        outs, ref = run_pair(ctx, dtype, n, seed)
        (l_ws, r_ws), (l_na, r_na) = outs
        assert l_na == l_ws, (n, l_na, l_ws)
        assert np.array_equal(r_na, r_ws)
        tol = 1e-12 if dtype == np.float64 else 1e-6
        assert abs(l_na - ref) <= tol * ref


def test_noalloc_loss_rejects_bad_arguments(ctx):
    b = hx.hx_buffer_create(ctx, 4096)
    o = hx.hx_buffer_create(ctx, 8)
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_loss_noalloc(ctx, hx.HX_F32, 2048, b, b, 0, o)  # 8 KiB > buffer
    assert e.value.status == hx.HX_ERR_RANGE
    with pytest.raises(hx.HxError) as e:
        hx.hx_launch_loss_noalloc(ctx, 7, 16, b, b, 0, o)
    assert e.value.status == hx.HX_ERR_ARG
    hx.hx_buffer_destroy(ctx, b)
    hx.hx_buffer_destroy(ctx, o)
