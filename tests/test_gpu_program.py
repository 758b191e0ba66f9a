"""Runtime-compiled kernels on the GPU: the paper's two benchmark kernels
written as user programs (Sec. V-A.1's 3-point stencil and Sec. V-A.2's
k(x) = sqrt(sin^2 x + cos^2 x)) run through Algorithm 1's futures (copy in,
kernel, copy out per partition, joined by when_all) and checked against the
oracle; argument errors; the hazard checker sees program operations."""
import numpy as np
import pytest

import oracle
from conftest import rel_max

pytestmark = pytest.mark.gpu
hx = pytest.importorskip("paper_1810_11482_amd")
from hxutil import download, upload  # noqa: E402

SRC = r'''
extern "C" __global__ void kmap(double* x, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { double v = x[i]; x[i] = sqrt(sin(v) * sin(v) + cos(v) * cos(v)); }
}
extern "C" __global__ void kprk(const double* x, double* y, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        long il = i == 0 ? n - 1 : i - 1, ir = i == n - 1 ? 0 : i + 1;
        y[i] = (0.5 * x[il] + x[i]) + 0.5 * x[ir];
    }
}
extern "C" __global__ void kaxpy(float* y, const float* x, float a, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + y[i];
}
'''


@pytest.fixture
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0, check=True)
    yield c
    hx.hx_ctx_destroy(c)


@pytest.fixture
def prog(ctx):
    p = hx.hx_program_create(ctx, SRC, "bench_kernels.hip")
    hx.hx_program_build(ctx, p)
    yield p
    hx.hx_program_destroy(ctx, p)


@pytest.mark.parametrize("n,parts", [(1 << 20, 4), (300007, 7), (5, 2)])
def test_partition_benchmark_with_futures(ctx, prog, n, parts):
    """Algorithm 1: per partition H2D -> k -> D2H, every partition in flight,
    joined once; x_i = i as in the oracle's partition kernel."""
    host = np.arange(n, dtype=np.float64)
    out = np.full(n, -1.0)
    bounds = [(p * n // parts, (p + 1) * n // parts - p * n // parts) for p in range(parts)]
    bufs = [hx.hx_buffer_create(ctx, max(s, 1) * 8) for _, s in bounds]
    evs = []
    for (o, s), b in zip(bounds, bufs):
        if s == 0:
            continue
        e1 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, host.ctypes.data + o * 8, b, 0, 0, 0,
                                                   s * 8))
        e2 = hx.hx_program_run(ctx, prog, "kmap", [hx.karg_buffer(b), hx.karg_value(np.int64(s))],
                               ((s + 255) // 256,), (256,), deps=[e1])
        e3 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, out.ctypes.data + o * 8, b, 0, 0, 0,
                                                   s * 8), [e2])
        evs.append(e3)
    assert hx.hx_wait(ctx, hx.hx_when_all(ctx, evs)) == hx.HX_OK, hx.hx_last_error(ctx)
    ref = oracle.partition_kernel(0, n)
    assert np.max(np.abs(out - ref)) <= 1e-15
    assert hx.hx_hazard_count(ctx) == 0, hx.hx_hazard_report(ctx)


def test_prk_stencil_program(ctx, prog):
    x = np.random.default_rng(3).uniform(-1, 1, 100003)
    bx = upload(ctx, x)
    by = hx.hx_buffer_create(ctx, x.nbytes)
    ev = hx.hx_program_run(ctx, prog, "kprk",
                           [hx.karg_buffer(bx, access=hx.HX_ACCESS_READ),
                            hx.karg_buffer(by, access=hx.HX_ACCESS_WRITE),
                            hx.karg_value(np.int64(x.size))], ((x.size + 127) // 128,), (128,))
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    got = download(ctx, by, x.size, np.float64)
    assert rel_max(got, oracle.prk_stencil(x)) <= 1e-15


def test_value_argument_and_offsets(ctx, prog):
    n = 1000
    x = np.arange(2 * n, dtype=np.float32)
    y = np.ones(2 * n, dtype=np.float32)
    bx, by = upload(ctx, x), upload(ctx, y)
    # second halves only, through buffer offsets
    ev = hx.hx_program_run(ctx, prog, "kaxpy",
                           [hx.karg_buffer(by, n * 4), hx.karg_buffer(bx, n * 4, hx.HX_ACCESS_READ),
                            hx.karg_value(np.float32(0.5)), hx.karg_value(np.int32(n))],
                           (4,), (256,))
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    got = download(ctx, by, 2 * n, np.float32)
    assert np.array_equal(got[:n], y[:n])
    assert np.array_equal(got[n:], 0.5 * x[n:] + 1.0)


def test_program_errors(ctx, prog):
    b = hx.hx_buffer_create(ctx, 64)
    bad = [
        (dict(kernel="nosuch", args=[], grid=(1,), block=(64,)), hx.HX_ERR_ARG),
        (dict(kernel="kmap", args=[hx.karg_buffer(b)], grid=(0,), block=(64,)), hx.HX_ERR_ARG),
        (dict(kernel="kmap", args=[hx.karg_buffer(b)], grid=(1,), block=(2048,)), hx.HX_ERR_ARG),
        (dict(kernel="kmap", args=[hx.karg_buffer(b, 65)], grid=(1,), block=(64,)),
         hx.HX_ERR_RANGE),
        (dict(kernel="kmap", args=[hx.karg_buffer(b, 0, 0)], grid=(1,), block=(64,)),
         hx.HX_ERR_ARG),
        (dict(kernel="kmap", args=[hx.karg_buffer(b + 1)], grid=(1,), block=(64,)),
         hx.HX_ERR_INVALID),
    ]
    for kw, st in bad:
        with pytest.raises(hx.HxError) as e:
            hx.hx_program_run(ctx, prog, **kw)
        assert e.value.status == st, kw
    assert hx.hx_program_function(ctx, prog, "kmap") != 0


def test_unordered_program_writes_are_flagged(ctx, prog):
    n = 4096
    b = upload(ctx, np.zeros(n, np.float64))
    args = [hx.karg_buffer(b), hx.karg_value(np.int64(n))]
    e1 = hx.hx_program_run(ctx, prog, "kmap", args, (16,), (256,))
    e2 = hx.hx_program_run(ctx, prog, "kmap", args, (16,), (256,))  # no order to e1
    hx.hx_wait(ctx, hx.hx_when_all(ctx, [e1, e2]))
    assert hx.hx_hazard_count(ctx) >= 1
    n0 = hx.hx_hazard_count(ctx)
    e3 = hx.hx_program_run(ctx, prog, "kmap", args, (16,), (256,))
    e4 = hx.hx_program_run(ctx, prog, "kmap", args, (16,), (256,), deps=[e3])
    hx.hx_wait(ctx, e4)
    assert hx.hx_hazard_count(ctx) == n0
