"""Runtime compilation (the program object) on a host-only context: source
that compiles, source that does not (the compiler's messages come back),
build options, and the errors of running without a device.  hiprtc compiles
for gfx950 without a GPU, so these run on the CPU."""
import pytest

hx = pytest.importorskip("paper_1810_11482_amd")

SRC = r'''
extern "C" __global__ void kmap(double* x, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { double v = x[i]; x[i] = sqrt(sin(v) * sin(v) + cos(v) * cos(v)); }
}
#ifndef SCALE
#error SCALE must be defined
#endif
extern "C" __global__ void kscale(float* x, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= SCALE;
}
'''


@pytest.fixture
def ctx():
    c = hx.hx_ctx_create(-1)
    yield c
    hx.hx_ctx_destroy(c)


def test_build_with_options(ctx):
    p = hx.hx_program_create(ctx, SRC, "kernels.hip")
    hx.hx_program_build(ctx, p, ["-DSCALE=2.0f"])
    assert "error" not in hx.hx_program_log(ctx, p)
    with pytest.raises(hx.HxError) as e:  # a program builds once
        hx.hx_program_build(ctx, p, ["-DSCALE=2.0f"])
    assert e.value.status == hx.HX_ERR_ARG
    hx.hx_program_destroy(ctx, p)


def test_compile_errors_carry_the_log(ctx):
    p = hx.hx_program_create(ctx, SRC, "kernels.hip")
    with pytest.raises(hx.HxError) as e:
        hx.hx_program_build(ctx, p)  # SCALE undefined
    assert e.value.status == hx.HX_ERR_ARG
    assert "SCALE must be defined" in hx.hx_program_log(ctx, p)
    q = hx.hx_program_create(ctx, 'extern "C" __global__ void k(float* x) { x[0] = nope; }')
    with pytest.raises(hx.HxError):
        hx.hx_program_build(ctx, q)
    assert "nope" in hx.hx_program_log(ctx, q)


def test_run_needs_a_device_and_valid_handles(ctx):
    p = hx.hx_program_create(ctx, SRC)
    hx.hx_program_build(ctx, p, ["-DSCALE=1.0f"])
    with pytest.raises(hx.HxError) as e:
        hx.hx_program_run(ctx, p, "kmap", [], (1,), (64,))
    assert e.value.status == hx.HX_ERR_NO_DEVICE
    with pytest.raises(hx.HxError) as e:
        hx.hx_program_function(ctx, p, "kmap")  # built but not loaded on a host-only context
    assert e.value.status == hx.HX_ERR_ARG
    hx.hx_program_destroy(ctx, p)
    with pytest.raises(hx.HxError) as e:
        hx.hx_program_build(ctx, p)
    assert e.value.status == hx.HX_ERR_INVALID


def test_value_arguments_pack_numpy_scalars():
    import numpy as np
    a = hx.karg_value(np.float32(1.5))
    assert a.kind == hx.HX_ARG_VALUE and a.size == 4
    assert bytes(a.value[:4]) == np.float32(1.5).tobytes()
    b = hx.karg_value(np.int64(-3))
    assert b.size == 8 and bytes(b.value[:8]) == np.int64(-3).tobytes()
    with pytest.raises(ValueError):
        hx.karg_value(np.zeros(3))
