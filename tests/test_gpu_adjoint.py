"""GPU parity of the variable-coefficient step, its adjoint, the checkpointed
gradient and the autograd.Function, against the FP64 oracle adjoint.

Bars: FP64 GPU <= 1e-12 relative to the oracle (steps, gradients, loss), the
GPU FP64 inner-product identity <A u, v> = <u, A^T v> <= 1e-12; FP32 GPU
<= 1e-5 relative L2 against the FP64 oracle (errors printed per result)."""
import numpy as np
import pytest

import oracle
import workloads
from conftest import rel_l2, rel_max

pytestmark = pytest.mark.gpu
hx = pytest.importorskip("paper_1810_11482_amd")
from hxutil import download, upload  # noqa: E402

TOL = {np.float64: 1e-12, np.float32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    if hx.hx_device_count() == 0:
        pytest.skip("no GPU")
    c = hx.hx_ctx_create(0)
    yield c
    hx.hx_ctx_destroy(c)


def kappa_field(shape, seed, dtype):
    z = workloads.rng(600, seed).standard_normal(shape)
    return np.minimum(np.exp(-2 + 0.5 * z), 1.0).astype(dtype)


def wait(ctx, ev):
    assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, ev)


def code(dtype):
    return hx.HX_F64 if dtype == np.float64 else hx.HX_F32


SHAPES = [(1, 1), (1, 7), (9, 1), (5, 6), (33, 257), (70, 300), (128, 512)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape", SHAPES)
def test_forward_step(ctx, dtype, shape):
    u = workloads.uniform(shape, 601, shape[0] * 1000 + shape[1], -1, 1, dtype)
    k = kappa_field(shape, 1, dtype)
    bu, bk = upload(ctx, u), upload(ctx, k)
    bo = hx.hx_buffer_create(ctx, u.nbytes)
    wait(ctx, hx.hx_heat_vc_step(ctx, code(dtype), shape[1], shape[0], 0.2, bu, bk, bo))
    got = download(ctx, bo, shape, dtype)
    ref = oracle.heatvc_step(u.astype(np.float64), k.astype(np.float64), 0.2)
    assert rel_l2(got, ref) <= TOL[dtype] and rel_max(got, ref) <= 10 * TOL[dtype]
    for b in (bu, bk, bo):
        hx.hx_buffer_destroy(ctx, b)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_step(ctx, dtype, shape):
    u = workloads.uniform(shape, 602, shape[0] * 1000 + shape[1], -1, 1, dtype)
    lam = workloads.uniform(shape, 603, shape[0] * 1000 + shape[1], -1, 1, dtype)
    g0 = workloads.uniform(shape, 604, 0, -1, 1, dtype)
    k = kappa_field(shape, 2, dtype)
    bu, bl, bk, bg = upload(ctx, u), upload(ctx, lam), upload(ctx, k), upload(ctx, g0)
    bo = hx.hx_buffer_create(ctx, u.nbytes)
    wait(ctx, hx.hx_heat_vc_adjoint_step(ctx, code(dtype), shape[1], shape[0], 0.2, bu, bl, bk,
                                         bo, bg))
    lam_out = download(ctx, bo, shape, dtype)
    gk = download(ctx, bg, shape, dtype)
    f64 = lambda a: a.astype(np.float64)
    ref_l = oracle.heatvc_step_transpose(f64(lam), f64(k), 0.2)
    ref_g = oracle.heatvc_grad_kappa_step(f64(u), f64(lam), 0.2, f64(g0))
    assert rel_l2(lam_out, ref_l) <= TOL[dtype]
    assert rel_l2(gk, ref_g) <= TOL[dtype]
    for b in (bu, bl, bk, bg, bo):
        hx.hx_buffer_destroy(ctx, b)


@pytest.mark.parametrize("shape", [(1, 1), (40, 77), (256, 300)])
def test_gpu_fp64_inner_product_identity(ctx, shape):
    """<A u, v> = <u, A^T v> with the GPU step, the GPU adjoint step and the
    GPU FP64 dot; positive u, v so the sums do not cancel."""
    n = shape[0] * shape[1]
    u = workloads.uniform(shape, 605, 0)
    v = workloads.uniform(shape, 605, 1)
    k = kappa_field(shape, 3, np.float64)
    bu, bv, bk = upload(ctx, u), upload(ctx, v), upload(ctx, k)
    bAu = hx.hx_buffer_create(ctx, u.nbytes)
    bATv = hx.hx_buffer_create(ctx, u.nbytes)
    bg = upload(ctx, np.zeros(shape))
    bd = [hx.hx_buffer_create(ctx, 8) for _ in range(2)]
    work = hx.hx_buffer_create(ctx, 4096 * 8)
    wait(ctx, hx.hx_heat_vc_step(ctx, hx.HX_F64, shape[1], shape[0], 0.2, bu, bk, bAu))
    wait(ctx, hx.hx_heat_vc_adjoint_step(ctx, hx.HX_F64, shape[1], shape[0], 0.2, bu, bv, bk,
                                         bATv, bg))
    wait(ctx, hx.hx_launch_dot(ctx, hx.HX_F64, n, bAu, bv, bd[0], work))
    wait(ctx, hx.hx_launch_dot(ctx, hx.HX_F64, n, bu, bATv, bd[1], work))
    lhs = download(ctx, bd[0], 1, np.float64)[0]
    rhs = download(ctx, bd[1], 1, np.float64)[0]
    Au = download(ctx, bAu, shape, np.float64)
    err = abs(lhs - rhs) / (np.linalg.norm(Au) * np.linalg.norm(v))
    print(f"inner-product identity {shape}: {err:.2e}")
    assert err <= 1e-12
    assert abs(lhs - oracle.dot(Au, v)) <= 1e-12 * abs(lhs)
    for b in (bu, bv, bk, bAu, bATv, bg, work, *bd):
        hx.hx_buffer_destroy(ctx, b)


def gpu_grad(ctx, u0, kappa, y, dt, T, ckpt, dtype, seg_misaligned=False, rows=0):
    """(loss, lam0, dL/dkappa) from the library; seg_misaligned: the segment
    buffer is a view 4 bytes into its allocation, so the backward sweep
    recomputes its states by single steps instead of fused passes; rows: rows
    per wave (0: the library's choice)."""
    shape = u0.shape
    ny, nx = shape
    n = ny * nx
    S, nseg = hx.hx_vc_schedule(T, ckpt)
    es = np.dtype(dtype).itemsize
    bu0, bk, by = upload(ctx, u0.astype(dtype)), upload(ctx, kappa.astype(dtype)), \
        upload(ctx, y.astype(dtype))
    buT = hx.hx_buffer_create(ctx, n * es)
    bck = hx.hx_buffer_create(ctx, max(nseg - 1, 1) * n * es)
    bw = hx.hx_buffer_create(ctx, 2 * n * es)
    bseg_mem = hx.hx_buffer_create(ctx, max(S - 1, 1) * n * es + 16)
    bseg = hx.hx_buffer_wrap(ctx, hx.hx_buffer_ptr(ctx, bseg_mem)[0] + (4 if seg_misaligned else 0),
                             max(S - 1, 1) * n * es)
    blT = hx.hx_buffer_create(ctx, n * es)
    bl0 = hx.hx_buffer_create(ctx, n * es)
    bg64 = hx.hx_buffer_create(ctx, n * 8)
    bga = hx.hx_buffer_create(ctx, n * es)
    bloss = hx.hx_buffer_create(ctx, 8)
    work = hx.hx_buffer_create(ctx, 4096 * 8)
    a = hx.hx_vc_args(code(dtype), nx, ny, dt, T, ckpt, bu0, bk, buT, bck if nseg > 1 else 0,
                      bw if T > 1 else 0, bseg if S > 1 else 0, blT, bl0, bg64, bga, rows)
    e1 = hx.hx_heat_vc_forward(ctx, a)
    e2 = hx.hx_launch_loss(ctx, code(dtype), n, buT, by, blT, bloss, work, deps=[e1])
    e3 = hx.hx_heat_vc_backward(ctx, a, deps=[e2])
    wait(ctx, e3)
    for e in (e1, e2):
        hx.hx_event_release(ctx, e)
    loss = download(ctx, bloss, 1, np.float64)[0]
    lam0 = download(ctx, bl0, shape, dtype)
    gk = download(ctx, bg64, shape, np.float64)
    for b in (bu0, bk, by, buT, bck, bw, bseg, bseg_mem, blT, bl0, bg64, bga, bloss, work):
        hx.hx_buffer_destroy(ctx, b)
    return loss, lam0, gk


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape,T,ckpt", [((48, 70), 25, 0), ((33, 260), 17, 4), ((8, 8), 1, 0),
                                          ((64, 64), 10, 10), ((20, 300), 7, 3)])
def test_checkpointed_gradient_matches_oracle(ctx, dtype, shape, T, ckpt):
    u0 = workloads.gaussian_bumps(*shape, 3, 5.0, 610, np.float64).astype(dtype).astype(np.float64)
    kappa = kappa_field(shape, 4, dtype).astype(np.float64)
    y = workloads.uniform(shape, 611, 0, 0, 1, dtype).astype(np.float64)
    loss, lam0, gk = gpu_grad(ctx, u0, kappa, y, 0.2, T, ckpt, dtype)
    rl, rlam, rgk = oracle.heatvc_grad(u0, kappa, y, 0.2, T)
    e = (abs(loss - rl) / rl, rel_l2(lam0, rlam), rel_l2(gk, rgk))
    print(f"{dtype.__name__} {shape} T={T} S={ckpt}: loss {e[0]:.2e} lam0 {e[1]:.2e} gk {e[2]:.2e}")
    assert max(e) <= TOL[dtype]


def test_checkpoint_length_does_not_change_bits(ctx):
    shape, T = (40, 100), 12
    u0 = workloads.uniform(shape, 612, 0)
    kappa = kappa_field(shape, 5, np.float64)
    y = workloads.uniform(shape, 612, 1)
    ref = gpu_grad(ctx, u0, kappa, y, 0.2, T, 12, np.float64)  # one segment = keep everything
    for S in (1, 3, 5, 0):
        got = gpu_grad(ctx, u0, kappa, y, 0.2, T, S, np.float64)
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1])
        # the FP64 gradient total is folded once per segment, so its summation
        # grouping (not its terms) changes with S
        assert rel_l2(got[2], ref[2]) <= 1e-14


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_chunk_height_does_not_change_bits(ctx, dtype):
    """The rows per wave of the fused passes (the library's choice, which
    fills the device once, or the caller's) change how many halo rows are
    recomputed, not the result: loss, lam0 and the kappa gradient are the same
    bits at every height, one row per wave included."""
    shape, T, ckpt = (150, 496), 11, 4
    u0 = workloads.gaussian_bumps(*shape, 3, 5.0, 619, np.float64)
    kappa = kappa_field(shape, 12, np.float64)
    y = workloads.uniform(shape, 620, 0, 0, 1, np.float64)
    ref = gpu_grad(ctx, u0, kappa, y, 0.2, T, ckpt, dtype)
    for rows in (1, 7, 64, 1000):
        got = gpu_grad(ctx, u0, kappa, y, 0.2, T, ckpt, dtype, rows=rows)
        assert got[0] == ref[0], rows
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2]), rows


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,T,ckpt", [((64, 248), 20, 10), ((130, 496), 17, 5),
                                          ((40, 100), 12, 12), ((12, 8), 9, 3)])
def test_fused_recompute_equals_stepped_recompute(ctx, dtype, shape, T, ckpt):
    """The backward sweep's recomputation of each segment's states in fused
    passes that store every level (aligned segment buffer) gives the same
    loss, lam0 and kappa gradient bit for bit as single-step recomputation
    (the same segment buffer misaligned by 4 bytes)."""
    u0 = workloads.gaussian_bumps(*shape, 3, 5.0, 617, np.float64)
    kappa = kappa_field(shape, 11, np.float64)
    y = workloads.uniform(shape, 618, 0, 0, 1, np.float64)
    fused = gpu_grad(ctx, u0, kappa, y, 0.2, T, ckpt, dtype)
    stepped = gpu_grad(ctx, u0, kappa, y, 0.2, T, ckpt, dtype, seg_misaligned=True)
    assert fused[0] == stepped[0]
    assert np.array_equal(fused[1], stepped[1]) and np.array_equal(fused[2], stepped[2])


def test_fd_directional_fp64(ctx):
    shape, T = (30, 40), 15
    u0 = workloads.uniform(shape, 613, 0)
    kappa = kappa_field(shape, 6, np.float64)
    y = workloads.uniform(shape, 613, 1)
    loss, lam0, gk = gpu_grad(ctx, u0, kappa, y, 0.2, T, 0, np.float64)
    du = workloads.uniform(shape, 613, 2, -1, 1)
    dk = workloads.uniform(shape, 613, 3, -1, 1) * 0.01
    eps = 1e-4
    lp = gpu_grad(ctx, u0 + eps * du, kappa + eps * dk, y, 0.2, T, 0, np.float64)[0]
    lm = gpu_grad(ctx, u0 - eps * du, kappa - eps * dk, y, 0.2, T, 0, np.float64)[0]
    fd = (lp - lm) / (2 * eps)
    an = float(np.sum(lam0 * du) + np.sum(gk * dk))
    assert abs(fd - an) <= 1e-7 * abs(an)


def test_autograd_function(ctx):
    import torch
    from paper_1810_11482_amd.adjoint import HeatLoss, HeatVC
    shape, T = (60, 90), 16
    u0n = workloads.gaussian_bumps(*shape, 4, 6.0, 614, np.float64)
    kn = kappa_field(shape, 7, np.float64)
    yn = workloads.uniform(shape, 614, 1)
    for dt_ in (torch.float64, torch.float32):
        u0 = torch.tensor(u0n, dtype=dt_, device="cuda", requires_grad=True)
        k = torch.tensor(kn, dtype=dt_, device="cuda", requires_grad=True)
        y = torch.tensor(yn, dtype=dt_, device="cuda")
        loss = HeatLoss.apply(HeatVC.apply(u0, k, 0.2, T, 0), y)
        loss.backward()
        torch.cuda.synchronize()
        ref = oracle.heatvc_grad(u0.detach().cpu().double().numpy(),
                                 k.detach().cpu().double().numpy(), y.cpu().double().numpy(),
                                 0.2, T)
        tol = 1e-12 if dt_ == torch.float64 else 1e-5
        assert abs(loss.item() - ref[0]) <= tol * ref[0]
        assert rel_l2(u0.grad.cpu().double().numpy(), ref[1]) <= tol
        assert rel_l2(k.grad.cpu().double().numpy(), ref[2]) <= tol


def full_size_windows(ny, nx, T):
    """Oracle windows over the 8192^2 grid (a cell is exact 2T inside every cut:
    T forward and T adjoint steps): the four corners (a (4T+1)^2 window each,
    whose (2T+1)^2 corner block is exact), the four edge midpoints (2T+1 cells
    each), four cells where the kernel's 64-row chunks and 256-column strips
    meet, and four seeded interior cells (a (4T+21)^2 window each: its 21 x 21
    centre)."""
    m = 4 * T + 1
    h = 2 * T
    wins = [(0, 0, m, m), (0, nx - m, m, m), (ny - m, 0, m, m), (ny - m, nx - m, m, m),
            (0, nx // 2 - h, m, m), (ny - m, nx // 2 - h, m, m), (ny // 2 - h, 0, m, m),
            (ny // 2 - h, nx - m, m, m)]
    c = 4 * T + 21
    centres = [(64 * 37, 256 * 5), (64 * 100, 256 * 17), (64 * 7 + 1, 256 * 29 - 1),
               (64 * 120 - 1, 256 * 3 + 1)]
    rng = np.random.default_rng(23)
    centres += [(int(rng.integers(c, ny - c)), int(rng.integers(c, nx - c))) for _ in range(4)]
    wins += [(y - c // 2, x - c // 2, c, c) for y, x in centres]
    return wins


def test_full_size_against_oracle_windows(ctx):
    """8192^2, 100 steps, dt = 0.2, log-normal kappa clipped at 1, S = 10: the
    FP32 and FP64 gradients of the full run against the FP64 oracle cell by
    cell, on the oracle's light-cone windows (each window is an exact
    sub-problem for its cells 2T inside its cuts): corners, edges, the
    kernel's row-chunk and strip seams and random cells.  Also the FP32 run
    against the FP64 run on the whole grid, and the FP64 run's directional
    finite difference (exact in u0 for this quadratic loss, O(eps^2) in
    kappa)."""
    spec = workloads.VarCoef2D()
    u0, kappa, y = workloads.varcoef2d_inputs(spec)
    u0, kappa, y = u0.astype(np.float64), kappa.astype(np.float64), y.astype(np.float64)
    T = spec.steps
    res = {}
    for dt_ in (np.float64, np.float32):
        res[dt_] = gpu_grad(ctx, u0, kappa, y, spec.dt, T, spec.ckpt, dt_)
    refs_l, refs_g = [], []
    got = {dt_: ([], []) for dt_ in res}
    for w in full_size_windows(spec.ny, spec.nx, T):
        (r0, r1), (c0, c1), wl, wg = oracle.heatvc_grad_window(u0, kappa, y, spec.dt, T, *w)
        refs_l.append(wl.ravel())
        refs_g.append(wg.ravel())
        for dt_, (_, lam, gk) in res.items():
            got[dt_][0].append(lam[r0:r1, c0:c1].ravel())
            got[dt_][1].append(gk[r0:r1, c0:c1].ravel())
    rl, rg = np.concatenate(refs_l), np.concatenate(refs_g)
    for dt_ in res:
        gl, gg = np.concatenate(got[dt_][0]), np.concatenate(got[dt_][1])
        e = (rel_l2(gl, rl), rel_max(gl, rl), rel_l2(gg, rg), rel_max(gg, rg))
        print(f"full size {dt_.__name__} vs oracle windows ({rl.size} cells): lam0 rel L2 "
              f"{e[0]:.2e} max {e[1]:.2e}, dL/dkappa rel L2 {e[2]:.2e} max {e[3]:.2e}")
        assert e[0] <= TOL[dt_] and e[2] <= TOL[dt_], e
        assert e[1] <= 10 * TOL[dt_] and e[3] <= 10 * TOL[dt_], e
    l64, lam64, gk64 = res[np.float64]
    l32, lam32, gk32 = res[np.float32]
    e = (abs(l32 - l64) / l64, rel_l2(lam32, lam64), rel_l2(gk32, gk64))
    print(f"full size fp32 vs fp64: loss {e[0]:.2e} lam0 {e[1]:.2e} gk {e[2]:.2e}")
    assert max(e) <= 1e-5
    # directional finite difference of the FP64 run
    du = workloads.uniform(u0.shape, 615, 0, -1, 1)
    dk = workloads.uniform(u0.shape, 615, 1, -1, 1) * 0.01
    eps = 1e-4
    lp = gpu_grad(ctx, u0 + eps * du, kappa + eps * dk, y, spec.dt, T, spec.ckpt,
                  np.float64)[0]
    lm = gpu_grad(ctx, u0 - eps * du, kappa - eps * dk, y, spec.dt, T, spec.ckpt,
                  np.float64)[0]
    fd = (lp - lm) / (2 * eps)
    an = float(np.sum(lam64 * du) + np.sum(gk64 * dk))
    print(f"full size fp64 directional derivative: analytic {an:.10e} fd {fd:.10e}")
    assert abs(fd - an) <= 1e-6 * abs(an)


def vc_forward(ctx, u0, kappa, dt, T, ckpt, dtype):
    """u_T from hx_heat_vc_forward (fused passes where the grid is aligned)."""
    ny, nx = u0.shape
    n = ny * nx
    es = np.dtype(dtype).itemsize
    S, nseg = hx.hx_vc_schedule(T, ckpt)
    bu0, bk = upload(ctx, u0.astype(dtype)), upload(ctx, kappa.astype(dtype))
    buT = hx.hx_buffer_create(ctx, n * es)
    bck = hx.hx_buffer_create(ctx, max(nseg - 1, 1) * n * es)
    bw = hx.hx_buffer_create(ctx, 2 * n * es)
    a = hx.hx_vc_args(code(dtype), nx, ny, dt, T, ckpt, bu0, bk, buT, bck if nseg > 1 else 0,
                      bw if T > 1 else 0, 0, 0, 0, 0, 0, 0)
    wait(ctx, hx.hx_heat_vc_forward(ctx, a))
    out = download(ctx, buT, (ny, nx), dtype)
    cks = download(ctx, bck, (max(nseg - 1, 1), ny, nx), dtype)
    for b in (bu0, bk, buT, bck, bw):
        hx.hx_buffer_destroy(ctx, b)
    return out, cks[:nseg - 1]


def vc_stepped(ctx, u0, kappa, dt, T, dtype):
    """u_T by T single steps (hx_heat_vc_step), for bitwise comparison."""
    ny, nx = u0.shape
    bk = upload(ctx, kappa.astype(dtype))
    bufs = [upload(ctx, u0.astype(dtype)), hx.hx_buffer_create(ctx, u0.astype(dtype).nbytes)]
    for t in range(T):
        wait(ctx, hx.hx_heat_vc_step(ctx, code(dtype), nx, ny, dt, bufs[t % 2], bk,
                                     bufs[(t + 1) % 2]))
    out = download(ctx, bufs[T % 2], (ny, nx), dtype)
    for b in bufs + [bk]:
        hx.hx_buffer_destroy(ctx, b)
    return out


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,T,ckpt", [((300, 1000), 10, 10), ((130, 496), 7, 3),
                                          ((64, 248), 9, 0), ((5, 8), 4, 4), ((1, 4), 3, 0),
                                          ((257, 252), 13, 5)])
def test_fused_forward_equals_steps_and_oracle(ctx, dtype, shape, T, ckpt):
    """The forward run in fused passes of up to four steps (strips of 248
    output columns, chunks of the library's height, ragged at the ends): the same bits as T
    single steps, every checkpoint equal to the stepped state, and the oracle's
    forward to the suite's bar."""
    u0 = workloads.gaussian_bumps(*shape, 3, 7.0, 616, np.float64).astype(dtype)
    kappa = kappa_field(shape, 9, dtype)
    out, cks = vc_forward(ctx, u0, kappa, 0.2, T, ckpt, dtype)
    assert np.array_equal(out, vc_stepped(ctx, u0, kappa, 0.2, T, dtype))
    S, nseg = hx.hx_vc_schedule(T, ckpt)
    for k in range(nseg - 1):
        assert np.array_equal(cks[k], vc_stepped(ctx, u0, kappa, 0.2, (k + 1) * S, dtype)), k
    ref = oracle.heatvc_forward(u0.astype(np.float64), kappa.astype(np.float64), 0.2, T)
    assert rel_l2(out, ref) <= TOL[dtype] and rel_max(out, ref) <= 10 * TOL[dtype]
