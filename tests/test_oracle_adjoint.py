"""Pins for the oracle adjoint (CPU only).

  * inner-product identity <A u, v> = <u, A^T v> between the forward step and
    the scatter-form transposed step, on positive inputs, to 1e-12;
  * finite differences: L is quadratic in u0, so central differences carry no
    truncation error; in kappa the central difference is O(eps^2);
  * closed form: kappa = c everywhere, target 0, u0 = a Dirichlet mode phi gives
    L = mu^(2T) ||phi||^2 / 2, dL/du0 = mu^(2T) phi and
    sum_c dL/dkappa_c = -T dt w mu^(2T-1) ||phi||^2, where
    w = 4 sin^2(pi k/(2(ny+1))) + 4 sin^2(pi l/(2(nx+1))), mu = 1 - dt c w;
  * checkpointed sweeps equal the keep-everything sweep bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads
from conftest import rel_l2


def _kappa(ny, nx, seed):
    z = workloads.rng(110, seed).standard_normal((ny, nx))
    return np.minimum(np.exp(-2 + 0.5 * z), 1.0)


@pytest.mark.parametrize("ny,nx", [(1, 1), (1, 7), (9, 1), (16, 16), (45, 61)])
def test_inner_product_identity(ny, nx):
    kappa = _kappa(ny, nx, 0)
    u = workloads.uniform((ny, nx), 111, 0)
    v = workloads.uniform((ny, nx), 111, 1)
    Au = oracle.heatvc_step(u, kappa, 0.2)
    ATv = oracle.heatvc_step_transpose(v, kappa, 0.2)
    lhs, rhs = oracle.dot(Au, v), oracle.dot(u, ATv)
    assert abs(lhs - rhs) / (np.linalg.norm(Au) * np.linalg.norm(v)) < 1e-12
    # the face rule is symmetric, so A^T v is A v up to rounding order
    assert rel_l2(ATv, oracle.heatvc_step(v, kappa, 0.2)) < 1e-14


def test_fd_in_u0_is_exact_for_quadratic_loss():
    ny, nx, dt, T = 12, 14, 0.2, 9
    kappa = _kappa(ny, nx, 1)
    u0 = workloads.uniform((ny, nx), 112, 0)
    y = workloads.uniform((ny, nx), 112, 1)
    _, lam0, _ = oracle.heatvc_grad(u0, kappa, y, dt, T)
    for s in range(3):
        e = workloads.uniform((ny, nx), 112, 10 + s, -1, 1)
        eps = 1e-2
        lp = oracle.loss(oracle.heatvc_forward(u0 + eps * e, kappa, dt, T), y)
        lm = oracle.loss(oracle.heatvc_forward(u0 - eps * e, kappa, dt, T), y)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - oracle.dot(lam0, e)) < 1e-11 * max(1.0, abs(fd))


def test_fd_in_kappa_every_cell():
    """Every cell, including corners and edges (where the edge-face term acts)."""
    ny, nx, dt, T = 5, 6, 0.2, 8
    kappa = _kappa(ny, nx, 2)
    u0 = workloads.uniform((ny, nx), 113, 0)
    y = workloads.uniform((ny, nx), 113, 1)
    _, _, gk = oracle.heatvc_grad(u0, kappa, y, dt, T)
    eps = 1e-5
    fd = np.zeros_like(gk)
    for i in range(ny):
        for j in range(nx):
            kp = kappa.copy(); kp[i, j] += eps
            km = kappa.copy(); km[i, j] -= eps
            lp = oracle.loss(oracle.heatvc_forward(u0, kp, dt, T), y)
            lm = oracle.loss(oracle.heatvc_forward(u0, km, dt, T), y)
            fd[i, j] = (lp - lm) / (2 * eps)
    assert np.max(np.abs(fd - gk)) < 1e-7 * np.max(np.abs(gk))


def test_closed_form_single_mode():
    ny, nx, k, l, c, dt, T = 20, 26, 2, 3, 0.8, 0.2, 25
    i = np.arange(ny)[:, None]
    j = np.arange(nx)[None, :]
    phi = np.sin(np.pi * k * (i + 1) / (ny + 1)) * np.sin(np.pi * l * (j + 1) / (nx + 1))
    w = 4 * np.sin(np.pi * k / (2 * (ny + 1))) ** 2 + 4 * np.sin(np.pi * l / (2 * (nx + 1))) ** 2
    mu = 1 - dt * c * w
    nrm2 = float(np.sum(phi * phi))
    loss, lam0, gk = oracle.heatvc_grad(phi, np.full((ny, nx), c), np.zeros((ny, nx)), dt, T)
    assert abs(loss - 0.5 * mu ** (2 * T) * nrm2) < 1e-13 * nrm2
    assert np.max(np.abs(lam0 - mu ** (2 * T) * phi)) < 1e-13
    ref = -T * dt * w * mu ** (2 * T - 1) * nrm2
    assert abs(gk.sum() - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("T,S", [(10, 3), (10, 1), (10, 10), (10, 15), (7, 2), (1, 4)])
def test_checkpointed_equals_store_all_bitwise(T, S):
    ny, nx, dt = 11, 13, 0.2
    kappa = _kappa(ny, nx, 3)
    u0 = workloads.uniform((ny, nx), 114, 0)
    y = workloads.uniform((ny, nx), 114, 1)
    a = oracle.heatvc_grad(u0, kappa, y, dt, T, ckpt=0)
    b = oracle.heatvc_grad(u0, kappa, y, dt, T, ckpt=S)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_zero_steps():
    u0 = workloads.uniform((4, 5), 115, 0)
    y = workloads.uniform((4, 5), 115, 1)
    loss, lam0, gk = oracle.heatvc_grad(u0, np.ones((4, 5)) * 0.1, y, 0.2, 0)
    assert loss == oracle.loss(u0, y)
    assert np.array_equal(lam0, u0 - y) and not gk.any()


@pytest.mark.parametrize("win", [(0, 0, 40, 40), (20, 25, 37, 37), (50, 0, 60, 45),
                                 (-5, 60, 50, 40), (10, 10, 45, 38)])
def test_window_equals_whole_grid_inside_its_cone(win):
    """The light-cone window of the gradient (used to check full-size runs
    cell by cell): on its cells 2T inside every cut it returns the whole
    grid's lam0 and dL/dkappa bit for bit; the cells just outside that band
    differ, so the band is not wider than it must be."""
    ny, nx, dt, T = 90, 100, 0.2, 6
    kappa = _kappa(ny, nx, 5)
    u0 = workloads.gaussian_bumps(ny, nx, 5, 8.0, 112, np.float64)
    y = workloads.uniform((ny, nx), 112, 1)
    _, lam, gk = oracle.heatvc_grad(u0, kappa, y, dt, T)
    (r0, r1), (c0, c1), wl, wg = oracle.heatvc_grad_window(u0, kappa, y, dt, T, *win)
    assert wl.shape == (r1 - r0, c1 - c0) and wl.size > 0
    assert np.array_equal(wl, lam[r0:r1, c0:c1])
    assert np.array_equal(wg, gk[r0:r1, c0:c1])
    y0, x0, hy, hx = win
    if y0 > 0:  # one row closer to the top cut than allowed is wrong
        big = oracle.heatvc_grad(u0[y0:y0 + hy, max(x0, 0):x0 + hx],
                                 kappa[y0:y0 + hy, max(x0, 0):x0 + hx],
                                 y[y0:y0 + hy, max(x0, 0):x0 + hx], dt, T)[1]
        row = r0 - y0 - 1
        assert not np.array_equal(big[row], lam[r0 - 1, max(x0, 0):x0 + hx])
