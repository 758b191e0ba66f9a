"""Pins for the 2D oracles (CPU only).

Constant coefficient, zero-Dirichlet: the five-point operator separates, and
the 2D type-I DST diagonalises it with eigenvalues
1 - 4 r (sin^2(pi k / (2 (ny+1))) + sin^2(pi l / (2 (nx+1)))); any input's
result is therefore idstn(dstn(u0) * mu^T).

Variable coefficient: with kappa constant = c the update reduces to the
constant stencil with r = dt c (textbook special case); a hand-computed 1x2
example fixes every matrix entry including the edge-face rule; the operator is
symmetric (<Au, v> = <u, Av>) for any kappa because the face rule is; the
increment is linear in kappa.
"""
import json
import os

import numpy as np
import pytest
import scipy.fft

import oracle
import workloads
from conftest import rel_l2, rel_max

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def spectral_dirichlet2d(u0, r, steps):
    ny, nx = u0.shape
    ky = np.arange(1, ny + 1)[:, None]
    kx = np.arange(1, nx + 1)[None, :]
    mu = 1 - 4 * r * (np.sin(np.pi * ky / (2 * (ny + 1))) ** 2 +
                      np.sin(np.pi * kx / (2 * (nx + 1))) ** 2)
    return scipy.fft.idstn(scipy.fft.dstn(u0, type=1) * mu ** steps, type=1)


@pytest.mark.parametrize("ny,nx,r,steps", [(7, 9, 0.25, 10), (40, 33, 0.2, 60),
                                           (128, 96, 0.125, 200)])
def test_dirichlet2d_matches_dst_closed_form(ny, nx, r, steps):
    u0 = workloads.uniform((ny, nx), 96, ny * nx, -1, 1)
    got = oracle.heat2d_dirichlet(u0, r, steps)
    assert rel_l2(got, spectral_dirichlet2d(u0, r, steps)) < 1e-13


def test_dirichlet2d_separable_mode():
    ny, nx, k, l, r, steps = 30, 50, 3, 7, 0.2, 40
    i = np.arange(ny)[:, None]
    j = np.arange(nx)[None, :]
    phi = np.sin(np.pi * k * (i + 1) / (ny + 1)) * np.sin(np.pi * l * (j + 1) / (nx + 1))
    mu = 1 - 4 * r * (np.sin(np.pi * k / (2 * (ny + 1))) ** 2 +
                      np.sin(np.pi * l / (2 * (nx + 1))) ** 2)
    got = oracle.heat2d_dirichlet(phi, r, steps)
    assert np.max(np.abs(got - mu ** steps * phi)) < 1e-13


def test_dirichlet2d_invariants():
    u0 = workloads.uniform((37, 37), 97, 0)
    out = oracle.heat2d_dirichlet(u0, 0.25, 25)
    assert out.min() >= 0 and out.max() <= u0.max()
    t = oracle.heat2d_dirichlet(u0.T.copy(), 0.25, 25)
    assert rel_max(t.T, out) < 1e-14


def test_dirichlet2d_light_cone_bitwise():
    u0 = workloads.uniform((60, 70), 98, 0)
    full = oracle.heat2d_dirichlet(u0, 0.2, 12)
    pts = [(0, 0), (0, 69), (59, 0), (59, 69), (30, 35), (5, 64), (11, 12)]
    got = oracle.heat2d_dirichlet_at(u0, 0.2, 12, pts)
    assert np.array_equal(got, np.array([full[p] for p in pts]))


def test_varcoef_constant_kappa_reduces_to_constant_stencil():
    u0 = workloads.uniform((23, 31), 99, 0, -1, 1)
    kappa = np.full(u0.shape, 0.7)
    got = oracle.heatvc_forward(u0, kappa, 0.3, 15)
    ref = oracle.heat2d_dirichlet(u0, 0.3 * 0.7, 15)
    assert rel_max(got, ref) < 1e-13


def test_varcoef_hand_computed_1x2():
    """Fixture tests/golden/varcoef_1x2.json: the matrix of one step on a 1x2
    grid, derived by hand from the face rule (see the fixture's note)."""
    with open(os.path.join(GOLDEN, "varcoef_1x2.json")) as f:
        g = json.load(f)
    kappa = np.array(g["kappa"], dtype=float)
    A = np.array(g["A"], dtype=float)
    cols = []
    for c in range(2):
        e = np.zeros((1, 2))
        e[0, c] = 1.0
        cols.append(oracle.heatvc_step(e, kappa, g["dt"]).ravel())
    assert np.allclose(np.array(cols).T, A, rtol=0, atol=1e-15)


def test_varcoef_operator_symmetric_and_linear_in_kappa():
    ny, nx, dt = 19, 24, 0.2
    g = workloads.rng(100, 0)
    kappa = np.exp(-2 + 0.5 * g.standard_normal((ny, nx)))
    u = g.random((ny, nx))
    v = g.random((ny, nx))
    Au = oracle.heatvc_step(u, kappa, dt)
    Av = oracle.heatvc_step(v, kappa, dt)
    lhs, rhs = oracle.dot(Au, v), oracle.dot(u, Av)
    assert abs(lhs - rhs) / abs(lhs) < 1e-14
    k2 = g.random((ny, nx))
    inc = lambda k: oracle.heatvc_step(u, k, dt) - u
    assert rel_max(inc(kappa + k2), inc(kappa) + inc(k2)) < 1e-13


def test_varcoef_maximum_principle():
    ny, nx, dt = 33, 20, 0.2
    kappa = np.minimum(np.exp(-2 + 0.5 * workloads.rng(101, 0).standard_normal((ny, nx))), 1.0)
    u = workloads.uniform((ny, nx), 101, 1)
    out = oracle.heatvc_forward(u, kappa, dt, 30)
    assert out.min() >= 0 and out.max() <= u.max()
