"""The D-step propagator the propagator form convolves with (host code, no
device): pinned to the binomial closed form at r = 1/4, to mass conservation
and symmetry for any r, and to the oracle stepping a unit impulse."""
import math

import numpy as np
import pytest

import oracle

hx = pytest.importorskip("paper_1810_11482_amd")


@pytest.mark.parametrize("D", [0, 1, 2, 7, 50, 64])
def test_quarter_rate_is_binomial(D):
    # [1/4, 1/2, 1/4] is the square of [1/2, 1/2]: p_j = C(2D, D + j) / 4^D
    p = hx.hx_propagator_coefficients(0.25, D)
    ref = np.array([math.comb(2 * D, k) for k in range(2 * D + 1)], dtype=np.float64) / 4.0 ** D
    assert p.shape == (2 * D + 1,)
    assert np.max(np.abs(p - ref) / ref) <= 1e-14


@pytest.mark.parametrize("r", [0.05, 0.2, 0.3, 0.45, 0.6])
def test_mass_and_symmetry(r):
    p = hx.hx_propagator_coefficients(r, 33)
    scale = np.abs(p).sum()                     # (|r| + |1-2r| + |r|)^33
    assert abs(p.sum() - 1.0) <= 1e-14 * scale  # sum of [r, 1-2r, r] is 1
    assert np.max(np.abs(p - p[::-1])) <= 1e-15 * scale   # the stencil is symmetric


@pytest.mark.parametrize("r,D", [(0.25, 50), (0.1, 20), (0.45, 64), (0.37, 9)])
def test_equals_oracle_stepping_an_impulse(r, D):
    # D oracle steps of a unit impulse on a ring wider than the light cone
    n = 2 * D + 9
    u = np.zeros(n)
    u[D + 4] = 1.0
    v = oracle.heat1d_periodic(u, r, D)
    p = hx.hx_propagator_coefficients(r, D)
    assert np.max(np.abs(v[4:4 + 2 * D + 1] - p)) <= 1e-15
    assert np.all(v[:4] == 0) and np.all(v[-4:] == 0)


def test_bad_arguments():
    with pytest.raises(hx.HxError):
        hx.hx_propagator_coefficients(0.25, -1)
    with pytest.raises(hx.HxError):
        hx.hx_propagator_coefficients(float("nan"), 3)
