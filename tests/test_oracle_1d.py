"""Pins for the 1D oracle (CPU only).

The oracle is checked against facts fixed outside itself:
  * the spectral closed form: the periodic heat operator is circulant, so the
    discrete Fourier modes are its eigenvectors with eigenvalues
    1 - 4 r sin^2(pi k / N); any input's result is ifft(fft(u0) * lambda^T);
  * exact rational arithmetic on tiny inputs;
  * invariants: conservation of the periodic sum, the maximum principle
    (r <= 1/2), shift equivariance, mirror equivariance, linearity;
  * the paper's own kernel (Sec. V-A.1): s = 0.5 x_{i-1} + x_i + 0.5 x_{i+1}
    is exactly twice the heat step at r = 1/4;
  * zero-Dirichlet: the DST-I modes sin(pi k (i+1)/(n+1)) with eigenvalues
    1 - 4 r sin^2(pi k / (2 (n+1))).
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft

import oracle
import workloads
from conftest import rel_l2, rel_max


def spectral_periodic(u0, r, steps):
    n = len(u0)
    k = np.arange(n)
    lam = 1.0 - 4.0 * r * np.sin(np.pi * k / n) ** 2
    return np.real(np.fft.ifft(np.fft.fft(u0) * lam ** steps))


@pytest.mark.parametrize("n,r,steps", [(16, 0.25, 7), (64, 0.1, 40), (1024, 0.25, 100),
                                       (4096, 0.4, 333), (1000, 0.05, 17)])
def test_periodic_matches_spectral_closed_form(n, r, steps):
    u0 = workloads.uniform(n, 90, n, -1, 1)
    got = oracle.heat1d_periodic(u0, r, steps)
    ref = spectral_periodic(u0, r, steps)
    assert rel_l2(got, ref) < 1e-13


@pytest.mark.parametrize("n,k,r,steps", [(16, 1, 0.25, 5), (16, 8, 0.25, 3), (64, 5, 0.2, 50),
                                         (1024, 127, 0.25, 100), (1024, 512, 0.1, 10)])
def test_sine_mode_decays_by_lambda_power(n, k, r, steps):
    i = np.arange(n)
    u0 = np.sin(2 * np.pi * k * i / n)
    lam = 1 - 4 * r * np.sin(np.pi * k / n) ** 2
    got = oracle.heat1d_periodic(u0, r, steps)
    assert np.max(np.abs(got - lam ** steps * u0)) < 1e-13 * steps


def test_full_size_modes_decay_exactly():
    """Noise-free 2^20 fp64 input of the cfg-1 modes after 100 steps; the decay
    1 - lambda_k^T ranges from 9e-10 (k=1) to 1.5e-5 (k=127), far above the
    1e-12 check, so a wrong r or a dropped term cannot hide."""
    spec = workloads.Periodic1D()
    u0 = workloads.periodic1d_u0(spec, with_noise=False)
    got = oracle.heat1d_periodic(u0, spec.r, spec.steps)
    i = np.arange(spec.n)
    ref = np.zeros(spec.n)
    for k in spec.modes:
        lam = 1 - 4 * spec.r * np.sin(np.pi * k / spec.n) ** 2
        ref += lam ** spec.steps * np.sin(2 * np.pi * k * i / spec.n)
    assert rel_l2(got, ref) < 1e-12
    # and the decay itself is visible well above that tolerance
    assert rel_l2(u0, ref) > 1e-7


def test_exact_rational_small():
    u0 = [3, -1, 4, 1, -5, 9, 2, -6, 5, 3, -5]
    exact = oracle.heat1d_periodic_exact(u0, Fraction(1, 4), 6)
    got = oracle.heat1d_periodic(np.array(u0, dtype=float), 0.25, 6)
    # dyadic data with r = 1/4 stays exactly representable in FP64 here
    assert [Fraction(x) for x in got] == exact
    exact3 = oracle.heat1d_periodic_exact(u0, Fraction(3, 10), 9)
    got3 = oracle.heat1d_periodic(np.array(u0, dtype=float), 0.3, 9)
    assert max(abs(float(e) - g) for e, g in zip(exact3, got3)) < 1e-13


def test_conservation_and_maximum_principle():
    u0 = workloads.uniform(5000, 91, 0)
    out = oracle.heat1d_periodic(u0, 0.5, 200)
    assert abs(out.sum() - u0.sum()) < 1e-10
    assert out.min() >= u0.min() - 1e-15 and out.max() <= u0.max() + 1e-15


def test_shift_and_mirror_equivariance():
    u0 = workloads.uniform(777, 92, 0, -1, 1)
    base = oracle.heat1d_periodic(u0, 0.23, 31)
    shifted = oracle.heat1d_periodic(np.roll(u0, 123), 0.23, 31)
    assert np.array_equal(shifted, np.roll(base, 123))  # same arithmetic per cell
    mirrored = oracle.heat1d_periodic(u0[::-1].copy(), 0.23, 31)
    assert rel_max(mirrored[::-1], base) < 1e-14


def test_linearity_modes_plus_noise():
    spec = workloads.Periodic1D(n=4096)
    clean = workloads.periodic1d_u0(spec, with_noise=False)
    noisy = workloads.periodic1d_u0(spec)
    a = oracle.heat1d_periodic(noisy, 0.25, 100)
    b = oracle.heat1d_periodic(noisy - clean, 0.25, 100)
    ref = spectral_periodic(clean, 0.25, 100)
    assert rel_l2(a - b, ref) < 1e-12


def test_paper_kernel_is_twice_heat_step_quarter():
    x = workloads.uniform(1001, 93, 0, -1, 1)
    s = oracle.prk_stencil(x)
    h = oracle.heat1d_periodic(x, 0.25, 1)
    assert np.max(np.abs(s - 2 * h)) <= 4 * np.finfo(float).eps * np.max(np.abs(x))


def test_partition_kernel_is_one():
    k = oracle.partition_kernel(0, 100000)
    assert np.max(np.abs(k - 1.0)) < 4e-16


def test_light_cone_window_is_bitwise_equal():
    u0 = workloads.uniform(3000, 94, 0)
    full = oracle.heat1d_periodic(u0, 0.25, 50)
    idx = [0, 1, 49, 50, 1499, 2950, 2999]
    assert np.array_equal(oracle.heat1d_periodic_at(u0, 0.25, 50, idx), full[idx])


@pytest.mark.parametrize("n,r,steps", [(31, 0.25, 20), (500, 0.4, 123)])
def test_dirichlet_matches_dst_closed_form(n, r, steps):
    u0 = workloads.uniform(n, 95, n, -1, 1)
    k = np.arange(1, n + 1)
    mu = 1 - 4 * r * np.sin(np.pi * k / (2 * (n + 1))) ** 2
    ref = scipy.fft.idst(scipy.fft.dst(u0, type=1) * mu ** steps, type=1)
    assert rel_l2(oracle.heat1d_dirichlet(u0, r, steps), ref) < 1e-13
