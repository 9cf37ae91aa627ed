"""Pins for oracle.filters: closed form, orthogonality, moments, minimum phase."""
import numpy as np
import pytest

from oracle import filters

NUS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10]


def test_db2_closed_form():
    s3 = np.sqrt(3.0)
    ref = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0))
    assert np.allclose(filters.daubechies(2), ref, atol=1e-15, rtol=0)


def test_haar():
    assert np.allclose(filters.daubechies(1), [2 ** -0.5, 2 ** -0.5], atol=1e-16)


@pytest.mark.parametrize("nu", NUS)
def test_orthonormal_shifts(nu):
    h = filters.daubechies(nu)
    assert abs(h.sum() - np.sqrt(2.0)) < 1e-14
    for m in range(nu):
        dot = np.dot(h[: h.size - 2 * m], h[2 * m:])
        assert abs(dot - (1.0 if m == 0 else 0.0)) < 1e-14


@pytest.mark.parametrize("nu", NUS)
def test_vanishing_moments(nu):
    g = filters.wavelet(nu)
    c = np.arange(-nu + 1, nu + 1, dtype=float)
    for a in range(nu):
        assert abs(np.sum(g * c ** a)) < 1e-9 * max(1.0, np.abs(c).max() ** a)
    # the nu-th moment does not vanish
    assert abs(np.sum(g * c ** nu)) > 1e-6


@pytest.mark.parametrize("nu", [2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_minimum_phase(nu):
    h = filters.daubechies(nu)
    # sum_k h_k z^(2nu-1-k) = (1 + z)^nu Q(z); the zeros of Q lie inside the unit circle
    binom = np.poly1d([1.0, 1.0]) ** nu
    quot, rem = np.polydiv(h, binom.coeffs)
    # the division's rounding grows with the degree
    assert np.abs(rem).max() < (1e-12 if nu <= 8 else 1e-11)
    assert quot.size == nu
    assert (np.abs(np.roots(quot)) < 1).all()


def test_wavelet_filter_is_quadrature_mirror():
    for nu in NUS:
        h, g = filters.daubechies(nu), filters.wavelet(nu)
        assert abs(np.dot(h, g)) < 1e-14
        assert abs(np.dot(g, g) - 1) < 1e-14
