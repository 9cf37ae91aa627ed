"""Pins for oracle.cascade: partition, refinement consistency, Haar, quadrature."""
import numpy as np
import pytest

from oracle import cascade, filters


@pytest.mark.parametrize("nu", [1, 2, 4, 8])
@pytest.mark.parametrize("r", [0, 1, 3, 5])
def test_integral_one_and_zero_mean(nu, r):
    assert abs(cascade.phi_cells(nu, r).values.sum() - 1) < 1e-13
    assert abs(cascade.psi_cells(nu, r).values.sum()) < 1e-13


@pytest.mark.parametrize("nu", [2, 3, 8])
def test_children_sum_to_parent(nu):
    for r in range(0, 5):
        p, c = cascade.phi_cells(nu, r), cascade.phi_cells(nu, r + 1)
        s = np.arange(p.lo, p.lo + p.values.size)
        assert np.allclose(c.take(2 * s) + c.take(2 * s + 1), p.values, atol=1e-15)
        p, c = cascade.psi_cells(nu, r), cascade.psi_cells(nu, r + 1)
        assert np.allclose(c.take(2 * s) + c.take(2 * s + 1), p.values, atol=1e-15)


def test_haar_cells():
    for r in range(5):
        P = cascade.phi_cells(1, r)
        assert P.lo == 0 and np.allclose(P.values, 2.0 ** -r)
        Q = cascade.psi_cells(1, r)
        half = 1 << max(r - 1, 0)
        if r >= 1:
            assert np.allclose(Q.values[:half], 2.0 ** -r) and np.allclose(Q.values[half:], -2.0 ** -r)


@pytest.mark.parametrize("nu", [2, 4])
def test_point_value_quadrature_converges(nu):
    errs = []
    exact = cascade.phi_cells(nu, 0).values
    for R in (6, 8, 10):
        pts = cascade.phi_points(nu, R)
        step = 2.0 ** -R
        approx = []
        for s in range(-nu + 1, nu):
            a = (s + nu - 1) << R
            seg = pts[a:a + (1 << R) + 1]
            approx.append(step * (seg.sum() - 0.5 * (seg[0] + seg[-1])))
        errs.append(np.abs(np.array(approx) - exact).max())
    assert errs[-1] < 1e-5
    assert errs[0] > 8 * errs[1] > 64 * errs[2] * 0.5


@pytest.mark.parametrize("nu", [1, 2, 4, 8])
def test_first_moment_exact(nu):
    # The integral of x phi(x) is sum_c c h_c / sqrt(2) (two-scale relation with sum h = sqrt 2).
    # The cell-midpoint sum reproduces it exactly at every level: its change from level r
    # to r+1 is the integral of phi against a 1-periodic zero-mean square wave, which
    # vanishes because the integer translates of phi sum to one.
    h = filters.daubechies(nu)
    c = np.arange(-nu + 1, nu + 1)
    m1 = np.dot(c, h) / np.sqrt(2.0)
    for r in (0, 2, 5, 9):
        P = cascade.phi_cells(nu, r)
        s = np.arange(P.lo, P.lo + P.values.size)
        assert abs(np.sum(P.values * (s + 0.5) * 2.0 ** -r) - m1) < 1e-13
