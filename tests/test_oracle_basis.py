"""Pins for oracle.halfline / oracle.basis: the boundary-corrected interval basis.

Reading under test (Sec. 3.2): vanishing-moment-preserving boundary functions
with staggered supports [0, nu+m] / [-m-nu, 0].  The pins are properties the
paper states for this basis: orthonormality, supports, polynomial reproduction
(vanishing moments preserved at the edges), zero-mean wavelets.  Orthonormality
is checked by trapezoid quadrature of point values from the point-value
cascade, a path that does not use the exact half-line Gram matrix.
"""
import numpy as np
import pytest

from oracle import basis, cascade, halfline
from oracle import operator as op


def _trap_gram(F, R):
    w = np.full(F.shape[0], 2.0 ** -R)
    w[0] *= 0.5
    w[-1] *= 0.5
    return F.T @ (F * w[:, None])


@pytest.mark.parametrize("nu", [2, 3, 4, 8])
def test_halfline_gram_against_quadrature(nu):
    G = halfline.gram_left(nu)
    R = 13
    pts = cascade.phi_points(nu, R)
    step = 2.0 ** -R
    lo = (-nu + 1) << R
    for k in range(-nu + 1, nu - 1):
        for kp in range(k, nu - 1):
            # integral over [0, inf) of phi(x-k) phi(x-kp) on the grid x = i 2^-R
            x0 = 0
            x1 = (min(k, kp) + nu) << R
            i = np.arange(x0, x1 + 1)
            a = i - (k << R) - lo
            b = i - (kp << R) - lo
            fa = np.where((a >= 0) & (a < pts.size), pts[np.clip(a, 0, pts.size - 1)], 0)
            fb = np.where((b >= 0) & (b < pts.size), pts[np.clip(b, 0, pts.size - 1)], 0)
            prod = fa * fb
            approx = step * (prod.sum() - 0.5 * (prod[0] + prod[-1]))
            assert abs(approx - float(G(k, kp))) < 2e-6


@pytest.mark.parametrize("nu", [1, 2, 3, 4, 8, 9, 10])
def test_staggered_supports_and_signs(nu):
    from oracle import filters
    g = filters.wavelet(nu)
    for side in ("left", "right"):
        sc = halfline.edge_scaling(nu, side)
        wv = halfline.edge_wavelets(nu, side)
        for m in range(nu):
            keys = [k for k, v in sc[m].items() if abs(float(v)) > 1e-40]
            if side == "left":
                assert max(keys) == m and float(sc[m][m]) > 0
                wkeys = [k for k, v in wv[m].items() if abs(float(v)) > 1e-30]
                assert max(wkeys) == nu + 2 * m
                assert (float(wv[m][nu + 2 * m]) > 0) == (g[-1] > 0)
            else:
                assert min(keys) == -m - 1 and float(sc[m][-m - 1]) > 0
                wkeys = [k for k, v in wv[m].items() if abs(float(v)) > 1e-30]
                assert min(wkeys) == -nu - 2 * m - 1
                assert (float(wv[m][-nu - 2 * m - 1]) > 0) == (g[0] > 0)


@pytest.mark.parametrize("nu,j", [(2, 3), (2, 4), (3, 3), (4, 4)])
def test_interval_basis_orthonormal_by_quadrature(nu, j):
    j0 = 0 if nu == 1 else int(np.ceil(np.log2(2 * nu)))
    R = 14 if nu <= 2 else 13
    cols = [basis.scaling_function_points(nu, j0, m, R) for m in range(1 << j0)]
    for k in range(j0, j):
        cols += [basis.wavelet_points(nu, k, m, R) for m in range(1 << k)]
    F = np.array(cols).T
    Gm = _trap_gram(F, R)
    assert np.abs(Gm - np.eye(Gm.shape[0])).max() < 5e-5


def _interval_basis_points(nu, j, j0, R):
    cols = [basis.scaling_function_points(nu, j0, m, R) for m in range(1 << j0)]
    for k in range(j0, j):
        cols += [basis.wavelet_points(nu, k, m, R) for m in range(1 << k)]
    return np.array(cols).T


@pytest.mark.parametrize("nu,j", [(6, 5), (8, 5)])
def test_interval_basis_orthonormal_by_extrapolated_quadrature(nu, j):
    """Orthonormality of the interval basis for the long filters (Sec. 3.2).

    The boundary functions are nonzero with nonzero slope at the ends, so the
    trapezoid error is c h^2 (it falls by 4 per halving, checked below); one
    Richardson step (4 G_h/2 - G_h) / 3 removes that term.  Point values come
    from the point-value cascade, not from the half-line Gram matrix.
    """
    j0 = int(np.ceil(np.log2(2 * nu)))
    G12 = _trap_gram(_interval_basis_points(nu, j, j0, 12), 12)
    G13 = _trap_gram(_interval_basis_points(nu, j, j0, 13), 13)
    eye = np.eye(G12.shape[0])
    e12, e13 = np.abs(G12 - eye).max(), np.abs(G13 - eye).max()
    assert 3.5 < e12 / e13 < 4.5
    assert np.abs((4 * G13 - G12) / 3 - eye).max() < 1e-6


@pytest.mark.parametrize("nu,j,q", [(1, 4, 1), (2, 4, 1), (2, 5, 2), (3, 4, 1), (4, 5, 1), (6, 5, 1), (8, 6, 1),
                                    (9, 6, 1), (10, 6, 1)])
def test_polynomial_reproduction(nu, j, q):
    cfg = op.Config(nu, j, q)
    C = basis.multiscale(nu, j, cfg.j0, cfg.J).toarray()
    i = np.arange(cfg.N, dtype=float)
    x0, x1 = i / cfg.N, (i + 1) / cfg.N
    scale = np.linalg.norm(C, axis=0).max()
    for a in range(nu + 1):
        target = (x1 ** (a + 1) - x0 ** (a + 1)) / (a + 1)       # exact cell integrals of t^a
        coef, *_ = np.linalg.lstsq(C, target, rcond=None)
        res = np.linalg.norm(C @ coef - target) / np.linalg.norm(target)
        if a < nu:
            assert res < 1e-11, (a, res)
        else:
            assert res > 1e-12, (a, res)     # degree nu is not reproduced


@pytest.mark.parametrize("nu,j", [(2, 4), (4, 5), (8, 6), (10, 6)])
def test_wavelets_have_zero_mean(nu, j):
    cfg = op.Config(nu, j, 1)
    for k in range(cfg.j0, j):
        W = basis.block(nu, k, cfg.J, False).toarray()
        assert np.abs(W.sum(axis=0)).max() < 1e-13
