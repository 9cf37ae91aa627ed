"""Pins for the periodic extension (Sec. 3.2) in the oracle.

The paper defines the periodic basis by adding to each function crossing an
end of [0, 1] its translate by the period; Prop. 4.2 prints the Walsh
coefficients of the periodic edge functions.  Pins: the Haar case (nothing
wraps), orthonormality against point-value quadrature, the partition of unity
(constant functions are reproduced), zero-mean wavelets, the norm bound, that
the linear function is not reproduced (the point of Fig. 4), and the printed
periodic formulas of Prop. 4.2 entry by entry against the plain definition.
"""
import numpy as np
import pytest

from oracle import basis, cascade, walsh
from oracle import operator as op


def _walsh_of_cells(values, q, s):
    return sum(walsh.walsh(s, r, q) * values[r] for r in range(1 << q))


def test_haar_periodic_equals_haar():
    for per in (False, True):
        A = op.matrix_1d(op.Config(1, 4, 1, 0, per=per))
        if per:
            assert np.array_equal(A, Ab)
        Ab = A


@pytest.mark.parametrize("nu,j", [(2, 3), (4, 4), (3, 3)])
def test_periodic_basis_orthonormal_by_quadrature(nu, j):
    j0 = int(np.ceil(np.log2(2 * nu)))

    def gram(R):
        cols = [basis.periodic_points(nu, j0, m, R, True) for m in range(1 << j0)]
        for k in range(j0, j):
            cols += [basis.periodic_points(nu, k, m, R, False) for m in range(1 << k)]
        F = np.array(cols).T
        w = np.full(F.shape[0], 2.0 ** -R)
        w[0] *= 0.5
        w[-1] *= 0.5
        return F.T @ (F * w[:, None])

    # periodic functions: the trapezoid rule has no endpoint error term; Richardson for safety
    G13 = gram(13)
    G12 = gram(12)
    eye = np.eye(G13.shape[0])
    assert np.abs((4 * G13 - G12) / 3 - eye).max() < 1e-5


@pytest.mark.parametrize("nu,j,q", [(2, 5, 1), (4, 6, 2), (8, 6, 1)])
def test_periodic_constants_norm_and_zero_mean(nu, j, q):
    cfg = op.Config(nu, j, q, per=True)
    C = basis.multiscale(nu, j, cfg.j0, cfg.J, per=True).toarray()
    A = op.matrix_1d(cfg)
    x1 = C.sum(axis=0)
    e0 = np.zeros(cfg.N)
    e0[0] = 1
    assert np.abs(A @ x1 - e0).max() < 1e-13
    assert np.abs(A[0, 1 << cfg.j0:]).max() < 1e-14
    s = np.linalg.svd(A, compute_uv=False)
    assert s.max() <= 1 + 1e-12 and s.min() > 0.05
    # the linear function t is not in the periodic space (it is in the boundary-corrected one)
    i = np.arange(cfg.N, dtype=float)
    cells_t = ((i + 1) ** 2 - i ** 2) / (2.0 * cfg.N ** 2)
    coef, *_ = np.linalg.lstsq(C, cells_t, rcond=None)
    assert np.linalg.norm(C @ coef - cells_t) / np.linalg.norm(cells_t) > 1e-3


@pytest.mark.parametrize("nu,j,q", [(2, 4, 1), (4, 5, 2), (3, 4, 3)])
def test_proposition_4_2_periodic(nu, j, q):
    """Prop. 4.2 (per): the printed sums for the periodic edge functions against the plain definition."""
    cfg = op.Config(nu, j, q, per=True)
    A = op.scaling_matrix_1d(cfg)
    M, N = cfg.M, cfg.N
    Phi = cascade.phi_cells(nu, q)

    def W_phi(l, s):
        # Walsh coefficient at s of phi_{0,-l} restricted to [0, 1): cells of phi(x + l)
        return _walsh_of_cells(Phi.take((l << q) + np.arange(1 << q)), q, s)

    for n in range(0, N, max(1, N // 64)):
        s = n >> j
        for m in list(range(nu)) + list(range(M - nu, M)):
            if m < nu:
                val = sum(walsh.walsh(n, M + m + l, j) * W_phi(l, s) for l in range(-nu + 1, -m))
                val += sum(walsh.walsh(n, m + l, j) * W_phi(l, s) for l in range(-m, nu))
            else:
                val = sum(walsh.walsh(n, l + m, j) * W_phi(l, s) for l in range(-nu + 1, M - m))
                val += sum(walsh.walsh(n, l + m - M, j) * W_phi(l, s) for l in range(M - m, nu))
            assert abs(2 ** (-j / 2) * val - A[n, m]) < 1e-14


@pytest.mark.parametrize("nu,j,q", [(2, 3, 1), (3, 3, 1)])
def test_periodic_fubini_dense_equals_separable(nu, j, q):
    cfg = op.Config(nu, j, q, per=True)
    A2 = op.dense_2d(cfg)
    blocks = op.Blocks2D(cfg)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((cfg.M, cfg.M))
    assert np.abs(A2 @ X.ravel() - op.forward_2d_full(blocks, X).ravel()).max() < 1e-13
    s = np.linalg.svd(A2, compute_uv=False)
    assert s.max() <= 1 + 1e-12
