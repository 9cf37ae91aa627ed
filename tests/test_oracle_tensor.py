"""Pins for the tensor-product 2D basis in the oracle.

Sec. 5 (Fubini) makes every entry of the 2D section a product of 1D entries;
with the tensor-product basis r_{c1} (x) r_{c2} the section is exactly the
Kronecker product of the 1D section.  Pins: the Kronecker product of the 1D
basis columns built one by one (dense_2d), the singular values shared with the
isotropic basis (both are orthonormal bases of V_j (x) V_j, so the two sections
differ by an orthogonal change of coordinates), equality when j0 = j (no
wavelet level), and the adjoint identity.
"""
import numpy as np
import pytest

from oracle import operator as op


@pytest.mark.parametrize("nu,j,q,per", [(2, 3, 1, False), (3, 3, 1, False), (2, 3, 2, True), (1, 3, 1, False)])
def test_tensor_section_is_the_kronecker_product(nu, j, q, per):
    cfg = op.Config(nu, j, q, per=per, tensor=True)
    A2 = op.dense_2d(cfg)
    A1 = op.matrix_1d(cfg)
    assert np.abs(A2 - np.kron(A1, A1)).max() < 1e-15
    rng = np.random.default_rng(5)
    X = rng.standard_normal((cfg.M, cfg.M))
    assert np.abs(op.forward_2d_tensor(A1, X).ravel() - A2 @ X.ravel()).max() < 1e-13
    omega = np.sort(rng.choice(cfg.N ** 2, cfg.N ** 2 // 3, replace=False))
    yv = rng.standard_normal(omega.size)
    assert np.abs(op.adjoint_2d_tensor(A1, yv, omega).ravel() - A2[omega].T @ yv).max() < 1e-13


@pytest.mark.parametrize("nu,j,q", [(2, 4, 1), (3, 5, 1)])
def test_tensor_and_isotropic_bases_share_singular_values(nu, j, q):
    iso = op.dense_2d(op.Config(nu, j, q))
    ten = op.dense_2d(op.Config(nu, j, q, tensor=True))
    s_iso = np.linalg.svd(iso, compute_uv=False)
    s_ten = np.linalg.svd(ten, compute_uv=False)
    assert np.abs(s_iso - s_ten).max() < 1e-12
    assert not np.allclose(iso, ten)  # two or more wavelet levels: the bases differ
    # with no wavelet level both bases are phi (x) phi
    a = op.dense_2d(op.Config(nu, 3, q, 3))
    b = op.dense_2d(op.Config(nu, 3, q, 3, tensor=True))
    assert np.array_equal(a, b)
