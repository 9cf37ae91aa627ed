"""Pins for the d-dimensional and unequal-sided sections in the oracle.

Sec. 5 splits the 2D inner products into 1D ones by Fubini, and the same
splitting holds for any d-fold tensor product; Sec. 4 reaches other sizes of
the 1D section through padding, which along each axis of a tensor basis is an
axis with its own j.  The oracle applies the 1D sections axis by axis (mode
products).  Pins, none of which reuses that path:
* at d = 2 the d-dimensional functions equal the 2D ones, which are pinned on
  their own (Haar closed form, Kronecker matrix, Table 1);
* at d = 3 and for unequal sides the result equals the matrix built column by
  column from Kronecker products of single 1D basis-function columns
  (dense_nd; whole at tiny sizes, sampled columns above);
* separable coefficients a (x) b (x) c map to (A a) (x) (B b) (x) (C c);
* the isotropic and tensor bases are orthonormal bases of the same space, so
  the two sections share their singular values, which for the tensor basis
  are the products of the 1D singular values;
* the adjoint identity on a sparse Omega.
"""
import numpy as np
import pytest

from oracle import operator as op


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("nu,j,q,per", [(2, 4, 1, False), (4, 4, 1, False), (2, 4, 2, True), (1, 3, 1, False)])
def test_two_dimensions_reduce_to_the_2d_oracle(nu, j, q, per):
    cfg = op.Config(nu, j, q, per=per)
    B = op.Blocks2D(cfg)
    A1 = op.matrix_1d(cfg)
    rng = _rng(1)
    X = rng.standard_normal((cfg.M, cfg.M))
    omega = np.sort(rng.choice(cfg.N ** 2, cfg.N ** 2 // 4, replace=False))
    assert np.abs(op.forward_nd_iso(B, X, omega) - op.forward_2d_full(B, X, omega)).max() < 1e-13
    assert np.abs(op.forward_nd_tensor([A1, A1], X, omega) - op.forward_2d_tensor(A1, X, omega)).max() < 1e-13
    yv = rng.standard_normal(omega.size)
    assert np.abs(op.adjoint_nd_iso(B, yv, 2, omega) - op.adjoint_2d_full(B, yv, omega)).max() < 1e-13
    assert np.abs(op.adjoint_nd_tensor([A1, A1], yv, omega) - op.adjoint_2d_tensor(A1, yv, omega)).max() < 1e-13


@pytest.mark.parametrize("nu,j,q,j0,per", [(1, 3, 1, 0, False), (1, 3, 1, 1, True), (2, 3, 1, 2, False),
                                           (2, 3, 1, 2, True)])
def test_three_dimensions_match_the_kronecker_columns(nu, j, q, j0, per):
    cfg = op.Config(nu, j, q, j0, per=per)
    rng = _rng(2)
    X = rng.standard_normal((cfg.M,) * 3)
    omega = np.sort(rng.choice(cfg.N ** 3, cfg.N ** 3 // 5, replace=False))
    yv = rng.standard_normal(omega.size)
    D_iso = op.dense_nd([cfg] * 3, tensor=False)
    B = op.Blocks2D(cfg)
    assert np.abs(op.forward_nd_iso(B, X).ravel() - D_iso @ X.ravel()).max() < 1e-13
    assert np.abs(op.adjoint_nd_iso(B, yv, 3, omega).ravel() - D_iso[omega].T @ yv).max() < 1e-13
    D_ten = op.dense_nd([cfg] * 3, tensor=True)
    A1 = op.matrix_1d(cfg)
    assert np.abs(op.forward_nd_tensor([A1] * 3, X).ravel() - D_ten @ X.ravel()).max() < 1e-13
    assert np.abs(op.adjoint_nd_tensor([A1] * 3, yv, omega).ravel() - D_ten[omega].T @ yv).max() < 1e-13
    if j - j0 >= 2:
        assert not np.allclose(D_iso, D_ten)  # two or more levels: the bases differ
    else:
        assert np.abs(D_iso - D_ten).max() < 1e-15  # at most one level: the same functions
    # same space, both orthonormal: equal singular values, products of the 1D ones
    s_iso = np.linalg.svd(D_iso, compute_uv=False)
    s_ten = np.linalg.svd(D_ten, compute_uv=False)
    s1 = np.linalg.svd(A1, compute_uv=False)
    prod = np.sort(np.einsum("a,b,c->abc", s1, s1, s1).ravel())[::-1]
    assert np.abs(s_iso - s_ten).max() < 1e-12
    assert np.abs(s_ten - prod).max() < 1e-12


@pytest.mark.parametrize("nu,j,q,per", [(2, 4, 1, False), (3, 5, 1, False), (2, 4, 1, True)])
def test_three_dimensions_sampled_columns_with_two_levels(nu, j, q, per):
    """db2 at 16^3 and db3 at 32^3: the isotropic and tensor sections on 48 sampled unit
    coefficient vectors, against the same columns built one by one."""
    cfg = op.Config(nu, j, q, per=per)
    assert j - cfg.j0 >= 2
    rng = _rng(3)
    cols = np.sort(rng.choice(cfg.M ** 3, 48, replace=False))
    B = op.Blocks2D(cfg)
    A1 = op.matrix_1d(cfg)
    D_iso = op.dense_nd([cfg] * 3, tensor=False, columns=cols)
    D_ten = op.dense_nd([cfg] * 3, tensor=True, columns=cols)
    for i, c in enumerate(cols):
        e = np.zeros(cfg.M ** 3)
        e[c] = 1.0
        e = e.reshape((cfg.M,) * 3)
        assert np.abs(op.forward_nd_iso(B, e).ravel() - D_iso[:, i]).max() < 1e-13
        assert np.abs(op.forward_nd_tensor([A1] * 3, e).ravel() - D_ten[:, i]).max() < 1e-13


@pytest.mark.parametrize("js,nu,q,per", [((2, 4), 2, 1, False), ((4, 2), 2, 2, False), ((3, 2, 4), 2, 1, False),
                                         ((3, 4), 1, 1, True)])
def test_unequal_sides_match_the_kronecker_columns(js, nu, q, per):
    j0 = 2 if nu == 2 else 1
    cfgs = [op.Config(nu, j, q, j0, per=per) for j in js]
    mats = [op.matrix_1d(c) for c in cfgs]
    D = op.dense_nd(cfgs, tensor=True)
    K = mats[0]
    for A in mats[1:]:
        K = np.kron(K, A)
    assert np.abs(D - K).max() < 1e-15
    rng = _rng(4)
    X = rng.standard_normal(tuple(c.M for c in cfgs))
    assert np.abs(op.forward_nd_tensor(mats, X).ravel() - D @ X.ravel()).max() < 1e-13
    omega = np.sort(rng.choice(D.shape[0], D.shape[0] // 3, replace=False))
    yv = rng.standard_normal(omega.size)
    assert np.abs(op.adjoint_nd_tensor(mats, yv, omega).ravel() - D[omega].T @ yv).max() < 1e-13


def test_separable_coefficients_map_to_separable_samples():
    """X = a (x) b (x) c on unequal sides: alpha = (A a) (x) (B b) (x) (C c)."""
    cfgs = [op.Config(4, 5, 1), op.Config(4, 3, 1), op.Config(4, 4, 2)]
    mats = [op.matrix_1d(c) for c in cfgs]
    rng = _rng(5)
    vecs = [rng.standard_normal(c.M) for c in cfgs]
    X = np.einsum("a,b,c->abc", *vecs)
    expect = np.einsum("a,b,c->abc", *[A @ v for A, v in zip(mats, vecs)])
    assert np.abs(op.forward_nd_tensor(mats, X) - expect).max() < 1e-13


@pytest.mark.parametrize("tensor", [False, True])
def test_adjoint_identity_in_three_dimensions(tensor):
    cfg = op.Config(4, 5, 1)
    rng = _rng(6)
    X = rng.standard_normal((cfg.M,) * 3)
    omega = np.sort(rng.choice(cfg.N ** 3, cfg.N ** 3 // 8, replace=False))
    yv = rng.standard_normal(omega.size)
    if tensor:
        mats = [op.matrix_1d(cfg)] * 3
        ax, aty = op.forward_nd_tensor(mats, X, omega), op.adjoint_nd_tensor(mats, yv, omega)
    else:
        B = op.Blocks2D(cfg)
        ax, aty = op.forward_nd_iso(B, X, omega), op.adjoint_nd_iso(B, yv, 3, omega)
    lhs, rhs = float(ax @ yv), float(np.sum(X * aty))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
