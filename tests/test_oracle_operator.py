"""Pins for oracle.operator: the dense Walsh-to-wavelet section and its 2D form."""
import numpy as np
import pytest

from oracle import basis, cascade, halfline, walsh
from oracle import operator as op
from tests import inputs
from tests.conftest import read_golden


def test_haar_closed_form_scaling_basis():
    # Remark on Haar reconstruction: for nu = 1 the section in the scaling basis is
    # M^-1/2 times the M x M sequency Hadamard matrix, and Walsh rows n >= M vanish.
    cfg = op.Config(1, 4, 2, 0)
    A = op.scaling_matrix_1d(cfg)
    M = cfg.M
    ref = np.zeros((cfg.N, M))
    ref[:M] = walsh.walsh_matrix(4) / np.sqrt(M)
    assert np.abs(A - ref).max() < 1e-15


def test_haar_closed_form_wavelet_basis():
    # Textbook Haar functions: phi = 1 on [0,1), psi_{k,m} = 2^{k/2} (+1 on the left half,
    # -1 on the right half of [m 2^-k, (m+1) 2^-k)); cell integrals written out directly.
    j, q = 4, 1
    cfg = op.Config(1, j, q, 0)
    N = cfg.N
    cols = [np.full(N, 1.0 / N)]
    for k in range(j):
        w = N >> k
        for m in range(1 << k):
            c = np.zeros(N)
            c[m * w: m * w + w // 2] = 2 ** (k / 2) / N
            c[m * w + w // 2: (m + 1) * w] = -(2 ** (k / 2)) / N
            cols.append(c)
    ref = walsh.walsh_matrix(cfg.J) @ np.array(cols).T
    assert np.abs(op.matrix_1d(cfg) - ref).max() < 1e-15


@pytest.mark.parametrize("nu,j,q", [(2, 5, 1), (4, 6, 1), (4, 6, 2), (8, 6, 1), (3, 5, 2)])
def test_norm_at_most_one(nu, j, q):
    s = np.linalg.svd(op.matrix_1d(op.Config(nu, j, q)), compute_uv=False)
    assert s.max() <= 1 + 1e-12
    assert s.min() > 0.05


@pytest.mark.parametrize("nu", [2, 4])
def test_conditioning_improves_with_q(nu):
    smin = [np.linalg.svd(op.scaling_matrix_1d(op.Config(nu, 6, q)), compute_uv=False).min()
            for q in (1, 2, 3)]
    assert smin[0] < smin[1] < smin[2] < 1


def _table1():
    out = {}
    for ln in read_golden("table1_mu.txt"):
        name, dim, *vals = ln.split()
        out[(name, int(dim))] = [float(v) for v in vals]
    return out


def test_table1_db2_one_dimension():
    # soft pin: the DB2 row of Table 1 (M = 2^7) to 0.15 % (the printed values have 3 decimals)
    ref = _table1()[("DB2", 1)]
    for q in (1, 2, 3, 4):
        s = np.linalg.svd(op.scaling_matrix_1d(op.Config(2, 7, q)), compute_uv=False)
        assert abs(1 / s.min() - ref[q - 1]) / ref[q - 1] < 1.5e-3


def test_table1_db2_two_dimensions():
    # the 2D singular values are products of 1D ones (Fubini), so mu_2D = mu_1D(M = 2^5)^2
    ref = _table1()[("DB2", 2)]
    for q in (1, 2):
        s = np.linalg.svd(op.scaling_matrix_1d(op.Config(2, 5, q)), compute_uv=False)
        assert abs(1 / s.min() ** 2 - ref[q - 1]) / ref[q - 1] < 3e-3


@pytest.mark.parametrize("nu,j,q", [(2, 5, 1), (4, 6, 2), (8, 6, 1)])
def test_constant_and_linear_functions(nu, j, q):
    cfg = op.Config(nu, j, q)
    C = basis.multiscale(nu, j, cfg.j0, cfg.J).toarray()
    A = op.matrix_1d(cfg)
    # f = 1: coefficients are the integrals of the basis functions; the Walsh
    # coefficients of 1 are e_0.  Wavelet columns have zero in row n = 0.
    x1 = C.sum(axis=0)
    e0 = np.zeros(cfg.N)
    e0[0] = 1
    assert np.abs(A @ x1 - e0).max() < 1e-13
    assert np.abs(A[0, 1 << cfg.j0:]).max() < 1e-14
    # f(t) = t = 1/2 - sum_k 2^(-k-2) r_k(t), r_k the Rademacher function = w_{2^(k+1)-1}
    i = np.arange(cfg.N, dtype=float)
    cells_t = ((i + 1) ** 2 - i ** 2) / (2.0 * cfg.N ** 2)
    xt, *_ = np.linalg.lstsq(C, cells_t, rcond=None)
    ref = np.zeros(cfg.N)
    ref[0] = 0.5
    for k in range(cfg.J):
        ref[(1 << (k + 1)) - 1] = -(2.0 ** (-k - 2))
    assert np.abs(A @ xt - ref).max() < 1e-13


def _walsh_of_cells(values, q, s):
    """Walsh transform at s < 2^q of a function given by its 2^q cell integrals on [0,1)."""
    return sum(walsh.walsh(s, r, q) * values[r] for r in range(1 << q))


@pytest.mark.parametrize("nu,j,q", [(2, 4, 1), (4, 5, 2), (3, 4, 3)])
def test_lemma_3_3_and_proposition_4_2(nu, j, q):
    """Lemma 3.3 / Prop. 4.2 reproduce the plain-definition matrix entry by entry.

    Reading checked here: in the right-edge formula of Prop. 4.2 the factor is
    2^{-j/2} (as in every other formula), not 2^{j/2}.
    """
    cfg = op.Config(nu, j, q)
    A = op.scaling_matrix_1d(cfg)
    M, N = cfg.M, cfg.N
    Phi = cascade.phi_cells(nu, q)
    L = halfline.edge_scaling(nu, "left")
    R = halfline.edge_scaling(nu, "right")

    def cells_of(coef, l):
        # 2^q cell integrals on [0,1) of sum_t coef[t] phi(x + l - t)
        out = np.zeros(1 << q)
        for t, a in coef.items():
            out += float(a) * Phi.take(((l - t) << q) + np.arange(1 << q))
        return out

    for n in range(0, N, max(1, N // 64)):
        s = n >> j
        for m in range(M):
            if nu <= m < M - nu:          # Lemma 3.3 with h = phi, supp [-nu+1, nu]
                val = sum(walsh.walsh(n, (l + m) % M, j) * _walsh_of_cells(cells_of({0: 1}, l), q, s)
                          for l in range(-nu + 1, nu))
            elif m < nu:                   # Prop. 4.2, bd, left edge
                val = sum(walsh.walsh(n, l, j) * _walsh_of_cells(cells_of(L[m], l), q, s)
                          for l in range(0, nu + m))
            else:                          # Prop. 4.2, bd, right edge (factor 2^{-j/2})
                mm = M - 1 - m
                val = sum(walsh.walsh(n, l + M, j) * _walsh_of_cells(cells_of(R[mm], l), q, s)
                          for l in range(m - M - nu + 1, 0))
            assert abs(2 ** (-j / 2) * val - A[n, m]) < 1e-14


@pytest.mark.parametrize("nu,j,q", [(2, 3, 1), (1, 2, 1), (3, 3, 1)])
def test_fubini_dense_equals_separable(nu, j, q):
    cfg = op.Config(nu, j, q)
    A2 = op.dense_2d(cfg)
    blocks = op.Blocks2D(cfg)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((cfg.M, cfg.M))
    alpha = op.forward_2d_full(blocks, X)
    assert np.abs(A2 @ X.ravel() - alpha.ravel()).max() < 1e-13
    omega = np.sort(rng.choice(cfg.N * cfg.N, cfg.N * cfg.N // 3, replace=False))
    y = rng.standard_normal(omega.size)
    Xa = op.adjoint_2d_full(blocks, y, omega)
    assert np.abs(A2[omega].T @ y - Xa.ravel()).max() < 1e-13
    s = np.linalg.svd(A2, compute_uv=False)
    assert s.max() <= 1 + 1e-12


def test_sampled_rows_match_full():
    cfg = op.Config(2, 5, 1)
    full = op.Blocks2D(cfg)
    rows = np.array([0, 3, 17, 40, 63])
    part = op.Blocks2D(cfg, rows=rows)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((cfg.M, cfg.M))
    alpha = op.forward_2d_full(full, X)
    sub = op._forward_2d(part, full, X, None)
    assert np.abs(sub - alpha[rows]).max() < 1e-14


def test_sampled_1d_entries_equal_dense_products():
    """The sampled 1D forward / adjoint entries equal the dense product A x and A[omega]^T y."""
    cfg = op.Config(4, 7, 2, 3)
    A = op.matrix_1d(cfg)
    x = inputs.coefficients_1d(cfg.j, cfg.j0, 51)
    omega = inputs.uniform_omega(cfg.N, 0.3, 52)
    yv = inputs.sample_vector(omega.size, 53)
    ns = np.array([0, 1, 5, cfg.N // 2, cfg.N - 1, 77, 300])
    np.testing.assert_allclose(op.forward_entries_1d(cfg, x, ns), (A @ x)[ns], rtol=0, atol=1e-13)
    cs = np.array([0, 3, 8, 9, 15, 16, 64, 100, 127])
    np.testing.assert_allclose(op.adjoint_entries_1d(cfg, yv, omega, cs), (A[omega].T @ yv)[cs], rtol=0, atol=1e-13)


@pytest.mark.parametrize("nu,j,q", [(8, 6, 2), (4, 5, 1)])
def test_sampled_2d_entries_equal_full_products(nu, j, q):
    """The entry-by-entry 2D oracle equals the full separable products.

    forward_entries_2d, walsh_column and adjoint_entries_2d are the oracle for
    the full-size sampled checks; here they are compared with forward_2d_full,
    adjoint_2d_full and the block columns at a size with boundary rows and
    columns on both ends.
    """
    cfg = op.Config(nu, j, q)
    N, M = cfg.N, cfg.M
    blocks = op.Blocks2D(cfg)
    X = inputs.coefficients_2d(j, cfg.j0, 91)
    omega = inputs.multilevel_omega_2d(N, 0.3, 92, core=4)
    yv = inputs.sample_vector(omega.size, 93)
    alpha = op.forward_2d_full(blocks, X)
    rng = np.random.default_rng(94)
    n1 = np.concatenate([[0, 0, N - 1, N - 1, 1, N // 2], rng.integers(0, N, 40)])
    n2 = np.concatenate([[0, N - 1, 0, N - 1, N - 2, 3], rng.integers(0, N, 40)])
    np.testing.assert_allclose(op.forward_entries_2d(cfg, X, n1, n2), alpha[n1, n2], rtol=0, atol=1e-13)
    # each column of a 1D block is walsh_column of that basis function
    for kind, level, idx in [("phi", cfg.j0, 0), ("phi", cfg.j0, (1 << cfg.j0) - 1), ("phi", j - 1, nu + 1),
                             ("psi", cfg.j0, 1), ("psi", j - 1, 0), ("psi", j - 1, (1 << (j - 1)) - 1)]:
        ref = (blocks.phi if kind == "phi" else blocks.psi)[level][:, idx]
        np.testing.assert_allclose(op.walsh_column(cfg, kind, level, idx), ref, rtol=0, atol=1e-14)
    xa = op.adjoint_2d_full(blocks, yv, omega)
    pos = [(0, 0), (0, M - 1), (M - 1, 0), (M - 1, M - 1), (1, 2), (M // 2 - 1, M // 2), (nu, M - nu - 1),
           (3, 1), (M // 2 + 1, 5)]
    got = op.adjoint_entries_2d(cfg, yv, omega, pos)
    np.testing.assert_allclose(got, [xa[a, b] for a, b in pos], rtol=0, atol=1e-13)


def test_row_restricted_products_sum_to_full():
    """forward_2d_rows / adjoint_2d_rows restrict the full products to row sets."""
    cfg = op.Config(4, 5, 1)
    blocks = op.Blocks2D(cfg)
    X = inputs.coefficients_2d(5, cfg.j0, 81)
    Y = inputs.sample_vector(cfg.N * cfg.N, 82).reshape(cfg.N, cfg.N)
    alpha = op.forward_2d_full(blocks, X)
    rows_a, rows_b = np.arange(0, 23), np.arange(23, cfg.N)
    np.testing.assert_allclose(op.forward_2d_rows(blocks, X, rows_a), alpha[rows_a], rtol=0, atol=1e-14)
    xa = op.adjoint_2d_rows(blocks, Y[rows_a], rows_a) + op.adjoint_2d_rows(blocks, Y[rows_b], rows_b)
    np.testing.assert_allclose(xa, op.adjoint_2d_full(blocks, Y.ravel()), rtol=0, atol=1e-13)
