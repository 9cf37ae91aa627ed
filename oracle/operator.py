"""Dense products with the Walsh-to-wavelet section and its adjoint.

Test infrastructure (see the package header).

1D.  With J = j + q (N = 2^J Walsh functions, M = 2^j wavelet functions),
the matrix of Sec. 4 composed with the change of basis of the Remark on
compressive sensing is  A[n, c] = <r_c, w_n>,  r_c the c-th function of
C_{psi,j}.  w_n (n < N) is constant on each cell [i/N, (i+1)/N) (Def. 3.1
with the non-terminating expansion), so A = H C exactly, with
H[n, i] = w_n(i/N) from Def. 3.1 and C the cell integrals (module basis).
Forward: y = A[Omega, :] x; adjoint: x = A[Omega, :]^T y (everything is
real; Omega in increasing order as in the Notation section).

2D.  Sampling functions w_{n1} (x) w_{n2}, reconstruction functions the
isotropic 2D wavelet basis in the quadtree layout (reading: the paper
defines only phi (x) phi and Algorithm 2; the 2D wavelet convention is the
standard square one).  By Fubini (Sec. 5) every entry is a product of 1D
entries, so alpha = sum over (level, band) of A_a X_band A_b^T with the 1D
blocks A_a, A_b of B_{phi,k} / B_{psi,k}; y = alpha[Omega] in increasing
linear index n1 N + n2, n1 belonging to the first coordinate.

Tensor-product 2D basis (the alternative to the isotropic one): the
functions r_{c1} (x) r_{c2} of the 1D multiscale basis, so the section is the
Kronecker product of the 1D section with itself (forward_2d_tensor).

d dimensions and unequal sides (forward_nd_* / adjoint_nd_*): the same
splitting with one 1D section per axis (mode products), in the tensor basis
(any sides) or the isotropic one (equal sides, octant layout).

Parity status: pinned (Haar closed form, norm bound, polynomial
reproduction, Fubini against the dense Kronecker matrix, Table 1 for DB2;
the tensor basis against the Kronecker product of 1D basis columns and by
the singular values it shares with the isotropic basis of the same space;
the d-dimensional functions against the 2D ones at d = 2, against columns
built one by one from 1D basis functions at d = 3 and for unequal sides,
separable inputs, and shared singular values).
"""
import numpy as np
import scipy.sparse as sp

from . import basis, walsh


def walsh_rows(J, rows, C):
    """Rows `rows` of H C (H = Walsh matrix of order 2^J), C sparse (2^J x K).

    Each chunk of rows of H is generated once and multiplied with all K
    columns; C is expanded to a dense array when it fits in 2 GiB, so that
    the product is one BLAS matrix product per chunk.
    """
    out = np.empty((len(rows), C.shape[1]))
    dense = C.toarray() if C.shape[0] * C.shape[1] <= (1 << 28) else None
    step = 256
    for a in range(0, len(rows), step):
        Hr = walsh.walsh_matrix(J, rows=rows[a:a + step])
        out[a:a + step] = Hr @ dense if dense is not None else (C.T @ Hr.T).T
    return out


def walsh_cols(J, C):
    """Full H C, built in row chunks."""
    return walsh_rows(J, np.arange(1 << J), C)


class Config:
    """Sizes of one operator: M = 2^j per dimension, N = 2^(j+q), coarse level j0;
    per=True selects the periodic extension instead of the boundary functions;
    tensor=True the tensor-product 2D basis instead of the isotropic one."""

    def __init__(self, nu, j, q, j0=None, per=False, tensor=False):
        if j0 is None:
            j0 = max(0, int(np.ceil(np.log2(2 * nu)))) if nu >= 2 else 0
        if q < 1 or j < j0 or (1 << j0) < 2 * nu and nu >= 2:
            raise ValueError("invalid (nu, j, q, j0)")
        self.nu, self.j, self.q, self.j0, self.per, self.tensor = nu, j, q, j0, per, tensor
        self.J = j + q
        self.M, self.N = 1 << j, 1 << (j + q)


def matrix_1d(cfg):
    """Dense N x M matrix A of the wavelet basis C_{psi,j}."""
    C = basis.multiscale(cfg.nu, cfg.j, cfg.j0, cfg.J, cfg.per)
    return walsh_cols(cfg.J, C)


def scaling_matrix_1d(cfg):
    """Dense N x M matrix of the scaling basis B_{phi,j} (P_N U P_M of Sec. 4)."""
    C = basis.block(cfg.nu, cfg.j, cfg.J, True, cfg.per)
    return walsh_cols(cfg.J, C)


def forward_1d(A, x, omega=None):
    y = A @ x
    return y if omega is None else y[np.asarray(omega)]


def adjoint_1d(A, y, omega=None):
    if omega is None:
        return A.T @ y
    return A[np.asarray(omega)].T @ y


class Blocks2D:
    """1D Walsh-coefficient blocks A_phi[k], A_psi[k] (N x 2^k) for the 2D basis."""

    def __init__(self, cfg, rows=None):
        self.cfg = cfg
        rows = np.arange(cfg.N) if rows is None else np.asarray(rows)
        self.rows = rows
        nu, J = cfg.nu, cfg.J
        # every block is H C_block for the same Walsh rows: one product with
        # the blocks' cell-integral matrices side by side
        keys = [("phi", cfg.j0)]
        for k in range(cfg.j0, cfg.j):
            keys += [("phi", k)] if k != cfg.j0 else []
            keys += [("psi", k)]
        parts = [basis.block(nu, k, J, kind == "phi", cfg.per) for kind, k in keys]
        allcols = walsh_rows(J, rows, sp.hstack(parts).tocsc())
        self.phi, self.psi = {}, {}
        c = 0
        for (kind, k), part in zip(keys, parts):
            (self.phi if kind == "phi" else self.psi)[k] = allcols[:, c:c + part.shape[1]]
            c += part.shape[1]

    def bands(self):
        """Yield (row slice, col slice, first-dim block, second-dim block)."""
        c = self.cfg
        s0 = slice(0, 1 << c.j0)
        yield s0, s0, self.phi[c.j0], self.phi[c.j0]
        for k in range(c.j0, c.j):
            lo, hi = slice(0, 1 << k), slice(1 << k, 1 << (k + 1))
            yield lo, hi, self.phi[k], self.psi[k]
            yield hi, lo, self.psi[k], self.phi[k]
            yield hi, hi, self.psi[k], self.psi[k]


def _forward_2d(rows_blocks, col_blocks, X, omega):
    """alpha[rows_blocks.rows, col_blocks.rows] = sum_bands A_a X_band A_b^T."""
    cfg = rows_blocks.cfg
    alpha = np.zeros((len(rows_blocks.rows), len(col_blocks.rows)))
    it_r = rows_blocks.bands()
    it_c = col_blocks.bands()
    for (rs, cs, Aa, _), (_, _, _, Bb) in zip(it_r, it_c):
        alpha += Aa @ X[rs, cs] @ Bb.T
    if omega is None:
        return alpha
    return alpha.ravel()[np.asarray(omega)]


def forward_2d_full(blocks, X, omega=None):
    """Full N x N alpha (blocks must hold all N rows)."""
    return _forward_2d(blocks, blocks, X, omega)


def adjoint_2d_full(blocks, y, omega=None):
    """x = A^T P_Omega^T y with the full blocks; returns the M x M quadtree array."""
    cfg = blocks.cfg
    if omega is None:
        Y = np.asarray(y).reshape(cfg.N, cfg.N)
    else:
        Y = np.zeros(cfg.N * cfg.N)
        Y[np.asarray(omega)] = y
        Y = Y.reshape(cfg.N, cfg.N)
    X = np.zeros((cfg.M, cfg.M))
    for rs, cs, Aa, Bb in blocks.bands():
        X[rs, cs] += Aa.T @ Y @ Bb
    return X


def forward_2d_rows(blocks, X, rows):
    """Rows n1 in `rows` of the full N x N alpha: sum over bands of A_a[rows] X_band A_b^T."""
    rows = np.asarray(rows)
    alpha = np.zeros((rows.size, blocks.cfg.N))
    for rs, cs, Aa, Bb in blocks.bands():
        alpha += Aa[rows] @ X[rs, cs] @ Bb.T
    return alpha


def adjoint_2d_rows(blocks, Y_rows, rows):
    """x = A^T y for a sample array y that vanishes outside the rows n1 in `rows`;
    Y_rows holds those rows (len(rows) x N).  Summed over disjoint row sets this
    is adjoint_2d_full."""
    rows = np.asarray(rows)
    cfg = blocks.cfg
    X = np.zeros((cfg.M, cfg.M))
    for rs, cs, Aa, Bb in blocks.bands():
        X[rs, cs] += Aa[rows].T @ Y_rows @ Bb
    return X


# ---------------------------------------------------------------------------
# Tensor-product 2D basis: the functions r_{c1} (x) r_{c2}, r the 1D multiscale
# basis C_{psi,j}, x[c1, c2] their coefficients.  By Fubini (Sec. 5) the
# section is the Kronecker product of the 1D section with itself.

def forward_2d_tensor(A1, X, omega=None):
    """alpha = A1 X A1^T (A1 the dense N x M 1D section), gathered on omega."""
    alpha = A1 @ np.asarray(X) @ A1.T
    return alpha if omega is None else alpha.ravel()[np.asarray(omega)]


def adjoint_2d_tensor(A1, y, omega=None):
    """X = A1^T Y A1 with Y the N x N array holding y on omega (zero elsewhere)."""
    N = A1.shape[0]
    if omega is None:
        Y = np.asarray(y).reshape(N, N)
    else:
        Y = np.zeros(N * N)
        Y[np.asarray(omega)] = y
        Y = Y.reshape(N, N)
    return A1.T @ Y @ A1


def quadtree_functions(cfg, c1, c2):
    """For quadtree position (c1, c2): ((kind1, level1, idx1), (kind2, level2, idx2))."""
    j0 = cfg.j0
    if c1 < (1 << j0) and c2 < (1 << j0):
        return ("phi", j0, c1), ("phi", j0, c2)
    k = max(int(c1).bit_length(), int(c2).bit_length()) - 1
    if c1 < (1 << k):
        return ("phi", k, c1), ("psi", k, c2 - (1 << k))
    if c2 < (1 << k):
        return ("psi", k, c1 - (1 << k)), ("phi", k, c2)
    return ("psi", k, c1 - (1 << k)), ("psi", k, c2 - (1 << k))


def dense_2d(cfg):
    """Dense (N^2 x M^2) matrix by Kronecker products of 1D columns (tiny sizes only)."""
    J, nu = cfg.J, cfg.nu
    cols = {}

    def col(kind, level, idx):
        key = (kind, level, idx)
        if key not in cols:
            if cfg.per:
                i, v = basis.periodic_cells(nu, level, idx, J, kind == "phi")
            else:
                f = basis.scaling_function_cells if kind == "phi" else basis.wavelet_cells
                i, v = f(nu, level, idx, J)
            c = np.zeros(cfg.N)
            c[i] = v
            cols[key] = walsh.walsh_matrix(J) @ c
        return cols[key]

    A2 = np.zeros((cfg.N * cfg.N, cfg.M * cfg.M))
    for c1 in range(cfg.M):
        for c2 in range(cfg.M):
            if cfg.tensor:
                f1, f2 = basis.position_1d(c1, cfg.j0), basis.position_1d(c2, cfg.j0)
                f1, f2 = (f1[1], f1[0], f1[2]), (f2[1], f2[0], f2[2])
            else:
                f1, f2 = quadtree_functions(cfg, c1, c2)
            A2[:, c1 * cfg.M + c2] = np.kron(col(*f1), col(*f2))
    return A2


# ---------------------------------------------------------------------------
# Entry-by-entry evaluation for sizes where the full product is too costly.

def forward_entries_2d(cfg, X, n1s, n2s):
    """alpha[n1s[i], n2s[i]] for each i, from rows of the 1D blocks (plain sums)."""
    n1s, n2s = np.asarray(n1s), np.asarray(n2s)
    rows = np.unique(np.concatenate([n1s, n2s]))
    B = Blocks2D(cfg, rows=rows)
    pos = {int(r): i for i, r in enumerate(rows)}
    i1 = np.array([pos[int(v)] for v in n1s])
    i2 = np.array([pos[int(v)] for v in n2s])
    out = np.zeros(n1s.size)
    for rs, cs, Aa, Bb in B.bands():
        out += np.einsum("ia,ab,ib->i", Aa[i1], X[rs, cs], Bb[i2])
    return out


def walsh_column(cfg, kind, level, idx):
    """Column <f, w_n>, n < N, of one 1D basis function (kind 'phi' or 'psi')."""
    if cfg.per:
        cells, vals = basis.periodic_cells(cfg.nu, level, idx, cfg.J, kind == "phi")
    else:
        f = basis.scaling_function_cells if kind == "phi" else basis.wavelet_cells
        cells, vals = f(cfg.nu, level, idx, cfg.J)
    out = np.zeros(cfg.N)
    step = 1024
    for a in range(0, cfg.N, step):
        H = walsh.walsh_matrix_bits(cfg.J, rows=np.arange(a, min(cfg.N, a + step)), cols=cells)
        out[a:a + step] = H @ vals
    return out


def adjoint_entries_2d(cfg, y, omega, positions):
    """x[c1, c2] = sum_i A2[omega_i, (c1, c2)] y_i for each quadtree position (plain sums)."""
    omega = np.asarray(omega)
    n1, n2 = omega // cfg.N, omega % cfg.N
    out = []
    for c1, c2 in positions:
        f1, f2 = quadtree_functions(cfg, c1, c2)
        a1 = walsh_column(cfg, *f1)
        a2 = walsh_column(cfg, *f2)
        out.append(np.dot(a1[n1] * a2[n2], y))
    return np.array(out)


def forward_entries_1d(cfg, x, ns, C=None):
    """y_n = sum_c A[n, c] x_c for each n in ns, as sum_i w_n(i/N) f[i] with f = C x
    the cell integrals of the function sum_c x_c r_c (plain sums, no fast transform)."""
    C = basis.multiscale(cfg.nu, cfg.j, cfg.j0, cfg.J, cfg.per) if C is None else C
    f = C @ np.asarray(x, dtype=np.float64)
    ns = np.asarray(ns)
    out = np.empty(ns.size)
    step = 64
    for a in range(0, ns.size, step):
        H = walsh.walsh_matrix_bits(cfg.J, rows=ns[a:a + step], cols=np.arange(cfg.N))
        out[a:a + step] = H @ f
    return out


def adjoint_entries_1d(cfg, y, omega, cs, C=None):
    """(A[omega]^T y)_c for each position c in cs: the column of one basis function
    restricted to omega, against y (plain sums)."""
    C = basis.multiscale(cfg.nu, cfg.j, cfg.j0, cfg.J, cfg.per) if C is None else C
    omega = np.arange(cfg.N) if omega is None else np.asarray(omega)
    out = []
    for c in cs:
        col = C[:, int(c)]
        cells = col.indices
        H = walsh.walsh_matrix_bits(cfg.J, rows=omega, cols=cells)
        out.append(np.dot(H @ col.data, y))
    return np.array(out)



# ---------------------------------------------------------------------------
# d dimensions and unequal sides.  Sec. 5 splits the 2D inner products into
# 1D ones (Fubini); the same splitting holds for any d-fold tensor product.
# Sampling functions w_{n_0} (x) ... (x) w_{n_{d-1}}; y lists alpha in
# increasing linear index over the row-major N_0 x ... x N_{d-1} array.
# Two reconstruction bases:
# * tensor: the products r_{c_0} (x) ... (x) r_{c_{d-1}} of the 1D multiscale
#   bases of the axes, whose sizes may differ (M_a = 2^{j_a}, N_a = 2^{j_a+q}).
#   The section is the Kronecker product of the 1D sections, applied here one
#   axis at a time (mode products);
# * isotropic (equal sides): the d-dimensional analogue of the quadtree
#   layout.  The coarse cube [0, 2^{j0})^d holds phi_{j0} (x) ... (x) phi_{j0};
#   at each level k the cube [0, 2^{k+1})^d holds 2^d - 1 detail blocks, one
#   per nonzero beta in {0, 1}^d, at offset 2^k along the axes with
#   beta_a = 1, holding psi_k along those axes and phi_k along the others.

def mode_apply(mats, X):
    """Y = X x_0 mats[0] x_1 mats[1] ... : matrix mats[a] acts on axis a of X."""
    Y = np.asarray(X, dtype=np.float64)
    for a, A in enumerate(mats):
        Y = np.moveaxis(np.tensordot(A, Y, axes=([1], [a])), 0, a)
    return Y


def _scatter_samples(shape, y, omega):
    """The array of the given shape holding y at the linear indices omega (zero elsewhere)."""
    size = int(np.prod(shape))
    if omega is None:
        return np.asarray(y, dtype=np.float64).reshape(shape)
    Y = np.zeros(size)
    Y[np.asarray(omega)] = y
    return Y.reshape(shape)


def forward_nd_tensor(mats, X, omega=None):
    """alpha = X with the 1D section mats[a] (N_a x M_a) applied along each axis a."""
    alpha = mode_apply(mats, X)
    return alpha if omega is None else alpha.ravel()[np.asarray(omega)]


def adjoint_nd_tensor(mats, y, omega=None):
    """X = Y with mats[a]^T applied along each axis, Y holding y on omega."""
    Y = _scatter_samples(tuple(A.shape[0] for A in mats), y, omega)
    return mode_apply([A.T for A in mats], Y)


def octant_bands(cfg, d):
    """Yield (slices, kinds, level) of the isotropic d-dimensional basis."""
    import itertools
    s0 = slice(0, 1 << cfg.j0)
    yield (s0,) * d, ("phi",) * d, cfg.j0
    for k in range(cfg.j0, cfg.j):
        lo, hi = slice(0, 1 << k), slice(1 << k, 1 << (k + 1))
        for beta in itertools.product((0, 1), repeat=d):
            if any(beta):
                yield tuple(hi if b else lo for b in beta), tuple("psi" if b else "phi" for b in beta), k


def forward_nd_iso(blocks, X, omega=None):
    """Isotropic basis: alpha = sum over blocks of X_block with the 1D blocks
    A_phi[k] / A_psi[k] (Blocks2D, all N rows) applied along each axis."""
    X = np.asarray(X, dtype=np.float64)
    d, N = X.ndim, blocks.cfg.N
    alpha = np.zeros((N,) * d)
    for sl, kinds, k in octant_bands(blocks.cfg, d):
        alpha += mode_apply([blocks.phi[k] if kd == "phi" else blocks.psi[k] for kd in kinds], X[sl])
    return alpha if omega is None else alpha.ravel()[np.asarray(omega)]


def adjoint_nd_iso(blocks, y, d, omega=None):
    """Its transpose: the M^d array of coefficients from y on omega."""
    cfg = blocks.cfg
    Y = _scatter_samples((cfg.N,) * d, y, omega)
    X = np.zeros((cfg.M,) * d)
    for sl, kinds, k in octant_bands(cfg, d):
        X[sl] += mode_apply([(blocks.phi[k] if kd == "phi" else blocks.psi[k]).T for kd in kinds], Y)
    return X


def octree_functions(cfg, cs):
    """For isotropic position cs = (c_0, ..., c_{d-1}): the 1D function (kind, level, idx) per axis."""
    j0 = cfg.j0
    if all(c < (1 << j0) for c in cs):
        return [("phi", j0, int(c)) for c in cs]
    k = max(int(c).bit_length() for c in cs) - 1
    return [("phi", k, int(c)) if c < (1 << k) else ("psi", k, int(c) - (1 << k)) for c in cs]


def dense_nd(cfgs, tensor, columns=None):
    """Dense (prod N_a) x (prod M_a) matrix, column by column as Kronecker products
    of the 1D Walsh columns of the basis functions (tiny sizes only).  cfgs: one
    Config per axis (equal ones for the isotropic basis); columns: the linear
    coefficient indices to build (all by default), in that order."""
    cols = {}

    def col(a, kind, level, idx):
        key = (a, kind, level, idx)
        if key not in cols:
            cols[key] = walsh_column(cfgs[a], kind, level, idx)
        return cols[key]

    shape_m = [c.M for c in cfgs]
    if columns is None:
        columns = range(int(np.prod(shape_m)))
    columns = list(columns)
    A = np.zeros((int(np.prod([c.N for c in cfgs])), len(columns)))
    for ci, flat in enumerate(columns):
        cs = np.unravel_index(int(flat), shape_m)
        if tensor:
            fs = []
            for a, c in enumerate(cs):
                level, kind, idx = basis.position_1d(c, cfgs[a].j0)
                fs.append((kind, level, idx))
        else:
            fs = octree_functions(cfgs[0], cs)
        v = np.ones(1)
        for a, f in enumerate(fs):
            v = np.kron(v, col(a, *f))
        A[:, ci] = v
    return A
