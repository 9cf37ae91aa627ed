"""Cell integrals of the wavelet bases on [0, 1] (Sec. 3.2).

Test infrastructure (see the package header).

For a level k >= J0 the scaling basis B_{phi,k} is, in this order,
  phi^left_m (m = 0..nu-1), interior phi_{k,m} (m = nu .. 2^k-nu-1),
  phi^right_{2^k-1-m} (m = 2^k-nu .. 2^k-1),
and B_{psi,k} is the same with psi.  Boundary functions are dilated as in
Sec. 3.2: phi^bd_{k,m}(x) = 2^{k/2} phi^left_m(2^k x) on the left and
2^{k/2} phi^right_{2^k-1-m}(2^k (x - 1)) on the right.  The multiscale basis
is C_{psi,j} = B_{phi,J0} u B_{psi,J0} u ... u B_{psi,j-1}.

Each function is returned by its cell integrals c[i] over the 2^J cells
[i 2^-J, (i+1) 2^-J) of [0, 1], built from the cascade cell integrals of
phi (Phi_r) and psi (Psi_r):
  interior phi_{k,m}:  c[i] = 2^{-k/2} Phi_{J-k}[i - m 2^{J-k}]
  interior psi_{k,m}:  c[i] = 2^{-k/2} Psi_{J-k}[i - m 2^{J-k}]
  boundary functions:  the same for each translate in their coefficient
                       vectors, keeping only cells inside [0, 1).

Periodic extension (per=True in block / multiscale): every function of
level k is periodised with period 1 (Sec. 3.2), no boundary functions.

Parity status: pinned by polynomial reproduction, orthonormality against
point-value quadrature, zero mean of wavelets and the Haar closed form; the
periodic basis by orthonormality against quadrature, the partition of unity,
the Haar case and the periodic formulas of Prop. 4.2.
"""
import functools

import numpy as np
import scipy.sparse as sp

from . import cascade, halfline


def _translate_cells(nu, level, t, J, scaling=True, extended=False):
    """(cell indices, values) of 2^{level/2} f(2^level x - t) on [0, 1), f = phi or psi."""
    r = J - level
    tab = cascade.phi_cells(nu, r) if scaling else cascade.psi_cells(nu, r)
    s = np.arange(tab.lo, tab.lo + tab.values.size)
    i = s + t * (1 << r)
    keep = (i >= 0) & (i < (1 << J))
    vals = tab.values_ld if extended else tab.values
    return i[keep], vals[keep] * (np.longdouble(2) ** (-level) if extended else 2.0 ** (-level)) ** 0.5


def _combo_cells(nu, level, coef, offset, J):
    """Cell integrals of sum_t coef[t] 2^{level/2} phi(2^level x - offset - t) on [0,1).

    Formed in extended precision (the coefficients cancel strongly), then rounded.
    """
    out = np.zeros(1 << J, dtype=np.longdouble)
    for t, a in coef.items():
        i, v = _translate_cells(nu, level, offset + t, J, extended=True)
        out[i] += np.longdouble(mp_str(a)) * v
    out = out.astype(np.float64)
    nz = np.nonzero(out)[0]
    return nz, out[nz]


def mp_str(a):
    import mpmath as mp
    return mp.nstr(a, 40) if isinstance(a, mp.mpf) else repr(float(a))


@functools.lru_cache(maxsize=None, typed=True)
def _edge_float(nu):
    return (halfline.edge_scaling(nu, "left"), halfline.edge_scaling(nu, "right"),
            halfline.edge_wavelets(nu, "left"), halfline.edge_wavelets(nu, "right"))


def scaling_function_cells(nu, k, m, J):
    """Cell integrals of the m-th function of B_{phi,k}."""
    L, R, _, _ = _edge_float(nu)
    size = 1 << k
    if m < nu:
        return _combo_cells(nu, k, L[m], 0, J)
    if m >= size - nu:
        return _combo_cells(nu, k, R[size - 1 - m], size, J)
    return _translate_cells(nu, k, m, J, scaling=True)


def wavelet_cells(nu, k, m, J):
    """Cell integrals of the m-th function of B_{psi,k}."""
    _, _, WL, WR = _edge_float(nu)
    size = 1 << k
    if m < nu:
        return _combo_cells(nu, k + 1, WL[m], 0, J)
    if m >= size - nu:
        return _combo_cells(nu, k + 1, WR[size - 1 - m], 2 * size, J)
    return _translate_cells(nu, k, m, J, scaling=False)


def periodic_cells(nu, k, m, J, scaling=True):
    """Cell integrals of the periodic-extension function phi^per_{k,m} (psi^per_{k,m}).

    Sec. 3.2 (periodic extension): a function crossing an end of [0, 1] is the
    sum of its restriction and that of the translate by +-2^k positions, i.e.
    sum_t f_{k, m + t 2^k} restricted to [0, 1] (for 2^k >= 2 nu only t = -1, 0,
    1 can meet [0, 1]).  Its cell integrals at resolution 2^-J are those of
    f_{k,m} with the cell index taken modulo 2^J.
    """
    r = J - k
    tab = cascade.phi_cells(nu, r) if scaling else cascade.psi_cells(nu, r)
    s = np.arange(tab.lo, tab.lo + tab.values.size)
    i = np.mod(s + m * (1 << r), 1 << J)
    out = np.zeros(1 << J)
    np.add.at(out, i, tab.values * 2.0 ** (-k / 2.0))
    nz = np.nonzero(out)[0]
    return nz, out[nz]


def check_level(nu, k, j0=None):
    if nu < 1:
        raise ValueError("nu must be >= 1")
    # Sec. 3.2: J0 >= ceil(log2(2 nu)) for nu >= 2 and J0 >= 0 for Haar (at k = 0 the
    # single Haar function is both the left and the right boundary function)
    if nu >= 2 and (1 << k) < 2 * nu:
        raise ValueError("level too coarse for the boundary construction: need 2^k >= 2 nu")


def block(nu, k, J, scaling, per=False):
    """Sparse (2^J x 2^k) matrix of cell integrals of B_{phi,k} or B_{psi,k}
    (boundary-corrected, or with per=True the periodic extension)."""
    check_level(nu, k)
    rows, cols, vals = [], [], []
    for m in range(1 << k):
        if per:
            i, v = periodic_cells(nu, k, m, J, scaling)
        else:
            i, v = (scaling_function_cells if scaling else wavelet_cells)(nu, k, m, J)
        rows.append(i)
        cols.append(np.full(i.size, m))
        vals.append(v)
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(1 << J, 1 << k))


def multiscale(nu, j, j0, J, per=False):
    """Sparse (2^J x 2^j) cell-integral matrix of C_{psi,j} in the paper's order."""
    parts = [block(nu, j0, J, True, per)]
    for k in range(j0, j):
        parts.append(block(nu, k, J, False, per))
    return sp.hstack(parts).tocsc()


def position_1d(c, j0):
    """Map a C_{psi,j} position c to (level, 'phi'|'psi', index)."""
    if c < (1 << j0):
        return j0, "phi", c
    k = int(c).bit_length() - 1
    return k, "psi", c - (1 << k)


# ---------------------------------------------------------------------------
# Point values on the grid i 2^-R (for the brute-force quadrature cross-check).
# They come from the point-value cascade, a path independent of the cell
# integrals and of the half-line Gram matrix.

def _translate_points(nu, level, t, R):
    """2^{level/2} phi(2^level x - t) at x = i 2^-R, i = 0 .. 2^R."""
    r = R - level
    pts = cascade.phi_points(nu, r)
    i = np.arange((1 << R) + 1)
    idx = i - t * (1 << r) - ((-nu + 1) << r)
    ok = (idx >= 0) & (idx < pts.size)
    out = np.zeros(i.size)
    out[ok] = pts[idx[ok]] * 2.0 ** (level / 2.0)
    return out


def _combo_points(nu, level, coef, offset, R):
    out = np.zeros((1 << R) + 1)
    for t, a in coef.items():
        out += float(a) * _translate_points(nu, level, offset + t, R)
    return out


def periodic_points(nu, k, m, R, scaling=True):
    """Point values of phi^per_{k,m} (psi^per_{k,m}) at x = i 2^-R, i = 0 .. 2^R: the sum of the
    translates f_{k, m + t 2^k}, t = -1, 0, 1 (point-value cascade)."""
    out = np.zeros((1 << R) + 1)
    for t in (-1, 0, 1):
        if scaling:
            out += _translate_points(nu, k, m + t * (1 << k), R)
        else:
            from . import filters
            g = filters.wavelet(nu)
            coef = {2 * (m + t * (1 << k)) + c: g[ci] for ci, c in enumerate(range(-nu + 1, nu + 1))}
            out += _combo_points(nu, k + 1, coef, 0, R)
    return out


def scaling_function_points(nu, k, m, R):
    L, Rr, _, _ = _edge_float(nu)
    size = 1 << k
    if m < nu:
        return _combo_points(nu, k, L[m], 0, R)
    if m >= size - nu:
        return _combo_points(nu, k, Rr[size - 1 - m], size, R)
    return _translate_points(nu, k, m, R)


def wavelet_points(nu, k, m, R):
    from . import filters
    _, _, WL, WR = _edge_float(nu)
    size = 1 << k
    if m < nu:
        return _combo_points(nu, k + 1, WL[m], 0, R)
    if m >= size - nu:
        return _combo_points(nu, k + 1, WR[size - 1 - m], 2 * size, R)
    g = filters.wavelet(nu)
    coef = {2 * m + c: g[ci] for ci, c in enumerate(range(-nu + 1, nu + 1))}
    return _combo_points(nu, k + 1, coef, 0, R)


def halfline_scaling_cells(nu, side, m, r, cells):
    """Cell integrals of phi^side_m over the sub-cells of the given unit cells.

    Returns (values, bound), arrays of shape (len(cells), 2^r): entry [i, t] of
    `values` is the integral of the boundary scaling function over
    [c + t 2^-r, c + (t+1) 2^-r), c = cells[i] (level-0 units, measured from the
    boundary point), summed in extended precision; `bound` is a rounding-error
    bound for that sum (64 eps_ld times the sum of the absolute terms; the
    terms cancel by up to six digits at nu = 8).
    """
    coef = halfline.edge_scaling(nu, side)[m]
    tab = cascade.phi_cells(nu, r)
    out = np.zeros((len(cells), 1 << r), dtype=np.longdouble)
    mag = np.zeros((len(cells), 1 << r), dtype=np.longdouble)
    sub = np.arange(1 << r)
    for i, c in enumerate(cells):
        for t, a in coef.items():
            term = np.longdouble(mp_str(a)) * tab.take((c - t) * (1 << r) + sub, extended=True)
            out[i] += term
            mag[i] += np.abs(term)
    eps = float(np.finfo(np.longdouble).eps)
    return out.astype(np.float64), (64 * eps * mag).astype(np.float64) + 1e-17
