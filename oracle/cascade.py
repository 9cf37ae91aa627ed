"""Cell integrals and point values of phi and psi by the cascade algorithm.

Test infrastructure (see the package header).

Sec. 3.2 notes that phi and psi have no closed form and are computed at
dyadic points by the cascade algorithm.  The operator only needs integrals
of phi over dyadic cells, so the cascade is run on cell integrals, which is
exact up to rounding (point values followed by a quadrature rule would
converge only like the Hoelder exponent of phi).

  Phi_r[s] = integral of phi over [s 2^-r, (s+1) 2^-r),   s in [(-nu+1) 2^r, nu 2^r).

From phi(x) = sqrt(2) sum_c h_c phi(2x - c):
  Phi_0[s]     = 2^-1/2 sum_c h_c (Phi_0[2s - c] + Phi_0[2s - c + 1])   (eigenvector, eigenvalue 1)
  Phi_{r}[s]   = 2^-1/2 sum_c h_c Phi_{r-1}[s - c 2^(r-1)]               (r >= 1)
  Psi_{r}[s]   = 2^-1/2 sum_c g_c Phi_{r-1}[s - c 2^(r-1)]               (r >= 1)
with sum_s Phi_0[s] = 1 fixing the scale (the integral of phi is 1).

Point values (used only by the brute-force cross-check): phi at the
integers is the eigenvector of phi(s) = sqrt(2) sum_c h_c phi(2s - c) with
sum_s phi(s) = 1, and phi(k 2^-(r+1)) follows from the same relation.

Pins: sum_s Phi_r[s] = 1, two children sum to their parent, the Haar case
(Phi_r = 2^-r on [0, 1)), the first moment of phi from the filter, and
trapezoid quadrature of the point values converging to the cell integrals.
"""
import functools

import numpy as np

from . import filters


class CellIntegrals:
    """Phi_r (or Psi_r) stored with an offset so that arr[s - lo] = value at s.

    `values_ld` holds the same numbers in x87 extended precision (64-bit
    mantissa); `values` is their float64 rounding.  The boundary functions are
    combinations of translates whose coefficients reach 1e7 and cancel by up to
    four digits (nu = 8), so their cell integrals are formed from `values_ld`.
    """

    def __init__(self, r, lo, values_ld):
        self.r = r
        self.lo = lo
        self.values_ld = np.asarray(values_ld, dtype=np.longdouble)
        self.values = self.values_ld.astype(np.float64)

    def __getitem__(self, s):
        i = s - self.lo
        if 0 <= i < self.values.size:
            return self.values[i]
        return 0.0

    def take(self, s, extended=False):
        """Vectorised lookup with zeros outside the support."""
        s = np.asarray(s) - self.lo
        ok = (s >= 0) & (s < self.values.size)
        src = self.values_ld if extended else self.values
        out = np.zeros(s.shape, dtype=src.dtype)
        out[ok] = src[s[ok]]
        return out


def _phi0(h, nu):
    cells = list(range(-nu + 1, nu))
    n = len(cells)
    T = np.zeros((n, n))
    for a, s in enumerate(cells):
        for ci, c in enumerate(range(-nu + 1, nu + 1)):
            for t in (2 * s - c, 2 * s - c + 1):
                if -nu + 1 <= t <= nu - 1:
                    T[a, t + nu - 1] += h[ci] / np.sqrt(2.0)
    w, v = np.linalg.eig(T)
    i = int(np.argmin(np.abs(w - 1.0)))
    if abs(w[i] - 1.0) > 1e-10:
        raise RuntimeError("refinement operator has no eigenvalue 1")
    vec = np.real(v[:, i]).astype(np.longdouble)
    vec /= vec.sum()
    # polish in extended precision: the other eigenvalues are at most 1/2 in modulus
    h_ld = _taps_ld(filters.scaling_mp(nu))
    Tld = np.zeros((n, n), dtype=np.longdouble)
    for a, s in enumerate(cells):
        for ci, c in enumerate(range(-nu + 1, nu + 1)):
            for t in (2 * s - c, 2 * s - c + 1):
                if -nu + 1 <= t <= nu - 1:
                    Tld[a, t + nu - 1] += h_ld[ci] / np.sqrt(np.longdouble(2))
    for _ in range(80):
        vec = Tld @ vec
        vec /= vec.sum()
    return vec


def _taps_ld(taps_mp):
    import mpmath as mp
    return [np.longdouble(mp.nstr(t, 40)) for t in taps_mp]


@functools.lru_cache(maxsize=None, typed=True)
def phi_cells(nu, r):
    """Phi_r for the Daubechies scaling function with nu vanishing moments."""
    if r == 0:
        return CellIntegrals(0, -nu + 1, _phi0(filters.daubechies(nu), nu))
    h = _taps_ld(filters.scaling_mp(nu))
    prev = phi_cells(nu, r - 1)
    lo, hi = (-nu + 1) << r, nu << r
    s = np.arange(lo, hi)
    out = np.zeros(s.size, dtype=np.longdouble)
    for ci, c in enumerate(range(-nu + 1, nu + 1)):
        out += h[ci] * prev.take(s - c * (1 << (r - 1)), extended=True)
    return CellIntegrals(r, lo, out / np.sqrt(np.longdouble(2)))


@functools.lru_cache(maxsize=None, typed=True)
def psi_cells(nu, r):
    """Psi_r, cell integrals of the wavelet psi at resolution 2^-r."""
    if r == 0:
        fine = psi_cells(nu, 1)
        s = np.arange(-nu + 1, nu)
        return CellIntegrals(0, -nu + 1, fine.take(2 * s, True) + fine.take(2 * s + 1, True))
    g = _taps_ld(filters.wavelet_mp(nu))
    prev = phi_cells(nu, r - 1)
    lo, hi = (-nu + 1) << r, nu << r
    s = np.arange(lo, hi)
    out = np.zeros(s.size, dtype=np.longdouble)
    for ci, c in enumerate(range(-nu + 1, nu + 1)):
        out += g[ci] * prev.take(s - c * (1 << (r - 1)), extended=True)
    return CellIntegrals(r, lo, out / np.sqrt(np.longdouble(2)))


@functools.lru_cache(maxsize=None, typed=True)
def phi_points(nu, r):
    """phi(k 2^-r) for k in [(-nu+1) 2^r, nu 2^r], point-value cascade."""
    h = filters.daubechies(nu)
    if r == 0:
        ints = list(range(-nu + 1, nu + 1))
        n = len(ints)
        T = np.zeros((n, n))
        for a, s in enumerate(ints):
            for ci, c in enumerate(range(-nu + 1, nu + 1)):
                t = 2 * s - c
                if -nu + 1 <= t <= nu:
                    T[a, t + nu - 1] += np.sqrt(2.0) * h[ci]
        w, v = np.linalg.eig(T)
        i = int(np.argmin(np.abs(w - 1.0)))
        vec = np.real(v[:, i])
        return vec / vec.sum()
    prev = phi_points(nu, r - 1)
    lo = (-nu + 1) << r
    k = np.arange(lo, (nu << r) + 1)
    out = np.zeros(k.size)
    # phi(k 2^-r) = sqrt2 sum_c h_c phi((k - c 2^(r-1)) 2^-(r-1)): a lookup on the level r-1 grid
    for ci, c in enumerate(range(-nu + 1, nu + 1)):
        j = k - c * (1 << (r - 1)) - ((-nu + 1) << (r - 1))
        ok = (j >= 0) & (j < prev.size)
        out[ok] += np.sqrt(2.0) * h[ci] * prev[j[ok]]
    return out
