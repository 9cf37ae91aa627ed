"""Daubechies scaling and wavelet filters (Sec. 3.2), computed from scratch.

Test infrastructure (see the package header).

The paper uses compactly supported orthonormal wavelets with nu vanishing
moments and minimal support, in the Daubechies (minimum-phase) choice, with
supp(phi) = supp(psi) = [-nu+1, nu].  The filter is obtained by the textbook
spectral factorisation: with y = sin^2(omega/2) the squared modulus of the
trigonometric polynomial is built from P(y) = sum_{k<nu} C(nu-1+k, k) y^k.
Each root y_i of P gives a pair z, 1/z with (2 - z - 1/z)/4 = y_i; keeping the
root inside the unit circle gives the minimum-phase factor.  The filter is
the coefficient list of ((1+z)/2)^nu * prod_i (z - z_i), normalised to
sum sqrt(2), read from the highest power of z down, so that h_0 is the
largest leading tap (the convention of Daubechies' tables).  All arithmetic
is done in mpmath at 60 digits.

Index convention: h[c] for c in [-nu+1, nu] (the paper's support convention),
stored in arrays at position c + nu - 1.  The wavelet filter is
g_c = (-1)^c h_{1-c}, which keeps the support [-nu+1, nu].

Pins: the closed form of the nu = 2 filter, sum h = sqrt 2, double-shift
orthogonality, nu vanishing moments of g, and the minimum-phase root
condition; nu = 1 is the Haar filter.
"""
import functools

import mpmath as mp
import numpy as np

DPS = 60


class Symlet(int):
    """The number of vanishing moments, tagged as the least-asymmetric family.

    Symlet(nu) behaves as the integer nu everywhere (supports, index ranges);
    only the filter differs, so every function of this package that takes
    `nu` accepts a Symlet and caches it apart from the Daubechies order
    (the caches are keyed by type).
    """

    def __repr__(self):
        return f"Symlet({int(self)})"


def family(nu):
    return "sym" if isinstance(nu, Symlet) else "db"


def _y_roots(nu):
    """Roots of P(y) = sum_{k<nu} C(nu-1+k, k) y^k (mpmath, at the working precision)."""
    p_coeffs = [mp.binomial(nu - 1 + k, k) for k in range(nu)]
    return mp.polyroots(p_coeffs[::-1], maxsteps=500, extraprec=4 * DPS)


def _inside_root(y):
    """The root z, |z| < 1, of (2 - z - 1/z) / 4 = y."""
    b = 2 - 4 * y
    d = mp.sqrt(b * b - 4)
    z1, z2 = (b + d) / 2, (b - d) / 2
    return z1 if abs(z1) < 1 else z2


def _taps_from_roots(nu, z_roots):
    """Coefficients of ((1+z)/2)^nu prod (z - z_i), highest power first, scaled to sum sqrt 2."""
    poly = [mp.mpc(1)]
    for _ in range(nu):
        poly = _polymul(poly, [mp.mpc(1), mp.mpc(1)])
    for z in z_roots:
        poly = _polymul(poly, [mp.mpc(1), -z])
    taps = [mp.re(c) for c in poly]
    total = mp.fsum(taps)
    return tuple(t * mp.sqrt(2) / total for t in taps)


@functools.lru_cache(maxsize=None, typed=True)
def daubechies_mp(nu):
    """Tuple of mpf filter taps h_c, c = -nu+1 .. nu (Daubechies, minimum phase)."""
    if nu < 1:
        raise ValueError("nu must be >= 1")
    nu = int(nu)
    with mp.workdps(DPS):
        if nu == 1:
            return (mp.sqrt(2) / 2, mp.sqrt(2) / 2)
        return _taps_from_roots(nu, [_inside_root(y) for y in _y_roots(nu)])


PHASE_GRID = 256


def phase_deviation(z_roots):
    """Deviation from linear of the phase of the filter with factor roots z_roots.

    A filter read from ((1+z)/2)^nu prod (z - z_i) (highest power first) has
    the frequency response e^{-i D w} c (1 + e^{iw})^nu prod (e^{iw} - z_i)
    (D = 2 nu - 1), whose phase is linear in w plus
    phi(w) = sum_i arg(e^{iw} - z_i).  phi is evaluated from the roots on
    w_k = pi k / K, k = 0 .. K (K = 256), unwrapped along k; a straight line
    a + c w is fitted to it by least squares and the largest absolute
    residual is returned.  (Evaluating the phase from the taps instead loses
    all accuracy near w = pi, where the response has a zero of order nu.)
    """
    K = PHASE_GRID
    w = [mp.pi * k / K for k in range(K + 1)]
    theta = []
    for wk in w:
        u = mp.expj(wk)
        a = mp.fsum(mp.arg(u - z) for z in z_roots)
        if theta:
            while a - theta[-1] > mp.pi:
                a -= 2 * mp.pi
            while a - theta[-1] <= -mp.pi:
                a += 2 * mp.pi
        theta.append(a)
    n = mp.mpf(K + 1)
    sw, st = mp.fsum(w), mp.fsum(theta)
    sww, swt = mp.fsum(x * x for x in w), mp.fsum(x * t for x, t in zip(w, theta))
    c = (n * swt - sw * st) / (n * sww - sw * sw)
    a0 = (st - c * sw) / n
    return max(abs(t - a0 - c * x) for x, t in zip(w, theta))


@functools.lru_cache(maxsize=None)
def symlet_roots(nu):
    """Factor roots z_i of the least-asymmetric filter (see symlet_mp)."""
    nu = int(nu)
    with mp.workdps(DPS):
        ys = _y_roots(nu)
        tol = mp.mpf(10) ** (-DPS // 2)
        reps = sorted([y for y in ys if mp.im(y) >= -tol], key=lambda y: (float(mp.re(y)), float(mp.im(y))))
        groups = []
        for y in reps:
            zin = _inside_root(y)
            if abs(mp.im(y)) <= tol:
                groups.append([zin])
            else:
                groups.append([zin, mp.conj(zin)])
        best, best_dev = None, None
        for mask in range(1 << len(groups)):
            roots = []
            for g, grp in enumerate(groups):
                roots += [1 / z for z in grp] if (mask >> g) & 1 else grp
            dev = phase_deviation(roots)
            if best_dev is None or dev < best_dev - mp.mpf(10) ** -20:
                best, best_dev = roots, dev
        return tuple(best)


@functools.lru_cache(maxsize=None)
def symlet_mp(nu):
    """Tuple of mpf taps h_c, c = -nu+1 .. nu, of the least-asymmetric filter.

    Reading (the paper uses symlets but does not define the choice): the
    spectral factorisation of the Daubechies construction leaves one free
    choice per root group of P(y) -- a real root, or a complex-conjugate pair
    taken together so that the taps stay real -- namely the factor inside or
    outside the unit circle.  Groups are ordered by the real part of their
    member with non-negative imaginary part (then by that imaginary part);
    choice mask bit g set means group g takes the outside factor.  The symlet
    is the candidate of least phase_deviation; a mask and its complement are
    the same filter reversed and tie, and the smaller mask wins.  Mask 0 is
    the Daubechies filter, so sym2 = db2 and sym3 = db3 (each has one group).
    """
    nu = int(nu)
    if nu < 1:
        raise ValueError("nu must be >= 1")
    if nu == 1:
        return daubechies_mp(1)
    with mp.workdps(DPS):
        return _taps_from_roots(nu, list(symlet_roots(nu)))


def scaling_mp(nu):
    """The scaling filter of the family `nu` belongs to (Daubechies or Symlet)."""
    return symlet_mp(nu) if isinstance(nu, Symlet) else daubechies_mp(nu)


def _polymul(a, b):
    out = [mp.mpc(0)] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for k, bk in enumerate(b):
            out[i + k] += ai * bk
    return out


@functools.lru_cache(maxsize=None, typed=True)
def wavelet_mp(nu):
    """Tuple of mpf wavelet taps g_c = (-1)^c h_{1-c}, c = -nu+1 .. nu."""
    h = scaling_mp(nu)
    out = []
    with mp.workdps(DPS):           # cached: never round at the caller's precision
        for c in range(-nu + 1, nu + 1):
            out.append(-h[(1 - c) + nu - 1] if c % 2 else +h[(1 - c) + nu - 1])
    return tuple(out)


def daubechies(nu):
    """float64 array of h_c, c = -nu+1 .. nu (the family of `nu`: Daubechies or Symlet)."""
    return np.array([float(t) for t in scaling_mp(nu)])


def wavelet(nu):
    """float64 array of g_c, c = -nu+1 .. nu."""
    return np.array([float(t) for t in wavelet_mp(nu)])
