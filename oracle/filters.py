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


@functools.lru_cache(maxsize=None)
def daubechies_mp(nu):
    """Tuple of mpf filter taps h_c, c = -nu+1 .. nu."""
    if nu < 1:
        raise ValueError("nu must be >= 1")
    with mp.workdps(DPS):
        if nu == 1:
            return (mp.sqrt(2) / 2, mp.sqrt(2) / 2)
        p_coeffs = [mp.binomial(nu - 1 + k, k) for k in range(nu)]
        y_roots = mp.polyroots(p_coeffs[::-1], maxsteps=500, extraprec=4 * DPS)
        z_roots = []
        for y in y_roots:
            b = 2 - 4 * y
            d = mp.sqrt(b * b - 4)
            z1, z2 = (b + d) / 2, (b - d) / 2
            z_roots.append(z1 if abs(z1) < 1 else z2)
        poly = [mp.mpc(1)]
        for _ in range(nu):
            poly = _polymul(poly, [mp.mpc(1), mp.mpc(1)])
        for z in z_roots:
            poly = _polymul(poly, [mp.mpc(1), -z])
        taps = [mp.re(c) for c in poly]
        total = mp.fsum(taps)
        return tuple(t * mp.sqrt(2) / total for t in taps)


def _polymul(a, b):
    out = [mp.mpc(0)] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for k, bk in enumerate(b):
            out[i + k] += ai * bk
    return out


@functools.lru_cache(maxsize=None)
def wavelet_mp(nu):
    """Tuple of mpf wavelet taps g_c = (-1)^c h_{1-c}, c = -nu+1 .. nu."""
    h = daubechies_mp(nu)
    out = []
    with mp.workdps(DPS):           # cached: never round at the caller's precision
        for c in range(-nu + 1, nu + 1):
            out.append(-h[(1 - c) + nu - 1] if c % 2 else +h[(1 - c) + nu - 1])
    return tuple(out)


def daubechies(nu):
    """float64 array of h_c, c = -nu+1 .. nu."""
    return np.array([float(t) for t in daubechies_mp(nu)])


def wavelet(nu):
    """float64 array of g_c, c = -nu+1 .. nu."""
    return np.array([float(t) for t in wavelet_mp(nu)])
