"""Boundary (vanishing-moment-preserving) functions on a half-line.

Test infrastructure (see the package header).

Sec. 3.2 replaces the scaling functions and wavelets that cross an end of
[0, 1] by boundary functions phi^left_m, psi^left_m (m = 0..nu-1) with
staggered supports [0, nu+m], and phi^right_m, psi^right_m with supports
[-m-nu, 0]; they are finite combinations of interior functions and keep
orthonormality and the vanishing moments (the construction of Cohen,
Daubechies and Vial).  The paper gives the supports and the staggering but
not the construction, so this module takes the following reading, written
from the mathematics:

* Left edge, scaling functions.  Interior translates phi(. - k), k >= nu,
  are kept.  The edge space is spanned by the polynomial tails
  sum_{k=-nu+1}^{nu-1} p(k) phi(. - k) restricted to [0, inf), deg p < nu;
  with the interior translates it reproduces every polynomial of degree
  < nu on [0, inf).  S_m is the subspace of tails supported in [0, nu+m],
  i.e. with p(m+1) = ... = p(nu-1) = 0 (dimension m+1).  phi^left_m is the
  unit vector of S_m orthogonal to S_{m-1}, with a positive coefficient on
  the translate k = m.
* Right edge, scaling functions: the mirror statement on (-inf, 0] with the
  translates k in [-nu, nu-2], interior k <= -nu-1, phi^right_m supported in
  [-m-nu, 0] and a positive coefficient on the translate k = -m-1.
* Boundary wavelets: psi^left_m is the unit vector of
  Q_m = {f in V_1[0,inf) supported in [0, nu+m], orthogonal to V_0[0,inf)
  and to the interior wavelets psi(. - k), k >= nu} orthogonal to Q_{m-1}.
  Its coefficient on the level-1 translate 2^1/2 phi(2x - nu - 2m) (the
  right-most one that fits) has the sign of the interior wavelet's
  coefficient on its own right-most level-1 translate, g_nu.  Right edge:
  the mirror statement; the coefficient on the level-1 translate -nu-2m-1
  has the sign of g_{-nu+1}.  For Haar this makes every boundary function
  equal to the plain Haar function it replaces.

Every function is a coefficient vector over restricted translates (level 0
for scaling functions, level 1 for wavelets).  Inner products use the exact
half-line Gram matrix G[k, k'] = integral over [0, inf) of phi(x-k) phi(x-k'),
which follows from the two-scale relation
  G[k, k'] = sum_{c, c'} h_c h_{c'} G[2k + c, 2k' + c'],
with G = delta when either translate lies inside [0, inf) and 0 when either
lies inside (-inf, 0].  The right-edge Gram is delta - G.  The linear system
is solved in float64 and refined in mpmath; all further steps run in
mpmath at 60 digits, because the tails of the outermost translates have
norms near 1e-15 and carry coefficients near 1e7.

Parity status: pinned by orthonormality (against point-value quadrature),
support, polynomial reproduction of the resulting interval basis, and the
zero mean of every wavelet; the sign conventions are a reading.
"""
import functools

import mpmath as mp
import numpy as np

from . import filters

DPS = 60


@functools.lru_cache(maxsize=None, typed=True)
def gram_left(nu):
    """Return a function G(k, k') (mpf) of the left half-line Gram matrix."""
    with mp.workdps(DPS):
        h = filters.scaling_mp(nu)
        taps = list(range(-nu + 1, nu + 1))

        def known(a, b):
            if a >= nu - 1 or b >= nu - 1:
                return True, (mp.mpf(1) if a == b else mp.mpf(0))
            if a <= -nu or b <= -nu or abs(a - b) >= 2 * nu - 1:
                return True, mp.mpf(0)
            return False, None

        unknowns = [(a, b) for a in range(-nu + 1, nu - 1) for b in range(-nu + 1, nu - 1)
                    if not known(a, b)[0]]
        pos = {p: i for i, p in enumerate(unknowns)}
        n = len(unknowns)
        rows = []       # per unknown: (dict col -> coef, const) for x_i - sum coef x_j = const
        for (a, b) in unknowns:
            coef, const = {}, mp.mpf(0)
            for ci, c in enumerate(taps):
                for di, d in enumerate(taps):
                    w = h[ci] * h[di]
                    ok, v = known(2 * a + c, 2 * b + d)
                    if ok:
                        const += w * v
                    else:
                        j = pos[(2 * a + c, 2 * b + d)]
                        coef[j] = coef.get(j, mp.mpf(0)) + w
            rows.append((coef, const))
        if n == 0:
            sol = {}
            return lambda a, b: known(a, b)[1]
        A = np.eye(n)
        rhs = np.zeros(n)
        for i, (coef, const) in enumerate(rows):
            for j, w in coef.items():
                A[i, j] -= float(w)
            rhs[i] = float(const)
        x = [mp.mpf(v) for v in np.linalg.solve(A, rhs)]
        for _ in range(6):                       # iterative refinement in mpmath
            res = []
            for i, (coef, const) in enumerate(rows):
                r = const - x[i] + mp.fsum(w * x[j] for j, w in coef.items())
                res.append(r)
            delta = np.linalg.solve(A, np.array([float(r) for r in res]))
            x = [xi + mp.mpf(di) for xi, di in zip(x, delta)]
            if max(abs(r) for r in res) < mp.mpf(10) ** (-DPS + 8):
                break
        sol = {p: x[i] for i, p in enumerate(unknowns)}

    def G(a, b):
        ok, v = known(a, b)
        return v if ok else sol[(a, b)]

    return G


def _inner(u, v, G, side):
    """<f, g> for coefficient dicts {index: coef} over restricted translates."""
    total = mp.mpf(0)
    for a, ua in u.items():
        for b, vb in v.items():
            if side == "left":
                gab = G(a, b)
            else:
                gab = (mp.mpf(1) if a == b else mp.mpf(0)) - G(a, b)
            if gab != 0:
                total += ua * vb * gab
    return total


def _axpy(alpha, x, y):
    out = dict(y)
    for k, v in x.items():
        out[k] = out.get(k, mp.mpf(0)) + alpha * v
    return out


def _scale(alpha, x):
    return {k: alpha * v for k, v in x.items()}


@functools.lru_cache(maxsize=None, typed=True)
def edge_scaling(nu, side):
    """Boundary scaling functions as tuples of {level-0 translate: coef}.

    side 'left':  phi^left_m,  translates k in [-nu+1, nu-1].
    side 'right': phi^right_m, translates k in [-nu, nu-2].
    """
    G = gram_left(nu)
    with mp.workdps(DPS):
        out = []
        for m in range(nu):
            if side == "left":
                ks = range(-nu + 1, nu)
                roots = range(m + 1, nu)
                lead = m
            else:
                ks = range(-nu, nu - 1)
                roots = range(-nu, -m - 1)
                lead = -m - 1
            u = {}
            for k in ks:
                val = mp.mpf(1)
                for i in roots:
                    val *= (k - i)
                if val != 0:
                    u[k] = val
            for _ in range(2):                    # Gram-Schmidt, twice
                for e in out:
                    u = _axpy(-_inner(e, u, G, side), e, u)
            u = _scale(1 / mp.sqrt(_inner(u, u, G, side)), u)
            if u[lead] < 0:
                u = _scale(-1, u)
            out.append(u)
        return tuple(out)


def _level0_to_level1(coef0, nu, side, taps):
    """Rewrite a level-0 combination in level-1 restricted translates."""
    out = {}
    for k, a in coef0.items():
        for ci, c in enumerate(range(-nu + 1, nu + 1)):
            n = 2 * k + c
            if side == "left" and n + nu <= 0:
                continue                           # vanishes on [0, inf)
            if side == "right" and n - nu + 1 >= 0:
                continue                           # vanishes on (-inf, 0]
            out[n] = out.get(n, mp.mpf(0)) + a * taps[ci]
    return out


@functools.lru_cache(maxsize=None, typed=True)
def edge_wavelets(nu, side):
    """Boundary wavelets as tuples of {level-1 translate: coef}.

    The level-1 translates are 2^1/2 phi(2x - n) restricted to the half-line.
    """
    G = gram_left(nu)
    with mp.workdps(DPS):
        h = filters.scaling_mp(nu)
        g = filters.wavelet_mp(nu)
        scal = edge_scaling(nu, side)
        sgn = 1 if side == "left" else -1
        # level-1 edge scaling functions: same coefficients, level-1 translates
        e1 = [dict(f) for f in scal]
        # level-0 functions that may overlap [0, nu + nu] (left) or its mirror
        v0 = [_level0_to_level1(f, nu, side, h) for f in scal]
        interior = range(nu, 4 * nu + 2) if side == "left" else range(-nu - 1, -4 * nu - 3, -1)
        for k in interior:
            v0.append(_level0_to_level1({k: mp.mpf(1)}, nu, side, h))
        psi_int = [_level0_to_level1({k: mp.mpf(1)}, nu, side, g) for k in interior]
        constraints = v0 + psi_int
        out = []
        for m in range(nu):
            if side == "left":
                newest = nu + 2 * m
                fresh = range(nu, nu + 2 * m + 1)
            else:
                newest = -nu - 2 * m - 1
                fresh = range(-nu - 2 * m - 1, -nu)
            cands = e1 + [{n: mp.mpf(1)} for n in fresh]
            K = mp.matrix(len(constraints), len(cands))
            for i, cf in enumerate(constraints):
                for j, cd in enumerate(cands):
                    K[i, j] = _inner(cf, cd, G, side)
            U, S, V = mp.svd_r(K)
            svals = [S[i] for i in range(min(K.rows, K.cols))]
            smax = max(abs(s) for s in svals)
            null_idx = [i for i in range(K.cols)
                        if i >= len(svals) or abs(svals[i]) < smax * mp.mpf(10) ** (-DPS // 2)]
            if len(null_idx) != m + 1:
                raise RuntimeError(f"edge wavelet space Q_{m} has dimension {len(null_idx)}, expected {m + 1}")
            basis = []
            for i in null_idx:
                f = {}
                for j, cd in enumerate(cands):
                    f = _axpy(V[i, j], cd, f)
                basis.append(f)
            best, best_norm = None, mp.mpf(-1)
            for f in basis:
                for _ in range(2):
                    for e in out:
                        f = _axpy(-_inner(e, f, G, side), e, f)
                nrm = mp.sqrt(_inner(f, f, G, side))
                if nrm > best_norm:
                    best, best_norm = f, nrm
            f = _scale(1 / best_norm, best)
            lead = f.get(newest, mp.mpf(0))
            if abs(lead) < mp.mpf(10) ** -20:
                raise RuntimeError("boundary wavelet has no weight on its newest translate")
            ref = g[2 * nu - 1] if side == "left" else g[0]
            if (lead < 0) != (ref < 0):
                f = _scale(-1, f)
            out.append({k: v for k, v in f.items() if v != 0})
        del sgn
        return tuple(out)


def to_float(coef):
    """{index: mpf} -> (sorted int indices, float64 values)."""
    keys = sorted(coef)
    return np.array(keys, dtype=np.int64), np.array([float(coef[k]) for k in keys])
