"""Seeded synthetic inputs shared by the tests, smoke() and bench.py.

This module holds no arithmetic of the method: it only draws coefficient
vectors in the multiscale layout and sampling sets, from
numpy.random.Generator(PCG64(seed)).

Recipes (synthetic stand-ins for image-like data; the paper uses no dataset):
* coefficients: the coarse scaling block ~ N(0, 1); level-k details
  ~ N(0, 2^{-e k}) (variance, e = 1.5 in 1D and 2 in 2D) with exactly
  round(frac * count) of each level (each band in 2D) set to zero, chosen
  uniformly without replacement.
* multilevel Omega (2D): the full low-sequency square [0, core)^2, then dyadic
  annuli A_l = {core 2^(l-1) <= max(n1, n2) < core 2^l} sampled uniformly
  without replacement at density p_l = min(1, c 2^-l); c is water-filled so
  that |Omega| = round(density N^2) exactly.  1D: the same with intervals.
"""
import numpy as np


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _sparsify(rng, block, frac):
    flat = block.reshape(-1)
    k = int(round(frac * flat.size))
    if k:
        flat[rng.choice(flat.size, k, replace=False)] = 0.0
    return block


def coefficients_1d(j, j0, seed, exponent=1.5, zero_frac=0.8):
    """Vector of 2^j coefficients in C_{psi,j} order [a_j0 | d_j0 | ... | d_{j-1}]."""
    rng = rng_for(seed)
    x = np.empty(1 << j)
    x[: 1 << j0] = rng.standard_normal(1 << j0)
    for k in range(j0, j):
        d = rng.standard_normal(1 << k) * 2.0 ** (-exponent * k / 2)
        x[1 << k: 2 << k] = _sparsify(rng, d, zero_frac)
    return x


def coefficients_2d(j, j0, seed, exponent=2.0, zero_frac=0.9):
    """2^j x 2^j array in the quadtree layout (scaling block, then LH, HL, HH per level)."""
    rng = rng_for(seed)
    M = 1 << j
    X = np.empty((M, M))
    X[: 1 << j0, : 1 << j0] = rng.standard_normal((1 << j0, 1 << j0))
    for k in range(j0, j):
        lo, hi = slice(0, 1 << k), slice(1 << k, 2 << k)
        for rs, cs in ((lo, hi), (hi, lo), (hi, hi)):
            band = rng.standard_normal((1 << k, 1 << k)) * 2.0 ** (-exponent * k / 2)
            X[rs, cs] = _sparsify(rng, band, zero_frac)
    return X


def coefficients_nd(shape, seed, zero_frac=0.5):
    """Coefficients of the 3D and unequal-sided operators: standard normal, a share zeroed."""
    rng = rng_for(seed)
    return _sparsify(rng, rng.standard_normal(tuple(shape)), zero_frac)


def _annuli_2d(N, core):
    """Yield index arrays (linear n1 * N + n2) of the core square and the dyadic annuli."""
    n1, n2 = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    r = np.maximum(n1, n2).reshape(-1)
    lin = np.arange(N * N, dtype=np.int64)
    core = min(core, N)
    groups = [lin[r < core]]
    lo = core
    while lo < N:
        groups.append(lin[(r >= lo) & (r < 2 * lo)])
        lo *= 2
    return groups


def _annuli_1d(N, core):
    lin = np.arange(N, dtype=np.int64)
    core = min(core, N)
    groups = [lin[:core]]
    lo = core
    while lo < N:
        groups.append(lin[lo:2 * lo])
        lo *= 2
    return groups


def _water_fill(groups, target, rng):
    sizes = np.array([g.size for g in groups[1:]], dtype=float)
    base = groups[0].size
    if target <= base:
        pick = rng.choice(groups[0], target, replace=False)
        return np.sort(pick)
    levels = np.arange(1, len(groups))

    def count(c):
        return base + np.minimum(1.0, c * 2.0 ** -levels) @ sizes

    lo, hi = 0.0, 2.0 ** (len(groups) + 2)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if count(mid) < target else (lo, mid)
    p = np.minimum(1.0, hi * 2.0 ** -levels)
    take = np.round(p * sizes).astype(np.int64)
    take[-1] += target - base - take.sum()
    take = np.clip(take, 0, sizes.astype(np.int64))
    parts = [groups[0]]
    for g, k in zip(groups[1:], take):
        parts.append(rng.choice(g, int(k), replace=False))
    return np.sort(np.concatenate(parts))


def multilevel_omega_2d(N, density, seed, core=32):
    """Sorted int64 linear indices n1 * N + n2 of a multilevel variable-density subsample."""
    rng = rng_for(seed)
    target = int(round(density * N * N))
    return _water_fill(_annuli_2d(N, core), target, rng).astype(np.int64)


def multilevel_omega_1d(N, density, seed, core=32):
    rng = rng_for(seed)
    target = int(round(density * N))
    return _water_fill(_annuli_1d(N, core), target, rng).astype(np.int64)


def uniform_omega(total, density, seed):
    rng = rng_for(seed)
    k = int(round(density * total))
    return np.sort(rng.choice(total, k, replace=False)).astype(np.int64)


def sample_vector(m, seed):
    return rng_for(seed).standard_normal(m)


# The workloads of the benchmark and the parity tests (sizes from the paper's
# setting: M = 2^j per dimension, N = 2^(j+q)).
WORKLOADS = {
    "1d_db4_j10_q1": dict(dim=1, nu=4, j=10, q=1, j0=3, density=1.0, seed=1000),
    "2d_db4_j9_q1_25pct": dict(dim=2, nu=4, j=9, q=1, j0=3, density=0.25, seed=2000),
    "2d_db8_j11_q2_12.5pct": dict(dim=2, nu=8, j=11, q=2, j0=4, density=0.125, seed=3000),
    "2d_db4_j10_q1_25pct": dict(dim=2, nu=4, j=10, q=1, j0=3, density=0.25, seed=4000),
}


def workload_inputs(name):
    """(x, omega) for a named workload."""
    w = WORKLOADS[name]
    N = 1 << (w["j"] + w["q"])
    if w["dim"] == 1:
        x = coefficients_1d(w["j"], w["j0"], w["seed"])
        omega = None if w["density"] >= 1 else multilevel_omega_1d(N, w["density"], w["seed"] + 1)
    else:
        x = coefficients_2d(w["j"], w["j0"], w["seed"])
        omega = None if w["density"] >= 1 else multilevel_omega_2d(N, w["density"], w["seed"] + 1)
    return x, omega


def batch_specs(seed=5000, count=96):
    """The uneven batch: instance i of three groups of count/3, FP32.

    group 1: 1D, j = 12 + (i mod 5); group 2: 2D, j = 7 + (i mod 3);
    group 3: 2D, j = 10.  Daubechies order nu = (2, 4, 8)[i mod 3],
    q = 1 + floor(i / 3) mod 2, multilevel Omega of density ~ U[0.10, 0.30]
    with its own seed.  Returns a list of dicts (dim, nu, j, q, j0, density,
    seed) and leaves the arrays to `batch_instance`.
    """
    rng = rng_for(seed)
    per = count // 3
    specs = []
    for i in range(count):
        g = i // per
        nu = (2, 4, 8)[i % 3]
        q = 1 + (i // 3) % 2
        j = (12 + i % 5) if g == 0 else (7 + i % 3) if g == 1 else 10
        j0 = max(1, (2 * nu - 1).bit_length())
        specs.append(dict(dim=1 if g == 0 else 2, nu=nu, j=j, q=q, j0=j0,
                          density=float(rng.uniform(0.10, 0.30)), seed=seed + 10 * (i + 1)))
    return specs


def batch_instance(spec):
    """(x, omega) of one batch instance."""
    N = 1 << (spec["j"] + spec["q"])
    if spec["dim"] == 1:
        return (coefficients_1d(spec["j"], spec["j0"], spec["seed"]),
                multilevel_omega_1d(N, spec["density"], spec["seed"] + 1))
    return (coefficients_2d(spec["j"], spec["j0"], spec["seed"]),
            multilevel_omega_2d(N, spec["density"], spec["seed"] + 1))

