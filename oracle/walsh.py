"""Sequency-ordered Walsh functions, written digit by digit from Def. 3.1.

Test infrastructure (see the package header).

For n >= 0 write n = sum_i n^(i) 2^(i-1) (digits least significant first)
and for x in [0, 1) write x = sum_i x^(i) 2^-i (digits most significant
first, never ending in repeated ones).  Def. 3.1 sets

    w_n(x) = (-1)^( sum_i (n^(i) + n^(i+1)) x^(i) ).

Only dyadic rationals x = k / 2^J are needed here; their expansion stops
after digit J, so the sum has J terms and uses digits n^(1..J+1).

Pins: Fig. 3 (eight functions drawn as sign patterns), orthogonality of the
matrix, "w_n has n sign changes" (Sec. 3.1), the three identities of
Lemma 3.2, and the Haar special case (Remark on Haar reconstruction).
"""
import numpy as np


def walsh(n, k, J):
    """w_n(k / 2^J) for integers n >= 0 and 0 <= k < 2^J, by Def. 3.1."""
    if not 0 <= k < (1 << J):
        raise ValueError("k must lie in [0, 2^J)")
    exponent = 0
    for i in range(1, J + 1):
        x_i = (k >> (J - i)) & 1          # i-th binary digit of k / 2^J
        n_i = (n >> (i - 1)) & 1          # digit n^(i)
        n_i1 = (n >> i) & 1               # digit n^(i+1)
        exponent += (n_i + n_i1) * x_i
    return -1 if exponent % 2 else 1


def walsh_matrix(J, rows=None, cols=None):
    """Matrix [w_n(k / 2^J)] for n in `rows`, k in `cols` (default: all < 2^J).

    The same digit sum as `walsh`, evaluated with numpy over the grid of
    (n, k) pairs.  Entries are +1 / -1 as float64.
    """
    size = 1 << J
    n = np.arange(size, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    k = np.arange(size, dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    exponent = np.zeros((n.size, k.size), dtype=np.int64)
    for i in range(1, J + 1):
        x_i = (k >> (J - i)) & 1
        n_pair = ((n >> (i - 1)) & 1) + ((n >> i) & 1)
        exponent += np.outer(n_pair, x_i)
    return np.where(exponent % 2 == 1, -1.0, 1.0)


def xor_dyadic(k1, k2):
    """x ⊕ y for x = k1 / 2^J, y = k2 / 2^J: digitwise XOR (Sec. 3.1)."""
    return k1 ^ k2


def walsh_matrix_bits(J, rows, cols):
    """Same matrix as `walsh_matrix`, via the parity of gray(n) AND bitrev_J(k).

    Def. 3.1 pairs digit n^(i) + n^(i+1) (bit i-1 of gray(n) = n xor (n >> 1))
    with the i-th binary digit of k / 2^J (bit J-i of k, i.e. bit i-1 of the
    J-bit reversal of k); the exponent is the number of common set bits.  Used
    for large sampled columns; pinned equal to `walsh_matrix` by the tests.
    """
    n = np.asarray(rows, dtype=np.int64)
    k = np.asarray(cols, dtype=np.int64)
    # digits beyond J do not enter (x has J digits); gray bit J-1 uses n^(J+1)
    gray = (n ^ (n >> 1)) & ((1 << J) - 1)
    rev = np.zeros_like(k)
    for b in range(J):
        rev |= ((k >> b) & 1) << (J - 1 - b)
    parity = np.bitwise_count(np.bitwise_and.outer(gray, rev)) & 1
    return np.where(parity == 1, -1.0, 1.0)
