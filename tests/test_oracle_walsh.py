"""Pins for oracle.walsh: Fig. 3, Lemma 3.2, orthogonality, sign changes."""
import numpy as np
import pytest

from oracle import walsh
from tests.conftest import read_golden


def test_fig3_first_eight_walsh_functions():
    rows = read_golden("fig3_walsh_signs.txt")
    expected = np.array([[1 if ch == "+" else -1 for ch in r] for r in rows])
    got = np.array([[walsh.walsh(n, k, 3) for k in range(8)] for n in range(8)])
    assert (got == expected).all()
    assert (walsh.walsh_matrix(3) == expected).all()


@pytest.mark.parametrize("J", [1, 2, 4, 6, 8])
def test_orthogonal_and_symmetric(J):
    H = walsh.walsh_matrix(J)
    N = 1 << J
    assert np.array_equal(H @ H.T, N * np.eye(N))
    # Lemma 3.2 (2): w_n(2^-J l) = w_l(2^-J n) for n, l < 2^J
    assert np.array_equal(H, H.T)


@pytest.mark.parametrize("J", [3, 5, 7])
def test_sequency_has_n_sign_changes(J):
    H = walsh.walsh_matrix(J)
    changes = (np.diff(H, axis=1) != 0).sum(axis=1)
    assert np.array_equal(changes, np.arange(1 << J))


def test_lemma_3_2_identities():
    rng = np.random.default_rng(0)
    J = 9
    for _ in range(400):
        n = int(rng.integers(0, 1 << 12))
        a, b = (int(v) for v in rng.integers(0, 1 << J, 2))
        # (1) w_n(x xor y) = w_n(x) w_n(y)
        assert walsh.walsh(n, walsh.xor_dyadic(a, b), J) == walsh.walsh(n, a, J) * walsh.walsh(n, b, J)
        # (3) w_n(2^-j x) = w_{floor(n / 2^j)}(x), x = a 2^-J, j = 3: 2^-3 a 2^-J = a 2^-(J+3)
        assert walsh.walsh(n, a, J + 3) == walsh.walsh(n >> 3, a, J)


def test_walsh_matrix_matches_scalar_definition():
    J = 6
    rows = [0, 1, 5, 63, 64, 100, 1000]
    Hm = walsh.walsh_matrix(J, rows=rows)
    for r, n in enumerate(rows):
        assert all(Hm[r, k] == walsh.walsh(n, k, J) for k in range(1 << J))


def test_high_index_rows_reduce_to_low_ones():
    # w_n with n >= 2^J on the 2^J grid: only digit n^(J+1) beyond the grid matters
    J = 5
    H = walsh.walsh_matrix(J, rows=np.arange(1 << (J + 2)))
    base = walsh.walsh_matrix(J)
    for n in range(1 << (J + 2)):
        low = n & ((1 << J) - 1)
        bit = (n >> J) & 1
        ref = base[low ^ ((1 << J) - 1) if bit else low]
        assert np.array_equal(H[n], ref)


def test_bitwise_form_equals_definition():
    rng = np.random.default_rng(4)
    for J in (1, 3, 7, 11):
        rows = rng.integers(0, 1 << (J + 3), 300)
        cols = rng.integers(0, 1 << J, 200)
        assert np.array_equal(walsh.walsh_matrix_bits(J, rows, cols), walsh.walsh_matrix(J, rows, cols))
