"""CPU tests of the C ABI: exports, descriptor validation, and the host planner's
tables against independent derivations from the oracle (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import basis, cascade, filters, halfline, walsh
from oracle import operator as op

abi = pytest.importorskip("paper_2106_00554_amd._abi")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def desc(nu, j, q, dim=1, j0=None, dtype=1, omega=None):
    """Descriptor for nu (an int: Daubechies; a filters.Symlet: symlets)."""
    j0 = (0 if nu == 1 else int(np.ceil(np.log2(2 * nu)))) if j0 is None else j0
    N = 1 << (j + q)
    fam = abi.WH2WAV_SYM if isinstance(nu, filters.Symlet) else abi.WH2WAV_DB
    d = abi.wh2wav_desc(dim=dim, j=j, q=q, j0=j0, nu=int(nu), family=fam, boundary=0, dtype=dtype,
                        m=N ** dim, omega=None, basis2d=0)
    keep = None
    if omega is not None:
        keep = np.ascontiguousarray(np.asarray(omega, dtype=np.int64))
        d.m = keep.size
        d.omega = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    return d, keep


def test_every_declared_symbol_is_exported():
    header = open(os.path.join(ROOT, "include", "wh2wav.h")).read()
    declared = set(re.findall(r"\b(wh2wav_[a-z_]+)\s*\(", header))
    assert declared == set(abi.EXPORTS)
    for name in declared:
        assert hasattr(abi.LIB, name)


@pytest.mark.parametrize("nu", [1, 2, 3, 4, 8, filters.Symlet(2), filters.Symlet(4), filters.Symlet(5),
                                filters.Symlet(6), filters.Symlet(8), filters.Symlet(10)])
def test_filters_match_oracle(nu):
    d, _ = desc(nu, max(4, int(np.ceil(np.log2(2 * nu))) + 1), 1)
    assert np.abs(np.array(abi.wh2wav_host_table(d, "h")) - filters.daubechies(nu)).max() < 2e-16
    assert np.abs(np.array(abi.wh2wav_host_table(d, "g")) - filters.wavelet(nu)).max() < 2e-16


@pytest.mark.parametrize("nu,j,q", [(1, 3, 1), (2, 4, 1), (4, 5, 2), (8, 6, 2), (3, 4, 3), (filters.Symlet(4), 5, 2),
                                    (filters.Symlet(6), 5, 1)])
def test_interior_table_matches_oracle(nu, j, q):
    d, _ = desc(nu, j, q)
    Q = 1 << q
    T = np.array(abi.wh2wav_host_table(d, "T")).reshape(2 * nu - 1, Q)
    Phi = cascade.phi_cells(nu, q)
    ref = np.zeros_like(T)
    for l in range(-nu + 1, nu):
        cells = Phi.take(l * Q + np.arange(Q))
        for s in range(Q):
            ref[l + nu - 1, s] = 2 ** (-j / 2) * sum(walsh.walsh(s, r, q) * cells[r] for r in range(Q))
    assert np.abs(T - ref).max() < 1e-15


@pytest.mark.parametrize("nu,j,q", [(1, 3, 1), (2, 4, 1), (4, 5, 2), (8, 6, 1), (3, 4, 2), (filters.Symlet(4), 5, 2),
                                    (filters.Symlet(5), 5, 1)])
def test_boundary_bands_match_oracle(nu, j, q):
    """Prop. 4.2 (bd): Walsh coefficients at s < 2^q of the boundary functions on each cell."""
    d, _ = desc(nu, j, q)
    Q, band = 1 << q, 2 * nu - 1
    BL = np.array(abi.wh2wav_host_table(d, "band_l")).reshape(band, nu, Q)
    BR = np.array(abi.wh2wav_host_table(d, "band_r")).reshape(band, nu, Q)
    # The oracle forms these boundary cell integrals in extended precision; its
    # own rounding bound (which grows with the cancellation, up to ~1e-13 at
    # nu = 8) sets the tolerance.
    for m in range(nu):
        left, lb = basis.halfline_scaling_cells(nu, "left", m, q, range(band))
        right, rb = basis.halfline_scaling_cells(nu, "right", m, q, range(-band, 0))
        for p in range(band):
            for side, table, cell, cells, err in (("L", BL, p, left[p], lb[p]), ("R", BR, p - band, right[p], rb[p])):
                supported = (cell <= nu + m - 1) if side == "L" else (cell >= -nu - m)
                for s in range(Q):
                    ref = 2 ** (-j / 2) * sum(walsh.walsh(s, r, q) * cells[r] for r in range(Q)) if supported else 0.0
                    tol = 2 ** (-j / 2) * err.sum() + 4e-16 * abs(ref) + 1e-17
                    assert abs(table[p, m, s] - ref) < tol, (side, m, p, s, tol)


@pytest.mark.parametrize("nu", [1, 2, 3, 4, 6, 8, filters.Symlet(4), filters.Symlet(6)])
def test_synthesis_blocks_match_oracle(nu):
    """Boundary blocks of the one-level synthesis matrix V_k + W_k -> V_{k+1}.

    The oracle never forms this matrix; here it is recovered by least squares
    from the oracle's cell integrals of B_{phi,k}, B_{psi,k} and B_{phi,k+1}.
    """
    j0 = 0 if nu == 1 else int(np.ceil(np.log2(2 * nu)))
    k = j0 + 1
    d, _ = desc(nu, k + 1, 1)
    rows, cols = 3 * nu - 1, 2 * nu
    SL = np.array(abi.wh2wav_host_table(d, "syn_l")).reshape(rows, cols)
    SR = np.array(abi.wh2wav_host_table(d, "syn_r")).reshape(rows, cols)
    J = k + 3
    fine = basis.block(nu, k + 1, J, True).toarray()
    coarse = np.hstack([basis.block(nu, k, J, True).toarray(), basis.block(nu, k, J, False).toarray()])
    S, *_ = np.linalg.lstsq(fine, coarse, rcond=None)
    half, size = 1 << k, 2 << k
    assert np.abs(S.T @ S - np.eye(size)).max() < 1e-12
    for c in range(nu):
        for kind in range(2):
            col_l = kind * half + c
            col_r = kind * half + (half - 1 - c)
            assert np.abs(S[:rows, col_l] - SL[:, kind * nu + c]).max() < 1e-13
            assert np.abs(S[rows:, col_l]).max() < 1e-13
            assert np.abs(S[size - rows:, col_r] - SR[:, kind * nu + c]).max() < 1e-13
            assert np.abs(S[:size - rows, col_r]).max() < 1e-13


def test_omega_row_offsets():
    rng = np.random.default_rng(1)
    nu, j, q = 2, 3, 1
    N = 1 << (j + q)
    omega = np.sort(rng.choice(N * N, 57, replace=False))
    d, keep = desc(nu, j, q, dim=2, omega=omega)
    rp = np.array(abi.wh2wav_host_table(d, "row_ptr"))
    ref = np.concatenate([[0], np.cumsum(np.bincount(omega // N, minlength=N))])
    assert np.array_equal(rp, ref)


@pytest.mark.parametrize("js,tensor", [((3, 3, 3), False), ((2, 3, 4), True), ((4, 2), True), ((3, 5), True)])
def test_omega_rows_of_three_dimensions_and_unequal_sides(js, tensor):
    """Rows of the sample bitmask: every axis but the last, row-major; row length N_last."""
    rng = np.random.default_rng(2)
    q = 1
    Ns = [1 << (ja + q) for ja in js]
    total = int(np.prod(Ns))
    omega = np.sort(rng.choice(total, total // 7, replace=False))
    d, keep = desc(2, 3, q, dim=len(js), omega=omega)
    d.basis2d = abi.WH2WAV_TENSOR if tensor else abi.WH2WAV_ISOTROPIC
    for a, ja in enumerate(js):
        d.j_axes[a] = ja
    rp = np.array(abi.wh2wav_host_table(d, "row_ptr"))
    ref = np.concatenate([[0], np.cumsum(np.bincount(omega // Ns[-1], minlength=total // Ns[-1]))])
    assert np.array_equal(rp, ref)


@pytest.mark.parametrize("dim,js,basis,code", [
    (2, (3, 4), 0, "EINVAL"),      # unequal sides need the tensor basis
    (3, (3, 3, 5), 0, "EINVAL"),
    (2, (3, 4, 3), 1, "EINVAL"),   # an entry beyond dim
    (1, (4, 0, 0), 0, "EINVAL"),   # no per-axis sizes in 1D
    (2, (1, 4), 1, "EINVAL"),      # below j0
    (3, (10, 10, 10), 1, "EUNSUPPORTED"),  # N_1 N_2 N_3 beyond 2^32
    (2, (15, 3), 1, "EUNSUPPORTED"),       # N_a beyond 2^15
])
def test_axis_validation(dim, js, basis, code):
    d, _ = desc(2, 3, 1, dim=dim)
    d.m = 0
    d.omega = ctypes.cast(ctypes.pointer(ctypes.c_int64(0)), ctypes.POINTER(ctypes.c_int64))
    d.basis2d = basis
    for a, ja in enumerate(js):
        d.j_axes[a] = ja
    with pytest.raises(abi.Wh2WavError) as e:
        abi.wh2wav_host_table(d, "h")
    assert e.value.code == getattr(abi, "WH2WAV_" + code)


@pytest.mark.parametrize("field,value", [("dim", 4), ("dim", 0), ("nu", 0), ("nu", 11), ("q", 0), ("j0", 1), ("j", 1),
                                         ("dtype", 5), ("family", 2), ("boundary", 2), ("boundary", -1), ("m", 5),
                                         ("basis2d", 2)])
def test_descriptor_validation(field, value):
    d, _ = desc(2, 4, 1)
    setattr(d, field, value)
    with pytest.raises(abi.Wh2WavError) as e:
        abi.wh2wav_host_table(d, "h")
    assert e.value.code in (abi.WH2WAV_EINVAL, abi.WH2WAV_EUNSUPPORTED)
    assert abi.wh2wav_last_error()


@pytest.mark.parametrize("omega", [[3, 2], [0, 0], [-1, 4], [0, 1 << 20]])
def test_omega_validation(omega):
    d, keep = desc(2, 4, 1, dim=1, omega=omega)
    with pytest.raises(abi.Wh2WavError) as e:
        abi.wh2wav_host_table(d, "row_ptr")
    assert e.value.code == abi.WH2WAV_EINVAL


def test_handles_that_were_never_created_are_rejected():
    """A pointer that no plan call returned is refused before it is dereferenced."""
    bogus = ctypes.c_void_p(0x1000)
    buf = ctypes.c_void_p(0x2000)
    for call in (lambda: abi.wh2wav_forward(bogus, buf, ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), None),
                 lambda: abi.wh2wav_adjoint(bogus, buf, ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), None),
                 lambda: abi.wh2wav_workspace_size(bogus),
                 lambda: abi.wh2wav_stage_count(bogus, 0),
                 lambda: abi.wh2wav_destroy(bogus),
                 lambda: abi.wh2wav_batch_workspace_size(bogus),
                 lambda: abi.wh2wav_batch_schedule(bogus),
                 lambda: abi.wh2wav_destroy_batch(bogus)):
        with pytest.raises(abi.Wh2WavError) as e:
            call()
        assert e.value.code == abi.WH2WAV_EINVAL
        assert "live" in abi.wh2wav_last_error()
    # NULL handles are a no-op for the destroy calls
    assert abi.LIB.wh2wav_destroy(None) == abi.WH2WAV_OK
    assert abi.LIB.wh2wav_destroy_batch(None) == abi.WH2WAV_OK


def test_sizes_beyond_the_supported_range_are_rejected():
    for dim, j, q in ((2, 14, 2), (1, 26, 3)):
        d, _ = desc(2, j, q, dim=dim)
        with pytest.raises(abi.Wh2WavError) as e:
            abi.wh2wav_host_table(d, "h")
        assert e.value.code == abi.WH2WAV_EUNSUPPORTED


def test_null_arguments_are_rejected():
    assert abi.LIB.wh2wav_plan(None, None) == abi.WH2WAV_EINVAL
    handle = ctypes.c_void_p()
    assert abi.LIB.wh2wav_plan(None, ctypes.byref(handle)) == abi.WH2WAV_EINVAL
    assert handle.value is None
    d, _ = desc(2, 4, 1)
    assert abi.LIB.wh2wav_host_table(ctypes.byref(d), 0, None, 0, None) == abi.WH2WAV_EINVAL
    assert abi.LIB.wh2wav_plan_batch(None, 0, ctypes.byref(handle)) == abi.WH2WAV_EINVAL
