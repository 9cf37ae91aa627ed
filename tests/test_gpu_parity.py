"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: relative l2 error <= 1e-12 in FP64 and <= 1e-5 in FP32; FP32 errors
are also reported against the FP64 GPU result.  Sizes span several tiles and every boundary
regime: j = J0 (no interior functions), Haar, empty and ragged Omega rows.
"""
import numpy as np
import pytest

from oracle import operator as op
from oracle.filters import Symlet
from tests import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu_pair(dim, nu, j, q, j0, dtype, x, omega, y_in, boundary="bd", basis2d="isotropic"):
    """Forward of x and adjoint of y_in through the C ABI; nu an int (Daubechies) or a Symlet."""
    from oracle.filters import family
    from paper_2106_00554_amd.operator import Wh2Wav
    print(f"[gpu] dim={dim} nu={nu!r} j={j} q={q} j0={j0} {boundary} {basis2d} {dtype} "
          f"m={'all' if omega is None else len(omega)}", flush=True)
    opr = Wh2Wav(dim, j, q, int(nu), j0, dtype, omega, family=family(nu), boundary=boundary, basis2d=basis2d)
    xt = torch.tensor(x, dtype=dtype, device="cuda")
    y = opr.forward(xt)
    yt = torch.tensor(y_in, dtype=dtype, device="cuda")
    xa = opr.adjoint(yt)
    torch.cuda.synchronize()
    return y.cpu().numpy(), xa.cpu().numpy()


CASES_1D = [
    # nu, j, q, j0, omega density (None = all)
    (1, 4, 1, 0, None), (1, 6, 3, 2, 0.4),
    (2, 2, 1, 2, None), (2, 5, 2, 2, 0.3), (2, 7, 1, 3, 0.5),
    (3, 3, 1, 3, None), (3, 6, 2, 3, 0.25),
    (4, 3, 2, 3, 0.6), (4, 10, 1, 3, None), (4, 8, 3, 3, 0.2),
    (6, 4, 1, 4, None), (8, 4, 2, 4, 0.5), (8, 7, 2, 4, None),
    # lines of 128 .. 2048 values: one workgroup per transform (wave line kernels)
    (3, 9, 2, 3, 0.3), (6, 10, 1, 4, 0.2), (8, 11, 1, 4, 0.15), (2, 11, 2, 2, None), (4, 9, 3, 3, 0.1),
    (4, 8, 4, 3, 0.3),  # q = 4: sixteen phase waves per workgroup
    (10, 7, 1, 5, 0.4),  # the longest filters
    (5, 8, 1, 4, 0.3), (7, 9, 1, 4, None), (9, 6, 2, 5, 0.5),  # the remaining orders
    (9, 9, 1, 5, 0.3), (10, 10, 2, 5, None),  # nu = 9, 10 on the wave line kernels
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nu,j,q,j0,dens", CASES_1D)
def test_parity_1d(nu, j, q, j0, dens, dtype):
    cfg = op.Config(nu, j, q, j0)
    seed = 100 * nu + 10 * j + q
    x = inputs.coefficients_1d(j, j0, seed)
    omega = None if dens is None else inputs.uniform_omega(cfg.N, dens, seed + 1)
    m = cfg.N if omega is None else omega.size
    yv = inputs.sample_vector(m, seed + 2)
    A = op.matrix_1d(cfg)
    y_ref = op.forward_1d(A, x, omega)
    x_ref = op.adjoint_1d(A, yv, omega)
    y, xa = gpu_pair(1, nu, j, q, j0, dtype, x, omega, yv)
    assert rel(y, y_ref) < TOL[dtype], rel(y, y_ref)
    assert rel(xa, x_ref) < TOL[dtype], rel(xa, x_ref)


CASES_2D = [
    (1, 3, 1, 0, None), (1, 4, 2, 1, 0.3),
    (2, 2, 1, 2, None), (2, 4, 1, 2, 0.25), (2, 5, 2, 2, 0.1),
    (3, 3, 2, 3, 0.5), (4, 3, 1, 3, None), (4, 5, 1, 3, 0.25),
    (6, 5, 1, 4, 0.3), (8, 4, 2, 4, 0.2), (8, 6, 1, 4, 0.125),
    (2, 5, 1, 5, 0.3),  # no wavelet level (j0 = j) at M = 32
    # nu > 8: analysis tiles on the small levels must be at least nu wide
    (9, 7, 1, 5, 0.3), (10, 6, 1, 5, None),
    (5, 6, 1, 4, 0.3), (7, 6, 2, 4, None),  # the remaining orders
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nu,j,q,j0,dens", CASES_2D)
def test_parity_2d(nu, j, q, j0, dens, dtype):
    cfg = op.Config(nu, j, q, j0)
    seed = 1000 + 100 * nu + 10 * j + q
    X = inputs.coefficients_2d(j, j0, seed)
    omega = None if dens is None else inputs.multilevel_omega_2d(cfg.N, dens, seed + 1, core=4)
    m = cfg.N ** 2 if omega is None else omega.size
    yv = inputs.sample_vector(m, seed + 2)
    blocks = op.Blocks2D(cfg)
    y_ref = op.forward_2d_full(blocks, X, omega).reshape(-1)
    x_ref = op.adjoint_2d_full(blocks, yv, omega)
    y, xa = gpu_pair(2, nu, j, q, j0, dtype, X, omega, yv)
    assert rel(y, y_ref) < TOL[dtype], rel(y, y_ref)
    assert rel(xa, x_ref) < TOL[dtype], rel(xa, x_ref)


def test_parity_dense_kronecker_tiny():
    """Brute force: the full N^2 x M^2 matrix by Kronecker products."""
    cfg = op.Config(2, 3, 1, 2)
    A2 = op.dense_2d(cfg)
    X = inputs.coefficients_2d(3, 2, 5)
    omega = inputs.uniform_omega(cfg.N ** 2, 0.4, 6)
    yv = inputs.sample_vector(omega.size, 7)
    y, xa = gpu_pair(2, 2, 3, 1, 2, torch.float64, X, omega, yv)
    assert rel(y, A2[omega] @ X.reshape(-1)) < 1e-12
    assert rel(xa.reshape(-1), A2[omega].T @ yv) < 1e-12


def test_1d_workload_db4_j10_q1():
    """1D plain path: db4, M = 2^10, q = 1, all N = 2^11 samples, FP64 (and FP32 vs FP64)."""
    w = inputs.WORKLOADS["1d_db4_j10_q1"]
    x, omega = inputs.workload_inputs("1d_db4_j10_q1")
    cfg = op.Config(w["nu"], w["j"], w["q"], w["j0"])
    A = op.matrix_1d(cfg)
    yv = inputs.sample_vector(cfg.N, 11)
    y64, x64 = gpu_pair(1, w["nu"], w["j"], w["q"], w["j0"], torch.float64, x, omega, yv)
    assert rel(y64, A @ x) < 1e-12
    assert rel(x64, A.T @ yv) < 1e-12
    y32, x32 = gpu_pair(1, w["nu"], w["j"], w["q"], w["j0"], torch.float32, x, omega, yv)
    assert rel(y32, A @ x) < 1e-5 and rel(y32, y64) < 1e-5
    assert rel(x32, A.T @ yv) < 1e-5 and rel(x32, x64) < 1e-5


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_workload_db4_j9_q1(dtype):
    """2D plain path: db4, M = 512^2, N = 1024^2, 25 % multilevel Omega, full oracle product."""
    name = "2d_db4_j9_q1_25pct"
    w = inputs.WORKLOADS[name]
    X, omega = inputs.workload_inputs(name)
    cfg = op.Config(w["nu"], w["j"], w["q"], w["j0"])
    blocks = op.Blocks2D(cfg)
    yv = inputs.sample_vector(omega.size, 21)
    y_ref = op.forward_2d_full(blocks, X, omega)
    x_ref = op.adjoint_2d_full(blocks, yv, omega)
    y, xa = gpu_pair(2, w["nu"], w["j"], w["q"], w["j0"], dtype, X, omega, yv)
    assert rel(y, y_ref) < TOL[dtype], rel(y, y_ref)
    assert rel(xa, x_ref) < TOL[dtype], rel(xa, x_ref)


def _boundary_heavy_positions(cfg, rng, count):
    M, nu = cfg.M, cfg.nu
    pos = [(0, 0), (0, M - 1), (M - 1, 0), (M - 1, M - 1), (1, 2), (M // 2 - 1, M // 2),
           (M // 2 + 3, M - 2), (nu, M // 2 + nu), (M - nu, M - nu - 1)]
    while len(pos) < count:
        pos.append(tuple(int(v) for v in rng.integers(0, M, 2)))
    return pos


@pytest.mark.timeout(900)
def test_2d_workload_db8_j11_q2():
    """2D large: db8, M = 2048^2, N = 8192^2, 12.5 % multilevel Omega.

    Run at full size in the configuration the benchmark times, in FP64 and
    FP32, and compared element by element with the separable oracle: all
    8,388,608 forward outputs and all 4,194,304 adjoint coefficients.  The
    FP32 errors are also stated against the FP64 GPU result.
    """
    name = "2d_db8_j11_q2_12.5pct"
    w = inputs.WORKLOADS[name]
    X, omega = inputs.workload_inputs(name)
    cfg = op.Config(w["nu"], w["j"], w["q"], w["j0"])
    yv = inputs.sample_vector(omega.size, 31)
    blocks = op.Blocks2D(cfg)
    y_ref = op.forward_2d_full(blocks, X, omega)
    x_ref = op.adjoint_2d_full(blocks, yv, omega)
    del blocks
    y64, x64 = gpu_pair(2, w["nu"], w["j"], w["q"], w["j0"], torch.float64, X, omega, yv)
    y32, x32 = gpu_pair(2, w["nu"], w["j"], w["q"], w["j0"], torch.float32, X, omega, yv)
    errs = {"fwd_f64_vs_oracle": rel(y64, y_ref), "adj_f64_vs_oracle": rel(x64, x_ref),
            "fwd_f32_vs_oracle": rel(y32, y_ref), "adj_f32_vs_oracle": rel(x32, x_ref),
            "fwd_f32_vs_f64": rel(y32, y64), "adj_f32_vs_f64": rel(x32, x64)}
    print("[2048^2 db8 q=2 relative l2 errors] " + ", ".join(f"{k} {v:.3e}" for k, v in errs.items()), flush=True)
    assert errs["fwd_f64_vs_oracle"] < 1e-12 and errs["adj_f64_vs_oracle"] < 1e-12
    assert errs["fwd_f32_vs_oracle"] < 1e-5 and errs["adj_f32_vs_oracle"] < 1e-5
    assert errs["fwd_f32_vs_f64"] < 1e-5 and errs["adj_f32_vs_f64"] < 1e-5
    print(f"[2048^2 db8 q=2 max abs deviation / max abs value] fwd f32 "
          f"{np.abs(y32 - y_ref).max() / np.abs(y_ref).max():.3e}, adj f32 "
          f"{np.abs(x32 - x_ref).max() / np.abs(x_ref).max():.3e}", flush=True)


@pytest.mark.timeout(900)
def test_2d_periodic_db8_j11_q2():
    """The periodic extension (Sec. 3.2) at the benchmark's full size: db8,
    M = 2048^2, N = 8192^2, 12.5 % multilevel Omega.  Its wavelet levels take
    the same tiled kernels as the boundary-corrected basis with indices
    modulo each level's size, including the 64^2 synthesis and 32^2 analysis
    tiles that only this size reaches.  Every output and every coefficient
    against the separable oracle, FP64 and FP32.
    """
    name = "2d_db8_j11_q2_12.5pct"
    w = inputs.WORKLOADS[name]
    X, omega = inputs.workload_inputs(name)
    cfg = op.Config(w["nu"], w["j"], w["q"], w["j0"], per=True)
    yv = inputs.sample_vector(omega.size, 37)
    blocks = op.Blocks2D(cfg)
    y_ref = op.forward_2d_full(blocks, X, omega)
    x_ref = op.adjoint_2d_full(blocks, yv, omega)
    del blocks
    args = (2, w["nu"], w["j"], w["q"], w["j0"])
    y64, x64 = gpu_pair(*args, torch.float64, X, omega, yv, boundary="per")
    y32, x32 = gpu_pair(*args, torch.float32, X, omega, yv, boundary="per")
    errs = {"fwd_f64": rel(y64, y_ref), "adj_f64": rel(x64, x_ref),
            "fwd_f32": rel(y32, y_ref), "adj_f32": rel(x32, x_ref)}
    print("[2048^2 db8 q=2 periodic relative l2 errors] " + ", ".join(f"{k} {v:.3e}" for k, v in errs.items()),
          flush=True)
    assert errs["fwd_f64"] < 1e-12 and errs["adj_f64"] < 1e-12
    assert errs["fwd_f32"] < 1e-5 and errs["adj_f32"] < 1e-5


@pytest.mark.timeout(900)
def test_2d_tensor_db8_j11_q2():
    """The tensor-product basis at the benchmark's full size: db8, M = 2048^2,
    N = 8192^2, 12.5 % multilevel Omega.  Its wavelet stage runs every level
    of a 2048-value line in one workgroup, rows, transpose, rows.  Every
    output and every coefficient against the oracle's A1 X A1^T (the dense
    1D section applied along both axes), FP64 and FP32.
    """
    name = "2d_db8_j11_q2_12.5pct"
    w = inputs.WORKLOADS[name]
    X, omega = inputs.workload_inputs(name)
    cfg = op.Config(w["nu"], w["j"], w["q"], w["j0"], tensor=True)
    yv = inputs.sample_vector(omega.size, 41)
    A1 = op.matrix_1d(cfg)
    y_ref = op.forward_2d_tensor(A1, X, omega)
    x_ref = op.adjoint_2d_tensor(A1, yv, omega)
    del A1
    args = (2, w["nu"], w["j"], w["q"], w["j0"])
    y64, x64 = gpu_pair(*args, torch.float64, X, omega, yv, basis2d="tensor")
    y32, x32 = gpu_pair(*args, torch.float32, X, omega, yv, basis2d="tensor")
    errs = {"fwd_f64": rel(y64, y_ref), "adj_f64": rel(x64, x_ref),
            "fwd_f32": rel(y32, y_ref), "adj_f32": rel(x32, x_ref)}
    print("[2048^2 db8 q=2 tensor relative l2 errors] " + ", ".join(f"{k} {v:.3e}" for k, v in errs.items()),
          flush=True)
    assert errs["fwd_f64"] < 1e-12 and errs["adj_f64"] < 1e-12
    assert errs["fwd_f32"] < 1e-5 and errs["adj_f32"] < 1e-5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_2d_j12_sampled(dtype):
    """2D beyond the wave kernels: db4, M = 4096^2, q = 1, 10 % Omega.

    Generic line kernels; the 2048^2 wavelet level runs untransposed through
    the direct (two-pass) synthesis and analysis tiles with 64^2 / 32^2 tiles,
    which no smaller size reaches.  Sampled forward and adjoint entries from
    the oracle, and the adjoint identity at full size.
    """
    cfg = op.Config(4, 12, 1, 3)
    X = inputs.coefficients_2d(12, 3, 1234)
    omega = inputs.multilevel_omega_2d(cfg.N, 0.1, 1235)
    yv = inputs.sample_vector(omega.size, 1236)
    y, xa = gpu_pair(2, 4, 12, 1, 3, dtype, X, omega, yv)
    rng = np.random.default_rng(7)
    N = cfg.N
    edge = np.flatnonzero((omega // N < 4) | (omega // N >= N - 4) | (omega % N < 4) | (omega % N >= N - 4))
    pick = np.concatenate([rng.choice(omega.size, 48, replace=False), rng.choice(edge, min(16, edge.size), replace=False)])
    ref = op.forward_entries_2d(cfg, X, omega[pick] // N, omega[pick] % N)
    assert rel(y[pick], ref) < TOL[dtype], rel(y[pick], ref)
    pos = _boundary_heavy_positions(cfg, rng, 6)
    xref = op.adjoint_entries_2d(cfg, yv, omega, pos)
    got = np.array([xa[c1, c2] for c1, c2 in pos])
    assert rel(got, xref) < TOL[dtype], rel(got, xref)
    lhs, rhs = np.dot(y.astype(np.float64), yv), np.sum(X * xa.astype(np.float64))
    assert abs(lhs - rhs) / (np.linalg.norm(y) * np.linalg.norm(yv)) < TOL[dtype]


def test_empty_omega():
    from paper_2106_00554_amd.operator import Wh2Wav
    for dim in (1, 2):
        opr = Wh2Wav(dim, 4, 1, 2, 2, torch.float64, omega=np.zeros(0, dtype=np.int64))
        x = torch.randn(opr.x_shape, dtype=torch.float64, device="cuda")
        y = opr.forward(x)
        assert y.numel() == 0
        xa = opr.adjoint(torch.zeros(0, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert torch.count_nonzero(xa).item() == 0


def test_ragged_rows_and_determinism():
    """Omega with whole empty rows and a single full row; bitwise-repeatable output."""
    nu, j, q, j0 = 4, 5, 1, 3
    cfg = op.Config(nu, j, q, j0)
    N = cfg.N
    rows = [0, 1, 5, N - 1]
    omega = np.sort(np.concatenate([np.arange(r * N, r * N + N, 3 if r else 1) for r in rows])).astype(np.int64)
    X = inputs.coefficients_2d(j, j0, 77)
    yv = inputs.sample_vector(omega.size, 78)
    blocks = op.Blocks2D(cfg)
    y1, x1 = gpu_pair(2, nu, j, q, j0, torch.float64, X, omega, yv)
    y2, x2 = gpu_pair(2, nu, j, q, j0, torch.float64, X, omega, yv)
    assert np.array_equal(y1, y2) and np.array_equal(x1, x2)
    assert rel(y1, op.forward_2d_full(blocks, X, omega)) < 1e-12
    assert rel(x1, op.adjoint_2d_full(blocks, yv, omega)) < 1e-12


def test_call_errors_are_reported():
    from paper_2106_00554_amd import _abi
    from paper_2106_00554_amd.operator import Wh2Wav
    opr = Wh2Wav(1, 4, 1, 2, 2, torch.float64)
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(_abi.Wh2WavError):
        _abi.wh2wav_forward(opr._plan, x.data_ptr(), x.data_ptr(), opr.workspace.data_ptr(), None)
    with pytest.raises(_abi.Wh2WavError):
        _abi.wh2wav_forward(opr._plan, x.data_ptr(), None, opr.workspace.data_ptr(), None)
    with pytest.raises(ValueError):
        opr.forward(torch.zeros(16, dtype=torch.float32, device="cuda"))


# Sizes and orders served by the wave-level kernels (M = 2^7 .. 2^11).  On the
# short lines (M = 128, 256 and db6/db8 at 512) the boundary values and the
# table-product halo span several lanes.
CASES_2D_WAVE = [
    (2, 9, 1, 2, 0.25), (3, 9, 2, 3, None), (4, 9, 3, 3, 0.125),
    (4, 10, 1, 3, None), (6, 10, 1, 4, 0.3), (8, 10, 1, 4, 0.2), (2, 10, 2, 2, 0.15),
    (2, 7, 1, 2, 0.3), (8, 7, 1, 4, None), (6, 7, 2, 4, 0.25), (4, 7, 3, 3, 0.3),
    (4, 7, 1, 7, 0.3),  # j0 = j: no wavelet level
    (3, 8, 1, 3, 0.2), (8, 8, 2, 4, 0.15), (6, 9, 1, 4, 0.2), (8, 9, 1, 4, None),
    (3, 7, 4, 3, 0.2),  # q = 4: sixteen phase waves per row workgroup
    (5, 8, 1, 4, 0.2), (7, 9, 2, 4, None), (5, 10, 1, 4, 0.25), (7, 7, 1, 4, 0.3),  # odd orders 5 and 7
    (4, 11, 1, 3, 0.1), (2, 11, 1, 2, None),  # 2048-value lines: two phase groups in the adjoint column pass (FP32)
    (9, 8, 1, 5, 0.2), (10, 10, 1, 5, None), (10, 7, 2, 5, 0.3), (9, 10, 2, 5, 0.25),  # nu = 9, 10 up to M = 1024
    (10, 9, 1, 5, 0.2), (9, 9, 3, 5, None),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nu,j,q,j0,dens", CASES_2D_WAVE)
def test_parity_2d_wave_kernels(nu, j, q, j0, dens, dtype):
    cfg = op.Config(nu, j, q, j0)
    seed = 5000 + 100 * nu + 10 * j + q
    X = inputs.coefficients_2d(j, j0, seed)
    omega = None if dens is None else inputs.multilevel_omega_2d(cfg.N, dens, seed + 1)
    m = cfg.N ** 2 if omega is None else omega.size
    yv = inputs.sample_vector(m, seed + 2)
    blocks = op.Blocks2D(cfg)
    y_ref = op.forward_2d_full(blocks, X, omega).reshape(-1)
    x_ref = op.adjoint_2d_full(blocks, yv, omega)
    y, xa = gpu_pair(2, nu, j, q, j0, dtype, X, omega, yv)
    assert rel(y, y_ref) < TOL[dtype], rel(y, y_ref)
    assert rel(xa, x_ref) < TOL[dtype], rel(xa, x_ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nu,j,q,j0", [(2, 9, 1, 7), (4, 9, 1, 8), (3, 10, 1, 6)])
def test_parity_2d_large_coarse_level(nu, j, q, j0, dtype):
    """Coarse level J0 at or above the LDS-resident limit of the 2D wavelet kernels."""
    cfg = op.Config(nu, j, q, j0)
    X = inputs.coefficients_2d(j, j0, 600 + j0)
    omega = inputs.multilevel_omega_2d(cfg.N, 0.2, 601)
    yv = inputs.sample_vector(omega.size, 602)
    blocks = op.Blocks2D(cfg)
    y, xa = gpu_pair(2, nu, j, q, j0, dtype, X, omega, yv)
    assert rel(y, op.forward_2d_full(blocks, X, omega)) < TOL[dtype]
    assert rel(xa, op.adjoint_2d_full(blocks, yv, omega)) < TOL[dtype]


def test_destroyed_plans_are_rejected():
    """Use after destroy and a second destroy fail with EINVAL instead of touching freed memory."""
    from paper_2106_00554_amd import _abi
    d = _abi.wh2wav_desc(dim=2, j=5, q=1, j0=3, nu=4, family=0, boundary=0, dtype=1, m=64 * 64, omega=None)
    plan = _abi.wh2wav_plan(d)
    nbytes = _abi.wh2wav_workspace_size(plan)
    x = torch.randn(32 * 32, dtype=torch.float64, device="cuda")
    y = torch.empty(64 * 64, dtype=torch.float64, device="cuda")
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.float64, device="cuda")
    _abi.wh2wav_forward(plan, x.data_ptr(), y.data_ptr(), ws.data_ptr(), None)
    torch.cuda.synchronize()
    _abi.wh2wav_destroy(plan)
    for call in (lambda: _abi.wh2wav_forward(plan, x.data_ptr(), y.data_ptr(), ws.data_ptr(), None),
                 lambda: _abi.wh2wav_workspace_size(plan), lambda: _abi.wh2wav_destroy(plan)):
        with pytest.raises(_abi.Wh2WavError) as e:
            call()
        assert e.value.code == _abi.WH2WAV_EINVAL


CASES_SYMLETS = [
    # dim, symlet order, j, q, j0, omega density: generic and wave kernels, 1D and 2D
    (1, 4, 8, 1, 3, None), (1, 6, 11, 2, 4, 0.2), (1, 5, 6, 2, 4, 0.5),
    (2, 4, 6, 1, 3, 0.3), (2, 5, 7, 2, 4, None), (2, 8, 9, 1, 4, 0.2), (2, 6, 10, 1, 4, 0.25),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,nu,j,q,j0,dens", CASES_SYMLETS)
def test_parity_symlets(dim, nu, j, q, j0, dens, dtype):
    """Symlets (least-asymmetric filters, Sec. 3.2 / Table 1) through every kernel family."""
    sym = Symlet(nu)
    cfg = op.Config(sym, j, q, j0)
    seed = 7000 + 100 * nu + 10 * j + q + dim
    if dim == 1:
        x = inputs.coefficients_1d(j, j0, seed)
        omega = None if dens is None else inputs.uniform_omega(cfg.N, dens, seed + 1)
        m = cfg.N if omega is None else omega.size
        yv = inputs.sample_vector(m, seed + 2)
        A = op.matrix_1d(cfg)
        y_ref, x_ref = op.forward_1d(A, x, omega), op.adjoint_1d(A, yv, omega)
    else:
        x = inputs.coefficients_2d(j, j0, seed)
        omega = None if dens is None else inputs.multilevel_omega_2d(cfg.N, dens, seed + 1)
        m = cfg.N ** 2 if omega is None else omega.size
        yv = inputs.sample_vector(m, seed + 2)
        blocks = op.Blocks2D(cfg)
        y_ref = op.forward_2d_full(blocks, x, omega).reshape(-1)
        x_ref = op.adjoint_2d_full(blocks, yv, omega)
    y, xa = gpu_pair(dim, sym, j, q, j0, dtype, x, omega, yv)
    assert rel(y, y_ref) < TOL[dtype], rel(y, y_ref)
    assert rel(xa, x_ref) < TOL[dtype], rel(xa, x_ref)


CASES_PERIODIC = [
    # dim, nu (int: Daubechies, negative: symlet of that order), j, q, j0, omega density
    (1, 1, 4, 1, 0, None), (1, 2, 5, 1, 2, 0.4), (1, 4, 8, 2, 3, None), (1, 8, 10, 1, 4, 0.3), (1, 3, 12, 1, 3, 0.2),
    (1, -4, 7, 2, 3, 0.5),
    (2, 2, 4, 1, 2, None), (2, 4, 5, 2, 3, 0.3), (2, 3, 6, 1, 3, 0.25),   # generic line kernels
    (2, 4, 7, 1, 3, 0.3), (2, 8, 9, 2, 4, 0.15), (2, 6, 10, 1, 4, None),  # wave line kernels
    (2, 2, 8, 3, 2, 0.2), (2, -6, 8, 1, 4, 0.25), (2, 8, 4, 1, 4, 0.5),   # j0 = j
    (2, 1, 5, 1, 0, 0.3), (2, 1, 9, 1, 0, None),  # Haar from J0 = 0: one-value blocks in the coarse kernel
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,nu,j,q,j0,dens", CASES_PERIODIC)
def test_parity_periodic(dim, nu, j, q, j0, dens, dtype):
    """Periodic extension (Sec. 3.2, Prop. 4.2 "per") through the generic and wave kernels."""
    nu = Symlet(-nu) if nu < 0 else nu
    cfg = op.Config(nu, j, q, j0, per=True)
    seed = 9000 + 100 * int(nu) + 10 * j + q + dim
    if dim == 1:
        x = inputs.coefficients_1d(j, j0, seed)
        omega = None if dens is None else inputs.uniform_omega(cfg.N, dens, seed + 1)
        m = cfg.N if omega is None else omega.size
        yv = inputs.sample_vector(m, seed + 2)
        A = op.matrix_1d(cfg)
        y_ref, x_ref = op.forward_1d(A, x, omega), op.adjoint_1d(A, yv, omega)
    else:
        x = inputs.coefficients_2d(j, j0, seed)
        omega = None if dens is None else inputs.multilevel_omega_2d(cfg.N, dens, seed + 1, core=4)
        m = cfg.N ** 2 if omega is None else omega.size
        yv = inputs.sample_vector(m, seed + 2)
        blocks = op.Blocks2D(cfg)
        y_ref = op.forward_2d_full(blocks, x, omega).reshape(-1)
        x_ref = op.adjoint_2d_full(blocks, yv, omega)
    y, xa = gpu_pair(dim, nu, j, q, j0, dtype, x, omega, yv, boundary="per")
    assert rel(y, y_ref) < TOL[dtype], rel(y, y_ref)
    assert rel(xa, x_ref) < TOL[dtype], rel(xa, x_ref)


CASES_TENSOR = [
    # nu, j, q, j0, omega density, boundary
    (2, 4, 1, 2, None, "bd"), (4, 6, 2, 3, 0.3, "bd"), (3, 5, 1, 3, 0.25, "per"),   # generic line kernels
    (4, 8, 1, 3, 0.2, "bd"), (8, 9, 1, 4, 0.15, "bd"), (2, 10, 1, 2, 0.2, "per"),  # wave line kernels
    (6, 7, 2, 4, None, "bd"),
    (2, 6, 1, 6, 0.3, "bd"),     # no wavelet level (j0 = j)
    (8, 8, 2, 4, 0.2, "per"),    # db8 periodic on the one-workgroup line kernels
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nu,j,q,j0,dens,boundary", CASES_TENSOR)
def test_parity_tensor_basis(nu, j, q, j0, dens, boundary, dtype):
    """Tensor-product 2D basis (Kronecker product of the 1D section, Sec. 5)."""
    cfg = op.Config(nu, j, q, j0, per=boundary == "per", tensor=True)
    seed = 11000 + 100 * nu + 10 * j + q
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((cfg.M, cfg.M))
    omega = None if dens is None else inputs.multilevel_omega_2d(cfg.N, dens, seed + 1, core=4)
    m = cfg.N ** 2 if omega is None else omega.size
    yv = inputs.sample_vector(m, seed + 2)
    A1 = op.matrix_1d(cfg)
    y_ref = op.forward_2d_tensor(A1, x, omega).reshape(-1)
    x_ref = op.adjoint_2d_tensor(A1, yv, omega)
    y, xa = gpu_pair(2, nu, j, q, j0, dtype, x, omega, yv, boundary=boundary, basis2d="tensor")
    assert rel(y, y_ref) < TOL[dtype], rel(y, y_ref)
    assert rel(xa, x_ref) < TOL[dtype], rel(xa, x_ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nu,j,q,j0,dens", [(4, 10, 1, 3, None), (8, 11, 2, 4, 0.2), (2, 7, 4, 2, 0.3),
                                            (6, 9, 3, 4, None), (3, 8, 1, 3, 0.0)])
def test_1d_one_launch_equals_the_stages(nu, j, q, j0, dens, dtype):
    """1D lines of up to 2048 values run as one launch per direction (wavelet
    levels in LDS fused with the line transform); the staged calls run the
    separate kernels.  Both use the same device arithmetic: equal bit for bit."""
    from paper_2106_00554_amd import _abi
    from paper_2106_00554_amd.operator import Wh2Wav
    cfg = op.Config(nu, j, q, j0)
    seed = 500 + 10 * nu + j
    omega = None if dens is None else (np.zeros(0, np.int64) if dens == 0 else
                                       inputs.uniform_omega(cfg.N, dens, seed + 1))
    opr = Wh2Wav(1, j, q, nu, j0, dtype, omega)
    x = torch.tensor(inputs.coefficients_1d(j, j0, seed), dtype=dtype, device="cuda")
    yv = torch.tensor(inputs.sample_vector(opr.m, seed + 2), dtype=dtype, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    y_whole, x_whole = opr.forward(x), opr.adjoint(yv)
    y_st, x_st = torch.empty_like(y_whole), torch.empty_like(x_whole)
    for s in range(_abi.wh2wav_stage_count(opr._plan, 0)):
        _abi.wh2wav_forward_stage(opr._plan, s, x.data_ptr(), y_st.data_ptr(), opr.workspace.data_ptr(), st)
    for s in range(_abi.wh2wav_stage_count(opr._plan, 1)):
        _abi.wh2wav_adjoint_stage(opr._plan, s, yv.data_ptr(), x_st.data_ptr(), opr.workspace.data_ptr(), st)
    torch.cuda.synchronize()
    assert torch.equal(y_st, y_whole) and torch.equal(x_st, x_whole)
