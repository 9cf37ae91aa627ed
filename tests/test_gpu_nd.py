"""GPU parity of the three-dimensional and unequal-sided operators against the oracle.

Sec. 5 splits the d-fold inner products into 1D ones; the HIP path runs the
wavelet levels (isotropic: per level and axis on the whole array; tensor:
every level of an axis in one launch of the LDS line kernel), then the line
transform along each axis with that axis's tables, the last pass gathering
Omega.  The
oracle applies the dense 1D sections axis by axis (forward_nd_*), pinned in
tests/test_oracle_nd.py.  Bar: relative l2 <= 1e-12 (FP64), <= 1e-5 (FP32).
"""
import numpy as np
import pytest

from oracle import operator as op
from tests import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_pair(js, nu, q, j0, per, tensor, X, omega, yv):
    cfgs = [op.Config(nu, ja, q, j0, per=per) for ja in js]
    if tensor:
        mats = [op.matrix_1d(c) for c in cfgs]
        return op.forward_nd_tensor(mats, X, omega).ravel(), op.adjoint_nd_tensor(mats, yv, omega)
    B = op.Blocks2D(cfgs[0])
    return op.forward_nd_iso(B, X, omega).ravel(), op.adjoint_nd_iso(B, yv, len(js), omega)


def gpu_pair(js, nu, q, j0, per, tensor, dtype, X, omega, yv):
    from paper_2106_00554_amd.operator import Wh2Wav
    print(f"[gpu nd] js={js} nu={nu} q={q} j0={j0} per={per} tensor={tensor} {dtype} "
          f"m={'all' if omega is None else len(omega)}", flush=True)
    opr = Wh2Wav(len(js), js[0], q, nu, j0, dtype, omega, boundary="per" if per else "bd",
                 basis2d="tensor" if tensor else "isotropic", j_axes=js)
    assert opr.x_shape == tuple(1 << ja for ja in js)
    y = opr.forward(torch.tensor(X, dtype=dtype, device="cuda"))
    xa = opr.adjoint(torch.tensor(yv, dtype=dtype, device="cuda"))
    torch.cuda.synchronize()
    return y.cpu().numpy(), xa.cpu().numpy()


CASES = [
    # js, nu, q, j0, per, tensor, Omega density (None = all)
    ((3, 3, 3), 1, 1, 0, False, False, None),
    ((3, 3, 3), 1, 1, 0, False, True, 0.3),
    ((4, 4, 4), 2, 1, 2, False, False, 0.2),
    ((4, 4, 4), 2, 1, 2, False, True, None),
    ((4, 4, 4), 3, 2, 3, True, False, 0.1),
    ((5, 5, 5), 4, 1, 3, False, False, 0.15),
    ((5, 5, 5), 4, 1, 3, True, True, 0.15),
    ((5, 5, 5), 8, 1, 4, False, False, 0.1),
    ((3, 4, 5), 2, 1, 2, False, True, 0.25),
    ((5, 3, 4), 4, 2, 3, True, True, 0.05),
    ((4, 7), 2, 1, 2, False, True, 0.3),
    ((7, 4), 4, 2, 3, True, True, None),
    ((3, 9), 2, 1, 2, False, True, 0.1),
    ((6, 5), 8, 1, 4, False, True, 0.2),
    ((4, 4), 2, 1, 2, False, True, 0.0),  # empty Omega: forward writes nothing, adjoint zeros
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("js,nu,q,j0,per,tensor,dens", CASES)
def test_parity_nd(js, nu, q, j0, per, tensor, dens, dtype):
    seed = 7000 + 100 * nu + 10 * sum(js) + q + (1 if per else 0) + (2 if tensor else 0)
    X = inputs.coefficients_nd(tuple(1 << ja for ja in js), seed)
    total = int(np.prod([1 << (ja + q) for ja in js]))
    omega = None if dens is None else inputs.uniform_omega(total, dens, seed + 1)
    m = total if omega is None else omega.size
    yv = inputs.sample_vector(m, seed + 2)
    y_ref, x_ref = oracle_pair(js, nu, q, j0, per, tensor, X, omega, yv)
    y, xa = gpu_pair(js, nu, q, j0, per, tensor, dtype, X, omega, yv)
    assert y.shape == (m,)
    if m:
        assert rel(y, y_ref) < TOL[dtype], rel(y, y_ref)
        assert rel(xa, x_ref) < TOL[dtype], rel(xa, x_ref)
    else:
        assert not np.any(xa)


@pytest.mark.parametrize("tensor", [False, True])
def test_three_dimensions_at_64_cubed(tensor):
    """db4 q = 1 at 64^3 (N^3 = 2^21 samples, 12.5 % Omega) in FP32 and FP64,
    every output against the oracle, FP32 also against FP64."""
    js, nu, q, j0 = (6, 6, 6), 4, 1, 3
    X = inputs.coefficients_nd((64, 64, 64), 7700)
    omega = inputs.uniform_omega(128 ** 3, 0.125, 7701)
    yv = inputs.sample_vector(omega.size, 7702)
    y_ref, x_ref = oracle_pair(js, nu, q, j0, False, tensor, X, omega, yv)
    y64, x64 = gpu_pair(js, nu, q, j0, False, tensor, torch.float64, X, omega, yv)
    y32, x32 = gpu_pair(js, nu, q, j0, False, tensor, torch.float32, X, omega, yv)
    print(f"[64^3 tensor={tensor}] fwd f64 {rel(y64, y_ref):.2e} f32 {rel(y32, y_ref):.2e} "
          f"(vs f64 {rel(y32, y64):.2e}); adj f64 {rel(x64, x_ref):.2e} f32 {rel(x32, x_ref):.2e}", flush=True)
    assert rel(y64, y_ref) < 1e-12 and rel(x64, x_ref) < 1e-12
    assert rel(y32, y_ref) < 1e-5 and rel(x32, x_ref) < 1e-5


@pytest.mark.timeout(600)
def test_unequal_sides_2048_by_256():
    """The tensor basis with unequal sides at 2048 x 256 (db4, q = 1, 12.5 %
    Omega), FP32 and FP64, every output against the oracle: 2048-value lines
    along a strided axis in the wavelet stage and both line passes."""
    js, nu, q, j0 = (11, 8), 4, 1, 3
    X = inputs.coefficients_nd((2048, 256), 7900)
    omega = inputs.uniform_omega(4096 * 512, 0.125, 7901)
    yv = inputs.sample_vector(omega.size, 7902)
    y_ref, x_ref = oracle_pair(js, nu, q, j0, False, True, X, omega, yv)
    y64, x64 = gpu_pair(js, nu, q, j0, False, True, torch.float64, X, omega, yv)
    y32, x32 = gpu_pair(js, nu, q, j0, False, True, torch.float32, X, omega, yv)
    print(f"[2048 x 256 tensor] fwd f64 {rel(y64, y_ref):.2e} f32 {rel(y32, y_ref):.2e}; "
          f"adj f64 {rel(x64, x_ref):.2e} f32 {rel(x32, x_ref):.2e}", flush=True)
    assert rel(y64, y_ref) < 1e-12 and rel(x64, x_ref) < 1e-12
    assert rel(y32, y_ref) < 1e-5 and rel(x32, x_ref) < 1e-5


@pytest.mark.parametrize("js,tensor", [((4, 4, 4), False), ((3, 5, 4), True), ((6, 3), True)])
def test_stages_compose_to_the_whole(js, tensor):
    """Stages 0..2 run one by one equal the whole call, bit for bit."""
    from paper_2106_00554_amd import _abi
    from paper_2106_00554_amd.operator import Wh2Wav
    q, nu, j0 = 1, 2, 2
    total = int(np.prod([1 << (ja + q) for ja in js]))
    omega = inputs.uniform_omega(total, 0.2, 7800)
    opr = Wh2Wav(len(js), js[0], q, nu, j0, torch.float64, omega, basis2d="tensor" if tensor else "isotropic",
                 j_axes=js)
    x = torch.tensor(inputs.coefficients_nd(opr.x_shape, 7801), dtype=torch.float64, device="cuda")
    yv = torch.tensor(inputs.sample_vector(opr.m, 7802), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    assert _abi.wh2wav_stage_count(opr._plan, 0) == 3 and _abi.wh2wav_stage_count(opr._plan, 1) == 3
    y_whole, x_whole = opr.forward(x), opr.adjoint(yv)
    y_st = torch.empty_like(y_whole)
    x_st = torch.empty_like(x_whole)
    for s in range(3):
        _abi.wh2wav_forward_stage(opr._plan, s, x.data_ptr(), y_st.data_ptr(), opr.workspace.data_ptr(), st)
    for s in range(3):
        _abi.wh2wav_adjoint_stage(opr._plan, s, yv.data_ptr(), x_st.data_ptr(), opr.workspace.data_ptr(), st)
    torch.cuda.synchronize()
    assert torch.equal(y_st, y_whole) and torch.equal(x_st, x_whole)


def test_three_dimensional_instances_in_a_batch():
    """3D and unequal-sided instances in one batch graph equal their single plans."""
    from paper_2106_00554_amd.operator import Wh2Wav, Wh2WavBatch
    specs = [dict(dim=3, j=4, q=1, nu=2, j0=2, dtype=torch.float32, omega=inputs.uniform_omega(32 ** 3, 0.2, 7900)),
             dict(dim=2, j=5, q=1, nu=4, j0=3, dtype=torch.float64, basis2d="tensor", j_axes=(5, 3)),
             dict(dim=3, j=3, q=2, nu=1, j0=0, dtype=torch.float64, basis2d="tensor", j_axes=(3, 4, 2))]
    b = Wh2WavBatch(specs)
    xs = [torch.tensor(inputs.coefficients_nd(shp, 7910 + i), dtype=sp["dtype"], device="cuda")
          for i, (shp, sp) in enumerate(zip(b.x_shapes, specs))]
    ys = b.forward(xs)
    xa = b.adjoint(ys)
    torch.cuda.synchronize()
    for sp, x, y, x2 in zip(specs, xs, ys, xa):
        single = Wh2Wav(sp["dim"], sp["j"], sp["q"], sp["nu"], sp["j0"], sp["dtype"], sp.get("omega"),
                        basis2d=sp.get("basis2d", "isotropic"), j_axes=sp.get("j_axes"))
        assert torch.equal(single.forward(x), y)
        assert torch.equal(single.adjoint(y), x2)
