"""wh2wav_forward_noalloc: the forward product with the library's fixed
workspace array, against wh2wav_forward with a caller-allocated workspace,
through the C ABI.  Two calls in a row, the second with a smaller input, so
that the second runs on what the first left in the shared array."""
import numpy as np
import pytest

from tests import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _plan(dim, nu, j, q, j0, dtype, omega):
    from paper_2106_00554_amd import _abi
    from paper_2106_00554_amd.operator import make_desc
    desc, keep = make_desc(dim, j, q, nu, j0, dtype, omega)
    plan = _abi.wh2wav_plan(desc)
    del keep
    return plan, int(desc.m)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_forward_matches_forward(dtype):
    from paper_2106_00554_amd import _abi
    # 1024^2 db4 q=1 (workspace 16 MiB in FP32, 32 MiB in FP64), then a 1D db8 2^12 q=2 line
    cases = [(2, 4, 10, 1, 3, 0.25), (1, 8, 12, 2, 4, 0.2)]
    stream = torch.cuda.current_stream().cuda_stream
    for dim, nu, j, q, j0, dens in cases:
        N = 1 << (j + q)
        print(f"[noalloc] dim={dim} nu={nu} j={j} q={q} {dtype}", flush=True)
        omega = (inputs.multilevel_omega_2d(N, dens, 7 + j) if dim == 2
                 else inputs.uniform_omega(N, dens, 7 + j))
        x_np = inputs.coefficients_2d(j, j0, 5 + j) if dim == 2 else inputs.coefficients_1d(j, j0, 5 + j)
        plan, m = _plan(dim, nu, j, q, j0, dtype, omega)
        try:
            nbytes = _abi.wh2wav_workspace_size(plan)
            assert nbytes <= _abi.WH2WAV_NOALLOC_MAX_WORKSPACE
            x = torch.tensor(x_np, dtype=dtype, device="cuda")
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            y_ref = torch.empty(m, dtype=dtype, device="cuda")
            y = torch.full((m,), float("nan"), dtype=dtype, device="cuda")
            _abi.wh2wav_forward(plan, x.data_ptr(), y_ref.data_ptr(), ws.data_ptr(), stream)
            _abi.wh2wav_forward_noalloc(plan, x.data_ptr(), y.data_ptr(), stream)
            torch.cuda.synchronize()
            yr, yn = y_ref.cpu().numpy(), y.cpu().numpy()
            err = np.linalg.norm(yn - yr) / np.linalg.norm(yr)
            assert err < (1e-5 if dtype == torch.float32 else 1e-12), err
            assert np.array_equal(yn, yr)
        finally:
            _abi.wh2wav_destroy(plan)


def test_noalloc_rejects_oversized_workspace():
    from paper_2106_00554_amd import _abi
    # 2048^2 db8 q=2 FP32 needs about 100 MB of workspace
    plan, m = _plan(2, 8, 11, 2, 4, torch.float32, None)
    try:
        assert _abi.wh2wav_workspace_size(plan) > _abi.WH2WAV_NOALLOC_MAX_WORKSPACE
        x = torch.zeros((2048, 2048), dtype=torch.float32, device="cuda")
        y = torch.zeros(m, dtype=torch.float32, device="cuda")
        with pytest.raises(_abi.Wh2WavError) as e:
            _abi.wh2wav_forward_noalloc(plan, x.data_ptr(), y.data_ptr(), None)
        assert e.value.code == _abi.WH2WAV_EUNSUPPORTED
    finally:
        _abi.wh2wav_destroy(plan)
