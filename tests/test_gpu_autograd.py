"""Autograd and FISTA through the HIP operator.

* the gradient of 0.5 ||P_Omega A x - y||^2 taken by autograd equals the
  oracle's A^T (A x - y) at 64^2 (FP64 to 1e-12, FP32 to 1e-5);
* central finite differences in 32 seeded directions at 1024^2, q = 1, db4:
  f is quadratic, so the central difference equals <grad f, v> up to rounding;
* gradcheck / gradgradcheck at a tiny size (FP64);
* FISTA iterates equal a plain numpy FISTA on the oracle's dense matrix;
* a leading batch dimension equals per-instance products.
"""
import numpy as np
import pytest

from oracle import operator as op
from tests import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make_op(nu, j, q, j0, dtype, omega):
    from paper_2106_00554_amd.operator import Wh2Wav
    print(f"[gpu] operator nu={nu} j={j} q={q} j0={j0} {dtype} m={len(omega)}", flush=True)
    return Wh2Wav(2, j, q, nu, j0, dtype, omega)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_autograd_gradient_equals_oracle_adjoint(dtype, tol):
    from paper_2106_00554_amd import autograd as ag
    nu, j, q, j0 = 4, 6, 1, 3
    cfg = op.Config(nu, j, q, j0)
    omega = inputs.multilevel_omega_2d(cfg.N, 0.25, 71)
    X = inputs.coefficients_2d(j, j0, 70)
    Xt = inputs.coefficients_2d(j, j0, 72)
    blocks = op.Blocks2D(cfg)
    y = op.forward_2d_full(blocks, Xt, omega).reshape(-1) + 0.01 * inputs.sample_vector(omega.size, 73)
    r = op.forward_2d_full(blocks, X, omega).reshape(-1) - y
    g_ref = op.adjoint_2d_full(blocks, r, omega)
    opr = make_op(nu, j, q, j0, dtype, omega)
    x = torch.tensor(X, dtype=dtype, device="cuda", requires_grad=True)
    yt = torch.tensor(y, dtype=dtype, device="cuda")
    res = ag.forward(opr, x) - yt
    loss = 0.5 * torch.dot(res, res)
    loss.backward()
    torch.cuda.synchronize()
    assert rel(x.grad.cpu().numpy(), g_ref) < tol
    assert abs(loss.item() - 0.5 * r @ r) <= tol * 0.5 * (r @ r)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-3)])
def test_finite_differences_1024(dtype, tol):
    """cfg of the reconstruction example: db4, M = 1024^2, q = 1, 25 % multilevel Omega.

    f(x) = 0.5 ||P A x - y||^2 is quadratic, so the central difference
    [f(x + e v) - f(x - e v)] / 2e equals <grad f, v> up to rounding for any e.
    Each direction is a Gaussian w plus (||w|| / ||grad||) grad, so <grad, v> is
    about ||w|| ||grad|| and a gradient of the wrong sign or size fails by far;
    the loss is summed in FP64.  The mismatch is measured against |<grad, v>|:
    the FP32 bound follows from the FP32 forward error (about 4e-7 relative),
    which the difference quotient magnifies by about ||x|| / ||grad||."""
    from paper_2106_00554_amd import autograd as ag
    name = "2d_db4_j10_q1_25pct"
    w = inputs.WORKLOADS[name]
    Xtrue, omega = inputs.workload_inputs(name)
    opr = make_op(w["nu"], w["j"], w["q"], w["j0"], dtype, omega)
    xt = torch.tensor(Xtrue, dtype=dtype, device="cuda")
    y0 = ag.forward(opr, xt)
    noise = torch.tensor(inputs.sample_vector(opr.m, 4001), dtype=dtype, device="cuda")
    y = y0 + 0.01 * y0.norm() / noise.norm() * noise
    x = torch.tensor(inputs.coefficients_2d(w["j"], w["j0"], 4002), dtype=dtype, device="cuda",
                     requires_grad=True)

    def f(z):
        r = (ag.forward(opr, z) - y).double()
        return 0.5 * torch.dot(r, r)

    loss = f(x)
    (grad,) = torch.autograd.grad(loss, x)
    rng = inputs.rng_for(4003)
    worst = 0.0
    with torch.no_grad():
        gn = grad.double().norm()
        for _ in range(32):
            wv = torch.tensor(rng.standard_normal(opr.x_shape), dtype=torch.float64, device="cuda")
            v = (wv + (wv.norm() / gn) * grad.double()).to(dtype)
            eps = (x.norm() / v.norm()).item()
            fp, fm = f(x + eps * v).item(), f(x - eps * v).item()
            fd = (fp - fm) / (2 * eps)
            exact = torch.sum(grad.double() * v.double()).item()
            worst = max(worst, abs(fd - exact) / abs(exact))
    print(f"worst FD mismatch relative to <grad, v>: {worst:.3e}")
    assert worst < tol


def test_gradcheck_tiny():
    from paper_2106_00554_amd import autograd as ag
    nu, j, q, j0 = 2, 4, 1, 2
    cfg = op.Config(nu, j, q, j0)
    omega = inputs.uniform_omega(cfg.N ** 2, 0.3, 81)
    opr = make_op(nu, j, q, j0, torch.float64, omega)
    x = torch.tensor(inputs.coefficients_2d(j, j0, 82), device="cuda", requires_grad=True)
    yv = torch.tensor(inputs.sample_vector(opr.m, 83), device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda z: ag.forward(opr, z), (x,), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradcheck(lambda z: ag.adjoint(opr, z), (yv,), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradgradcheck(lambda z: ag.forward(opr, z), (x,), eps=1e-6, atol=1e-8)


def _numpy_fista(A, y, lam, iters):
    """Beck-Teboulle FISTA with L = 1 on a dense matrix (plain numpy)."""
    x = np.zeros(A.shape[1])
    z = x.copy()
    t = 1.0
    out = []
    for _ in range(iters):
        g = A.T @ (A @ z - y)
        u = z - g
        x_new = np.sign(u) * np.maximum(np.abs(u) - lam, 0.0)
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        z = x_new + (t - 1.0) / t_new * (x_new - x)
        x, t = x_new, t_new
        out.append(x.copy())
    return out


def test_fista_matches_dense_oracle():
    from paper_2106_00554_amd import autograd as ag
    nu, j, q, j0 = 2, 5, 1, 2
    cfg = op.Config(nu, j, q, j0)
    omega = inputs.multilevel_omega_2d(cfg.N, 0.3, 91, core=8)
    A = op.dense_2d(cfg)[omega]
    xtrue = inputs.coefficients_2d(j, j0, 92).reshape(-1)
    y = A @ xtrue + 0.01 * np.linalg.norm(A @ xtrue) / np.sqrt(omega.size) * inputs.sample_vector(omega.size, 93)
    lam = 0.01 * np.abs(A.T @ y).max()
    ref = _numpy_fista(A, y, lam, 15)
    opr = make_op(nu, j, q, j0, torch.float64, omega)
    got = []
    ag.fista(opr, torch.tensor(y, device="cuda"), lam, 15,
             callback=lambda k, x: got.append(x.detach().cpu().numpy().reshape(-1)))
    for k in (0, 4, 14):
        assert rel(got[k], ref[k]) < 1e-10, (k, rel(got[k], ref[k]))
    obj = [0.5 * np.sum((A @ g - y) ** 2) + lam * np.abs(g).sum() for g in got]
    assert obj[-1] < obj[0]


def test_batched_leading_dimension():
    from paper_2106_00554_amd import autograd as ag
    nu, j, q, j0 = 4, 5, 1, 3
    cfg = op.Config(nu, j, q, j0)
    omega = inputs.multilevel_omega_2d(cfg.N, 0.25, 95, core=4)
    opr = make_op(nu, j, q, j0, torch.float64, omega)
    xs = torch.tensor(np.stack([inputs.coefficients_2d(j, j0, 96 + b) for b in range(3)]), device="cuda")
    yb = ag.forward(opr, xs)
    for b in range(3):
        assert torch.equal(yb[b], opr.forward(xs[b].contiguous()))
    xb = ag.adjoint(opr, yb)
    for b in range(3):
        assert torch.equal(xb[b], opr.adjoint(yb[b].contiguous()))


def test_graphed_gradient_and_fista_match_eager():
    """The HIP-graph forms replayed several times, with eager work in between, equal the eager forms."""
    from paper_2106_00554_amd import autograd as ag
    name = "2d_db4_j10_q1_25pct"
    w = inputs.WORKLOADS[name]
    Xtrue, omega = inputs.workload_inputs(name)
    for dtype in (torch.float64, torch.float32):
        opr = make_op(w["nu"], w["j"], w["q"], w["j0"], dtype, omega)
        y = ag.forward(opr, torch.tensor(Xtrue, dtype=dtype, device="cuda")).detach()
        gg = ag.GraphedGradient(opr, y)
        for seed in (501, 502, 503):
            xv = torch.tensor(inputs.coefficients_2d(w["j"], w["j0"], seed), dtype=dtype, device="cuda")
            got = gg(xv).clone()
            z = xv.clone().requires_grad_(True)
            r = ag.forward(opr, z) - y
            (ref,) = torch.autograd.grad(0.5 * torch.dot(r, r), z)
            torch.cuda.synchronize()
            assert rel(got.cpu().numpy(), ref.cpu().numpy()) < (1e-12 if dtype == torch.float64 else 1e-5)
        lam = 0.01 * float(opr.adjoint(y).abs().max())
        x_eager = ag.fista(opr, y, lam, 12)
        x_graph = ag.fista_graphed(opr, y, lam, 12)
        x_graph2 = ag.fista_graphed(opr, y, lam, 12)
        torch.cuda.synchronize()
        tol = 1e-12 if dtype == torch.float64 else 1e-5
        assert rel(x_graph.cpu().numpy(), x_eager.cpu().numpy()) < tol
        assert torch.equal(x_graph, x_graph2)
