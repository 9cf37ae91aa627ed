"""Reconstruction methods on top of the operator, and its extreme singular values.

Every solver of Sec. 1.2 needs only products with P_Omega U P_M and its
adjoint (the conjugate-gradient method for generalised sampling; SPGL1 or
Chambolle and Pock's primal-dual method for compressive sensing), so each one
here takes a `Wh2Wav` operator and calls its forward / adjoint HIP kernels;
what remains is vector arithmetic on torch tensors on the same device.

* `generalised_sampling`: the least-squares problem (GS_approx) of Sec. 1.2,
  min ||A z - y||_2, by conjugate gradients on the normal equations (CGLS:
  the residual and the adjoint residual are updated with one forward and one
  adjoint product per iteration).
* `pbdw`: the PBDW approximation of Sec. 1.2: the measured Walsh samples
  where they exist, and the generalised-sampling reconstruction's Walsh
  coefficients (from an operator with more samples, K > N) elsewhere.
* `qcbp`: quadratically constrained basis pursuit (QCBP) of Sec. 1.2,
  min ||z||_1 subject to ||A z - y||_2^2 <= eta, by the Chambolle-Pock
  primal-dual iteration with step sizes tau sigma ||A||^2 < 1 (||A|| <= 1,
  Sec. 2: the section of a unitary matrix).
* `extreme_singular_values`: sigma_min and sigma_max of A by the Lanczos
  process on A^T A with full reorthogonalisation; mu = 1 / sigma_min is the
  quantity of Table 1.
"""
import math

import torch


def generalised_sampling(op, y, iters=200, tol=1e-12, x0=None):
    """argmin_z ||A z - y||_2 (A = op) by CGLS; returns (z, relative residual history).

    Stops when ||A^T r|| <= tol ||A^T y|| or after `iters` iterations."""
    dt = op.dtype
    z = torch.zeros(op.x_shape, dtype=dt, device=op.device) if x0 is None else x0.clone()
    r = y - op.forward(z) if x0 is not None else y.clone()
    s = op.adjoint(r)
    p = s.clone()
    gamma = torch.dot(s.reshape(-1), s.reshape(-1))
    g0 = math.sqrt(float(gamma))
    hist = []
    for _ in range(iters):
        if g0 == 0 or math.sqrt(float(gamma)) <= tol * g0:
            break
        q = op.forward(p)
        alpha = gamma / torch.dot(q, q)
        z = z + alpha * p
        r = r - alpha * q
        s = op.adjoint(r)
        gamma_new = torch.dot(s.reshape(-1), s.reshape(-1))
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        hist.append(math.sqrt(float(gamma)) / g0)
    return z, hist


def pbdw(op_k, z_gs, y_first, first):
    """PBDW Walsh coefficients up to K: A_K z_gs with the measured samples put back.

    op_k: operator with all K samples (full Omega); z_gs: the generalised
    sampling coefficients; y_first: the measured samples; first: the linear
    indices of the measured samples in op_k's output order."""
    w = op_k.forward(z_gs)
    w[first] = y_first
    return w


def qcbp(op, y, eta, iters=500, tau=0.99, sigma=0.99, x0=None):
    """min ||z||_1 s.t. ||A z - y||_2^2 <= eta, by Chambolle-Pock; returns z.

    Primal z, dual p for F(u) = indicator of the ball ||u - y|| <= sqrt(eta):
      p <- p + sigma A zbar;  p <- p - sigma proj_ball(p / sigma)
      z_new <- soft(z - tau A^T p, tau);  zbar <- 2 z_new - z."""
    eps = math.sqrt(eta)
    dt = op.dtype
    z = torch.zeros(op.x_shape, dtype=dt, device=op.device) if x0 is None else x0.clone()
    zbar = z.clone()
    p = torch.zeros_like(y)
    for _ in range(iters):
        v = p + sigma * op.forward(zbar)
        u = v / sigma - y
        nu = torch.linalg.vector_norm(u)
        scale = torch.clamp(eps / torch.clamp(nu, min=torch.finfo(dt).tiny), max=1.0)
        p = v - sigma * (y + scale * u)
        z_new = torch.nn.functional.softshrink(z - tau * op.adjoint(p), tau)
        zbar = 2 * z_new - z
        z = z_new
    return z


def extreme_singular_values(op, iters=None, seed=0):
    """(sigma_min, sigma_max) of A = op by Lanczos on A^T A with full reorthogonalisation.

    With iters >= the number of columns the Krylov space is the whole space and
    the Ritz values are the eigenvalues of A^T A up to rounding."""
    n = math.prod(op.x_shape)
    k = n if iters is None else min(iters, n)
    dt = op.dtype
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn(n, generator=g, dtype=torch.float64).to(device=op.device, dtype=dt)
    v = v / torch.linalg.vector_norm(v)
    V = torch.zeros((k, n), dtype=dt, device=op.device)
    alphas, betas = [], []
    beta = 0.0
    v_prev = torch.zeros_like(v)
    for i in range(k):
        V[i] = v
        w = op.adjoint(op.forward(v.reshape(op.x_shape))).reshape(-1)
        a = float(torch.dot(w, v))
        w = w - a * v - beta * v_prev
        # full reorthogonalisation (twice) against the basis so far
        for _ in range(2):
            w = w - V[: i + 1].T @ (V[: i + 1] @ w)
        alphas.append(a)
        beta = float(torch.linalg.vector_norm(w))
        if i == k - 1 or beta <= 1e-13 * max(1.0, abs(a)):
            break
        betas.append(beta)
        v_prev, v = v, w / beta
    T = torch.diag(torch.tensor(alphas, dtype=torch.float64))
    if betas:
        b = torch.tensor(betas[: len(alphas) - 1], dtype=torch.float64)
        T = T + torch.diag(b, 1) + torch.diag(b, -1)
    ev = torch.linalg.eigvalsh(T)
    return math.sqrt(max(float(ev[0]), 0.0)), math.sqrt(float(ev[-1]))
