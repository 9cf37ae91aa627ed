"""Differentiable form of the operator, and FISTA on top of it.

`forward(op, x)` computes y = P_Omega A x and records it for autograd.  The
gradient with respect to x is A^T P_Omega^T g, which is exactly the adjoint
product, so the backward calls the adjoint kernels (and the adjoint's
backward calls the forward kernels, so every order of derivative is
available).  A is real (Algorithm 1 works over the reals), so the adjoint is
the transpose.

Compressive-sensing solvers only need the two products (the paper's
reconstructions call a solver with the forward and the adjoint); `fista`
solves the l1-regularised least-squares problem

    min_x  0.5 || P_Omega A x - y ||^2 + lam || x ||_1

with the gradient of the smooth term taken through autograd.  The step 1/L
with L = 1 is valid because || P_Omega A || <= 1 (the section of an
orthogonal change of basis, Sec. 2).

A leading batch dimension is accepted: x of shape (B, *op.x_shape) maps to y
of shape (B, op.m), one product per instance.
"""
import torch


def _apply(fn, t, in_shape, out_shape, op):
    lead = tuple(t.shape[: t.dim() - len(in_shape)])
    if tuple(t.shape[len(lead):]) != tuple(in_shape):
        raise ValueError(f"expected trailing shape {tuple(in_shape)}, got {tuple(t.shape)}")
    t = t.contiguous()
    if not lead:
        return fn(t)
    flat = t.reshape((-1,) + tuple(in_shape))
    out = torch.empty((flat.shape[0],) + tuple(out_shape), dtype=op.dtype, device=op.device)
    for b in range(flat.shape[0]):
        fn(flat[b], out=out[b])
    return out.reshape(lead + tuple(out_shape))


class _Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, op):
        ctx.op = op
        return _apply(op.forward, x.detach(), op.x_shape, (op.m,), op)

    @staticmethod
    def backward(ctx, g):
        return _Adjoint.apply(g, ctx.op), None


class _Adjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, op):
        ctx.op = op
        return _apply(op.adjoint, y.detach(), (op.m,), op.x_shape, op)

    @staticmethod
    def backward(ctx, g):
        return _Forward.apply(g, ctx.op), None


def forward(op, x):
    """y = P_Omega A x, differentiable in x."""
    return _Forward.apply(x, op)


def adjoint(op, y):
    """x = A^T P_Omega^T y, differentiable in y."""
    return _Adjoint.apply(y, op)


class Wh2WavLayer(torch.nn.Module):
    """nn.Module holding one operator: layer(x) = P_Omega A x."""

    def __init__(self, op):
        super().__init__()
        self.op = op

    def forward(self, x):
        return forward(self.op, x)

    def adjoint(self, y):
        return adjoint(self.op, y)


def soft_threshold(z, t):
    """sign(z) max(|z| - t, 0) for t >= 0, one elementwise kernel."""
    return torch.nn.functional.softshrink(z, t) if t > 0 else z.clone()


def objective(op, x, y, lam):
    r = forward(op, x) - y
    return 0.5 * torch.dot(r.reshape(-1), r.reshape(-1)) + lam * x.abs().sum()


class GraphedGradient:
    """The gradient A^T P_Omega^T (P_Omega A x - y) of 0.5 ||P_Omega A x - y||^2,
    taken through autograd once and replayed as a HIP graph.

    The captured step is the autograd vector-Jacobian product of the residual
    r = forward(op, x) - y with r itself (the gradient of the half squared
    norm without forming the norm: no reduction kernel in the graph).  The
    forward and the adjoint kernels run on the capturing stream with the
    operator's preallocated workspace; the graph is replayed on the current
    stream.  `x` and `y` are copied into static buffers before each replay;
    the returned tensor is the graph's static output (overwritten by the next
    call)."""

    def __init__(self, op, y):
        self.op = op
        self.x = torch.zeros(op.x_shape, dtype=op.dtype, device=op.device, requires_grad=True)
        self.y = y.detach().clone()
        side = torch.cuda.Stream(device=op.device)
        side.wait_stream(torch.cuda.current_stream(op.device))
        with torch.cuda.stream(side):
            for _ in range(2):  # warm-up outside capture
                self._step()
        torch.cuda.current_stream(op.device).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.grad = self._step()

    def _step(self):
        r = forward(self.op, self.x) - self.y
        (g,) = torch.autograd.grad(r, self.x, grad_outputs=r)
        return g

    def __call__(self, x, y=None):
        with torch.no_grad():
            self.x.copy_(x)
            if y is not None:
                self.y.copy_(y)
        self.graph.replay()
        return self.grad


def fista(op, y, lam, iters, x0=None, L=1.0, callback=None):
    """FISTA (Beck and Teboulle) for 0.5 ||P_Omega A x - y||^2 + lam ||x||_1.

    The gradient of the smooth term at the extrapolated point is obtained by
    autograd through `forward` (its backward is the adjoint kernel).  Returns
    the last iterate.  `callback(k, x)` is called after each iteration if
    given.
    """
    x = torch.zeros(op.x_shape, dtype=op.dtype, device=op.device) if x0 is None else x0.clone()
    z = x.clone()
    t = 1.0
    step = 1.0 / L
    for k in range(iters):
        z = z.detach().requires_grad_(True)
        r = forward(op, z) - y
        loss = 0.5 * torch.dot(r, r)
        (grad,) = torch.autograd.grad(loss, z)
        with torch.no_grad():
            x_new = soft_threshold(torch.add(z, grad, alpha=-step), step * lam)
            t_new = 0.5 * (1.0 + (1.0 + 4.0 * t * t) ** 0.5)
            # z = x_new + beta (x_new - x), beta = (t - 1) / t_new: lerp with
            # weight 1 + beta >= 1 evaluates exactly this expression
            z = torch.lerp(x, x_new, 1.0 + (t - 1.0) / t_new)
        x, t = x_new, t_new
        if callback is not None:
            callback(k, x)
    return x


def fista_graphed(op, y, lam, iters, x0=None, L=1.0):
    """FISTA with one iteration captured as a HIP graph and replayed `iters` times.

    Same iteration as `fista` (gradient through autograd at the extrapolated
    point, soft thresholding, momentum).  The momentum weights 1 + (t_k - 1) /
    t_{k+1} do not depend on the data, so they are precomputed into a device
    array that the graph indexes with a device-side counter."""
    dt, dev = op.dtype, op.device
    ws, t = [], 1.0
    for _ in range(iters):
        t_new = 0.5 * (1.0 + (1.0 + 4.0 * t * t) ** 0.5)
        ws.append(1.0 + (t - 1.0) / t_new)
        t = t_new
    weights = torch.tensor(ws + [1.0], dtype=dt, device=dev)
    k = torch.zeros(1, dtype=torch.long, device=dev)
    x = torch.zeros(op.x_shape, dtype=dt, device=dev) if x0 is None else x0.detach().clone()
    z = x.clone().requires_grad_(True)
    yy = y.detach().clone()
    step = 1.0 / L

    def iteration():
        r = forward(op, z) - yy
        (g,) = torch.autograd.grad(r, z, grad_outputs=r)
        with torch.no_grad():
            x_new = soft_threshold(torch.add(z, g, alpha=-step), step * lam)
            w = weights.index_select(0, k).reshape(())
            z.copy_(torch.lerp(x, x_new, w))
            x.copy_(x_new)
            k.add_(1)

    # warm-up on a side stream (two iterations), then restart from x0
    x_start, z_start = x.clone(), z.detach().clone()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        for _ in range(2):
            iteration()
    torch.cuda.current_stream(dev).wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        iteration()
    with torch.no_grad():
        x.copy_(x_start)
        z.copy_(z_start)
        k.zero_()
    for _ in range(iters):
        graph.replay()
    return x.detach().clone()
