"""torch-facing wrapper of the C ABI: device memory and streams only.

`Wh2Wav` owns one plan (include/wh2wav.h) and its workspace; `forward` and
`adjoint` hand device pointers and the current HIP stream to
wh2wav_forward / wh2wav_adjoint.  All arithmetic happens in libwh2wav.so.
"""
import math

import numpy as np
import torch

from . import _abi

_DTYPES = {torch.float32: _abi.WH2WAV_F32, torch.float64: _abi.WH2WAV_F64}


def default_j0(nu):
    """Smallest coarse level allowed by Sec. 3.2: ceil(log2(2 nu)) (0 for Haar)."""
    return 0 if nu == 1 else int(math.ceil(math.log2(2 * nu)))


_FAMILIES = {"db": _abi.WH2WAV_DB, "sym": _abi.WH2WAV_SYM}
_BOUNDARIES = {"bd": _abi.WH2WAV_BD, "per": _abi.WH2WAV_PER}
_BASES = {"isotropic": _abi.WH2WAV_ISOTROPIC, "tensor": _abi.WH2WAV_TENSOR}


def axis_sizes(dim, j, j_axes=None):
    """Per-axis j of an operator: j_axes (dim entries, 0 taking j) or j on every axis."""
    if dim == 1:
        return (j,)
    js = tuple(j for _ in range(dim)) if j_axes is None else tuple(int(v) or j for v in j_axes)
    if len(js) != dim:
        raise ValueError(f"j_axes needs {dim} entries")
    return js


def make_desc(dim, j, q, nu, j0=None, dtype=torch.float64, omega=None, family="db", boundary="bd",
              basis2d="isotropic", j_axes=None):
    """Build a wh2wav_desc; returns (desc, keepalive) -- keep the second alive until planned.

    family: "db" (Daubechies) or "sym" (least-asymmetric symlets); boundary:
    "bd" (vanishing-moment-preserving boundary functions) or "per" (periodic);
    basis2d: "isotropic" (quadtree / octant layout) or "tensor" (products of 1D
    basis functions), for dim 2 and 3; j_axes: per-axis j (tensor basis), or
    None for j on every axis."""
    j0 = default_j0(nu) if j0 is None else j0
    js = axis_sizes(dim, j, j_axes)
    total = 1
    for ja in js:
        total *= 1 << (ja + q)
    if omega is None:
        m, ptr, keep = total, None, None
    else:
        keep = np.ascontiguousarray(np.asarray(omega, dtype=np.int64))
        m = int(keep.size)
        ptr = keep.ctypes.data_as(_abi.ctypes.POINTER(_abi.ctypes.c_int64)) if m else \
            _abi.ctypes.cast(_abi.ctypes.pointer(_abi.ctypes.c_int64(0)), _abi.ctypes.POINTER(_abi.ctypes.c_int64))
    jx = (_abi.ctypes.c_int * 3)(*([0, 0, 0] if j_axes is None else list(j_axes) + [0] * (3 - len(j_axes))))
    desc = _abi.wh2wav_desc(dim=dim, j=j, q=q, j0=j0, nu=nu, family=_FAMILIES[family],
                            boundary=_BOUNDARIES[boundary], dtype=_DTYPES[dtype], m=m, omega=ptr,
                            basis2d=_BASES[basis2d], j_axes=jx)
    return desc, keep


class Wh2Wav:
    """y = P_Omega A x and x = A^T P_Omega^T y on the current CUDA/HIP device."""

    def __init__(self, dim, j, q, nu, j0=None, dtype=torch.float64, omega=None, device=None, family="db",
                 boundary="bd", basis2d="isotropic", j_axes=None):
        self.dim, self.j, self.q, self.nu, self.family, self.boundary = dim, j, q, nu, family, boundary
        self.basis2d = basis2d
        self.j0 = default_j0(nu) if j0 is None else j0
        self.dtype = dtype
        self.M, self.N = 1 << j, 1 << (j + q)
        self.j_axes = axis_sizes(dim, j, j_axes)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        desc, keep = make_desc(dim, j, q, nu, self.j0, dtype, omega, family, boundary, basis2d, j_axes)
        self.m = int(desc.m)
        with torch.cuda.device(self.device):
            self._plan = _abi.wh2wav_plan(desc)
        del keep
        nbytes = _abi.wh2wav_workspace_size(self._plan)
        self.workspace = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)

    @property
    def x_shape(self):
        return tuple(1 << ja for ja in self.j_axes)

    @property
    def y_shape(self):
        """Shape of the full Walsh sample array (N_1, ..., N_dim)."""
        return tuple(1 << (ja + self.q) for ja in self.j_axes)

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def _check(self, t, shape, name):
        if t.device != self.device or t.dtype != self.dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {tuple(shape)} "
                             f"on {self.device}; got {tuple(t.shape)} {t.dtype} {t.device}")

    def forward(self, x, out=None):
        self._check(x, self.x_shape, "x")
        y = torch.empty(self.m, dtype=self.dtype, device=self.device) if out is None else out
        self._check(y, (self.m,), "y")
        _abi.wh2wav_forward(self._plan, x.data_ptr(), y.data_ptr(), self.workspace.data_ptr(), self._stream())
        return y

    def adjoint(self, y, out=None):
        self._check(y, (self.m,), "y")
        x = torch.empty(self.x_shape, dtype=self.dtype, device=self.device) if out is None else out
        self._check(x, self.x_shape, "x")
        _abi.wh2wav_adjoint(self._plan, y.data_ptr(), x.data_ptr(), self.workspace.data_ptr(), self._stream())
        return x

    def close(self):
        if getattr(self, "_plan", None) is not None:
            _abi.wh2wav_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Wh2WavBatch:
    """Many independent operators, one graph launch per direction.

    `specs` is a list of dicts with the keys of `Wh2Wav` (dim, j, q, nu and
    optionally j0, dtype, omega).  `forward(xs)` returns the list of
    P_Omega_i A_i xs[i]; `adjoint(ys)` the list of A_i^T P_Omega_i^T ys[i].
    Calls with the same tensors replay a captured graph (see
    wh2wav_forward_batch); `tune` runs the schedule autotuner.
    """

    def __init__(self, specs, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        descs, keeps = [], []
        self.x_shapes, self.ms, self.dtypes = [], [], []
        for sp in specs:
            dtype = sp.get("dtype", torch.float64)
            d, k = make_desc(sp["dim"], sp["j"], sp["q"], sp["nu"], sp.get("j0"), dtype, sp.get("omega"),
                             sp.get("family", "db"), sp.get("boundary", "bd"), sp.get("basis2d", "isotropic"),
                             sp.get("j_axes"))
            descs.append(d)
            keeps.append(k)
            self.x_shapes.append(tuple(1 << ja for ja in axis_sizes(sp["dim"], sp["j"], sp.get("j_axes"))))
            self.ms.append(int(d.m))
            self.dtypes.append(dtype)
        with torch.cuda.device(self.device):
            self._batch = _abi.wh2wav_plan_batch(descs)
        del keeps
        nbytes = _abi.wh2wav_batch_workspace_size(self._batch)
        self.workspace = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)

    def __len__(self):
        return len(self.ms)

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def _check(self, ts, shapes, name):
        if len(ts) != len(self):
            raise ValueError(f"{name}: expected {len(self)} tensors, got {len(ts)}")
        for i, (t, shp, dt) in enumerate(zip(ts, shapes, self.dtypes)):
            if t.device != self.device or t.dtype != dt or not t.is_contiguous() or tuple(t.shape) != tuple(shp):
                raise ValueError(f"{name}[{i}] must be a contiguous {dt} tensor of shape {tuple(shp)} on "
                                 f"{self.device}")

    def new_outputs(self, direction):
        shapes = [(m,) for m in self.ms] if direction == 0 else self.x_shapes
        return [torch.empty(s, dtype=dt, device=self.device) for s, dt in zip(shapes, self.dtypes)]

    def forward(self, xs, ys=None):
        ys = self.new_outputs(0) if ys is None else ys
        self._check(xs, self.x_shapes, "xs")
        self._check(ys, [(m,) for m in self.ms], "ys")
        _abi.wh2wav_forward_batch(self._batch, [t.data_ptr() for t in xs], [t.data_ptr() for t in ys],
                                  self.workspace.data_ptr(), self._stream())
        return ys

    def adjoint(self, ys, xs=None):
        xs = self.new_outputs(1) if xs is None else xs
        self._check(ys, [(m,) for m in self.ms], "ys")
        self._check(xs, self.x_shapes, "xs")
        _abi.wh2wav_adjoint_batch(self._batch, [t.data_ptr() for t in ys], [t.data_ptr() for t in xs],
                                  self.workspace.data_ptr(), self._stream())
        return xs

    def schedule(self):
        return _abi.wh2wav_batch_schedule(self._batch)

    def set_mode(self, mode):
        """"branches": every instance's own kernels in graph branches; "fused": the
        small instances as fused launches, one per round of their stages."""
        _abi.wh2wav_batch_set_mode(self._batch, {"branches": _abi.WH2WAV_BATCH_BRANCHES,
                                                 "fused": _abi.WH2WAV_BATCH_FUSED}[mode])

    def mode(self):
        """(mode name, instances in the fused launches, fused launches per forward call)."""
        m, n, k = _abi.wh2wav_batch_mode(self._batch)
        return ("branches", "fused")[m], n, k

    def set_schedule(self, branches, order):
        _abi.wh2wav_batch_set_schedule(self._batch, branches, order)

    def tune(self, xs, ys, xa, reps=5):
        """Time every schedule on these buffers, keep the fastest; returns its ms per pair."""
        self._check(xs, self.x_shapes, "xs")
        self._check(ys, [(m,) for m in self.ms], "ys")
        self._check(xa, self.x_shapes, "xa")
        return _abi.wh2wav_batch_tune(self._batch, [t.data_ptr() for t in xs], [t.data_ptr() for t in ys],
                                      [t.data_ptr() for t in xa], self.workspace.data_ptr(), self._stream(), reps)

    def close(self):
        if getattr(self, "_batch", None) is not None:
            _abi.wh2wav_destroy_batch(self._batch)
            self._batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

