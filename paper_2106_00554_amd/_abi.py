"""ctypes binding of the C ABI declared in include/wh2wav.h (argument marshalling only).

Every function here has the name of the C entry point it wraps.  Nothing
computes: pointers and sizes go through unchanged, and a failing status is
turned into an exception carrying wh2wav_last_error().  There is no fallback:
if libwh2wav.so is missing the import of this module fails.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwh2wav.so")

WH2WAV_OK = 0
WH2WAV_EINVAL = -1
WH2WAV_EUNSUPPORTED = -2
WH2WAV_ENOMEM = -3
WH2WAV_EHIP = -4
WH2WAV_EINTERNAL = -5

WH2WAV_F32 = 0
WH2WAV_F64 = 1
WH2WAV_DB = 0
WH2WAV_SYM = 1
WH2WAV_BD = 0
WH2WAV_PER = 1
WH2WAV_ISOTROPIC = 0
WH2WAV_TENSOR = 1
WH2WAV_BATCH_BRANCHES = 0
WH2WAV_BATCH_FUSED = 1

TABLES = {"h": 0, "g": 1, "T": 2, "band_l": 3, "band_r": 4, "syn_l": 5, "syn_r": 6, "row_ptr": 7}

# every symbol the header declares
EXPORTS = ("wh2wav_plan", "wh2wav_workspace_size", "wh2wav_forward", "wh2wav_adjoint",
           "wh2wav_stage_count", "wh2wav_forward_stage", "wh2wav_adjoint_stage",
           "wh2wav_destroy", "wh2wav_last_error", "wh2wav_host_table",
           "wh2wav_plan_batch", "wh2wav_batch_workspace_size", "wh2wav_forward_batch",
           "wh2wav_adjoint_batch", "wh2wav_batch_schedule", "wh2wav_batch_set_schedule",
           "wh2wav_batch_tune", "wh2wav_destroy_batch", "wh2wav_forward_noalloc",
           "wh2wav_batch_set_mode", "wh2wav_batch_mode")

# size of the library's fixed workspace array used by wh2wav_forward_noalloc
WH2WAV_NOALLOC_MAX_WORKSPACE = 32 << 20


class wh2wav_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("j", ctypes.c_int),
        ("q", ctypes.c_int),
        ("j0", ctypes.c_int),
        ("nu", ctypes.c_int),
        ("family", ctypes.c_int),
        ("boundary", ctypes.c_int),
        ("dtype", ctypes.c_int),
        ("m", ctypes.c_int64),
        ("omega", ctypes.POINTER(ctypes.c_int64)),
        ("basis2d", ctypes.c_int),
        ("j_axes", ctypes.c_int * 3),
    ]


class Wh2WavError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"wh2wav status {code}: {message}")
        self.code = code


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 (same soname
    # as /opt/rocm's, but torch's libraries ask for it by the unversioned name).
    # Loading torch first makes this library bind to that copy; loading this
    # library first would leave two runtimes in the process, and the second
    # one to initialise sees no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2106_00554_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.wh2wav_plan.argtypes = [ctypes.POINTER(wh2wav_desc), ctypes.POINTER(vp)]
    lib.wh2wav_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.wh2wav_forward.argtypes = [vp, vp, vp, vp, vp]
    lib.wh2wav_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.wh2wav_stage_count.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.wh2wav_forward_stage.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    lib.wh2wav_adjoint_stage.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    lib.wh2wav_destroy.argtypes = [vp]
    lib.wh2wav_last_error.argtypes = []
    lib.wh2wav_last_error.restype = ctypes.c_char_p
    lib.wh2wav_host_table.argtypes = [ctypes.POINTER(wh2wav_desc), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_double), sz, ctypes.POINTER(sz)]
    pp = ctypes.POINTER(vp)
    lib.wh2wav_plan_batch.argtypes = [ctypes.POINTER(wh2wav_desc), ctypes.c_int, ctypes.POINTER(vp)]
    lib.wh2wav_batch_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.wh2wav_forward_batch.argtypes = [vp, pp, pp, vp, vp]
    lib.wh2wav_adjoint_batch.argtypes = [vp, pp, pp, vp, vp]
    lib.wh2wav_batch_schedule.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.wh2wav_batch_set_schedule.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.wh2wav_batch_tune.argtypes = [vp, pp, pp, pp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    lib.wh2wav_destroy_batch.argtypes = [vp]
    lib.wh2wav_forward_noalloc.argtypes = [vp, vp, vp, vp]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.wh2wav_batch_set_mode.argtypes = [vp, ctypes.c_int]
    lib.wh2wav_batch_mode.argtypes = [vp, ip, ip, ip]
    for name in EXPORTS:
        if name != "wh2wav_last_error":
            getattr(lib, name).restype = ctypes.c_int
    return lib


LIB = _load()


def _check(code):
    if code != WH2WAV_OK:
        raise Wh2WavError(code, LIB.wh2wav_last_error().decode())
    return code


def wh2wav_plan(desc):
    handle = ctypes.c_void_p()
    _check(LIB.wh2wav_plan(ctypes.byref(desc), ctypes.byref(handle)))
    return handle


def wh2wav_workspace_size(plan):
    n = ctypes.c_size_t()
    _check(LIB.wh2wav_workspace_size(plan, ctypes.byref(n)))
    return n.value


def wh2wav_forward(plan, x_ptr, y_ptr, ws_ptr, stream_ptr):
    return _check(LIB.wh2wav_forward(plan, x_ptr, y_ptr, ws_ptr, stream_ptr))


def wh2wav_forward_noalloc(plan, x_ptr, y_ptr, stream_ptr):
    return _check(LIB.wh2wav_forward_noalloc(plan, x_ptr, y_ptr, stream_ptr))


def wh2wav_adjoint(plan, y_ptr, x_ptr, ws_ptr, stream_ptr):
    return _check(LIB.wh2wav_adjoint(plan, y_ptr, x_ptr, ws_ptr, stream_ptr))


def wh2wav_stage_count(plan, direction):
    n = ctypes.c_int()
    _check(LIB.wh2wav_stage_count(plan, direction, ctypes.byref(n)))
    return n.value


def wh2wav_forward_stage(plan, stage, x_ptr, y_ptr, ws_ptr, stream_ptr):
    return _check(LIB.wh2wav_forward_stage(plan, stage, x_ptr, y_ptr, ws_ptr, stream_ptr))


def wh2wav_adjoint_stage(plan, stage, y_ptr, x_ptr, ws_ptr, stream_ptr):
    return _check(LIB.wh2wav_adjoint_stage(plan, stage, y_ptr, x_ptr, ws_ptr, stream_ptr))


def wh2wav_destroy(plan):
    return _check(LIB.wh2wav_destroy(plan))


def wh2wav_last_error():
    return LIB.wh2wav_last_error().decode()


def wh2wav_host_table(desc, which):
    """Return the float64 host table `which` (name or index) as a Python list."""
    idx = TABLES[which] if isinstance(which, str) else int(which)
    count = ctypes.c_size_t()
    _check(LIB.wh2wav_host_table(ctypes.byref(desc), idx, None, 0, ctypes.byref(count)))
    buf = (ctypes.c_double * max(count.value, 1))()
    _check(LIB.wh2wav_host_table(ctypes.byref(desc), idx, buf, count.value, ctypes.byref(count)))
    return list(buf[:count.value])


def _ptr_array(ptrs):
    return (ctypes.c_void_p * max(len(ptrs), 1))(*[ctypes.c_void_p(int(p)) for p in ptrs])


def wh2wav_plan_batch(descs):
    arr = (wh2wav_desc * len(descs))(*descs)
    handle = ctypes.c_void_p()
    _check(LIB.wh2wav_plan_batch(arr, len(descs), ctypes.byref(handle)))
    return handle


def wh2wav_batch_workspace_size(batch):
    n = ctypes.c_size_t()
    _check(LIB.wh2wav_batch_workspace_size(batch, ctypes.byref(n)))
    return n.value


def wh2wav_forward_batch(batch, x_ptrs, y_ptrs, ws_ptr, stream_ptr):
    return _check(LIB.wh2wav_forward_batch(batch, _ptr_array(x_ptrs), _ptr_array(y_ptrs), ws_ptr, stream_ptr))


def wh2wav_adjoint_batch(batch, y_ptrs, x_ptrs, ws_ptr, stream_ptr):
    return _check(LIB.wh2wav_adjoint_batch(batch, _ptr_array(y_ptrs), _ptr_array(x_ptrs), ws_ptr, stream_ptr))


def wh2wav_batch_schedule(batch):
    b, o = ctypes.c_int(), ctypes.c_int()
    _check(LIB.wh2wav_batch_schedule(batch, ctypes.byref(b), ctypes.byref(o)))
    return b.value, o.value


def wh2wav_batch_set_schedule(batch, branches, order):
    return _check(LIB.wh2wav_batch_set_schedule(batch, branches, order))


def wh2wav_batch_tune(batch, x_ptrs, y_ptrs, xa_ptrs, ws_ptr, stream_ptr, reps):
    best = ctypes.c_float()
    _check(LIB.wh2wav_batch_tune(batch, _ptr_array(x_ptrs), _ptr_array(y_ptrs), _ptr_array(xa_ptrs), ws_ptr,
                                 stream_ptr, reps, ctypes.byref(best)))
    return best.value


def wh2wav_destroy_batch(batch):
    return _check(LIB.wh2wav_destroy_batch(batch))


def wh2wav_batch_set_mode(batch, mode):
    return _check(LIB.wh2wav_batch_set_mode(batch, mode))


def wh2wav_batch_mode(batch):
    """(mode, instances in the fused launches, fused launches per forward call)."""
    mode, n, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(LIB.wh2wav_batch_mode(batch, ctypes.byref(mode), ctypes.byref(n), ctypes.byref(k)))
    return mode.value, n.value, k.value
