"""ctypes binding of libfirls.so (include/firls.h), same names as the C ABI.

Only argument marshalling lives here: every step of a solve runs in the HIP
kernels of the library.  Device buffers are torch tensors on the current
HIP device (``torch.cuda``); streams are torch streams.  There is no CPU
fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfirls.so")

FIRLS_OK = 0
FIRLS_E_INVALID = -1
FIRLS_E_UNSUPPORTED = -2
FIRLS_E_HIP = -3
FIRLS_E_NOMEM = -4
FIRLS_E_NONFINITE = -5
FIRLS_E_SYNC = -6
FIRLS_E_BREAKDOWN = -7
FIRLS_W_MAXITER = 1
FIRLS_W_NONMONOTONE = 2
FIRLS_SCHED_PER_SHAPE = 0
FIRLS_SCHED_ACROSS = 1
FIRLS_SCHED_ACROSS_LARGEST_FIRST = 2
FIRLS_TEST_SYNC_TIMEOUT = 1
FIRLS_TEST_BREAKDOWN = 2
FIRLS_TEST_NONMONOTONE = 4
FIRLS_PSI_HAAR = 0
FIRLS_PSI_TV = 1
FIRLS_PSI_TV_PAPER = 2
FIRLS_OP_FOURIER = 0
FIRLS_OP_DENSE = 1
FIRLS_FP64 = 0
FIRLS_FP32 = 1
FIRLS_PC_PAPER = 0
FIRLS_PC_JACOBI = 1
FIRLS_PC_NONE = 2

EXPORTED = (
    "firls_create", "firls_destroy", "firls_workspace_bytes", "firls_slice_workspace_bytes", "firls_solve",
    "firls_solve_batched", "firls_solve_batched_noalloc", "firls_op_adjoint", "firls_op_weights",
    "firls_op_system", "firls_op_precond", "firls_op_objective",
    "firls_op_outer_step", "firls_profile", "firls_profile_read", "firls_profile_read_shape", "firls_last_error",
    "firls_cnn_param_count", "firls_cnn_create", "firls_cnn_destroy", "firls_cnn_set_params",
    "firls_cnn_get_params", "firls_cnn_forward", "firls_cnn_gradients", "firls_cnn_train_step",
    "firls_solve_batched_learned", "firls_set_graphs", "firls_set_chunk", "firls_set_paired", "firls_test_sync_timeout", "firls_test_hooks", "firls_autotune",
    "firls_set_schedule", "firls_get_schedule", "firls_get_paired",
)
PROF_CLASSES = 15


class firls_shape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("psi", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("n_groups", ctypes.c_int32), ("group_ptr", ctypes.POINTER(ctypes.c_int32)),
                ("group_idx", ctypes.POINTER(ctypes.c_int32)), ("channels", ctypes.c_int32),
                ("op", ctypes.c_int32), ("m", ctypes.c_int32), ("A", ctypes.POINTER(ctypes.c_double))]


class firls_config(ctypes.Structure):
    _fields_ = [("n_shapes", ctypes.c_int32), ("shapes", ctypes.POINTER(firls_shape)),
                ("max_slices", ctypes.c_int32), ("prec", ctypes.c_int32), ("eps", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("pcg_iters", ctypes.c_int32),
                ("outer_tol", ctypes.c_double), ("pcg_rtol", ctypes.c_double), ("precond", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class firls_slice(ctypes.Structure):
    _fields_ = [("shape_id", ctypes.c_int32), ("x_is_init", ctypes.c_int32), ("lambda_", ctypes.c_double),
                ("b", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("x", ctypes.c_void_p)]


class firls_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("slice_launches", ctypes.c_int64), ("ms", ctypes.c_double)]


class firls_report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("pcg_iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("F", ctypes.c_double), ("F_eps", ctypes.c_double),
                ("data", ctypes.c_double), ("rel_change", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# numpy views of the two batch records (same layout as the structures
# above), so a batch is marshalled column by column
SLICE_DTYPE = np.dtype([("shape_id", "<i4"), ("x_is_init", "<i4"), ("lambda_", "<f8"), ("b", "<u8"),
                        ("mask", "<u8"), ("x", "<u8")])
REPORT_DTYPE = np.dtype([("status", "<i4"), ("outer_iters", "<i4"), ("pcg_iters", "<i4"), ("converged", "<i4"),
                         ("F", "<f8"), ("F_eps", "<f8"), ("data", "<f8"), ("rel_change", "<f8")])
for _dt, _st in ((SLICE_DTYPE, firls_slice), (REPORT_DTYPE, firls_report)):
    assert _dt.itemsize == ctypes.sizeof(_st)
    assert all(_dt.fields[f][1] == getattr(_st, f).offset for f, _ in _st._fields_)


def check_tensor(t, what: str, dtype, numel: int, allow_none: bool = False, device: bool = True) -> None:
    """Rejects a buffer the kernels would misread: it must be a contiguous
    torch tensor of ``dtype`` with ``numel`` elements on the GPU (None only
    where ``allow_none``; ``device=False`` skips the device check).  The
    device is checked last, so every other check can be exercised with host
    tensors."""
    if t is None:
        if allow_none:
            return
        raise ValueError(f"{what} is required")
    if not hasattr(t, "data_ptr") or not hasattr(t, "is_contiguous"):
        raise TypeError(f"{what} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")
    if device and t.device.type != "cuda":
        raise ValueError(f"{what} must be on the GPU, got device {t.device}")


def _dtypes(prec: str):
    import torch
    return (torch.complex64, torch.float32) if prec == "fp32" else (torch.complex128, torch.float64)


def check_slice_item(it: dict, shapes, prec: str) -> None:
    """b, mask and x of one batch item against its shape: b holds n^2 C
    complex values (m for a dense sensing matrix), mask n^2 C bytes (may be
    None for a dense matrix), x n^2 C complex values."""
    import torch
    sid = int(it.get("shape_id", 0))
    if not 0 <= sid < len(shapes):
        raise ValueError(f"shape_id {sid} out of range")
    sh = shapes[sid]
    cplx, _ = _dtypes(prec)
    npx = sh.n * sh.n * sh.channels
    dense = sh.A is not None
    for dev in (False, True):    # every buffer's layout first, then where they live
        check_tensor(it["b"], "b", cplx, sh.A.shape[0] if dense else npx, device=dev)
        check_tensor(it["mask"], "mask", torch.uint8, npx, allow_none=dense, device=dev)
        check_tensor(it["x"], "x", cplx, npx, device=dev)


def slice_array(items, init: Optional[bool] = None, shapes=None, prec: Optional[str] = None) -> np.ndarray:
    """items (dicts with b, mask, x, lam, shape_id, x_is_init) -> firls_slice
    records; ``init`` overrides every x_is_init.  With ``shapes`` and
    ``prec`` every item's tensors are checked first (check_slice_item)."""
    if shapes is not None:
        for it in items:
            check_slice_item(it, shapes, prec)
    a = np.empty(len(items), SLICE_DTYPE)
    a["shape_id"] = [it.get("shape_id", 0) for it in items]
    a["x_is_init"] = ([bool(it.get("x_is_init", False)) for it in items] if init is None else bool(init))
    a["lambda_"] = [it["lam"] for it in items]
    a["b"] = [_ptr(it["b"]) for it in items]
    a["mask"] = [_ptr(it["mask"]) for it in items]
    a["x"] = [_ptr(it["x"]) for it in items]
    return a


def report_dicts(r: np.ndarray) -> List[dict]:
    names = r.dtype.names
    return [dict(zip(names, t)) for t in r.tolist()]


def _as(a: np.ndarray, st):
    return a.ctypes.data_as(ctypes.POINTER(st))


class Batch:
    """A batch marshalled once, for repeated solves of the same buffers (a
    serving loop that refills b, mask and x in place).  Holds the items, so
    their tensors stay alive.  Solves of a Batch return the reports as a
    numpy structured array with the fields of firls_report (one record per
    slice, in item order)."""

    def __init__(self, items: List[dict], init: Optional[bool] = None, shapes=None, prec: Optional[str] = None):
        self.items = list(items)
        self.slices = slice_array(self.items, init, shapes, prec)
        self.reports = np.zeros(len(self.items), REPORT_DTYPE)
        self.used = np.zeros(len(self.items), np.int32)

    def __len__(self):
        return len(self.items)


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfirls.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1411_5057_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sig = {
        "firls_create": ([ctypes.POINTER(firls_config), ctypes.POINTER(vp)], ctypes.c_int),
        "firls_destroy": ([vp], ctypes.c_int),
        "firls_workspace_bytes": ([ctypes.POINTER(firls_config)], ctypes.c_size_t),
        "firls_slice_workspace_bytes": ([vp, i32, i32], ctypes.c_size_t),
        "firls_solve": ([vp, vp, ctypes.POINTER(firls_slice), ctypes.POINTER(firls_report)], ctypes.c_int),
        "firls_solve_batched": ([vp, vp, i32, ctypes.POINTER(firls_slice), ctypes.POINTER(firls_report)], ctypes.c_int),
        "firls_solve_batched_noalloc": ([vp, vp, i32, ctypes.POINTER(firls_slice), ctypes.POINTER(firls_report)],
                                        ctypes.c_int),
        "firls_op_adjoint": ([vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "firls_op_weights": ([vp, vp, i32, vp, vp], ctypes.c_int),
        "firls_op_system": ([vp, vp, i32, vp, dbl, vp, vp, vp], ctypes.c_int),
        "firls_op_precond": ([vp, vp, i32, vp, dbl, vp, vp, vp], ctypes.c_int),
        "firls_op_objective": ([vp, vp, i32, vp, vp, dbl, vp, ctypes.POINTER(dbl)], ctypes.c_int),
        "firls_op_outer_step": ([vp, vp, i32, vp, vp, dbl, vp], ctypes.c_int),
        "firls_profile": ([vp, i32], ctypes.c_int),
        "firls_profile_read": ([vp, i32, ctypes.POINTER(firls_kernel_stat)], ctypes.c_int),
        "firls_profile_read_shape": ([vp, i32, i32, ctypes.POINTER(firls_kernel_stat)], ctypes.c_int),
        "firls_last_error": ([], ctypes.c_char_p),
        "firls_set_graphs": ([vp, i32], ctypes.c_int),
        "firls_set_chunk": ([vp, i32], ctypes.c_int),
        "firls_set_paired": ([vp, i32], ctypes.c_int),
        "firls_test_sync_timeout": ([vp, i32], ctypes.c_int),
        "firls_test_hooks": ([vp, i32], ctypes.c_int),
        "firls_set_schedule": ([vp, i32], ctypes.c_int),
        "firls_get_schedule": ([vp], ctypes.c_int),
        "firls_get_paired": ([vp], ctypes.c_int),
        "firls_autotune": ([vp, vp, i32, ctypes.POINTER(firls_slice), ctypes.POINTER(i32), ctypes.POINTER(i32)],
                           ctypes.c_int),
        "firls_cnn_param_count": ([], ctypes.c_int32),
        "firls_cnn_create": ([i32, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "firls_cnn_destroy": ([vp], ctypes.c_int),
        "firls_cnn_set_params": ([vp, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "firls_cnn_get_params": ([vp, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "firls_cnn_forward": ([vp, vp, i32, vp, vp], ctypes.c_int),
        "firls_cnn_gradients": ([vp, vp, i32, vp, vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(dbl)], ctypes.c_int),
        "firls_cnn_train_step": ([vp, vp, i32, vp, vp, ctypes.c_float, ctypes.POINTER(dbl)], ctypes.c_int),
        "firls_solve_batched_learned": ([vp, vp, vp, i32, ctypes.POINTER(firls_slice), ctypes.POINTER(firls_report),
                                         ctypes.POINTER(i32)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def firls_last_error() -> str:
    return load().firls_last_error().decode()


class FirlsError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where} failed with {code}: {firls_last_error()}")
        self.code = code


def _check(code: int, where: str) -> int:
    if code < 0:
        raise FirlsError(code, where)
    return code


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def firls_create(cfg: firls_config) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().firls_create(ctypes.byref(cfg), ctypes.byref(h)), "firls_create")
    return h


def firls_destroy(h) -> int:
    return load().firls_destroy(h)


def firls_workspace_bytes(cfg: firls_config) -> int:
    return int(load().firls_workspace_bytes(ctypes.byref(cfg)))


def firls_slice_workspace_bytes(h, shape_id: int, n: int) -> int:
    return int(load().firls_slice_workspace_bytes(h, shape_id, n))


def firls_solve(h, stream, sl: firls_slice, rep: firls_report) -> int:
    return _check(load().firls_solve(h, stream, ctypes.byref(sl), ctypes.byref(rep)), "firls_solve")


def firls_solve_batched(h, stream, n: int, slices, reports) -> int:
    return _check(load().firls_solve_batched(h, stream, n, slices, reports), "firls_solve_batched")


def firls_solve_batched_noalloc(h, stream, n: int, slices, reports) -> int:
    return _check(load().firls_solve_batched_noalloc(h, stream, n, slices, reports), "firls_solve_batched_noalloc")


def firls_op_adjoint(h, stream, shape_id, b, mask, x) -> int:
    return _check(load().firls_op_adjoint(h, stream, shape_id, b, mask, x), "firls_op_adjoint")


def firls_op_weights(h, stream, shape_id, x, d_out) -> int:
    return _check(load().firls_op_weights(h, stream, shape_id, x, d_out), "firls_op_weights")


def firls_op_system(h, stream, shape_id, mask, lam, x_w, p, q) -> int:
    return _check(load().firls_op_system(h, stream, shape_id, mask, lam, x_w, p, q), "firls_op_system")


def firls_op_precond(h, stream, shape_id, mask, lam, x_w, r, z) -> int:
    return _check(load().firls_op_precond(h, stream, shape_id, mask, lam, x_w, r, z), "firls_op_precond")


def firls_op_objective(h, stream, shape_id, b, mask, lam, x):
    out = (ctypes.c_double * 3)()
    _check(load().firls_op_objective(h, stream, shape_id, b, mask, lam, x, out), "firls_op_objective")
    return tuple(out)


def firls_op_outer_step(h, stream, shape_id, b, mask, lam, x) -> int:
    return _check(load().firls_op_outer_step(h, stream, shape_id, b, mask, lam, x), "firls_op_outer_step")


def firls_profile(h, enable: bool) -> int:
    return _check(load().firls_profile(h, int(enable)), "firls_profile")


def firls_profile_read(h) -> dict:
    arr = (firls_kernel_stat * PROF_CLASSES)()
    m = _check(load().firls_profile_read(h, PROF_CLASSES, arr), "firls_profile_read")
    return {arr[i].name.decode(): {"launches": arr[i].launches, "slice_launches": arr[i].slice_launches,
                                   "ms": arr[i].ms} for i in range(m)}


def firls_profile_read_shape(h, shape_id: int) -> dict:
    arr = (firls_kernel_stat * PROF_CLASSES)()
    m = _check(load().firls_profile_read_shape(h, shape_id, PROF_CLASSES, arr), "firls_profile_read_shape")
    return {arr[i].name.decode(): {"launches": arr[i].launches, "slice_launches": arr[i].slice_launches,
                                   "ms": arr[i].ms} for i in range(m)}


def firls_cnn_param_count() -> int:
    return int(load().firls_cnn_param_count())


def firls_cnn_create(n: int, max_batch: int):
    h = ctypes.c_void_p()
    _check(load().firls_cnn_create(n, max_batch, ctypes.byref(h)), "firls_cnn_create")
    return h


def firls_cnn_destroy(h) -> int:
    return load().firls_cnn_destroy(h)


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def firls_cnn_set_params(h, params: np.ndarray) -> int:
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == firls_cnn_param_count()
    return _check(load().firls_cnn_set_params(h, _fptr(p)), "firls_cnn_set_params")


def firls_cnn_get_params(h) -> np.ndarray:
    p = np.empty(firls_cnn_param_count(), dtype=np.float32)
    _check(load().firls_cnn_get_params(h, _fptr(p)), "firls_cnn_get_params")
    return p


def firls_cnn_forward(h, stream, batch, zf, x0) -> int:
    return _check(load().firls_cnn_forward(h, stream, batch, zf, x0), "firls_cnn_forward")


def firls_cnn_gradients(h, stream, batch, zf, label):
    g = np.empty(firls_cnn_param_count(), dtype=np.float32)
    loss = ctypes.c_double()
    _check(load().firls_cnn_gradients(h, stream, batch, zf, label, _fptr(g), ctypes.byref(loss)),
           "firls_cnn_gradients")
    return g, loss.value


def firls_cnn_train_step(h, stream, batch, zf, label, lr: float) -> float:
    loss = ctypes.c_double()
    _check(load().firls_cnn_train_step(h, stream, batch, zf, label, float(lr), ctypes.byref(loss)),
           "firls_cnn_train_step")
    return loss.value


def firls_solve_batched_learned(h, net, stream, n, slices, reports, used) -> int:
    return _check(load().firls_solve_batched_learned(h, net, stream, n, slices, reports, used),
                  "firls_solve_batched_learned")


def flatten_params(layers) -> np.ndarray:
    """[(W [3,3,cin,cout], b [cout]) x 5] -> the ABI's float32 parameter order."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float64).ravel(), np.asarray(b, np.float64).ravel()])
                           for W, b in layers]).astype(np.float32)


def unflatten_params(flat: np.ndarray, channels=(2, 32, 32, 32, 32, 2)):
    out, o = [], 0
    for i in range(5):
        cin, cout = channels[i], channels[i + 1]
        W = flat[o:o + 9 * cin * cout].reshape(3, 3, cin, cout)
        o += 9 * cin * cout
        b = flat[o:o + cout]
        o += cout
        out.append((W.astype(np.float64), b.astype(np.float64)))
    return out


class Net:
    """Owns a firls_cnn (warm-start network for n x n images)."""

    def __init__(self, n: int, max_batch: int, params: Optional[np.ndarray] = None):
        self.n, self.max_batch = n, max_batch
        self.handle = firls_cnn_create(n, max_batch)
        if params is not None:
            self.set_params(params)

    def close(self):
        if self.handle:
            firls_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        firls_cnn_set_params(self.handle, params)

    def get_params(self) -> np.ndarray:
        return firls_cnn_get_params(self.handle)

    def _batch(self, *ts) -> int:
        """Checks complex64 [batch, n, n] buffers of one batch size."""
        import torch
        batch = int(ts[0].shape[0]) if hasattr(ts[0], "shape") and len(ts[0].shape) else 0
        if not 1 <= batch <= self.max_batch:
            raise ValueError(f"batch must be in 1..{self.max_batch}, got {batch}")
        for i, t in enumerate(ts):
            check_tensor(t, f"network buffer {i}", torch.complex64, batch * self.n * self.n)
        return batch

    def forward(self, zf, x0, stream=None):
        firls_cnn_forward(self.handle, _stream(stream), self._batch(zf, x0), _ptr(zf), _ptr(x0))

    def gradients(self, zf, label, stream=None):
        return firls_cnn_gradients(self.handle, _stream(stream), self._batch(zf, label), _ptr(zf), _ptr(label))

    def train_step(self, zf, label, lr, stream=None) -> float:
        return firls_cnn_train_step(self.handle, _stream(stream), self._batch(zf, label), _ptr(zf), _ptr(label), lr)


# ---------------------------------------------------------------------------
# Convenience layer over torch tensors
# ---------------------------------------------------------------------------

class Shape:
    """Python description of a firls_shape (group map as int32 numpy CSR)."""

    def __init__(self, n: int, psi: str, levels: int = 0, group_ptr=None, group_idx=None, channels: int = 1,
                 A=None):
        """A: optional dense sensing matrix (M x n^2, float64) in place of the
        masked FFT."""
        self.n, self.psi, self.levels, self.channels = int(n), psi, int(levels), int(channels)
        self.A = None if A is None else np.ascontiguousarray(A, dtype=np.float64)
        self.group_ptr = None if group_ptr is None else np.ascontiguousarray(group_ptr, dtype=np.int32)
        self.group_idx = None if group_idx is None else np.ascontiguousarray(group_idx, dtype=np.int32)

    def c(self) -> firls_shape:
        s = firls_shape()
        s.n = self.n
        s.psi = {"haar": FIRLS_PSI_HAAR, "tv": FIRLS_PSI_TV, "tvp": FIRLS_PSI_TV_PAPER}[self.psi]
        s.levels = self.levels
        s.channels = self.channels
        if self.A is not None:
            s.op = FIRLS_OP_DENSE
            s.m = self.A.shape[0]
            s.A = self.A.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if self.group_ptr is not None:
            s.n_groups = len(self.group_ptr) - 1
            s.group_ptr = self.group_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            s.group_idx = self.group_idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        return s


class Solver:
    """Owns a firls_handle.  Tensors: b, x complex64 (FP32) / complex128
    (FP64) n x n on the GPU, mask uint8 n x n (C x n x n, contiguous, for a
    shape with C contrasts)."""

    def __init__(self, shapes: Sequence[Shape], *, prec: str = "fp32", max_slices: int = 1,
                 eps: float = 1e-10, max_outer: int = 50, pcg_iters: int = 20,
                 outer_tol: float = 0.0, pcg_rtol: float = 0.0, precond: int = FIRLS_PC_PAPER,
                 workspace=None):
        """workspace: None (the library allocates its own), True (a torch
        buffer of firls_workspace_bytes(cfg) is allocated here and handed
        over), or a contiguous uint8 torch tensor on the GPU of at least
        that size; it is kept alive as long as the solver."""
        self.shapes = list(shapes)
        self._cshapes = (firls_shape * len(self.shapes))(*[s.c() for s in self.shapes])
        cfg = firls_config()
        cfg.n_shapes = len(self.shapes)
        cfg.shapes = self._cshapes
        cfg.max_slices = max_slices
        cfg.prec = FIRLS_FP32 if prec == "fp32" else FIRLS_FP64
        cfg.eps = eps
        cfg.max_outer = max_outer
        cfg.pcg_iters = pcg_iters
        cfg.outer_tol = outer_tol
        cfg.pcg_rtol = pcg_rtol
        cfg.precond = precond
        self.workspace = None
        if workspace is not None and workspace is not False:
            import torch
            need = firls_workspace_bytes(cfg)
            if workspace is True:
                workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
            check_tensor(workspace, "workspace", torch.uint8, workspace.numel())
            cfg.workspace = int(workspace.data_ptr())
            cfg.workspace_bytes = int(workspace.numel())
            self.workspace = workspace
        self.cfg = cfg
        self.prec = prec
        self.handle = firls_create(cfg)
        self.graphs = True

    def close(self):
        if self.handle:
            firls_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, it: dict) -> None:
        check_slice_item(it, self.shapes, self.prec)

    def _npx(self, shape_id: int) -> int:
        if not 0 <= shape_id < len(self.shapes):
            raise ValueError(f"shape_id {shape_id} out of range")
        sh = self.shapes[shape_id]
        return sh.n * sh.n * sh.channels

    def _vec(self, t, what: str, shape_id: int) -> None:
        check_tensor(t, what, _dtypes(self.prec)[0], self._npx(shape_id))

    def _mask(self, m, shape_id: int) -> None:
        import torch
        check_tensor(m, "mask", torch.uint8, self._npx(shape_id), allow_none=self.shapes[shape_id].A is not None)

    def solve(self, b, mask, x, lam: float, shape_id: int = 0, x_is_init: bool = False, stream=None) -> dict:
        self._check(dict(b=b, mask=mask, x=x, shape_id=shape_id))
        sl = firls_slice(shape_id, int(x_is_init), float(lam), _ptr(b), _ptr(mask), _ptr(x))
        rep = firls_report()
        firls_solve(self.handle, _stream(stream), sl, rep)
        return rep.as_dict()

    def prepare(self, items: List[dict], learned: bool = False) -> Batch:
        """Marshal a batch once (``learned``: for solve_batched_learned, whose
        slices all count as initialised)."""
        return Batch(items, True if learned else None, self.shapes, self.prec)

    def solve_batched(self, items, stream=None):
        """items: dicts with b, mask, x, lam, shape_id (0), x_is_init (False),
        or a Batch from prepare().  Returns one report dict per item (a
        structured array for a Batch)."""
        if isinstance(items, Batch):
            firls_solve_batched(self.handle, _stream(stream), len(items), _as(items.slices, firls_slice),
                                _as(items.reports, firls_report))
            return items.reports.copy()
        arr = slice_array(items, None, self.shapes, self.prec)
        reps = np.zeros(len(items), REPORT_DTYPE)
        firls_solve_batched(self.handle, _stream(stream), len(items), _as(arr, firls_slice), _as(reps, firls_report))
        return report_dicts(reps)

    def solve_batched_noalloc(self, items, stream=None):
        """firls_solve_batched_noalloc: as solve_batched, with every device
        buffer of the solve in the library's fixed per-GPU scratch (nothing
        is allocated); items as for solve_batched."""
        if isinstance(items, Batch):
            firls_solve_batched_noalloc(self.handle, _stream(stream), len(items), _as(items.slices, firls_slice),
                                        _as(items.reports, firls_report))
            return items.reports.copy()
        arr = slice_array(items, None, self.shapes, self.prec)
        reps = np.zeros(len(items), REPORT_DTYPE)
        firls_solve_batched_noalloc(self.handle, _stream(stream), len(items), _as(arr, firls_slice),
                                    _as(reps, firls_report))
        return report_dicts(reps)

    # single-operator entry points
    def adjoint(self, b, mask, x, shape_id=0, stream=None):
        self._check(dict(b=b, mask=mask, x=x, shape_id=shape_id))
        firls_op_adjoint(self.handle, _stream(stream), shape_id, _ptr(b), _ptr(mask), _ptr(x))

    def weights(self, x, d_out, shape_id=0, stream=None):
        self._vec(x, "x", shape_id)
        ncoef = self._npx(shape_id) * (1 if self.shapes[shape_id].psi == "haar" else 2)
        check_tensor(d_out, "d_out", _dtypes(self.prec)[1], ncoef)
        firls_op_weights(self.handle, _stream(stream), shape_id, _ptr(x), _ptr(d_out))

    def system(self, mask, lam, x_w, p, q, shape_id=0, stream=None):
        self._mask(mask, shape_id)
        for t, w in ((x_w, "x_w"), (p, "p"), (q, "q")):
            self._vec(t, w, shape_id)
        firls_op_system(self.handle, _stream(stream), shape_id, _ptr(mask), float(lam), _ptr(x_w), _ptr(p), _ptr(q))

    def precond(self, mask, lam, x_w, r, z, shape_id=0, stream=None):
        self._mask(mask, shape_id)
        for t, w in ((x_w, "x_w"), (r, "r"), (z, "z")):
            self._vec(t, w, shape_id)
        firls_op_precond(self.handle, _stream(stream), shape_id, _ptr(mask), float(lam), _ptr(x_w), _ptr(r), _ptr(z))

    def objective(self, b, mask, lam, x, shape_id=0, stream=None):
        self._check(dict(b=b, mask=mask, x=x, shape_id=shape_id))
        return firls_op_objective(self.handle, _stream(stream), shape_id, _ptr(b), _ptr(mask), float(lam), _ptr(x))

    def solve_batched_learned(self, net: "Net", items, stream=None):
        """Like solve_batched, started from the network (returns reports and
        the per-slice flag of whether the learned start was kept).  items may
        be a Batch from prepare(..., learned=True)."""
        if isinstance(items, Batch):
            firls_solve_batched_learned(self.handle, net.handle, _stream(stream), len(items),
                                        _as(items.slices, firls_slice), _as(items.reports, firls_report),
                                        _as(items.used, ctypes.c_int32))
            return items.reports.copy(), items.used.copy()
        arr = slice_array(items, True, self.shapes, self.prec)
        reps = np.zeros(len(items), REPORT_DTYPE)
        used = np.zeros(len(items), np.int32)
        firls_solve_batched_learned(self.handle, net.handle, _stream(stream), len(items), _as(arr, firls_slice),
                                    _as(reps, firls_report), _as(used, ctypes.c_int32))
        return report_dicts(reps), [int(u) for u in used]

    def set_graphs(self, enable: bool):
        _check(load().firls_set_graphs(self.handle, int(enable)), "firls_set_graphs")
        self.graphs = bool(enable)

    def set_chunk(self, chunk: int):
        _check(load().firls_set_chunk(self.handle, int(chunk)), "firls_set_chunk")

    def set_paired(self, enable: bool):
        _check(load().firls_set_paired(self.handle, int(enable)), "firls_set_paired")

    def test_sync_timeout(self, enable: bool):
        """Test hook: the paired pass's barrier times out at once (FIRLS_E_SYNC)."""
        _check(load().firls_test_sync_timeout(self.handle, int(enable)), "firls_test_sync_timeout")

    def set_schedule(self, schedule: int):
        """FIRLS_SCHED_*: per-shape launches or one launch per kernel class
        and position across the shapes of a mixed batch."""
        _check(load().firls_set_schedule(self.handle, int(schedule)), "firls_set_schedule")

    @property
    def schedule(self) -> int:
        return _check(load().firls_get_schedule(self.handle), "firls_get_schedule")

    @property
    def paired(self) -> bool:
        """Whether the paired PCG pass is on (set_paired, autotune)."""
        return _check(load().firls_get_paired(self.handle), "firls_get_paired") == 1

    def test_hooks(self, flags: int):
        """Test hooks (FIRLS_TEST_* bits; 0 clears them): forced conditions
        that make the error paths run."""
        _check(load().firls_test_hooks(self.handle, int(flags)), "firls_test_hooks")

    def autotune(self, items: List[dict], stream=None) -> int:
        """Picks the sub-batch size (returned), the launch mode (kept in
        ``self.graphs``: True for graph replay), the mixed-batch schedule and
        whether the paired PCG pass runs (``self.paired``) for these slices."""
        arr = slice_array(items, None, self.shapes, self.prec)
        chosen, graphs = ctypes.c_int32(), ctypes.c_int32()
        _check(load().firls_autotune(self.handle, _stream(stream), len(items), _as(arr, firls_slice),
                                     ctypes.byref(chosen), ctypes.byref(graphs)),
               "firls_autotune")
        self.graphs = bool(graphs.value)
        return chosen.value

    def profile(self, enable: bool):
        firls_profile(self.handle, enable)

    def profile_read(self, shape_id: Optional[int] = None) -> dict:
        """Per-class kernel totals, of every launch or of one shape's."""
        if shape_id is None:
            return firls_profile_read(self.handle)
        return firls_profile_read_shape(self.handle, shape_id)

    def outer_step(self, b, mask, lam, x, shape_id=0, stream=None):
        self._check(dict(b=b, mask=mask, x=x, shape_id=shape_id))
        firls_op_outer_step(self.handle, _stream(stream), shape_id, _ptr(b), _ptr(mask), float(lam), _ptr(x))
