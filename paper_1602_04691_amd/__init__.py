"""Python binding of libori.so: argument marshalling only.

Every step of the solve runs in the library's HIP kernels.  PyTorch is used
for device memory and streams: arrays are CUDA (HIP) tensors of dtype
complex128 (h, u0, u, x, y) or float64 (N), contiguous, on the current device.

The functions mirror the C ABI in include/ori.h (same names).  A missing or
unloadable library raises at import time of the first call: there is no
CPU fallback.
"""

import ctypes
import os

__all__ = [
    "OriError", "lib", "Grid", "SolveOpts", "SolveInfo", "Context",
    "ori_setup", "ori_create", "ori_load", "ori_solve", "ori_matvec", "ori_destroy",
    "ori_workspace_bytes", "ori_default_opts", "ori_profile_enable", "ori_profile_read",
    "ori_last_error", "ori_version",
    "ORI_OK", "ORI_ERR_INVALID_ARG", "ORI_ERR_OUT_OF_MEMORY", "ORI_ERR_DEVICE",
    "ORI_ERR_BREAKDOWN", "ORI_ERR_NOT_CONVERGED", "ORI_ERR_UNSUPPORTED",
    "ORI_FP64", "ORI_MIXED", "ORI_OP_SYSTEM", "ORI_OP_SYMMETRIC", "ORI_OP_GREEN",
    "ORI_PROVISION_FP64", "ORI_PROVISION_MIXED", "LIB_PATH", "solve",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libori.so")

ORI_OK, ORI_ERR_INVALID_ARG, ORI_ERR_OUT_OF_MEMORY, ORI_ERR_DEVICE = 0, 1, 2, 3
ORI_ERR_BREAKDOWN, ORI_ERR_NOT_CONVERGED, ORI_ERR_UNSUPPORTED = 4, 5, 6
ORI_FP64, ORI_MIXED = 0, 1
ORI_OP_SYSTEM, ORI_OP_SYMMETRIC, ORI_OP_GREEN = 0, 1, 2
ORI_PROVISION_FP64, ORI_PROVISION_MIXED = 1, 2

_STATUS_NAMES = {
    0: "ORI_OK", 1: "ORI_ERR_INVALID_ARG", 2: "ORI_ERR_OUT_OF_MEMORY", 3: "ORI_ERR_DEVICE",
    4: "ORI_ERR_BREAKDOWN", 5: "ORI_ERR_NOT_CONVERGED", 6: "ORI_ERR_UNSUPPORTED",
}


class OriError(RuntimeError):
    def __init__(self, status, message, info=None):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message
        self.info = info


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("side", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("cell_offset", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("use_x0", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("true_residual", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("matvecs", ctypes.c_int64), ("matvecs_c64", ctypes.c_int64),
                ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """The loaded libori.so (loaded on first use; raises if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_1602_04691_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "ori_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
            "ori_version": (ctypes.c_char_p, []),
            "ori_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Grid), I32, ctypes.POINTER(I64)]),
            "ori_create": (ctypes.c_int, [ctypes.POINTER(Grid), I32, I64, P, ctypes.POINTER(P)]),
            "ori_load": (ctypes.c_int, [P, D, P, P, P]),
            "ori_setup": (ctypes.c_int, [ctypes.POINTER(Grid), D, P, P, P, P, ctypes.POINTER(P)]),
            "ori_solve": (ctypes.c_int, [P, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveInfo)]),
            "ori_matvec": (ctypes.c_int, [P, I32, I32, P, P]),
            "ori_profile_enable": (ctypes.c_int, [P, I32]),
            "ori_profile_read": (ctypes.c_int, [P, I32, ctypes.POINTER(ctypes.c_char_p),
                                                ctypes.POINTER(D), ctypes.POINTER(I64), ctypes.POINTER(I32)]),
            "ori_destroy": (None, [P]),
            "ori_last_error": (ctypes.c_char_p, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def ori_version():
    return lib().ori_version().decode()


def ori_last_error(ctx=None):
    h = ctx.handle if isinstance(ctx, Context) else ctx
    return lib().ori_last_error(h).decode()


def _check(status, ctx=None, info=None):
    if status != ORI_OK:
        raise OriError(status, ori_last_error(ctx), info)


def _grid(n, side=1.0, origin=(0.0, 0.0, 0.0), cell_offset=0.5):
    g = Grid()
    g.n = int(n)
    g.side = float(side)
    for i in range(3):
        g.origin[i] = float(origin[i])
    g.cell_offset = float(cell_offset)
    return g


def _dev(t, dtype, P, what):
    """Pointer of a contiguous CUDA tensor with P entries of dtype (or None)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor on the GPU")
    if not t.is_cuda:
        raise ValueError(f"{what} must live on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() != P:
        raise ValueError(f"{what} must have n^3 = {P} entries (got {t.numel()})")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """An ori_ctx plus the grid it was made for."""

    def __init__(self, handle, n, stream):
        self.handle = handle
        self.n = n
        self.P = n ** 3
        self.stream = stream

    def close(self):
        if self.handle:
            lib().ori_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def ori_default_opts():
    o = SolveOpts()
    lib().ori_default_opts(ctypes.byref(o))
    return o


def ori_workspace_bytes(n, provision=ORI_PROVISION_FP64 | ORI_PROVISION_MIXED, side=1.0):
    b = ctypes.c_int64()
    _check(lib().ori_workspace_bytes(ctypes.byref(_grid(n, side)), provision, ctypes.byref(b)))
    return b.value


def ori_create(n, side=1.0, origin=(0.0, 0.0, 0.0), cell_offset=0.5,
               provision=ORI_PROVISION_FP64 | ORI_PROVISION_MIXED, mem_limit_bytes=0, stream=None):
    import torch
    h = ctypes.c_void_p()
    st = _stream(stream)
    _check(lib().ori_create(ctypes.byref(_grid(n, side, origin, cell_offset)), provision,
                            int(mem_limit_bytes), st, ctypes.byref(h)))
    return Context(h, int(n), stream if stream is not None else torch.cuda.current_stream())


def ori_load(ctx, k, h, N, u0):
    import torch
    _check(lib().ori_load(ctx.handle, float(k), _dev(h, torch.complex128, ctx.P, "h"),
                          _dev(N, torch.float64, ctx.P, "N"), _dev(u0, torch.complex128, ctx.P, "u0")), ctx)


def ori_setup(n, k, h, N, u0, side=1.0, origin=(0.0, 0.0, 0.0), cell_offset=0.5, stream=None):
    import torch
    P = int(n) ** 3
    hdl = ctypes.c_void_p()
    st = _stream(stream)
    _check(lib().ori_setup(ctypes.byref(_grid(n, side, origin, cell_offset)), float(k),
                           _dev(h, torch.complex128, P, "h"), _dev(N, torch.float64, P, "N"),
                           _dev(u0, torch.complex128, P, "u0"), st, ctypes.byref(hdl)))
    return Context(hdl, int(n), stream if stream is not None else torch.cuda.current_stream())


def ori_solve(ctx, u, tol=1e-10, max_iter=1000, precision=ORI_FP64, check_every=1, use_x0=False,
              inner_tol=1e-5, max_outer=10, true_residual=True, raise_on_error=True):
    """Solve into u (complex128 CUDA tensor, n^3).  Returns (status, info dict)."""
    import torch
    o = SolveOpts(float(tol), int(max_iter), int(precision), int(check_every), int(bool(use_x0)),
                  float(inner_tol), int(max_outer), int(bool(true_residual)))
    info = SolveInfo()
    st = lib().ori_solve(ctx.handle, ctypes.byref(o), _dev(u, torch.complex128, ctx.P, "u"), ctypes.byref(info))
    d = info.as_dict()
    if raise_on_error:
        _check(st, ctx, d)
    return st, d


def ori_matvec(ctx, x, y, op=ORI_OP_SYSTEM, precision=ORI_FP64):
    import torch
    _check(lib().ori_matvec(ctx.handle, int(op), int(precision), _dev(x, torch.complex128, ctx.P, "x"),
                            _dev(y, torch.complex128, ctx.P, "y")), ctx)


def ori_destroy(ctx):
    ctx.close()


def ori_profile_enable(ctx, enable=True):
    _check(lib().ori_profile_enable(ctx.handle, int(bool(enable))), ctx)


def ori_profile_read(ctx, max_kinds=64):
    names = (ctypes.c_char_p * max_kinds)()
    avg = (ctypes.c_double * max_kinds)()
    cnt = (ctypes.c_int64 * max_kinds)()
    count = ctypes.c_int32()
    _check(lib().ori_profile_read(ctx.handle, max_kinds, names, avg, cnt, ctypes.byref(count)), ctx)
    return {names[i].decode(): (avg[i], cnt[i]) for i in range(min(count.value, max_kinds))}


def solve(n, k, h, N, u0, side=1.0, origin=(0.0, 0.0, 0.0), cell_offset=0.5, **opts):
    """One-shot convenience: setup, solve, destroy.  Returns (u, info)."""
    import torch
    with ori_setup(n, k, h, N, u0, side, origin, cell_offset) as ctx:
        u = torch.empty(int(n) ** 3, dtype=torch.complex128, device=h.device)
        _, info = ori_solve(ctx, u, **opts)
    return u, info
