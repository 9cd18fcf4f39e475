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
    "OriError", "lib", "Grid", "SolveOpts", "SolveInfo", "Layout", "Context",
    "ori_setup", "ori_create", "ori_load", "ori_spectrum_cache", "ori_solve", "ori_matvec", "ori_green_noalloc", "ori_destroy",
    "ori_adjoint", "ori_gradient", "OriSolve", "ori_batch_info",
    "ori_charges", "ori_scattered_field", "ori_far_field",
    "ori_refraction_index", "ori_design_impedance", "ori_interpolation_difference",
    "ori_get_layout", "ori_set_layout", "ori_tune", "ori_check_guards",
    "ori_workspace_bytes", "ori_default_opts", "ori_profile_enable", "ori_profile_kinds", "ori_profile_read",
    "ori_last_error", "ori_version",
    "ORI_OK", "ORI_ERR_INVALID_ARG", "ORI_ERR_OUT_OF_MEMORY", "ORI_ERR_DEVICE",
    "ORI_ERR_BREAKDOWN", "ORI_ERR_NOT_CONVERGED", "ORI_ERR_UNSUPPORTED",
    "ORI_FP64", "ORI_MIXED", "ORI_OP_SYSTEM", "ORI_OP_SYMMETRIC", "ORI_OP_GREEN",
    "ORI_PROVISION_FP64", "ORI_PROVISION_MIXED", "LIB_PATH", "solve", "solve_many",
    "Group", "ori_group_create", "ori_group_load", "ori_group_load_all", "ori_group_solve", "ori_group_destroy",
    "ori_group_multi_iterations", "ori_release_cached_memory",
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
                ("max_outer", ctypes.c_int32), ("true_residual", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("multi", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("matvecs", ctypes.c_int64), ("matvecs_c64", ctypes.c_int64),
                ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Layout(ctypes.Structure):
    _fields_ = [("blk_lg", ctypes.c_int32), ("narrow", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("znarrow", ctypes.c_int32), ("zplan", ctypes.c_int32)]

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
            "ori_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Grid), I32, I32, ctypes.POINTER(I64)]),
            "ori_create": (ctypes.c_int, [ctypes.POINTER(Grid), I32, I32, I64, P, ctypes.POINTER(P)]),
            "ori_batch_info": (ctypes.c_int, [P, I32, ctypes.POINTER(SolveInfo)]),
            "ori_group_create": (ctypes.c_int, [ctypes.POINTER(Grid), I32, I32, P, ctypes.POINTER(P)]),
            "ori_group_load": (ctypes.c_int, [P, I32, D, P, P, P]),
            "ori_group_load_all": (ctypes.c_int, [P, ctypes.POINTER(D), ctypes.POINTER(P), ctypes.POINTER(P),
                                                  ctypes.POINTER(P)]),
            "ori_group_solve": (ctypes.c_int, [P, ctypes.POINTER(SolveOpts), ctypes.POINTER(P),
                                               ctypes.POINTER(SolveInfo)]),
            "ori_group_destroy": (None, [P]),
            "ori_group_multi_iterations": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
            "ori_load": (ctypes.c_int, [P, D, P, P, P]),
            "ori_spectrum_cache": (ctypes.c_int, [P, I32]),
            "ori_setup": (ctypes.c_int, [ctypes.POINTER(Grid), D, P, P, P, P, ctypes.POINTER(P)]),
            "ori_solve": (ctypes.c_int, [P, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveInfo)]),
            "ori_matvec": (ctypes.c_int, [P, I32, I32, P, P]),
            "ori_green_noalloc": (ctypes.c_int, [ctypes.POINTER(Grid), D, I32, P, P, P]),
            "ori_adjoint": (ctypes.c_int, [P, ctypes.POINTER(SolveOpts), P, P, P, P, ctypes.POINTER(SolveInfo)]),
            "ori_gradient": (ctypes.c_int, [P, ctypes.POINTER(SolveOpts), P, P, ctypes.POINTER(D), P,
                                            ctypes.POINTER(SolveInfo)]),
            "ori_profile_enable": (ctypes.c_int, [P, I32]),
            "ori_profile_kinds": (ctypes.c_int, [P, ctypes.c_char_p]),
            "ori_profile_read": (ctypes.c_int, [P, I32, ctypes.POINTER(ctypes.c_char_p),
                                                ctypes.POINTER(D), ctypes.POINTER(I64), ctypes.POINTER(I32)]),
            "ori_charges": (ctypes.c_int, [P, P, P]),
            "ori_scattered_field": (ctypes.c_int, [P, P, P, I64, P]),
            "ori_far_field": (ctypes.c_int, [P, P, P, I64, P]),
            "ori_refraction_index": (ctypes.c_int, [P, D, D, P, P, P, P]),
            "ori_design_impedance": (ctypes.c_int, [P, D, D, P, P, P, P]),
            "ori_interpolation_difference": (ctypes.c_int, [P, P, P, I64, D, ctypes.POINTER(D)]),
            "ori_get_layout": (ctypes.c_int, [P, I32, ctypes.POINTER(Layout)]),
            "ori_set_layout": (ctypes.c_int, [P, I32, ctypes.POINTER(Layout)]),
            "ori_tune": (ctypes.c_int, [P, I32, ctypes.POINTER(Layout), ctypes.POINTER(D)]),
            "ori_check_guards": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64)]),
            "ori_destroy": (None, [P]),
            "ori_release_cached_memory": (None, []),
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
    """An ori_ctx plus the grid and batch size it was made for."""

    def __init__(self, handle, n, stream, nrhs=1):
        self.handle = handle
        self.n = n
        self.P = n ** 3
        self.nrhs = nrhs
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


def ori_workspace_bytes(n, provision=ORI_PROVISION_FP64 | ORI_PROVISION_MIXED, side=1.0, nrhs=1):
    b = ctypes.c_int64()
    _check(lib().ori_workspace_bytes(ctypes.byref(_grid(n, side)), int(nrhs), provision, ctypes.byref(b)))
    return b.value


def ori_create(n, side=1.0, origin=(0.0, 0.0, 0.0), cell_offset=0.5,
               provision=ORI_PROVISION_FP64 | ORI_PROVISION_MIXED, mem_limit_bytes=0, stream=None, nrhs=1):
    import torch
    h = ctypes.c_void_p()
    st = _stream(stream)
    _check(lib().ori_create(ctypes.byref(_grid(n, side, origin, cell_offset)), int(nrhs), provision,
                            int(mem_limit_bytes), st, ctypes.byref(h)))
    return Context(h, int(n), stream if stream is not None else torch.cuda.current_stream(), int(nrhs))


def ori_load(ctx, k, h, N, u0):
    """u0: complex128 CUDA tensor of nrhs * n^3 entries (batch-major)."""
    import torch
    _check(lib().ori_load(ctx.handle, float(k), _dev(h, torch.complex128, ctx.P, "h"),
                          _dev(N, torch.float64, ctx.P, "N"),
                          _dev(u0, torch.complex128, ctx.nrhs * ctx.P, "u0")), ctx)


def ori_spectrum_cache(ctx, enable=True):
    """enable: ori_load reuses the kernel spectrum while k is unchanged (the
    default); False: every ori_load computes it again."""
    _check(lib().ori_spectrum_cache(ctx.handle, int(bool(enable))), ctx)


def ori_setup(n, k, h, N, u0, side=1.0, origin=(0.0, 0.0, 0.0), cell_offset=0.5, stream=None):
    import torch
    P = int(n) ** 3
    hdl = ctypes.c_void_p()
    st = _stream(stream)
    _check(lib().ori_setup(ctypes.byref(_grid(n, side, origin, cell_offset)), float(k),
                           _dev(h, torch.complex128, P, "h"), _dev(N, torch.float64, P, "N"),
                           _dev(u0, torch.complex128, P, "u0"), st, ctypes.byref(hdl)))
    return Context(hdl, int(n), stream if stream is not None else torch.cuda.current_stream())


def _opts(tol=1e-10, max_iter=1000, precision=ORI_FP64, check_every=1, use_x0=False, inner_tol=1e-5,
          max_outer=10, true_residual=True, graph=True, multi=True):
    return SolveOpts(float(tol), int(max_iter), int(precision), int(check_every), int(bool(use_x0)),
                     float(inner_tol), int(max_outer), int(bool(true_residual)), int(bool(graph)), int(bool(multi)))


def ori_solve(ctx, u, tol=1e-10, max_iter=1000, precision=ORI_FP64, check_every=1, use_x0=False,
              inner_tol=1e-5, max_outer=10, true_residual=True, graph=True, raise_on_error=True):
    """Solve into u (complex128 CUDA tensor, n^3).  Returns (status, info dict)."""
    import torch
    o = _opts(tol, max_iter, precision, check_every, use_x0, inner_tol, max_outer, true_residual, graph)
    info = SolveInfo()
    st = lib().ori_solve(ctx.handle, ctypes.byref(o), _dev(u, torch.complex128, ctx.nrhs * ctx.P, "u"),
                         ctypes.byref(info))
    d = info.as_dict()
    if raise_on_error:
        _check(st, ctx, d)
    return st, d


def ori_adjoint(ctx, u, f, g=None, lam=None, raise_on_error=True, **opts):
    """A^T lam = f; g = -c u (G0 lam).  Fills g and/or lam (CUDA tensors).  Returns (status, info)."""
    import torch
    o = _opts(**opts)
    info = SolveInfo()
    st = lib().ori_adjoint(ctx.handle, ctypes.byref(o), _dev(u, torch.complex128, ctx.P, "u"),
                           _dev(f, torch.complex128, ctx.P, "f"), _dev(g, torch.complex128, ctx.P, "g"),
                           _dev(lam, torch.complex128, ctx.P, "lam"), ctypes.byref(info))
    d = info.as_dict()
    if raise_on_error:
        _check(st, ctx, d)
    return st, d


def ori_gradient(ctx, u_target, u, dJdh, raise_on_error=True, **opts):
    """J = sum |u - t|^2 and dJdh (dJ = Re sum dJdh dh).  Returns (status, J, info)."""
    import torch
    o = _opts(**opts)
    info = SolveInfo()
    J = ctypes.c_double(float("nan"))
    st = lib().ori_gradient(ctx.handle, ctypes.byref(o), _dev(u_target, torch.complex128, ctx.P, "u_target"),
                            _dev(u, torch.complex128, ctx.P, "u"), ctypes.byref(J),
                            _dev(dJdh, torch.complex128, ctx.P, "dJdh"), ctypes.byref(info))
    d = info.as_dict()
    if raise_on_error:
        _check(st, ctx, d)
    return st, J.value, d


def ori_matvec(ctx, x, y, op=ORI_OP_SYSTEM, precision=ORI_FP64):
    import torch
    _check(lib().ori_matvec(ctx.handle, int(op), int(precision), _dev(x, torch.complex128, ctx.nrhs * ctx.P, "x"),
                            _dev(y, torch.complex128, ctx.nrhs * ctx.P, "y")), ctx)


def ori_green_noalloc(n, k, x, y, precision=ORI_FP64, side=1.0, origin=(0.0, 0.0, 0.0), cell_offset=0.5,
                      stream=None):
    """y = G0 x (complex128 CUDA tensors, n^3 entries) without a context and
    without allocating (static device workspace, n <= 64).  The work is
    enqueued on the stream and not waited for."""
    import torch
    P = int(n) ** 3
    _check(lib().ori_green_noalloc(ctypes.byref(_grid(n, side, origin, cell_offset)), float(k), int(precision),
                                   _dev(x, torch.complex128, P, "x"), _dev(y, torch.complex128, P, "y"),
                                   _stream(stream)))


def ori_batch_info(ctx, i):
    info = SolveInfo()
    _check(lib().ori_batch_info(ctx.handle, int(i), ctypes.byref(info)), ctx)
    return info.as_dict()


def ori_destroy(ctx):
    ctx.close()


def ori_group_destroy(group):
    group.close()


def ori_release_cached_memory():
    """Free the device blocks, pinned blocks and streams that destroyed
    contexts and groups left in the library's process-wide cache."""
    lib().ori_release_cached_memory()


def ori_charges(ctx, u, q=None):
    """q = -D u (cell charges) for a solution u of the loaded problem."""
    import torch
    if q is None:
        q = torch.empty(ctx.nrhs * ctx.P, dtype=torch.complex128, device=u.device)
    _check(lib().ori_charges(ctx.handle, _dev(u, torch.complex128, ctx.nrhs * ctx.P, "u"),
                             _dev(q, torch.complex128, ctx.nrhs * ctx.P, "q")), ctx)
    return q


def _points(x, what):
    import torch
    if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.is_cuda and x.is_contiguous()
            and x.dim() == 2 and x.shape[1] == 3):
        raise TypeError(f"{what} must be a contiguous CUDA float64 tensor of shape (M, 3)")
    return x


def ori_scattered_field(ctx, u, x, v=None):
    """v(x) = sum_p G(x, x_p) q_p at the rows of x (M, 3); returns v (nrhs * M)."""
    import torch
    x = _points(x, "x")
    M = x.shape[0]
    if v is None:
        v = torch.empty(ctx.nrhs * M, dtype=torch.complex128, device=x.device)
    _check(lib().ori_scattered_field(ctx.handle, _dev(u, torch.complex128, ctx.nrhs * ctx.P, "u"),
                                     ctypes.c_void_p(x.data_ptr()), M,
                                     _dev(v, torch.complex128, ctx.nrhs * M, "v")), ctx)
    return v


def ori_far_field(ctx, u, beta, A=None):
    """A(beta) = (1/4 pi) sum_p exp(-i k beta.x_p) q_p for unit rows of beta (M, 3)."""
    import torch
    beta = _points(beta, "beta")
    M = beta.shape[0]
    if A is None:
        A = torch.empty(ctx.nrhs * M, dtype=torch.complex128, device=beta.device)
    _check(lib().ori_far_field(ctx.handle, _dev(u, torch.complex128, ctx.nrhs * ctx.P, "u"),
                               ctypes.c_void_p(beta.data_ptr()), M,
                               _dev(A, torch.complex128, ctx.nrhs * M, "A")), ctx)
    return A


def ori_refraction_index(ctx, k, n0, h, N=None, c_S=4 * 3.141592653589793, n=None):
    """n = [n0^2 - c_S h N / k^2]^{1/2}, arg in [0, 2 pi) (P entries)."""
    import torch
    if n is None:
        n = torch.empty(ctx.P, dtype=torch.complex128, device=h.device)
    _check(lib().ori_refraction_index(ctx.handle, float(k), float(c_S), _dev(n0, torch.complex128, ctx.P, "n0"),
                                      _dev(h, torch.complex128, ctx.P, "h"), _dev(N, torch.float64, ctx.P, "N"),
                                      _dev(n, torch.complex128, ctx.P, "n")), ctx)
    return n


def ori_design_impedance(ctx, k, n0, n, N=None, c_S=4 * 3.141592653589793, h=None):
    """h = k^2 (n0^2 - n^2) / (c_S N): the impedance that creates n (P entries)."""
    import torch
    if h is None:
        h = torch.empty(ctx.P, dtype=torch.complex128, device=n.device)
    _check(lib().ori_design_impedance(ctx.handle, float(k), float(c_S), _dev(n0, torch.complex128, ctx.P, "n0"),
                                      _dev(n, torch.complex128, ctx.P, "n"), _dev(N, torch.float64, ctx.P, "N"),
                                      _dev(h, torch.complex128, ctx.P, "h")), ctx)
    return h


def ori_interpolation_difference(ctx, y, x_fine, n_fine, fine_offset=0.5):
    """Section 4 / Table 4: sup over the cells of ctx's grid of the mean |x_i - y_q|
    over the points of the fine grid (n_fine per side) inside each cell."""
    import torch
    out = ctypes.c_double()
    _check(lib().ori_interpolation_difference(ctx.handle, _dev(y, torch.complex128, ctx.P, "y"),
                                              _dev(x_fine, torch.complex128, int(n_fine) ** 3, "x_fine"),
                                              int(n_fine), float(fine_offset), ctypes.byref(out)), ctx)
    return out.value


def ori_get_layout(ctx, precision=ORI_FP64):
    out = Layout()
    _check(lib().ori_get_layout(ctx.handle, int(precision), ctypes.byref(out)), ctx)
    return out.as_dict()


def ori_set_layout(ctx, precision=ORI_FP64, blk_lg=4, narrow=0, prefetch=0, znarrow=0, zplan=0):
    lay = Layout(int(blk_lg), int(narrow), int(prefetch), int(znarrow), int(zplan))
    _check(lib().ori_set_layout(ctx.handle, int(precision), ctypes.byref(lay)), ctx)


def ori_tune(ctx, reps=0):
    """Autotune the pass layouts of a loaded context.  Returns
    {"fp64": (layout dict, ms per product), "c64": (...)}; the complex64 entry
    has ms = -1 when complex64 workspaces were not provisioned."""
    best = (Layout * 2)()
    ms = (ctypes.c_double * 2)()
    _check(lib().ori_tune(ctx.handle, int(reps), best, ms), ctx)
    return {"fp64": (best[0].as_dict(), ms[0]), "c64": (best[1].as_dict(), ms[1])}


def ori_check_guards(ctx):
    """Number of the context's workspaces whose trailing guard band was overwritten."""
    out = ctypes.c_int64()
    _check(lib().ori_check_guards(ctx.handle, ctypes.byref(out)), ctx)
    return out.value


def ori_profile_enable(ctx, enable=True):
    _check(lib().ori_profile_enable(ctx.handle, int(bool(enable))), ctx)


def ori_profile_kinds(ctx, kinds=None):
    """Time only these kernel kinds (list or comma-separated names, e.g. "zpass"); None: all."""
    if kinds is not None and not isinstance(kinds, str):
        kinds = ",".join(kinds)
    _check(lib().ori_profile_kinds(ctx.handle, None if kinds is None else kinds.encode()), ctx)


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


def _autograd_function():
    import torch

    class _OriSolve(torch.autograd.Function):
        """u = solution of eq. 2.19 for impedance h (and incident field u0).

        Forward and backward both run in libori.so: the backward is one
        adjoint COCG solve with the same operator (ori_adjoint).
        """

        @staticmethod
        def forward(fctx, h, u0, N, n, k, side, opts):
            ctx = ori_setup(n, k, h.detach().contiguous(), None if N is None else N.detach().contiguous(),
                            u0.detach().contiguous(), side=side)
            u = torch.empty(int(n) ** 3, dtype=torch.complex128, device=h.device)
            try:
                ori_solve(ctx, u, **opts)
            except BaseException:
                ctx.close()  # the workspaces are released at once, not at garbage collection
                raise
            fctx.ori = ctx
            fctx.opts = opts
            fctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(fctx, grad_u):
            (u,) = fctx.saved_tensors
            ctx = fctx.ori
            f = torch.conj(grad_u).resolve_conj().contiguous()
            g = torch.empty_like(u) if fctx.needs_input_grad[0] else None
            lam = torch.empty_like(u) if fctx.needs_input_grad[1] else None
            try:
                if g is not None or lam is not None:
                    o = {k: v for k, v in fctx.opts.items() if k != "use_x0"}
                    ori_adjoint(ctx, u, f, g=g, lam=lam, **o)
            finally:
                ctx.close()
            return (None if g is None else torch.conj(g), None if lam is None else torch.conj(lam),
                    None, None, None, None, None)

    return _OriSolve


_ORI_SOLVE_FN = None


def OriSolve(h, u0, n, k, N=None, side=1.0, **opts):
    """Differentiable solve: torch.autograd.Function applied to (h, u0)."""
    global _ORI_SOLVE_FN
    if _ORI_SOLVE_FN is None:
        _ORI_SOLVE_FN = _autograd_function()
    return _ORI_SOLVE_FN.apply(h, u0, N, int(n), float(k), float(side), dict(opts))


class Group:
    """An ori_group: independent problems (each its own grid) solved together."""

    def __init__(self, handle, ns, stream):
        self.handle = handle
        self.ns = [int(n) for n in ns]
        self.stream = stream

    def close(self):
        if self.handle:
            lib().ori_group_destroy(self.handle)
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


def ori_group_create(grids, provision=ORI_PROVISION_FP64 | ORI_PROVISION_MIXED, stream=None):
    """grids: one entry per problem, an int n or a dict with n, side, origin, cell_offset."""
    import torch
    specs = [g if isinstance(g, dict) else {"n": g} for g in grids]
    arr = (Grid * len(specs))()
    for i, g in enumerate(specs):
        arr[i] = _grid(g["n"], g.get("side", 1.0), g.get("origin", (0.0, 0.0, 0.0)), g.get("cell_offset", 0.5))
    h = ctypes.c_void_p()
    _check(lib().ori_group_create(arr, len(specs), provision, _stream(stream), ctypes.byref(h)))
    return Group(h, [g["n"] for g in specs], stream if stream is not None else torch.cuda.current_stream())


def ori_group_load(group, i, k, h, N, u0):
    import torch
    P = group.ns[i] ** 3
    _check(lib().ori_group_load(group.handle, int(i), float(k), _dev(h, torch.complex128, P, "h"),
                                _dev(N, torch.float64, P, "N"), _dev(u0, torch.complex128, P, "u0")))


def ori_group_load_all(group, ks, hs, Ns, u0s):
    """ori_group_load of every problem in one call (their loads run side by
    side); Ns may be None or hold None entries."""
    import torch
    M = len(group.ns)
    Ns = [None] * M if Ns is None else list(Ns)
    if not (len(ks) == len(hs) == len(Ns) == len(u0s) == M):
        raise ValueError(f"expected {M} entries per argument")
    ptr = lambda t, dt, i, what: _dev(t, dt, group.ns[i] ** 3, f"{what}[{i}]")
    k_arr = (ctypes.c_double * M)(*[float(k) for k in ks])
    h_arr = (ctypes.c_void_p * M)(*[ptr(h, torch.complex128, i, "h").value for i, h in enumerate(hs)])
    N_arr = (ctypes.c_void_p * M)(*[(ptr(N, torch.float64, i, "N") or ctypes.c_void_p()).value
                                    for i, N in enumerate(Ns)])
    u_arr = (ctypes.c_void_p * M)(*[ptr(u, torch.complex128, i, "u0").value for i, u in enumerate(u0s)])
    _check(lib().ori_group_load_all(group.handle, k_arr, h_arr, N_arr, u_arr))


def ori_group_multi_iterations(group):
    """COCG iterations run in one launch per kernel for all running problems."""
    out = ctypes.c_int64()
    _check(lib().ori_group_multi_iterations(group.handle, ctypes.byref(out)))
    return out.value


def ori_group_solve(group, us, raise_on_error=True, **opts):
    """Solve every problem of the group into us[i] (complex128 CUDA tensors).
    Returns (status, [info dict per problem])."""
    import torch
    M = len(group.ns)
    if len(us) != M:
        raise ValueError(f"expected {M} output tensors, got {len(us)}")
    ptrs = (ctypes.c_void_p * M)(*[_dev(u, torch.complex128, n ** 3, f"u[{i}]").value
                                   for i, (u, n) in enumerate(zip(us, group.ns))])
    infos = (SolveInfo * M)()
    o = _opts(**opts)
    st = lib().ori_group_solve(group.handle, ctypes.byref(o), ptrs, infos)
    d = [infos[i].as_dict() for i in range(M)]
    if raise_on_error:
        _check(st, None, d)
    return st, d


def solve_many(problems, **opts):
    """Independent problems of any sizes solved together as one group made
    for this call: the COCG iterations of all running problems in one launch
    per kernel where their padded lengths allow (ori_solve_opts.multi), each
    block of iterations one graph replay.  The group's device blocks and
    streams come from, and go back to, the library's process-wide cache, so
    calls in a loop allocate nothing after the first.  problems: dicts with
    n, k, h, N, u0 (CUDA tensors) and optionally side.  Returns a list of
    (u, info) in order; each result equals that problem's ori_solve bit for
    bit."""
    import torch
    grids = [{"n": int(p["n"]), "side": float(p.get("side", 1.0))} for p in problems]
    dev = problems[0]["h"].device
    with ori_group_create(grids) as g:
        ori_group_load_all(g, [p["k"] for p in problems], [p["h"] for p in problems],
                           [p.get("N") for p in problems], [p["u0"] for p in problems])
        us = [torch.empty(int(p["n"]) ** 3, dtype=torch.complex128, device=dev) for p in problems]
        _, infos = ori_group_solve(g, us, **opts)
    return list(zip(us, infos))
