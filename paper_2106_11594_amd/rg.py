"""Python binding of librg.so (see include/rg.h).

Argument marshalling only: every step of the update runs in the HIP kernels
behind the C ABI.  torch supplies device memory and the HIP stream.  Loading
fails loudly when the library has not been built
(``python -m paper_2106_11594_amd.build``); there is no fallback path.
"""
import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "rg.h")

RG_F32, RG_F64 = 0, 1
FLAG_NONFINITE, FLAG_RANK_CAPACITY, FLAG_DENOMINATOR = 0x1, 0x2, 0x4
OPT_NO_REPROJECT, OPT_GENERIC_KERNEL, OPT_SERIAL_CLASSES, OPT_ROW_BY_ROW = 0x1, 0x2, 0x4, 0x8
OPT_DEPENDENT_BLOCKS_ONLY = 0x10
OPT_ORTHOGONAL, OPT_ORTHONORMAL = 0x20, 0x40
OPT_ONE_WG_PER_STREAM = 0x80
OPT_EXPLICIT_REJECTIONS = 0x100
OK, E_INVALID, E_NOMEM, E_DEVICE, E_RANK_CAPACITY, E_NONFINITE, E_STATE, E_UNSUPPORTED = range(8)
_STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "HIP runtime error", 4: "rank capacity reached",
           5: "non-finite row or target", 6: "stream is flagged", 7: "unsupported size"}


class RGError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (status %d)" % (what, _STATUS.get(code, "?"), code))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("r_max", ctypes.c_int32), ("eps", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


_lib = None
_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64

_SIGS = {
    "rg_default_options": (None, [_p]),
    "rg_init": (ctypes.c_int, [_p, _i32, _p]),
    "rg_push_rows": (ctypes.c_int, [_p, _p, _p, _i64]),
    "rg_solution": (ctypes.c_int, [_p, _p]),
    "rg_rank": (ctypes.c_int, [_p, _p]),
    "rg_status_flags": (ctypes.c_int, [_p, _p]),
    "rg_reset": (ctypes.c_int, [_p]),
    "rg_check": (ctypes.c_int, [_p]),
    "rg_batch_init_ws": (ctypes.c_int, [_p, _i32, _p, _p, _p, _p, ctypes.c_size_t]),
    "rg_batch_check_layout": (ctypes.c_int, [_p, _p, _p, _i64, _i64]),
    "rg_batch_status": (ctypes.c_int, [_p, _p]),
    "rg_batch_classes": (ctypes.c_int, [_p, _p]),
    "rg_probe_lds_read": (ctypes.c_int, [_p, _i32, _i32, _p]),
    "rg_destroy": (ctypes.c_int, [_p]),
    "rg_batch_init": (ctypes.c_int, [_p, _i32, _p, _p, _p]),
    "rg_batch_push": (ctypes.c_int, [_p, _p, _p, _p, _p]),
    "rg_batch_plan": (ctypes.c_int, [_p, _p]),
    "rg_batch_solution": (ctypes.c_int, [_p, _p]),
    "rg_batch_rank": (ctypes.c_int, [_p, _p]),
    "rg_batch_flags": (ctypes.c_int, [_p, _p]),
    "rg_batch_get_state": (ctypes.c_int, [_p, _i32, _p, _p, _p, _p]),
    "rg_batch_adjoint": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p, _p]),
    "rg_batch_pinv": (ctypes.c_int, [_p, _p, _p, _p, _p]),
    "rg_workspace_bytes": (ctypes.c_size_t, [_i32, _p, _p, _i32]),
    "rg_class_count": (_i32, []),
    "rg_class_info": (ctypes.c_int, [_i32, _p, _p, _p]),
    "rg_class_fits": (ctypes.c_int, [_i32, _i32, _i32, _p]),
    "rg_set_class_rules": (ctypes.c_int, [_p, _p, _p, _i32]),
    "rg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rg_pinv_track_workspace_bytes": (ctypes.c_size_t, [_i32, _i32, _i32, _i32]),
    "rg_pinv_track": (ctypes.c_int, [_p, _p, _i32, _i32, _i32, _i32, ctypes.c_double, _p, _p, _p, _p, _p,
                                     ctypes.c_size_t, _p]),
    "rg_pinv_track_noalloc": (ctypes.c_int, [_p, _p, _i32, _i32, _i32, _i32, ctypes.c_double, _p, _p, _p, _p,
                                             _p]),
    "rg_pinv_track_rhs": (ctypes.c_int, [_p, _p, _i32, _i32, _i32, _i32, _i32, ctypes.c_double, _p, _p, _p, _p,
                                         _p, ctypes.c_size_t, _p]),
    "rg_pinv_track_noalloc_max_bytes": (ctypes.c_size_t, []),
}


def header_functions():
    """Names of the functions declared in include/rg.h."""
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(rg_\w+)\s*\(", src, flags=re.M)))


def lib():
    """Load librg.so once (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librg.so is not built; run `python -m paper_2106_11594_amd.build`")
        # torch first: librg.so then binds to the HIP runtime torch has loaded, so
        # the streams and device pointers torch hands over belong to that runtime
        # (loading librg.so first can bring in a second HIP runtime).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code, what):
    if code != 0:
        raise RGError(code, what)


def _torch():
    import torch
    return torch


def _dtype_code(dtype):
    torch = _torch()
    if dtype in ("f32", np.float32, torch.float32):
        return RG_F32, torch.float32
    if dtype in ("f64", np.float64, torch.float64):
        return RG_F64, torch.float64
    raise ValueError("dtype must be float32 or float64")


def _dev(t, dtype, what, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) tensor" % what)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s" % (what, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements" % (what, numel))
    return ctypes.c_void_p(t.data_ptr())


class Batch:
    """B independent recursive least-squares streams (rg_batch_* calls)."""

    def __init__(self, ms, r_max=None, dtype="f32", eps=None, stream=None, flags=0, workspace=None):
        """workspace: optional caller-owned device tensor (uint8, at least
        workspace_bytes(ms, r_max, dtype) bytes, 256-byte aligned) that holds
        the handle's device state instead of a library allocation
        (rg_batch_init_ws); it must outlive the handle."""
        torch = _torch()
        L = lib()
        self.code, self.tdtype = _dtype_code(dtype)
        self.ms = np.ascontiguousarray(ms, dtype=np.int32).reshape(-1)
        self.B = int(self.ms.shape[0])
        self.r_max = None if r_max is None else np.ascontiguousarray(r_max, dtype=np.int32).reshape(-1)
        self.x_off = np.zeros(self.B, dtype=np.int64)
        self.x_off[1:] = np.cumsum(self.ms[:-1].astype(np.int64))
        self.n_x = int(self.ms.astype(np.int64).sum())
        if stream is None:
            stream = torch.cuda.current_stream()
        self.torch_stream = stream
        opt = Options()
        L.rg_default_options(ctypes.byref(opt))
        opt.dtype = self.code
        opt.eps = -1.0 if eps is None else float(eps)
        opt.stream = ctypes.c_void_p(stream.cuda_stream)
        opt.flags = int(flags)
        self._opt = opt
        h = ctypes.c_void_p()
        rp = None if self.r_max is None else self.r_max.ctypes.data_as(_p)
        if workspace is None:
            _check(L.rg_batch_init(ctypes.byref(h), self.B, self.ms.ctypes.data_as(_p), rp, ctypes.byref(opt)),
                   "rg_batch_init")
        else:
            _check(L.rg_batch_init_ws(ctypes.byref(h), self.B, self.ms.ctypes.data_as(_p), rp, ctypes.byref(opt),
                                      _dev(workspace, None, "workspace"),
                                      workspace.numel() * workspace.element_size()), "rg_batch_init_ws")
        self._workspace = workspace
        self._h = h

    @property
    def handle(self):
        return self._h

    def plan(self, rows_hint=None):
        rh = None if rows_hint is None else np.ascontiguousarray(rows_hint, dtype=np.int64)
        _check(lib().rg_batch_plan(self._h, None if rh is None else rh.ctypes.data_as(_p)), "rg_batch_plan")

    def push(self, gamma, y, row_ptr, gamma_off):
        torch = _torch()
        _check(lib().rg_batch_push(self._h, _dev(gamma, self.tdtype, "gamma"), _dev(y, self.tdtype, "y"),
                                   _dev(row_ptr, torch.int64, "row_ptr", self.B + 1),
                                   _dev(gamma_off, torch.int64, "gamma_off", self.B)), "rg_batch_push")

    def solution(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.n_x, dtype=self.tdtype, device="cuda")
        _check(lib().rg_batch_solution(self._h, _dev(out, self.tdtype, "x", self.n_x)), "rg_batch_solution")
        return out

    def rank(self):
        r = np.zeros(self.B, dtype=np.int32)
        _check(lib().rg_batch_rank(self._h, r.ctypes.data_as(_p)), "rg_batch_rank")
        return r

    def flags(self):
        f = np.zeros(self.B, dtype=np.uint32)
        _check(lib().rg_batch_flags(self._h, f.ctypes.data_as(_p)), "rg_batch_flags")
        return f

    def classes(self):
        """Kernel class of every stream (rg_batch_classes; -1 = generic kernel)."""
        c = np.zeros(self.B, dtype=np.int32)
        _check(lib().rg_batch_classes(self._h, c.ctypes.data_as(_p)), "rg_batch_classes")
        return c

    def status(self):
        """Per-stream status codes (rg_batch_status): OK, E_NONFINITE,
        E_RANK_CAPACITY or E_STATE."""
        st = np.zeros(self.B, dtype=np.int32)
        _check(lib().rg_batch_status(self._h, st.ctypes.data_as(_p)), "rg_batch_status")
        return st

    def check_layout(self, gamma, y, row_ptr, gamma_off):
        """Host-side check of a packed row layout (rg_batch_check_layout);
        raises RGError(E_INVALID) when it is inconsistent."""
        torch = _torch()
        _check(lib().rg_batch_check_layout(self._h, _dev(row_ptr, torch.int64, "row_ptr", self.B + 1),
                                           _dev(gamma_off, torch.int64, "gamma_off", self.B),
                                           int(y.numel()), int(gamma.numel())), "rg_batch_check_layout")

    def reset(self):
        _check(lib().rg_reset(self._h), "rg_reset")

    def get_state(self, b):
        """(C, Ct, Pinv, w) of stream b as device tensors (rank-sized)."""
        torch = _torch()
        r = int(self.rank()[b])
        m = int(self.ms[b])
        C = torch.empty((r, m), dtype=self.tdtype, device="cuda")
        Ct = torch.empty((r, m), dtype=self.tdtype, device="cuda")
        P = torch.empty((r, r), dtype=torch.float64, device="cuda")
        w = torch.empty(r, dtype=torch.float64, device="cuda")
        if r:
            _check(lib().rg_batch_get_state(self._h, int(b), _dev(C, None, "C"), _dev(Ct, None, "Ct"),
                                            _dev(P, None, "P"), _dev(w, None, "w")), "rg_batch_get_state")
        return C, Ct, P, w

    def adjoint(self, A, Y, row_ptr, a_off, g, dA=None, dY=None):
        torch = _torch()
        if dA is None:
            dA = torch.empty_like(A)
        if dY is None:
            dY = torch.empty_like(Y)
        _check(lib().rg_batch_adjoint(self._h, _dev(A, self.tdtype, "A"), _dev(Y, self.tdtype, "Y"),
                                      _dev(row_ptr, torch.int64, "row_ptr", self.B + 1),
                                      _dev(a_off, torch.int64, "a_off", self.B),
                                      _dev(g, self.tdtype, "g", self.n_x),
                                      _dev(dA, self.tdtype, "dA", A.numel()),
                                      _dev(dY, self.tdtype, "dY", Y.numel())), "rg_batch_adjoint")
        return dA, dY

    def pinv(self, A, row_ptr, a_off, out=None):
        """A^+ of every stream (Theorem 1), packed like A: stream b's m x n_b
        pseudoinverse, row-major, at a_off[b]."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(A)
        _check(lib().rg_batch_pinv(self._h, _dev(A, self.tdtype, "A"),
                                   _dev(row_ptr, torch.int64, "row_ptr", self.B + 1),
                                   _dev(a_off, torch.int64, "a_off", self.B),
                                   _dev(out, self.tdtype, "Ap", A.numel())), "rg_batch_pinv")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().rg_destroy(self._h), "rg_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One stream: rg_init / rg_push_rows / rg_solution / rg_rank."""

    def __init__(self, m, r_max=None, dtype="f32", eps=None, stream=None, flags=0):
        torch = _torch()
        L = lib()
        self.code, self.tdtype = _dtype_code(dtype)
        self.m = int(m)
        if stream is None:
            stream = torch.cuda.current_stream()
        opt = Options()
        L.rg_default_options(ctypes.byref(opt))
        opt.dtype = self.code
        opt.r_max = 0 if r_max is None else int(r_max)
        opt.eps = -1.0 if eps is None else float(eps)
        opt.stream = ctypes.c_void_p(stream.cuda_stream)
        opt.flags = int(flags)
        h = ctypes.c_void_p()
        _check(L.rg_init(ctypes.byref(h), self.m, ctypes.byref(opt)), "rg_init")
        self._h = h

    def push_rows(self, gamma, y):
        k = int(y.numel())
        _check(lib().rg_push_rows(self._h, _dev(gamma, self.tdtype, "gamma", k * self.m),
                                  _dev(y, self.tdtype, "y", k), k), "rg_push_rows")

    def solution(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.m, dtype=self.tdtype, device="cuda")
        _check(lib().rg_solution(self._h, _dev(out, self.tdtype, "x", self.m)), "rg_solution")
        return out

    def rank(self):
        r = ctypes.c_int32()
        _check(lib().rg_rank(self._h, ctypes.byref(r)), "rg_rank")
        return r.value

    def flags(self):
        f = ctypes.c_uint32()
        _check(lib().rg_status_flags(self._h, ctypes.byref(f)), "rg_status_flags")
        return f.value

    def check(self):
        """rg_check: the stream's condition as a status code (synchronises)."""
        return int(lib().rg_check(self._h))

    def get_state(self):
        """(C, Ct, Pinv, w) as device tensors (rank-sized; rg_batch_get_state)."""
        torch = _torch()
        r = self.rank()
        C = torch.empty((r, self.m), dtype=self.tdtype, device="cuda")
        Ct = torch.empty((r, self.m), dtype=self.tdtype, device="cuda")
        P = torch.empty((r, r), dtype=torch.float64, device="cuda")
        w = torch.empty(r, dtype=torch.float64, device="cuda")
        if r:
            _check(lib().rg_batch_get_state(self._h, 0, _dev(C, None, "C"), _dev(Ct, None, "Ct"),
                                            _dev(P, None, "P"), _dev(w, None, "w")), "rg_batch_get_state")
        return C, Ct, P, w

    def reset(self):
        _check(lib().rg_reset(self._h), "rg_reset")

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().rg_destroy(self._h), "rg_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(ms, r_max=None, dtype="f32"):
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    rp = None if r_max is None else np.ascontiguousarray(r_max, dtype=np.int32)
    code = RG_F64 if dtype in ("f64", np.float64) else RG_F32
    return int(lib().rg_workspace_bytes(len(ms), ms.ctypes.data_as(_p),
                                        None if rp is None else rp.ctypes.data_as(_p), code))


def _autograd_function():
    import torch

    class RGSolve(torch.autograd.Function):
        """x_b = A_b^+ Y_b for equal-shape problems, by rank-Greville on the GPU.

        forward: A (B, n, m), Y (B, n) -> x (B, m); every row of problem b is
        pushed through Algorithm 1 in order (rg_batch_push), then
        x_b = Ct_b^T w_b (rg_batch_solution).
        backward: the adjoint kernel (rg_batch_adjoint) gives dL/dA and dL/dY
        at constant rank from the maintained factorisation.
        """

        @staticmethod
        def forward(ctx, A, Y, eps, r_max):
            B, n, m = A.shape
            A = A.contiguous()
            Y = Y.contiguous()
            h = Batch(np.full(B, m, np.int32), r_max=None if r_max is None else np.full(B, r_max, np.int32),
                      dtype=A.dtype, eps=eps)
            row_ptr = torch.arange(0, (B + 1) * n, n, dtype=torch.int64, device=A.device)
            a_off = torch.arange(0, B * n * m, n * m, dtype=torch.int64, device=A.device)
            h.plan(np.full(B, n, np.int64))
            h.push(A.view(-1), Y.view(-1), row_ptr, a_off)
            x = h.solution().view(B, m)
            ctx.h = h
            ctx.save_for_backward(A, Y, row_ptr, a_off)
            return x

        @staticmethod
        def backward(ctx, gx):
            A, Y, row_ptr, a_off = ctx.saved_tensors
            dA, dY = ctx.h.adjoint(A.view(-1), Y.view(-1), row_ptr, a_off, gx.contiguous().view(-1))
            return dA.view_as(A), dY.view_as(Y), None, None

    return RGSolve


_RGSolve = None


def rg_solve(A, Y, eps=None, r_max=None):
    """Differentiable batched minimum-norm least squares (see RGSolve)."""
    global _RGSolve
    if _RGSolve is None:
        _RGSolve = _autograd_function()
    return _RGSolve.apply(A, Y, eps, r_max)


# ---- kernel size classes ------------------------------------------------------

def pinv_track_workspace_bytes(B, n, m, r_max):
    """Device bytes rg_pinv_track needs for B problems of n x m with capacity r_max."""
    return int(lib().rg_pinv_track_workspace_bytes(B, n, m, r_max))


def pinv_track_noalloc(A, Y, Ap, X, rank, flags, r_max=None, eps=None, stream=None):
    """rg_pinv_track_noalloc: as pinv_track, into caller-provided outputs
    (Ap [B x m x n], X [B x m], rank [B], flags [B]; FP64 / int32 CUDA
    tensors), with the workspace taken from the library's fixed device array:
    nothing is allocated by the call."""
    torch = _torch()
    B, n, m = A.shape
    if r_max is None:
        r_max = max(1, min(n, m))
    if stream is None:
        stream = torch.cuda.current_stream()
    null = ctypes.c_void_p(0)
    _check(lib().rg_pinv_track_noalloc(_dev(A, torch.float64, "A") if n else null,
                                       _dev(Y, torch.float64, "Y") if n else null, B, n, m, r_max,
                                       -1.0 if eps is None else float(eps),
                                       _dev(Ap, torch.float64, "Ap", B * m * n) if n else null,
                                       _dev(X, torch.float64, "X", B * m), _dev(rank, torch.int32, "rank", B),
                                       _dev(flags, torch.int32, "flags", B), ctypes.c_void_p(stream.cuda_stream)),
           "rg_pinv_track_noalloc")


def pinv_track_noalloc_max_bytes():
    return int(lib().rg_pinv_track_noalloc_max_bytes())


def pinv_track(A, Y, r_max=None, eps=None, stream=None):
    """Theorems 2 and 3: push every row of A (B x n x m, or n x m) with targets
    Y (B x n, or n; or with q right-hand sides B x n x q, or n x q) and
    maintain A^+ row by row (FP64, CUDA tensors).  Returns (Ap [B x m x n],
    X [B x m] or [B x m x q], rank [B] int32, flags [B] int32), with the batch
    dimension dropped for a 2-D A.  r_max defaults to min(n, m); eps=None
    takes the default threshold of Section 3."""
    torch = _torch()
    squeeze = A.dim() == 2
    if squeeze:
        A, Y = A.unsqueeze(0), Y.unsqueeze(0)
    if A.dim() != 3 or Y.shape[:2] != A.shape[:2] or Y.dim() not in (2, 3):
        raise ValueError("A must be B x n x m and Y B x n or B x n x q")
    multi = Y.dim() == 3
    q = int(Y.shape[2]) if multi else 1
    Y = Y.contiguous()
    B, n, m = A.shape
    if r_max is None:
        r_max = max(1, min(n, m))
    dev = A.device
    nbytes = pinv_track_workspace_bytes(B, n, m, r_max)
    if nbytes == 0:
        raise RGError(1, "rg_pinv_track_workspace_bytes")
    if stream is None:
        stream = torch.cuda.current_stream()
    # outputs and workspace come from the caching allocator on the stream the
    # kernel runs on, so none of them is reused while the kernel still runs
    with torch.cuda.stream(stream):
        Ap = torch.empty((B, m, n), dtype=torch.float64, device=dev)
        X = torch.empty((B, m, q) if multi else (B, m), dtype=torch.float64, device=dev)
        rank = torch.empty(B, dtype=torch.int32, device=dev)
        flags = torch.empty(B, dtype=torch.int32, device=dev)
        work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    null = ctypes.c_void_p(0)
    _check(lib().rg_pinv_track_rhs(_dev(A, torch.float64, "A") if n else null,
                                   _dev(Y, torch.float64, "Y") if n else null, B, n, m, q, r_max,
                                   -1.0 if eps is None else float(eps),
                                   _dev(Ap, None, "Ap") if n else null, _dev(X, None, "X"), _dev(rank, None, "rank"),
                                   _dev(flags, None, "flags"), _dev(work, None, "work"), nbytes,
                                   ctypes.c_void_p(stream.cuda_stream)), "rg_pinv_track_rhs")
    if squeeze:
        return Ap[0], X[0], rank[0], flags[0]
    return Ap, X, rank, flags


def class_count():
    """Number of on-chip kernel classes for FP32 streams (rg_class_count)."""
    return int(lib().rg_class_count())


def class_info(cls):
    """(rank capacity, largest m, threads per stream) of class cls."""
    r, m, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().rg_class_info(int(cls), ctypes.byref(r), ctypes.byref(m), ctypes.byref(t)), "rg_class_info")
    return r.value, m.value, t.value


def class_fits(cls, m, r_max):
    """Whether class cls can hold a stream with m regressors and capacity r_max."""
    f = ctypes.c_int32()
    _check(lib().rg_class_fits(int(cls), int(m), int(r_max), ctypes.byref(f)), "rg_class_fits")
    return bool(f.value)


def set_class_rules(rules):
    """Install placement rules [(m_hi, r_max_hi, cls), ...] for later handles
    (rg_set_class_rules); an empty list restores the default placement."""
    import numpy as np
    rules = list(rules)
    a = np.array([r[0] for r in rules] or [0], dtype=np.int32)
    b = np.array([r[1] for r in rules] or [0], dtype=np.int32)
    c = np.array([r[2] for r in rules] or [0], dtype=np.int32)
    _check(lib().rg_set_class_rules(a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p),
                                    c.ctypes.data_as(ctypes.c_void_p), len(rules)), "rg_set_class_rules")


LDS_PROBE_BYTES_PER_THREAD_ITER = 128
LDS_PROBE_THREADS = 256


def probe_lds_read(out, blocks, iters, stream=None):
    """rg_probe_lds_read: enqueue the LDS read-bandwidth probe; out is a CUDA
    float32 tensor of blocks * 256 elements.  Returns the bytes it reads."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().rg_probe_lds_read(_dev(out, torch.float32, "out", blocks * LDS_PROBE_THREADS), int(blocks),
                                   int(iters), ctypes.c_void_p(stream.cuda_stream)), "rg_probe_lds_read")
    return blocks * LDS_PROBE_THREADS * LDS_PROBE_BYTES_PER_THREAD_ITER * iters
