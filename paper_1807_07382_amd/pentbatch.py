"""Thin ctypes binding of libpentbatch.so (C ABI in include/pentbatch.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  torch is used for device memory and streams; a torch tensor of
shape (n, batch) with unit stride along the batch axis *is* the interleaved,
batch-fastest layout (ld = tensor.stride(0)).

The library is loaded on first use.  If it is missing this module raises --
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PENTBATCH_LIB names another build of the same sources (the sanitizer job's)
LIB_PATH = os.environ.get("PENTBATCH_LIB") or os.path.join(HERE, "libpentbatch.so")

OK = 0
INVALID_VALUE = 1
ZERO_PIVOT = 2
OUT_OF_MEMORY = 3
HIP_ERROR = 4
NOT_CONVERGED = 5
SIZE_MISMATCH = 6
NOT_SUPPORTED = 7
TIMEOUT = 8

# group solve modes (pent_group_solve)
GROUP_FP64 = 0
GROUP_MIXED = 1       # rejected with NOT_SUPPORTED (see the header)
GROUP_PER_MATRIX = 2

# every symbol include/pentbatch.h declares: name -> (restype, argtypes)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double
SIGNATURES = {
    "pent_factor": (_P, [_I64, _P, _P, _P, _P, _P]),
    "pent_factor_d4": (_P, [_I64, _D]),
    "pent_destroy": (_I, [_P]),
    "pent_solve": (_I, [_P, _P, _I64, _I64, _P]),
    "pent_solve_noalloc": (_I, [_P, _P, _I64, _I64, _P]),
    "pent_solve_tiled": (_I, [_P, _P, _I64, _I64, _I64, _P]),
    "pent_solve_strided": (_I, [_P, _P, _I64, _I64, _P]),
    "pent_solve_mixed": (_I, [_P, _P, _I, _I64, _P, _I64, _I64, _I, _P, _P, ctypes.c_size_t, _P]),
    "pent_mixed_workspace_size": (ctypes.c_size_t, [_P, _I64]),
    "pent_mixed_workspace_size_ex": (ctypes.c_size_t, [_P, _I64, _I, _I]),
    "pent_set_refine_tolerance": (_I, [_P, _D]),
    "pent_backward_error": (_I, [_P, _P, _I, _I64, _P, _I64, _I64, _P, _P, ctypes.c_size_t, _P]),
    "pent_group_create": (_P, [ctypes.POINTER(_P), _I64]),
    "pent_group_workspace_size": (ctypes.c_size_t, [_P, ctypes.POINTER(_I64)]),
    "pent_group_solve": (_I, [_P, ctypes.POINTER(_P), ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                              _I, _P, ctypes.c_size_t, _P]),
    "pent_group_destroy": (_I, [_P]),
    "pent_group_set_variant": (_I, [_P, _I]),
    "pent_group_check": (_I, [_P]),
    "pent_group_capture": (_P, [_P, ctypes.POINTER(_P), ctypes.POINTER(_I64),
                                ctypes.POINTER(_I64), _I, _I, _P, ctypes.c_size_t, _P]),
    "pent_graph_launch": (_I, [_P, _P]),
    "pent_graph_destroy": (_I, [_P]),
    "pent_autotune": (_I, [_P, _I64, ctypes.POINTER(_I), ctypes.POINTER(_I),
                           ctypes.POINTER(_D), _P]),
    "pent_group_autotune": (_I, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I),
                                 ctypes.POINTER(_D), _P]),
    "pent_ch2d_rhs": (_I, [_P, _P, _I64, _I64, _I64, _P, _D, _P]),
    "pent_ch2d_step": (_I, [_P, _P, _P, _P, _I64, _I64, _I64, _P, _D, _P]),
    "pent_cyclic_factor": (_P, [_I64, _P, _P, _P, _P, _P]),
    "pent_cyclic_factor_d4": (_P, [_I64, _D]),
    "pent_cyclic_solve": (_I, [_P, _P, _I64, _I64, _P]),
    "pent_cyclic_cn_rhs": (_I, [_P, _P, _I64, _P, _I64, _I64, _P]),
    "pent_cyclic_bordering": (_I, [_P, _P, _P]),
    "pent_cyclic_destroy": (_I, [_P]),
    "pent_cyclic_cn_step": (_I, [_P, _P, _I64, _P, _I64, _I64, _P]),
    "pent_cyclic_set_schedule": (_I, [_P, _I, _I]),
    "pent_cyclic_query_schedule": (_I, [_P, _I64, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "pent_cyclic_check": (_I, [_P]),
    "pent_rewrite_workspace_size": (ctypes.c_size_t, [_I64, _I64]),
    "pent_solve_rewrite": (_I, [_I64, _P, _P, _P, _P, _P, _I64, _P, _I64, _I64, _P,
                                ctypes.c_size_t, _P]),
    "pent_rewrite_check": (_I, [_P, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "pent_get_factors": (_I, [_P, _P, _P, _P, _P]),
    "pent_get_diagonals": (_I, [_P, _P, _P, _P, _P, _P]),
    "pent_size": (_I64, [_P]),
    "pent_set_schedule": (_I, [_P, _I, _I]),
    "pent_check": (_I, [_P]),
    "pent_query_schedule": (_I, [_P, _I64, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "pent_stream_copy": (_I, [_P, _I64, _P, _I64, _I64, _I64, _P]),
    "pent_stream_copy_shaped": (_I, [_P, _I64, _P, _I64, _I64, _I64, _I, _I, _P]),
    "pent_last_status": (_I, []),
    "pent_last_pivot_row": (_I64, []),
    "pent_status_string": (ctypes.c_char_p, [_I]),
}

_lib = None


class PentError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().pent_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


class ZeroPivotError(PentError):
    def __init__(self, row: int):
        super().__init__(ZERO_PIVOT, f"factorisation stopped at row {row}")
        self.row = row


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1807_07382_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int, what: str):
    if st != OK:
        raise PentError(st, what)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _torch_stream(stream):
    """The torch stream a solve is enqueued on (torch's current one for None;
    a raw hipStream_t handle is wrapped)."""
    import torch
    if stream is None:
        return torch.cuda.current_stream()
    if isinstance(stream, int):
        return torch.cuda.ExternalStream(stream)
    return stream


def _dptr(t, dtype_name: str):
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != getattr(torch, dtype_name):
        raise ValueError(f"expected {dtype_name}, got {t.dtype}")
    return t.data_ptr()


class Plan:
    """A factored matrix (pent_handle).  Free with close() or a with-block."""

    def __init__(self, handle: int, n: int):
        self._h = handle
        self.n = n

    # -- construction ------------------------------------------------------
    @classmethod
    def factor(cls, a, b, c, d, e) -> "Plan":
        """Factor the matrix with HOST diagonals a..e (float64 sequences of
        length n, row-indexed)."""
        import numpy as np
        arrs = [np.ascontiguousarray(np.asarray(x, dtype=np.float64)) for x in (a, b, c, d, e)]
        n = arrs[2].shape[0]
        if any(x.shape != (n,) for x in arrs):
            raise ValueError("diagonals must all have shape (n,)")
        h = lib().pent_factor(n, *[x.ctypes.data for x in arrs])
        return cls._made(h, n)

    @classmethod
    def factor_d4(cls, n: int, sigma: float) -> "Plan":
        """Factor I + sigma*D4 (non-periodic), assembled on the device."""
        h = lib().pent_factor_d4(int(n), float(sigma))
        return cls._made(h, n)

    @classmethod
    def _made(cls, h, n):
        if not h:
            st = lib().pent_last_status()
            if st == ZERO_PIVOT:
                raise ZeroPivotError(int(lib().pent_last_pivot_row()))
            raise PentError(st, "factor")
        return cls(h, int(n))

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if self._h:
            _check(lib().pent_destroy(self._h), "destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- solves --------------------------------------------------------------
    def solve_(self, F, stream=None):
        """Overwrite F (cuda float64, shape (n, batch), unit batch stride) with
        A^{-1} F.  Asynchronous on ``stream`` (default: torch's current)."""
        if F.dim() != 2 or F.shape[0] != self.n or (F.shape[1] > 1 and F.stride(1) != 1):
            raise ValueError(f"F must have shape ({self.n}, batch) with unit batch stride")
        ld = F.stride(0) if F.shape[1] > 0 else F.shape[1]
        _check(lib().pent_solve(self._h, _dptr(F, "float64"), F.shape[1], max(ld, F.shape[1]),
                                _stream_ptr(stream)), "solve")
        return F

    def solve_strided_(self, F, stream=None):
        """Overwrite F (cuda float64, shape (batch, n), unit stride along n)
        with the solutions of its rows (system-major storage)."""
        if F.dim() != 2 or F.shape[1] != self.n or F.stride(1) != 1:
            raise ValueError(f"F must have shape (batch, {self.n}) with unit stride along n")
        _check(lib().pent_solve_strided(self._h, _dptr(F, "float64"), F.shape[0],
                                        max(F.stride(0), self.n), _stream_ptr(stream)),
               "solve_strided")
        return F

    def solve_mixed(self, F, X, refine_steps: int = 0, eta=None, work=None, stream=None):
        """X (cuda float64, shape (n, batch)) = A^{-1} F with F cuda float32 or
        float64 of the same shape; FP64 arithmetic, ``refine_steps``
        compensated-residual corrections, optional per-system backward error
        into ``eta`` (cuda float64, shape (batch,)).  ``work`` is allocated
        with torch when not given."""
        import torch
        if F.dim() != 2 or F.shape[0] != self.n or X.shape != F.shape:
            raise ValueError(f"F and X must have shape ({self.n}, batch)")
        m = F.shape[1]
        for t in (F, X):
            if m > 1 and t.stride(1) != 1:
                raise ValueError("unit batch stride required")
        fdt = {torch.float32: 1, torch.float64: 0}.get(F.dtype)
        if fdt is None:
            raise ValueError("F must be float32 or float64")
        nbytes = lib().pent_mixed_workspace_size_ex(self._h, m, int(refine_steps), int(eta is not None))
        if work is None and nbytes:
            # allocated on the solve's stream, so the caching allocator does
            # not hand it out again while the kernels there still use it
            with torch.cuda.stream(_torch_stream(stream)):
                work = torch.empty(nbytes, dtype=torch.uint8, device=F.device)
        wptr = work.data_ptr() if work is not None else None
        wlen = work.numel() * work.element_size() if work is not None else 0
        if eta is not None and (eta.dtype != torch.float64 or eta.numel() < m):
            raise ValueError("eta must be float64 with batch elements")
        _check(lib().pent_solve_mixed(self._h, F.data_ptr(), fdt, max(F.stride(0), m),
                                      _dptr(X, "float64"), max(X.stride(0), m), m,
                                      int(refine_steps), eta.data_ptr() if eta is not None else None,
                                      wptr, wlen, _stream_ptr(stream)), "solve_mixed")
        return X

    def backward_error(self, F, X, eta, work=None, stream=None):
        """eta[j] = ||F_j - A X_j||_inf / (||A||_inf ||X_j||_inf + ||F_j||_inf),
        residual evaluated compensated on the device."""
        import torch
        m = F.shape[1]
        fdt = {torch.float32: 1, torch.float64: 0}[F.dtype]
        if work is None:
            with torch.cuda.stream(_torch_stream(stream)):
                work = torch.empty(24 * max(m, 1), dtype=torch.uint8, device=F.device)
        _check(lib().pent_backward_error(self._h, F.data_ptr(), fdt, max(F.stride(0), m),
                                         _dptr(X, "float64"), max(X.stride(0), m), m,
                                         eta.data_ptr(), work.data_ptr(), work.numel(),
                                         _stream_ptr(stream)), "backward_error")
        return eta

    # -- inspection ----------------------------------------------------------
    def factors(self):
        import numpy as np
        out = [np.empty(self.n) for _ in range(4)]
        _check(lib().pent_get_factors(self._h, *[x.ctypes.data for x in out]), "get_factors")
        return tuple(out)

    def diagonals(self):
        import numpy as np
        out = [np.empty(self.n) for _ in range(5)]
        _check(lib().pent_get_diagonals(self._h, *[x.ctypes.data for x in out]), "get_diagonals")
        return tuple(out)

    def autotune(self, batch: int, stream=None):
        """Time the schedules for ``batch`` systems and keep the fastest;
        returns (kind, seg_rows, ms)."""
        k, sr, ms = _I(0), _I(0), _D(0.0)
        _check(lib().pent_autotune(self._h, int(batch), ctypes.byref(k), ctypes.byref(sr),
                                   ctypes.byref(ms), _stream_ptr(stream)), "autotune")
        return int(k.value), int(sr.value), float(ms.value)

    def schedule_for(self, batch: int):
        """(kind, seg_rows) pent_solve uses for ``batch`` systems."""
        k, sr = _I(0), _I(0)
        _check(lib().pent_query_schedule(self._h, int(batch), ctypes.byref(k), ctypes.byref(sr)),
               "query_schedule")
        return int(k.value), int(sr.value)

    def set_schedule(self, kind: int, seg_rows: int = 0):
        _check(lib().pent_set_schedule(self._h, int(kind), int(seg_rows)), "set_schedule")

    def check(self):
        """Raise PentError(TIMEOUT) if a single-pass solve on this handle gave
        up a wait since the last check, PentError(NOT_CONVERGED) if a refined
        solve missed the tolerance set by set_refine_tolerance (blocking)."""
        _check(lib().pent_check(self._h), "check")

    def set_refine_tolerance(self, tol: float):
        """Backward-error tolerance of solve_mixed (0 turns the check off)."""
        _check(lib().pent_set_refine_tolerance(self._h, float(tol)), "set_refine_tolerance")

    def mixed_workspace_size(self, batch: int, refine_steps: int = None, eta: bool = True) -> int:
        """Bytes of solve_mixed's workspace: for every refine_steps (None) or
        for one configuration."""
        if refine_steps is None:
            return int(lib().pent_mixed_workspace_size(self._h, int(batch)))
        return int(lib().pent_mixed_workspace_size_ex(self._h, int(batch), int(refine_steps),
                                                      int(bool(eta))))


class Group:
    """Several factored plans solved together (pent_group).  ``solve`` runs
    one launch for all matrices (mode GROUP_FP64) or one solve per matrix
    (mode GROUP_PER_MATRIX); GROUP_MIXED is rejected by the library."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (_P * len(self.plans))(*[p.handle for p in self.plans])
        self._g = lib().pent_group_create(arr, len(self.plans))
        if not self._g:
            raise PentError(lib().pent_last_status(), "group_create")
        self._work = None

    def _args(self, Fs):
        import torch
        if len(Fs) != len(self.plans):
            raise ValueError("one right-hand-side block per plan")
        for p, F in zip(self.plans, Fs):
            if F.dim() != 2 or F.shape[0] != p.n or F.dtype != torch.float64 or not F.is_cuda:
                raise ValueError("each block must be cuda float64 of shape (n_k, r_k)")
            if F.shape[1] > 1 and F.stride(1) != 1:
                raise ValueError("unit batch stride required")
        cnt = len(Fs)
        ptrs = (_P * cnt)(*[F.data_ptr() for F in Fs])
        batch = (_I64 * cnt)(*[F.shape[1] for F in Fs])
        ld = (_I64 * cnt)(*[max(F.stride(0), F.shape[1]) for F in Fs])
        return ptrs, batch, ld

    def workspace(self, Fs):
        import torch
        _, batch, _ = self._args(Fs)
        nbytes = lib().pent_group_workspace_size(self._g, batch)
        if self._work is None or self._work.numel() < nbytes:
            self._work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        return self._work

    def solve_(self, Fs, mode: int = 0, stream=None):
        ptrs, batch, ld = self._args(Fs)
        w = self.workspace(Fs)
        _check(lib().pent_group_solve(self._g, ptrs, batch, ld, int(mode), w.data_ptr(), w.numel(),
                                      _stream_ptr(stream)), "group_solve")
        return Fs

    def set_variant(self, variant: int):
        _check(lib().pent_group_set_variant(self._g, int(variant)), "group_set_variant")

    def check(self):
        """Raise if a device-side wait of the last solves timed out."""
        _check(lib().pent_group_check(self._g), "group_check")

    def autotune(self, Fs, stream=None):
        """Time the persistent kernel variants on scratch blocks shaped like
        ``Fs`` and keep the fastest; returns (variant, ms)."""
        _, batch, _ = self._args(Fs)
        v, ms = _I(0), _D(0.0)
        _check(lib().pent_group_autotune(self._g, batch, ctypes.byref(v), ctypes.byref(ms),
                                         _stream_ptr(stream)), "group_autotune")
        return int(v.value), float(ms.value)

    def capture(self, Fs, steps: int, mode: int = 0, stream=None):
        """Executable graph of ``steps`` group solves on ``stream`` (a
        torch.cuda.Stream, not the null stream)."""
        ptrs, batch, ld = self._args(Fs)
        w = self.workspace(Fs)
        gr = lib().pent_group_capture(self._g, ptrs, batch, ld, int(mode), int(steps),
                                      w.data_ptr(), w.numel(), _stream_ptr(stream))
        if not gr:
            raise PentError(lib().pent_last_status(), "group_capture")
        # the graph's kernels read these buffers: keep them (and the plans,
        # through the group) alive as long as the graph
        return Graph(gr, keep=(self, w, list(Fs)))

    def close(self):
        if self._g:
            _check(lib().pent_group_destroy(self._g), "group_destroy")
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An executable HIP graph of captured group solves.  It holds the group,
    its workspace and the right-hand-side blocks it was captured on."""

    def __init__(self, handle, keep=()):
        self._h = handle
        self._keep = keep

    def launch(self, stream=None):
        _check(lib().pent_graph_launch(self._h, _stream_ptr(stream)), "graph_launch")

    def close(self):
        if self._h:
            _check(lib().pent_graph_destroy(self._h), "graph_destroy")
            self._h = None
        self._keep = ()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SystemZeroPivotError(PentError):
    def __init__(self, system: int, row: int):
        super().__init__(ZERO_PIVOT, f"system {system} stopped at row {row}")
        self.system = system
        self.row = row


def solve_rewrite_(a, b, c, d, e, F, work=None, stream=None, check=False):
    """Overwrite F (cuda float64, shape (n, batch)) with the solutions of the
    systems whose own matrices are the columns of a..e (cuda float64, shape
    (n, batch), row-indexed), factoring every system in this call.  With
    ``check`` the call synchronises and raises SystemZeroPivotError."""
    import torch
    n, m = F.shape
    for x in (a, b, c, d, e):
        if x.shape != (n, m) or (m > 1 and x.stride(1) != 1) or x.stride(0) != a.stride(0):
            raise ValueError("diagonals must have F's shape, unit batch stride, one row stride")
    if m > 1 and F.stride(1) != 1:
        raise ValueError("F needs unit batch stride")
    nbytes = lib().pent_rewrite_workspace_size(n, m)
    if work is None:
        work = torch.empty(nbytes, dtype=torch.uint8, device=F.device)
    _check(lib().pent_solve_rewrite(n, *[_dptr(x, "float64") for x in (a, b, c, d, e)],
                                    max(a.stride(0), m), _dptr(F, "float64"), m,
                                    max(F.stride(0), m), work.data_ptr(),
                                    work.numel() * work.element_size(), _stream_ptr(stream)),
           "solve_rewrite")
    if check:
        sy, ro = _I64(0), _I64(0)
        st = lib().pent_rewrite_check(work.data_ptr(), n, ctypes.byref(sy), ctypes.byref(ro))
        if st == ZERO_PIVOT:
            raise SystemZeroPivotError(int(sy.value), int(ro.value))
        _check(st, "rewrite_check")
    return F


class Cyclic:
    """A factored periodic pentadiagonal matrix (pent_cyclic), solved by
    bordering.  Free with close() or a with-block."""

    def __init__(self, handle: int, n: int):
        self._h = handle
        self.n = n

    @classmethod
    def factor(cls, a, b, c, d, e) -> "Cyclic":
        """HOST diagonals a..e of length n, row-indexed with wrap-around."""
        import numpy as np
        arrs = [np.ascontiguousarray(np.asarray(x, dtype=np.float64)) for x in (a, b, c, d, e)]
        n = arrs[2].shape[0]
        if any(x.shape != (n,) for x in arrs):
            raise ValueError("diagonals must all have shape (n,)")
        return cls._made(lib().pent_cyclic_factor(n, *[x.ctypes.data for x in arrs]), n)

    @classmethod
    def factor_d4(cls, n: int, sigma: float) -> "Cyclic":
        """The periodic Crank-Nicolson matrix I + sigma*D4 (wrapped corners)."""
        return cls._made(lib().pent_cyclic_factor_d4(int(n), float(sigma)), n)

    @classmethod
    def _made(cls, h, n):
        if not h:
            st = lib().pent_last_status()
            if st == ZERO_PIVOT:
                raise ZeroPivotError(int(lib().pent_last_pivot_row()))
            raise PentError(st, "cyclic factor")
        return cls(h, int(n))

    def close(self):
        if self._h:
            _check(lib().pent_cyclic_destroy(self._h), "cyclic destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _shape_ok(self, F, name):
        if F.dim() != 2 or F.shape[0] != self.n or (F.shape[1] > 1 and F.stride(1) != 1):
            raise ValueError(f"{name} must have shape ({self.n}, batch) with unit batch stride")

    def solve_(self, F, stream=None):
        """Overwrite F (cuda float64, shape (n, batch)) with A^{-1} F."""
        self._shape_ok(F, "F")
        m = F.shape[1]
        _check(lib().pent_cyclic_solve(self._h, _dptr(F, "float64"), m, max(F.stride(0), m),
                                       _stream_ptr(stream)), "cyclic solve")
        return F

    def cn_rhs(self, C, R, stream=None):
        """R = 2C - AC (the explicit Crank-Nicolson half step), C and R cuda
        float64 of shape (n, batch), not overlapping."""
        self._shape_ok(C, "C")
        self._shape_ok(R, "R")
        if R.shape != C.shape:
            raise ValueError("C and R must have the same shape")
        m = C.shape[1]
        _check(lib().pent_cyclic_cn_rhs(self._h, _dptr(C, "float64"), max(C.stride(0), m),
                                        _dptr(R, "float64"), max(R.stride(0), m), m,
                                        _stream_ptr(stream)), "cyclic cn_rhs")
        return R

    def cn_step(self, C, X, stream=None):
        """X = A^{-1} (2C - AC): one Crank-Nicolson step from C into X (cuda
        float64, shape (n, batch), different buffers)."""
        self._shape_ok(C, "C")
        self._shape_ok(X, "X")
        if X.shape != C.shape:
            raise ValueError("C and X must have the same shape")
        m = C.shape[1]
        _check(lib().pent_cyclic_cn_step(self._h, _dptr(C, "float64"), max(C.stride(0), m),
                                         _dptr(X, "float64"), max(X.stride(0), m), m,
                                         _stream_ptr(stream)), "cyclic cn_step")
        return X

    def cn_steps_(self, C, steps: int, R=None, stream=None):
        """Advance ``steps`` Crank-Nicolson steps ping-ponging between C and
        R (scratch of C's shape, allocated when absent); returns (state,
        other buffer)."""
        import torch
        if R is None:
            R = torch.empty_like(C)
        for _ in range(int(steps)):
            self.cn_step(C, R, stream)
            C, R = R, C
        return C, R

    def set_schedule(self, kind: int, seg_rows: int = 64):
        """0 automatic, 1 E-solve + update kernels, 2 single pass."""
        _check(lib().pent_cyclic_set_schedule(self._h, int(kind), int(seg_rows)),
               "cyclic set_schedule")

    def schedule_for(self, batch: int, cn: bool = False):
        k, sr = _I(0), _I(0)
        _check(lib().pent_cyclic_query_schedule(self._h, int(batch), int(bool(cn)),
                                                ctypes.byref(k), ctypes.byref(sr)),
               "cyclic query_schedule")
        return int(k.value), int(sr.value)

    def check(self):
        """Raise PentError(TIMEOUT) if a single-pass wait ran out (blocking)."""
        _check(lib().pent_cyclic_check(self._h), "cyclic check")

    def bordering(self):
        """(Z = E^{-1} k of shape (n-2, 2), [C2 - h^T Z]^{-1} of shape (2, 2))."""
        import numpy as np
        Z = np.empty((self.n - 2, 2))
        Minv = np.empty((2, 2))
        _check(lib().pent_cyclic_bordering(self._h, Z.ctypes.data, Minv.ctypes.data), "bordering")
        return Z, Minv


def ch2d_rhs(C, R, dt, h: float, stream=None):
    """R = C + dt[k] * Lap_h(C^3 - C) for C, R of shape (ny, ninst, nx)
    (cuda float64, contiguous) and dt of shape (ninst,)."""
    ny, ninst, nx = C.shape
    for t in (C, R):
        if not t.is_contiguous() or t.shape != C.shape:
            raise ValueError("C and R must be contiguous (ny, ninst, nx)")
    if dt.numel() != ninst:
        raise ValueError("one dt per instance")
    _check(lib().pent_ch2d_rhs(_dptr(C, "float64"), _dptr(R, "float64"), ny, ninst, nx,
                               _dptr(dt, "float64"), float(h), _stream_ptr(stream)), "ch2d_rhs")
    return R


def ch2d_step(plan_x: "Plan", plan_y: "Plan", C, R, dt, h: float, stream=None):
    """One split-implicit Cahn-Hilliard step: C <- next state, R scratch."""
    ny, ninst, nx = C.shape
    for t in (C, R):
        if not t.is_contiguous() or t.shape != C.shape:
            raise ValueError("C and R must be contiguous (ny, ninst, nx)")
    _check(lib().pent_ch2d_step(plan_x.handle, plan_y.handle, _dptr(C, "float64"),
                                _dptr(R, "float64"), ny, ninst, nx, _dptr(dt, "float64"),
                                float(h), _stream_ptr(stream)), "ch2d_step")
    return C


def stream_copy(src, dst, stream=None):
    """dst = src (cuda float64, shape (n, batch), unit batch stride) through
    the single pass's block pattern: the layout's copy ceiling."""
    if src.shape != dst.shape or src.dim() != 2:
        raise ValueError("src and dst must have one (n, batch) shape")
    n, m = src.shape
    for t in (src, dst):
        if m > 1 and t.stride(1) != 1:
            raise ValueError("unit batch stride required")
    _check(lib().pent_stream_copy(_dptr(src, "float64"), max(src.stride(0), m), _dptr(dst, "float64"),
                                  max(dst.stride(0), m), n, m, _stream_ptr(stream)), "stream_copy")
    return dst


def stream_copy_shaped(src, dst, tiles_across: int, waves_down: int, stream=None):
    """stream_copy with another workgroup shape (tiles side by side x waves
    down the rows; see pent_stream_copy_shaped)."""
    if src.shape != dst.shape or src.dim() != 2:
        raise ValueError("src and dst must have one (n, batch) shape")
    n, m = src.shape
    for t in (src, dst):
        if m > 1 and t.stride(1) != 1:
            raise ValueError("unit batch stride required")
    _check(lib().pent_stream_copy_shaped(_dptr(src, "float64"), max(src.stride(0), m),
                                         _dptr(dst, "float64"), max(dst.stride(0), m), n, m,
                                         int(tiles_across), int(waves_down), _stream_ptr(stream)),
           "stream_copy_shaped")
    return dst
