"""Python binding of libtda (argument marshalling only).

Every step of the likelihood runs in the HIP library ``libtda.so`` built in this
directory (``python -m paper_2603_06010_amd.build``).  PyTorch provides device
memory and streams: tensors are passed by device pointer together with the
current HIP stream.  If the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

__all__ = ["TdaError", "Handle", "loglik_multi", "release_workspaces", "acf_estimate",
           "load_library", "LIB_PATH",
           "timing_enable", "timing_read", "Server", "Plan",
           "PREC_FP64", "PREC_MIXED", "EXPORTED_SYMBOLS"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtda.so")
PREC_FP64, PREC_MIXED, PREC_GS, PREC_CDO = 0, 1, 2, 3
EXPORTED_SYMBOLS = [
    "tda_cov_build", "tda_factor", "tda_set_data", "tda_loglik", "tda_loglik_ex",
    "tda_loglik_terms", "tda_snr", "tda_whitened_residual", "tda_acf_estimate",
    "tda_loglik_multi", "tda_release_workspaces", "tda_info", "tda_destroy", "tda_status_str",
    "tda_last_error",
    "tda_loglik_fp64_noalloc",
    "tda_timing_enable", "tda_timing_read", "tda_plan_create", "tda_plan_execute",
    "tda_plan_destroy",
    "tda_server_create", "tda_server_add_dataset", "tda_server_submit", "tda_server_poll",
    "tda_server_wait", "tda_server_stats", "tda_server_destroy",
]

_STATUS = {0: "TDA_OK", 1: "TDA_EINVAL", 2: "TDA_ENOTSPD", 3: "TDA_ENOMEM", 4: "TDA_ESTATE",
           5: "TDA_ENODEV", 6: "TDA_EHIP", 7: "TDA_EINTERNAL", 8: "TDA_EAGAIN"}


class TdaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = _STATUS.get(status, str(status))


class _Segment(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("length", ctypes.c_int64)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_size_t),
                ("allocator", ctypes.POINTER(_Allocator))]


class _TorchAllocator:
    """tda_allocator backed by PyTorch's caching allocator on one device, so the handle's
    device memory is owned (and counted) by torch."""

    def __init__(self, device: int):
        import torch
        self.device = int(device)

        def _alloc(nbytes, _ctx):
            # the library calls this with the handle's device current
            try:
                dev = self.device if self.device >= 0 else torch.cuda.current_device()
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev)
            except Exception:  # out of memory: the library reports TDA_ENOMEM
                return None

        def _free(ptr, _ctx):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass

        self._fns = (_ALLOC_FN(_alloc), _FREE_FN(_free))
        self.struct = _Allocator(self._fns[0], self._fns[1], None)


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_eff", ctypes.c_int64), ("n_pad", ctypes.c_int64),
                ("n_segments", ctypes.c_int64), ("logdet", ctypes.c_double),
                ("fail_row", ctypes.c_int64), ("fail_segment", ctypes.c_int32),
                ("factored", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("data_set", ctypes.c_int32), ("device_bytes", ctypes.c_size_t)]


class _KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("count", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class _Work(ctypes.Structure):
    _fields_ = [("h", ctypes.c_void_p), ("d", ctypes.c_void_p), ("H", ctypes.c_void_p),
                ("B", ctypes.c_int64), ("ldh", ctypes.c_int64), ("out", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtda.so and declare its C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libtda.so not found at {path}; build it with "
                      "`python -m paper_2603_06010_amd.build`")
    L = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.tda_cov_build.argtypes = [vp, i64, i64, vp, vp, i64, vp, ctypes.POINTER(vp)]
    L.tda_factor.argtypes = [vp]
    L.tda_set_data.argtypes = [vp, vp, vp]
    L.tda_loglik.argtypes = [vp, vp, vp, i64, i64, vp, vp]
    L.tda_loglik_ex.argtypes = [vp, vp, vp, i64, i64, vp, i32, vp]
    L.tda_loglik_terms.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp, i32, vp]
    L.tda_snr.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp, vp, i32, vp]
    L.tda_loglik_fp64_noalloc.argtypes = [vp, vp, vp, i64, i64, vp, vp]
    L.tda_whitened_residual.argtypes = [vp, vp, vp, i64, i64, vp, vp, i64, vp]
    L.tda_acf_estimate.argtypes = [vp, i64, i64, i32, i64, vp, vp]
    L.tda_loglik_multi.argtypes = [vp, i64, i32, vp]
    L.tda_release_workspaces.argtypes = [i32]
    L.tda_info.argtypes = [vp, ctypes.POINTER(_Info)]
    L.tda_destroy.argtypes = [vp]
    L.tda_status_str.argtypes = [ctypes.c_int]
    L.tda_status_str.restype = ctypes.c_char_p
    L.tda_last_error.argtypes = []
    L.tda_last_error.restype = ctypes.c_char_p
    L.tda_timing_enable.argtypes = [i32]
    L.tda_timing_read.argtypes = [vp, i32, ctypes.POINTER(i32), i32]
    for f in ("tda_cov_build", "tda_factor", "tda_set_data", "tda_loglik", "tda_loglik_ex",
              "tda_loglik_terms", "tda_snr", "tda_whitened_residual", "tda_acf_estimate",
              "tda_loglik_multi", "tda_info", "tda_destroy", "tda_timing_enable",
              "tda_timing_read", "tda_loglik_fp64_noalloc", "tda_release_workspaces"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        msg = _lib.tda_last_error().decode(errors="replace")
        raise TdaError(status, msg)


_ENOMEM = 3


def _call(fn, *args):
    """Call a library entry point; on TDA_ENOMEM hand PyTorch's cached device memory back
    to the driver once and try again (handle buffers come from torch's caching allocator,
    which keeps what it frees, while the library's own workspaces use hipMalloc)."""
    st = fn(*args)
    if st == _ENOMEM:
        import torch
        torch.cuda.empty_cache()
        st = fn(*args)
    _check(st)


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64:
        raise TypeError("expected float64")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _precision(p) -> int:
    if p in (None,):
        return None
    if isinstance(p, str):
        return {"fp64": PREC_FP64, "mixed": PREC_MIXED, "gs": PREC_GS, "cdo": PREC_CDO}[p.lower()]
    return int(p)


class Handle:
    """One detector's noise model: covariance blocks, FP64 factor and evaluations.

    acf: float64[>= longest segment]; N: samples; gap_mask: uint8[N] (1 = excluded) or None;
    segments: [(offset, length), ...] or None for one segment [0, N).
    allocator: "torch" (default) passes PyTorch's caching allocator as the handle's
    tda_allocator, so torch owns and counts its device memory; "hip" lets the library
    call hipMalloc itself.
    """

    def __init__(self, acf, N: int, gap_mask=None, segments: Optional[Sequence] = None,
                 precision="fp64", device: int = -1, hbm_budget: int = 0,
                 compact: bool = False, allocator: str = "torch"):
        L = load_library()
        self._h = ctypes.c_void_p()
        self._alloc = None
        if allocator == "torch":
            self._alloc = _TorchAllocator(device)
        elif allocator != "hip":
            raise ValueError("allocator must be 'torch' or 'hip'")
        acf = np.ascontiguousarray(acf, dtype=np.float64)
        self._acf = acf
        mask_ptr = None
        if gap_mask is not None:
            m = np.ascontiguousarray(gap_mask, dtype=np.uint8)
            if m.shape != (N,):
                raise ValueError("gap_mask must have length N")
            self._mask = m
            mask_ptr = m.ctypes.data
        seg_arr, nseg = None, 0
        if segments is not None:
            nseg = len(segments)
            seg_arr = (_Segment * max(nseg, 1))(*[_Segment(int(o), int(l)) for o, l in segments])
        opt = _Options(ctypes.sizeof(_Options), _precision(precision), int(device),
                       1 if compact else 0, int(hbm_budget),
                       ctypes.pointer(self._alloc.struct) if self._alloc else None)
        h = ctypes.c_void_p()
        _call(L.tda_cov_build, acf.ctypes.data, len(acf), int(N), mask_ptr,
              ctypes.cast(seg_arr, ctypes.c_void_p) if seg_arr is not None else None,
              nseg, ctypes.byref(opt), ctypes.byref(h))
        self._h = h
        self.N = int(N)
        self.precision = _precision(precision)

    @property
    def ptr(self):
        return self._h.value

    def factor(self):
        _call(_lib.tda_factor, self._h)
        return self

    def set_data(self, d, stream=None):
        _call(_lib.tda_set_data, self._h, _ptr(d), _stream(stream))

    def loglik(self, d, H, out=None, precision=None, stream=None):
        import torch
        if H.dim() != 2:
            raise ValueError("H must be 2-D")
        B = H.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=H.device)
        if B == 0:
            return out
        if H.stride(1) != 1:
            raise ValueError("H rows must be contiguous")
        p = self.precision if precision is None else _precision(precision)
        _call(_lib.tda_loglik_ex, self._h, _ptr(d), _ptr(H), B, H.stride(0), _ptr(out), p,
              _stream(stream))
        return out

    def loglik_noalloc(self, d, H, out, stream=None):
        """FP64 logL through tda_loglik_fp64_noalloc (no device allocation; `out` given)."""
        if H.dim() != 2 or H.stride(1) != 1:
            raise ValueError("H must be 2-D with contiguous rows")
        _check(_lib.tda_loglik_fp64_noalloc(self._h, _ptr(d), _ptr(H), H.shape[0], H.stride(0),
                                            _ptr(out), _stream(stream)))
        return out

    def loglik_terms(self, d, H, precision=None, want_dh=True, want_hh=True, stream=None):
        """(logL, <d,h>, <h,h>) per template through tda_loglik_terms; an inner product
        not asked for comes back as None."""
        import torch
        if H.dim() != 2:
            raise ValueError("H must be 2-D")
        if H.stride(1) != 1:
            raise ValueError("H rows must be contiguous")
        B = H.shape[0]
        mk = lambda: torch.empty(B, dtype=torch.float64, device=H.device)
        out = mk()
        dh = mk() if want_dh else None
        hh = mk() if want_hh else None
        if B == 0:
            return out, dh, hh
        p = self.precision if precision is None else _precision(precision)
        _call(_lib.tda_loglik_terms, self._h, _ptr(d), _ptr(H), B, H.stride(0), _ptr(out),
              _ptr(dh) if dh is not None else None, _ptr(hh) if hh is not None else None, p,
              _stream(stream))
        return out, dh, hh

    def whitened_residual(self, d, H, stream=None):
        """(logL, W): W[b] = L^-1 (d - h_b) over the retained samples (segments
        concatenated), from the FP64 solve, through tda_whitened_residual."""
        import torch
        if H.dim() != 2:
            raise ValueError("H must be 2-D")
        if H.stride(1) != 1:
            raise ValueError("H rows must be contiguous")
        B = H.shape[0]
        n_eff = self.info()["n_eff"]
        out = torch.empty(B, dtype=torch.float64, device=H.device)
        W = torch.empty((B, n_eff), dtype=torch.float64, device=H.device)
        if B == 0:
            return out, W
        _call(_lib.tda_whitened_residual, self._h, _ptr(d), _ptr(H), B, H.stride(0), _ptr(out),
              _ptr(W), W.stride(0), _stream(stream))
        return out, W

    def snr(self, d, H, precision=None, stream=None):
        """Time-domain SNRs per template (Sec. II.B item 7) through tda_snr, computed in
        the library: {"loglik", "rho_mf" = <d,h>/sqrt(<h,h>), "rho_opt" = sqrt(<h,h>),
        "rho_eff2" = <d,d> - <r,r>}."""
        import torch
        if H.dim() != 2:
            raise ValueError("H must be 2-D")
        if H.stride(1) != 1:
            raise ValueError("H rows must be contiguous")
        B = H.shape[0]
        mk = lambda: torch.empty(B, dtype=torch.float64, device=H.device)
        out, mf, opt, eff2 = mk(), mk(), mk(), mk()
        if B:
            p = self.precision if precision is None else _precision(precision)
            _call(_lib.tda_snr, self._h, _ptr(d), _ptr(H), B, H.stride(0), _ptr(out), _ptr(mf),
                  _ptr(opt), _ptr(eff2), p, _stream(stream))
        return {"loglik": out, "rho_mf": mf, "rho_opt": opt, "rho_eff2": eff2}

    def info(self) -> dict:
        i = _Info()
        _check(_lib.tda_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in _Info._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.tda_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(on: bool = True):
    """Record HIP events around every library kernel launch (see tda_timing_read)."""
    _check(load_library().tda_timing_enable(1 if on else 0))


def timing_read(reset: bool = True) -> dict:
    """{kernel name: (launch count, total ms)} of the launches timed so far."""
    L = load_library()
    arr = (_KernelTime * 64)()
    n = ctypes.c_int32()
    _check(L.tda_timing_read(ctypes.cast(arr, ctypes.c_void_p), 64, ctypes.byref(n),
                             1 if reset else 0))
    return {arr[k].name.decode(): (arr[k].count, arr[k].total_ms) for k in range(min(n.value, 64))}


ACF_DIRECT, ACF_WELCH = 0, 1


def acf_estimate(x, n_lags, method="welch", seg_len=None, stream=None):
    """Autocovariance of the device float64 strain x through tda_acf_estimate; returns a
    new device tensor of n_lags values."""
    import torch
    L = load_library()
    m = {"direct": ACF_DIRECT, "welch": ACF_WELCH}[method] if isinstance(method, str) else int(method)
    if x.dtype != torch.float64 or x.dim() != 1 or not x.is_contiguous():
        raise ValueError("x must be a contiguous 1-D float64 tensor")
    out = torch.empty(n_lags, dtype=torch.float64, device=x.device)
    _call(L.tda_acf_estimate, _ptr(x), x.shape[0], n_lags, m, int(seg_len or 0), _ptr(out),
          _stream(stream))
    return out


def loglik_multi(items, precision="fp64", stream=None):
    """items: sequence of (Handle, d, H, out) -- items sharing `out` are summed."""
    L = load_library()
    arr = (_Work * max(len(items), 1))()
    for k, (h, d, H, out) in enumerate(items):
        arr[k] = _Work(h.ptr, _ptr(d), _ptr(H), H.shape[0], H.stride(0), _ptr(out))
    _call(L.tda_loglik_multi, ctypes.cast(arr, ctypes.c_void_p), len(items),
          _precision(precision), _stream(stream))


def release_workspaces(device=None):
    """Free the workspaces batched evaluations keep between calls (tda_release_workspaces)."""
    L = load_library()
    _check(L.tda_release_workspaces(-1 if device is None else int(device)))


class _ServerOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("staging_bytes", ctypes.c_size_t), ("dataset_budget_bytes", ctypes.c_size_t)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("templates", ctypes.c_int64), ("max_queue_depth", ctypes.c_int64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("mean_templates_per_launch", ctypes.c_double), ("busy_s", ctypes.c_double)]


def _declare_server(L):
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.tda_server_create.argtypes = [vp, ctypes.POINTER(vp)]
    L.tda_server_add_dataset.argtypes = [vp, vp, vp, ctypes.POINTER(i32)]
    L.tda_server_submit.argtypes = [vp, i32, vp, i64, i64, vp, ctypes.POINTER(ctypes.c_uint64)]
    L.tda_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32)]
    L.tda_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double]
    L.tda_server_stats.argtypes = [vp, ctypes.POINTER(_ServerStats), i32]
    L.tda_server_destroy.argtypes = [vp]
    for f in ("tda_server_create", "tda_server_add_dataset", "tda_server_submit",
              "tda_server_poll", "tda_server_wait", "tda_server_stats", "tda_server_destroy"):
        getattr(L, f).restype = ctypes.c_int


class Server:
    """Continuous-batching request server over resident datasets (see tda.h)."""

    EAGAIN = 8

    def __init__(self, precision="mixed", n_slots=2, max_batch=1024, max_queue=1 << 16,
                 staging_bytes=64 << 20, dataset_budget_bytes=0, device=-1):
        L = load_library()
        _declare_server(L)
        opt = _ServerOptions(ctypes.sizeof(_ServerOptions), int(device), _precision(precision),
                             int(n_slots), int(max_batch), int(max_queue), int(staging_bytes),
                             int(dataset_budget_bytes))
        s = ctypes.c_void_p()
        _call(L.tda_server_create, ctypes.byref(opt), ctypes.byref(s))
        self._s = s
        self._keep = []

    def add_dataset(self, handle: Handle, d) -> int:
        i = ctypes.c_int32()
        _call(_lib.tda_server_add_dataset, self._s, handle.ptr, _ptr(d), ctypes.byref(i))
        self._keep.append((handle, d))
        return i.value

    def submit(self, dataset: int, H, out) -> Optional[int]:
        """Returns a ticket, or None if the request was not admitted (TDA_EAGAIN)."""
        t = ctypes.c_uint64()
        st = _lib.tda_server_submit(self._s, int(dataset), _ptr(H), H.shape[0], H.stride(0),
                                    _ptr(out), ctypes.byref(t))
        if st == self.EAGAIN:
            return None
        _check(st)
        return t.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int32()
        _check(_lib.tda_server_poll(self._s, ticket, ctypes.byref(done)))
        return bool(done.value)

    def wait(self, ticket: int, timeout_s: float = 60.0):
        _check(_lib.tda_server_wait(self._s, ticket, float(timeout_s)))

    def stats(self, reset=False) -> dict:
        st = _ServerStats()
        _check(_lib.tda_server_stats(self._s, ctypes.byref(st), 1 if reset else 0))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value:
            _lib.tda_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Frozen batched evaluation, optionally replayed as a HIP graph (see tda.h)."""

    def __init__(self, items, precision="mixed"):
        L = load_library()
        vp = ctypes.c_void_p
        L.tda_plan_create.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(vp)]
        L.tda_plan_execute.argtypes = [vp, vp, ctypes.c_int32]
        L.tda_plan_destroy.argtypes = [vp]
        for f in ("tda_plan_create", "tda_plan_execute", "tda_plan_destroy"):
            getattr(L, f).restype = ctypes.c_int
        arr = (_Work * len(items))()
        for k, (h, d, H, out) in enumerate(items):
            arr[k] = _Work(h.ptr, _ptr(d), _ptr(H), H.shape[0], H.stride(0), _ptr(out))
        self._keep = list(items)
        p = vp()
        _call(L.tda_plan_create, ctypes.cast(arr, vp), len(items), _precision(precision),
              ctypes.byref(p))
        self._p = p

    def execute(self, stream=None, graph=False):
        _check(_lib.tda_plan_execute(self._p, _stream(stream), 1 if graph else 0))

    def close(self):
        if getattr(self, "_p", None) is not None and self._p.value:
            _lib.tda_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
