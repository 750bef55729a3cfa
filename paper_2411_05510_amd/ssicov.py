"""Thin Python binding of libssicov.so (include/ssicov.h).

Argument marshalling only: every step of the identification runs in the
library's HIP kernels.  Device buffers are torch CUDA tensors; all calls are
ordered on the context's stream, which defaults to torch's current stream so
that torch allocations and library work stay ordered.  There is no fallback:
if the library is missing or no gfx950 device is present, calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
# SSI_LIBRARY selects another build of the same library (the host-sanitized
# one of build.build_sanitized, for the sanitizer test)
LIB_PATH = os.environ.get("SSI_LIBRARY") or os.path.join(HERE, "libssicov.so")

SSI_OK, SSI_EINVAL, SSI_ENOMEM, SSI_EDEVICE, SSI_ENOCONV, SSI_EINTERNAL, SSI_EBUSY = range(7)
SVD_FULL, SVD_RANDOMIZED = 0, 1
PREC_FP32, PREC_BF16, PREC_BF16X3, PREC_BF16X6, PREC_FP8 = 0, 1, 2, 3, 4
CORR_FP32, CORR_BF16X6, CORR_F16X3 = 0, 1, 2

# Every symbol include/ssicov.h declares.
EXPORTED = (
    "ssi_create", "ssi_destroy", "ssi_synchronize", "ssi_workspace_bytes",
    "ssi_validate", "ssi_output_layout", "ssi_pole_offset", "ssi_workspace_estimate",
    "ssi_tau", "ssi_lag_rule", "ssi_default_rank", "ssi_status_string",
    "ssi_last_error", "ssi_identify", "ssi_correlate", "ssi_toeplitz",
    "ssi_sketch", "ssi_rsvd", "ssi_svd_full", "ssi_modal", "ssi_set_profiling",
    "ssi_profile_read", "ssi_set_lag_streams", "ssi_set_graphs", "ssi_set_autotune",
    "ssi_set_corr_mode", "ssi_tuned_splits", "ssi_footprint", "ssi_server_create", "ssi_server_destroy",
    "ssi_server_submit", "ssi_server_poll", "ssi_server_wait", "ssi_server_result",
    "ssi_server_release", "ssi_server_get_stats", "ssi_server_last_error", "ssi_stability",
    "ssi_stability_noalloc", "ssi_stability_noalloc_max_slots",
    "ssi_set_eig_max_sweeps", "ssi_set_product_tile_rows", "ssi_set_eig_workgroups", "ssi_set_allocator",
    "ssi_identify_result", "ssi_result_fetch",
    "ssi_result_dims", "ssi_result_poles", "ssi_result_singular_values", "ssi_result_free",
)

POLE_HC, POLE_STABLE_ORDER, POLE_STABLE_LAG, POLE_STABLE = 1, 2, 4, 8

STAGES = ("corr_mfma", "corr_reduce", "toeplitz", "sketch", "products", "orth",
          "small_svd", "shift_ls", "eig", "corr_split")


class SSIError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[status {status}] {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [
        ("fs", ctypes.c_double),
        ("lags", ctypes.POINTER(ctypes.c_int32)),
        ("n_lags", ctypes.c_int32),
        ("order_min", ctypes.c_int32),
        ("order_max", ctypes.c_int32),
        ("order_step", ctypes.c_int32),
        ("svd", ctypes.c_int32),
        ("rank", ctypes.c_int32),
        ("oversample", ctypes.c_int32),
        ("power_iters", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("prec", ctypes.c_int32),
        ("omega", ctypes.c_void_p),
        ("omega_ld", ctypes.c_int64),
        ("refine", ctypes.c_int32),
    ]


class _Layout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("n_lags", "n_orders", "sigma_per_lag", "pole_cap", "l", "n_corr")]


class _StabilityParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("xi_max", "mpc_min", "mpd_max", "alpha_f", "alpha_xi", "alpha_mac")]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("slot", ctypes.c_int32),
                ("t_submit_us", ctypes.c_double), ("t_start_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double), ("footprint", ctypes.c_size_t)]


class _HostResult(ctypes.Structure):
    _fields_ = [("layout", _Layout), ("sigma", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("f", ctypes.c_void_p), ("xi", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("phi", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("queued", ctypes.c_int32),
                ("running", ctypes.c_int32), ("peak_inflight", ctypes.c_int32),
                ("peak_bytes", ctypes.c_uint64), ("held_bytes", ctypes.c_uint64),
                ("budget", ctypes.c_uint64)]


class _Output(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("sigma", "count", "f", "xi", "mu", "phi", "flags")]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def lib() -> ctypes.CDLL:
    """Load libssicov.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        # torch ships its own HIP runtime; load it first so that this library
        # binds to the same one and shares its devices, streams and memory
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_uint64)
        P = ctypes.POINTER(_Params)
        sig = {
            "ssi_create": ([ctypes.c_int, vp, ctypes.POINTER(vp)], ctypes.c_int),
            "ssi_destroy": ([vp], None),
            "ssi_synchronize": ([vp], ctypes.c_int),
            "ssi_workspace_bytes": ([vp], ctypes.c_size_t),
            "ssi_validate": ([P, i32, i64], ctypes.c_int),
            "ssi_output_layout": ([P, i32, i64, ctypes.POINTER(_Layout)], ctypes.c_int),
            "ssi_pole_offset": ([P, i32], i32),
            "ssi_workspace_estimate": ([P, i32, i64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
            "ssi_tau": ([i32, ctypes.c_double], ctypes.c_double),
            "ssi_lag_rule": ([ctypes.c_double, ctypes.c_double, ctypes.c_double], i32),
            "ssi_default_rank": ([i64], i32),
            "ssi_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "ssi_last_error": ([], ctypes.c_char_p),
            "ssi_identify": ([vp, vp, i32, i64, i64, P, ctypes.POINTER(_Output)], ctypes.c_int),
            "ssi_correlate": ([vp, vp, i32, i64, i64, i32, vp], ctypes.c_int),
            "ssi_toeplitz": ([vp, vp, i32, i32, vp, i64], ctypes.c_int),
            "ssi_sketch": ([vp, u64, u32, i64, i32, vp, i64], ctypes.c_int),
            "ssi_rsvd": ([vp, vp, i64, i64, i32, i32, i32, i32, i32, vp, u64, u32, vp, vp],
                         ctypes.c_int),
            "ssi_svd_full": ([vp, vp, i64, i64, i32, vp, vp], ctypes.c_int),
            "ssi_modal": ([vp, vp, vp, i64, i32, i32, P, i32, ctypes.POINTER(_Output)],
                          ctypes.c_int),
            "ssi_set_profiling": ([vp, ctypes.c_int], ctypes.c_int),
            "ssi_profile_read": ([vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int32), i32], ctypes.c_int),
            "ssi_set_lag_streams": ([vp, i32], ctypes.c_int),
            "ssi_set_graphs": ([vp, ctypes.c_int], ctypes.c_int),
            "ssi_set_autotune": ([vp, ctypes.c_int], ctypes.c_int),
            "ssi_set_corr_mode": ([vp, i32], ctypes.c_int),
            "ssi_tuned_splits": ([vp, i32, i32, i32, i32, i32], i32),
            "ssi_footprint": ([P, i32, i64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
            "ssi_server_create": ([ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)],
                                  ctypes.c_int),
            "ssi_server_destroy": ([vp], None),
            "ssi_server_submit": ([vp, vp, i32, i64, i64, P, ctypes.POINTER(u64)], ctypes.c_int),
            "ssi_server_poll": ([vp, u64, ctypes.POINTER(_RequestInfo)], ctypes.c_int),
            "ssi_server_wait": ([vp, u64, ctypes.POINTER(_RequestInfo)], ctypes.c_int),
            "ssi_server_result": ([vp, u64, ctypes.POINTER(ctypes.POINTER(_HostResult))],
                                  ctypes.c_int),
            "ssi_server_release": ([vp, u64], ctypes.c_int),
            "ssi_server_get_stats": ([vp, ctypes.POINTER(_ServerStats)], ctypes.c_int),
            "ssi_server_last_error": ([], ctypes.c_char_p),
            "ssi_stability": ([vp, P, i32, ctypes.POINTER(_Output),
                               ctypes.POINTER(_StabilityParams), vp, vp, vp], ctypes.c_int),
            "ssi_stability_noalloc": ([vp, P, i32, ctypes.POINTER(_Output),
                                       ctypes.POINTER(_StabilityParams), vp, vp, vp],
                                      ctypes.c_int),
            "ssi_stability_noalloc_max_slots": ([], i64),
            "ssi_set_eig_max_sweeps": ([vp, i32], ctypes.c_int),
            "ssi_set_product_tile_rows": ([vp, i32], ctypes.c_int),
            "ssi_set_eig_workgroups": ([vp, i32], ctypes.c_int),
            "ssi_set_allocator": ([vp, _ALLOC_FN, _RELEASE_FN, vp], ctypes.c_int),
            "ssi_identify_result": ([vp, vp, i32, i64, i64, P, ctypes.POINTER(vp)],
                                    ctypes.c_int),
            "ssi_result_fetch": ([vp, P, i32, ctypes.POINTER(_Output), ctypes.POINTER(vp)],
                                 ctypes.c_int),
            "ssi_result_dims": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                 ctypes.POINTER(i32)], ctypes.c_int),
            "ssi_result_poles": ([vp, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.POINTER(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.POINTER(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.POINTER(ctypes.POINTER(ctypes.c_float)),
                                  ctypes.POINTER(i32)], ctypes.c_int),
            "ssi_result_singular_values": ([vp, i32, ctypes.POINTER(i32),
                                            ctypes.POINTER(ctypes.POINTER(ctypes.c_double))],
                                           ctypes.c_int),
            "ssi_result_free": ([vp], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != SSI_OK:
        raise SSIError(status, lib().ssi_last_error().decode())


def _check_srv(status: int) -> None:
    if status != SSI_OK:
        raise SSIError(status, lib().ssi_server_last_error().decode())


# ------------------------------------------------------------ parameters
@dataclasses.dataclass
class Params:
    """Identification parameters (see ssi_params in include/ssicov.h)."""
    fs: float
    lags: Sequence[int]
    order_min: int
    order_max: int
    order_step: int = 2
    svd: int = SVD_RANDOMIZED
    rank: int = 0
    oversample: int = 0
    power_iters: int = 0
    seed: int = 0
    prec: int = PREC_FP32
    omega: object = None        # optional caller sketch: device tensor (m_max, k + p) float32
    refine: int = 0             # reduced precision: last `refine` power iterations in full precision

    def c(self) -> _Params:
        arr = (ctypes.c_int32 * len(self.lags))(*[int(v) for v in self.lags])
        om = None if self.omega is None else _ptr(self.omega)
        ld = 0 if self.omega is None else int(self.omega.stride(0))
        p = _Params(float(self.fs), arr, len(self.lags), int(self.order_min),
                    int(self.order_max), int(self.order_step), int(self.svd),
                    int(self.rank), int(self.oversample), int(self.power_iters),
                    int(self.seed) & 0xFFFFFFFFFFFFFFFF, int(self.prec), om, ld,
                    int(self.refine))
        p._keep = arr  # keep the lag array alive with the struct
        return p

    @property
    def orders(self) -> List[int]:
        return list(range(self.order_min, self.order_max + 1, self.order_step))


def validate(p: Params, l: int, n: int) -> None:
    cp = p.c()
    _check(lib().ssi_validate(ctypes.byref(cp), l, n))


def output_layout(p: Params, l: int, n: int) -> dict:
    cp = p.c()
    lay = _Layout()
    _check(lib().ssi_output_layout(ctypes.byref(cp), l, n, ctypes.byref(lay)))
    return {name: getattr(lay, name) for name, _ in _Layout._fields_}


def pole_offset(p: Params, order_index: int) -> int:
    cp = p.c()
    return int(lib().ssi_pole_offset(ctypes.byref(cp), order_index))


def workspace_estimate(p: Params, l: int, n: int) -> int:
    cp = p.c()
    out = ctypes.c_size_t()
    _check(lib().ssi_workspace_estimate(ctypes.byref(cp), l, n, ctypes.byref(out)))
    return int(out.value)


def footprint(p: Params, l: int, n: int) -> int:
    """Device bytes one identification of these sizes holds (admission)."""
    cp = p.c()
    out = ctypes.c_size_t()
    _check(lib().ssi_footprint(ctypes.byref(cp), l, n, ctypes.byref(out)))
    return int(out.value)


def tau(jb: int, fs: float) -> float:
    return float(lib().ssi_tau(jb, fs))


def lag_rule(fs: float, f0: float, factor: float = 10.0) -> int:
    return int(lib().ssi_lag_rule(fs, f0, factor))


def default_rank(t_size: int) -> int:
    return int(lib().ssi_default_rank(t_size))


# --------------------------------------------------------------- context
def _ptr(t) -> int:
    return int(t.data_ptr())


class Context:
    """A library context on one GPU, ordered on a HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        handle = ctypes.c_void_p()
        _check(lib().ssi_create(device, ctypes.c_void_p(stream.cuda_stream),
                                ctypes.byref(handle)))
        self._h = handle
        self.device = device

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().ssi_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self) -> None:
        _check(lib().ssi_synchronize(self._h))

    @property
    def workspace_bytes(self) -> int:
        return int(lib().ssi_workspace_bytes(self._h))

    def set_profiling(self, enable: bool) -> None:
        _check(lib().ssi_set_profiling(self._h, 1 if enable else 0))

    def set_lag_streams(self, n: int) -> None:
        _check(lib().ssi_set_lag_streams(self._h, n))

    def set_graphs(self, enable: bool) -> None:
        _check(lib().ssi_set_graphs(self._h, 1 if enable else 0))

    def set_autotune(self, enable: bool) -> None:
        _check(lib().ssi_set_autotune(self._h, 1 if enable else 0))

    def set_product_tile_rows(self, rows: int) -> None:
        _check(lib().ssi_set_product_tile_rows(self._h, rows))

    def set_eig_workgroups(self, n: int) -> None:
        """Workgroups of the eigen-analysis launch (0: one per CU)."""
        _check(lib().ssi_set_eig_workgroups(self._h, n))

    def set_eig_max_sweeps(self, sweeps_per_row: int) -> None:
        _check(lib().ssi_set_eig_max_sweeps(self._h, sweeps_per_row))

    def use_torch_allocator(self, enable: bool = True) -> None:
        """Workspace from torch's caching allocator (ssi_set_allocator)."""
        import torch
        if not enable:
            _check(lib().ssi_set_allocator(self._h, _ALLOC_FN(), _RELEASE_FN(), None))
            self._alloc_cbs = None
            return
        dev, stream = self.device, self._stream

        def _alloc(nbytes, _user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            except Exception:
                return None

        def _release(ptr, _user):
            torch.cuda.caching_allocator_delete(ptr)

        cbs = (_ALLOC_FN(_alloc), _RELEASE_FN(_release))
        _check(lib().ssi_set_allocator(self._h, cbs[0], cbs[1], None))
        self._alloc_cbs = cbs          # the callbacks must outlive the context's use of them

    def set_corr_mode(self, mode: int) -> None:
        """CORR_FP32, CORR_BF16X6 or CORR_F16X3 (the default) for the correlation products."""
        _check(lib().ssi_set_corr_mode(self._h, mode))

    def tuned_splits(self, kind: int, trans: bool, m: int, n: int, k: int) -> int:
        return int(lib().ssi_tuned_splits(self._h, kind, 1 if trans else 0, m, n, k))

    def profile_read(self) -> dict:
        """{stage: (total ms, calls)} accumulated since the last read."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_int32 * n)()
        _check(lib().ssi_profile_read(self._h, ms, calls, n))
        return {name: (float(ms[i]), int(calls[i])) for i, name in enumerate(STAGES)}

    # ---------------------------------------------------------- stages
    def correlate(self, y, n_corr: int, out=None):
        """R (n_corr, l, l) float32 of the device record y (l, n) float32."""
        import torch
        l, n = y.shape
        if out is None:
            out = torch.empty((n_corr, l, l), dtype=torch.float32, device=y.device)
        _check(lib().ssi_correlate(self._h, _ptr(y), l, n, y.stride(0), n_corr, _ptr(out)))
        return out

    def toeplitz(self, r, jb: int, ldt: Optional[int] = None, out=None):
        import torch
        l = r.shape[1]
        m = jb * l
        if ldt is None:
            ldt = m
        if out is None:
            out = torch.empty((m, ldt), dtype=torch.float32, device=r.device)
        _check(lib().ssi_toeplitz(self._h, _ptr(r), l, jb, _ptr(out), ldt))
        return out

    def sketch(self, seed: int, stream: int, m: int, ell: int, out=None):
        import torch
        if out is None:
            out = torch.empty((m, ell), dtype=torch.float32, device=f"cuda:{self.device}")
        _check(lib().ssi_sketch(self._h, seed & 0xFFFFFFFFFFFFFFFF, stream, m, ell, _ptr(out),
                                out.stride(0)))
        return out

    def rsvd(self, t, k: int, p: int, q: int, omega=None, seed: int = 0, stream: int = 0,
             prec: int = PREC_FP32, refine: int = 0):
        """(U (m, k) float64, sigma (k,) float64) of the device matrix t (m, ldt) float32."""
        import torch
        m = t.shape[0]
        u = torch.empty((m, k), dtype=torch.float64, device=t.device)
        s = torch.empty((k,), dtype=torch.float64, device=t.device)
        om = _ptr(omega) if omega is not None else None
        _check(lib().ssi_rsvd(self._h, _ptr(t), m, t.stride(0), k, p, q, prec, refine, om,
                              seed & 0xFFFFFFFFFFFFFFFF, stream, _ptr(u), _ptr(s)))
        return u, s

    def svd_full(self, t, k: int):
        import torch
        m = t.shape[0]
        u = torch.empty((m, k), dtype=torch.float64, device=t.device)
        s = torch.empty((k,), dtype=torch.float64, device=t.device)
        _check(lib().ssi_svd_full(self._h, _ptr(t), m, t.stride(0), k, _ptr(u), _ptr(s)))
        return u, s

    def stability(self, out: "Output", l: int, xi_max: float = 0.10, mpc_min: float = 0.60,
                  mpd_max: float = 0.50, alpha_f: float = 0.01, alpha_xi: float = 0.03,
                  alpha_mac: float = 0.02, noalloc: bool = False, into=None):
        """(mpc, mpd, flags) device tensors [n_lags, pole_cap] of the poles in out.
        noalloc: call ssi_stability_noalloc (static scratch).  into: caller's
        (mpc, mpd, flags) tensors to write instead of new ones."""
        import torch
        lay = out.layout
        shape = (lay["n_lags"], lay["pole_cap"])
        dev = out.f.device
        if into is None:
            mpc = torch.zeros(shape, dtype=torch.float64, device=dev)
            mpd = torch.zeros(shape, dtype=torch.float64, device=dev)
            flags = torch.zeros(shape, dtype=torch.uint8, device=dev)
        else:
            mpc, mpd, flags = into
        cp = out.params.c()
        co = out.c()
        sp = _StabilityParams(xi_max, mpc_min, mpd_max, alpha_f, alpha_xi, alpha_mac)
        fn = lib().ssi_stability_noalloc if noalloc else lib().ssi_stability
        _check(fn(self._h, ctypes.byref(cp), l, ctypes.byref(co), ctypes.byref(sp), _ptr(mpc),
                  _ptr(mpd), _ptr(flags)))
        return mpc, mpd, flags

    # --------------------------------------------------- identification
    def alloc_output(self, p: Params, l: int, n: int) -> "Output":
        import torch
        lay = output_layout(p, l, n)
        dev = f"cuda:{self.device}"
        nl, no, cap = lay["n_lags"], lay["n_orders"], lay["pole_cap"]
        return Output(
            layout=lay, params=p,
            sigma=torch.zeros((nl, lay["sigma_per_lag"]), dtype=torch.float64, device=dev),
            count=torch.zeros((nl, no), dtype=torch.int32, device=dev),
            f=torch.zeros((nl, cap), dtype=torch.float64, device=dev),
            xi=torch.zeros((nl, cap), dtype=torch.float64, device=dev),
            mu=torch.zeros((nl, cap, 2), dtype=torch.float64, device=dev),
            phi=torch.zeros((nl, cap, l, 2), dtype=torch.float32, device=dev),
            flags=torch.zeros((nl, no), dtype=torch.int32, device=dev),
        )

    def modal(self, u, sigma, l: int, p: Params, lag_index: int, out: "Output"):
        cp = p.c()
        m, k = u.shape
        co = out.c()
        _check(lib().ssi_modal(self._h, _ptr(u), _ptr(sigma), m, k, l, ctypes.byref(cp),
                               lag_index, ctypes.byref(co)))
        return out

    def identify(self, y, p: Params, out: Optional["Output"] = None) -> "Output":
        """Enqueue the whole identification of the record y (l, n): a device
        tensor, or a host (CPU) tensor that the library copies in."""
        l, n = y.shape
        if out is None:
            out = self.alloc_output(p, l, n)
        cp = p.c()
        co = out.c()
        _check(lib().ssi_identify(self._h, _ptr(y), l, n, y.stride(0), ctypes.byref(cp),
                                  ctypes.byref(co)))
        return out

    def identify_result(self, y, p: Params) -> "Result":
        """Synchronous identification (ssi_identify_result) into a host result.
        y: device tensor, host tensor or numpy array (l, n) float32."""
        if isinstance(y, np.ndarray):
            y = np.ascontiguousarray(y, dtype=np.float32)
            l, n = y.shape
            ptr, ld = y.ctypes.data, y.strides[0] // 4
        else:
            l, n = y.shape
            ptr, ld = _ptr(y), y.stride(0)
        cp = p.c()
        h = ctypes.c_void_p()
        st = lib().ssi_identify_result(self._h, ptr, l, n, ld, ctypes.byref(cp), ctypes.byref(h))
        res = Result(h) if h.value else None
        if st != SSI_OK:
            err = SSIError(st, lib().ssi_last_error().decode())
            err.result = res
            raise err
        return res

    def fetch(self, out: "Output", l: int) -> "Result":
        """Host result of the device outputs (ssi_result_fetch)."""
        cp = out.params.c()
        co = out.c()
        h = ctypes.c_void_p()
        st = lib().ssi_result_fetch(self._h, ctypes.byref(cp), l, ctypes.byref(co),
                                    ctypes.byref(h))
        res = Result(h) if h.value else None
        if st != SSI_OK:
            err = SSIError(st, lib().ssi_last_error().decode())
            err.result = res
            raise err
        return res


@dataclasses.dataclass
class Output:
    """Device output buffers of one identification (see ssi_output)."""
    layout: dict
    params: Params
    sigma: object
    count: object
    f: object
    xi: object
    mu: object
    phi: object
    flags: object

    def c(self) -> _Output:
        return _Output(*[_ptr(getattr(self, n)) for n in
                         ("sigma", "count", "f", "xi", "mu", "phi", "flags")])

    def poles(self, lag_index: int, order_index: int) -> dict:
        """Host copy of the poles of one (lag, order)."""
        p = self.params
        off = pole_offset(p, order_index)
        cnt = int(self.count[lag_index, order_index].item())
        sl = slice(off, off + cnt)
        mu = self.mu[lag_index, sl].cpu().numpy()
        phi = self.phi[lag_index, sl].cpu().numpy().astype(np.float64)
        return {
            "f": self.f[lag_index, sl].cpu().numpy(),
            "xi": self.xi[lag_index, sl].cpu().numpy(),
            "mu": mu[:, 0] + 1j * mu[:, 1],
            "phi": phi[..., 0] + 1j * phi[..., 1],
            "flag": int(self.flags[lag_index, order_index].item()),
        }


class Result:
    """Host result of one identification (ssi_result_* accessors)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().ssi_result_free(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def dims(self) -> dict:
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().ssi_result_dims(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"n_lags": a.value, "n_orders": b.value, "l": c.value}

    def poles(self, lag_index: int, order_index: int) -> dict:
        order, cnt, flag = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        pd = [ctypes.POINTER(ctypes.c_double)() for _ in range(3)]
        pf = ctypes.POINTER(ctypes.c_float)()
        _check(lib().ssi_result_poles(self._h, lag_index, order_index, ctypes.byref(order),
                                      ctypes.byref(cnt), *[ctypes.byref(x) for x in pd],
                                      ctypes.byref(pf), ctypes.byref(flag)))
        k, l = cnt.value, self.dims()["l"]

        def arr(ptr, n, dt):
            return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dt).copy() if n else \
                np.zeros(0, dt)

        mu = arr(pd[2], 2 * k, np.float64).reshape(k, 2)
        phi = arr(pf, 2 * k * l, np.float64).reshape(k, l, 2)
        return {"order": order.value, "f": arr(pd[0], k, np.float64),
                "xi": arr(pd[1], k, np.float64), "mu": mu[:, 0] + 1j * mu[:, 1],
                "phi": phi[..., 0] + 1j * phi[..., 1], "flag": flag.value}

    def singular_values(self, lag_index: int) -> np.ndarray:
        n = ctypes.c_int32()
        p = ctypes.POINTER(ctypes.c_double)()
        _check(lib().ssi_result_singular_values(self._h, lag_index, ctypes.byref(n),
                                                ctypes.byref(p)))
        return np.ctypeslib.as_array(p, shape=(n.value,)).copy()


# --------------------------------------------------------------- serving
class Server:
    """Continuous-batching identification server (ssi_server_* in the header).

    submit() copies the host record and returns a ticket at once; the
    library's dispatcher admits requests to GPU slots as slots and device
    memory free up."""

    def __init__(self, device: int = 0, max_inflight: int = 8, hbm_budget: int = 0):
        cfg = _ServerConfig(device, max_inflight, hbm_budget)
        h = ctypes.c_void_p()
        _check_srv(lib().ssi_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().ssi_server_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def submit(self, y: np.ndarray, p: Params) -> int:
        y = np.ascontiguousarray(y, dtype=np.float32)
        l, n = y.shape
        cp = p.c()
        t = ctypes.c_uint64()
        _check_srv(lib().ssi_server_submit(self._h, y.ctypes.data, l, n, n, ctypes.byref(cp),
                                           ctypes.byref(t)))
        return int(t.value)

    @staticmethod
    def _info(inf: _RequestInfo) -> dict:
        return {"status": inf.status, "slot": inf.slot, "t_submit_us": inf.t_submit_us,
                "t_start_us": inf.t_start_us, "t_done_us": inf.t_done_us,
                "footprint": int(inf.footprint)}

    def poll(self, ticket: int):
        """Request info if finished, else None."""
        inf = _RequestInfo()
        st = lib().ssi_server_poll(self._h, ticket, ctypes.byref(inf))
        if st == SSI_EBUSY:
            return None
        _check_srv(st)
        return self._info(inf)

    def wait(self, ticket: int) -> dict:
        inf = _RequestInfo()
        _check_srv(lib().ssi_server_wait(self._h, ticket, ctypes.byref(inf)))
        return self._info(inf)

    def result(self, ticket: int) -> dict:
        """Host copies (numpy) of a finished request's outputs."""
        rp = ctypes.POINTER(_HostResult)()
        _check_srv(lib().ssi_server_result(self._h, ticket, ctypes.byref(rp)))
        r = rp.contents
        lay = {name: getattr(r.layout, name) for name, _ in _Layout._fields_}
        nl, no, cap, l = lay["n_lags"], lay["n_orders"], lay["pole_cap"], lay["l"]

        def arr(ptr, ctype, shape):
            n = int(np.prod(shape))
            buf = ctypes.cast(ptr, ctypes.POINTER(ctype * n)).contents
            return np.frombuffer(buf, dtype=np.dtype(ctype)).reshape(shape).copy()

        return {
            "layout": lay,
            "sigma": arr(r.sigma, ctypes.c_double, (nl, lay["sigma_per_lag"])),
            "count": arr(r.count, ctypes.c_int32, (nl, no)),
            "f": arr(r.f, ctypes.c_double, (nl, cap)),
            "xi": arr(r.xi, ctypes.c_double, (nl, cap)),
            "mu": arr(r.mu, ctypes.c_double, (nl, cap, 2)),
            "phi": arr(r.phi, ctypes.c_float, (nl, cap, l, 2)),
            "flags": arr(r.flags, ctypes.c_int32, (nl, no)),
        }

    def release(self, ticket: int) -> None:
        _check_srv(lib().ssi_server_release(self._h, ticket))

    def stats(self) -> dict:
        st = _ServerStats()
        _check_srv(lib().ssi_server_get_stats(self._h, ctypes.byref(st)))
        return {name: int(getattr(st, name)) for name, _ in _ServerStats._fields_}
