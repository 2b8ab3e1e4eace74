"""Thin Python binding of libsrmra.so (the C ABI declared in include/srmra.h).

Argument marshalling only: torch tensors are passed as raw device pointers and
the current torch stream as the HIP stream.  Every step of the EM computation
runs in the library's HIP kernels.  If the library is missing or cannot be
loaded, every call raises RuntimeError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libsrmra.so")

SRMRA_OK = 0
SRMRA_EINVAL = -1
SRMRA_EUNSUPPORTED = -2
SRMRA_EWORKSPACE = -3
SRMRA_EDEVICE = -4
SRMRA_ESCRATCH = -5
SRMRA_SCRATCH_BYTES = 64 << 20   # the library's per-device scratch array (srmra_em_step_noalloc)

SRMRA_FP32_PLAIN = FP32_PLAIN = 0
SRMRA_FP32_MFMA = FP32_MFMA = 1
SRMRA_BF16_SPLIT3 = BF16_SPLIT3 = 2
SRMRA_BF16_SPLIT4 = BF16_SPLIT4 = 3
SRMRA_FP32_FFT = FP32_FFT = 4
# block layouts of a tuning entry (srmra.h SRMRA_TILE_*)
SRMRA_TILE_TWO_PASS = 8
SRMRA_TILE_FUSED_8OBS = 16
SRMRA_TILE_FUSED_4OBS = 32
SRMRA_TILE_16X16 = 64
PRECISIONS = {"fp32_plain": FP32_PLAIN, "fp32_mfma": FP32_MFMA, "bf16_split3": BF16_SPLIT3,
              "bf16_split4": BF16_SPLIT4, "fp32_fft": FP32_FFT}

_lib = None
_lock = threading.Lock()

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_sz = ctypes.c_size_t
_f = ctypes.c_float


class SrmraError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class srmra_problem(ctypes.Structure):
    _fields_ = [
        ("y", _vp), ("prep", _vp), ("prep_bytes", _sz), ("N", _i64), ("L_low", _int),
        ("K", _int), ("x", _vp), ("log_rho", _vp), ("sigma", _f), ("x_new", _vp),
        ("rho_new", _vp), ("log_rho_new", _vp), ("loglik", _vp),
    ]


class srmra_tuning(ctypes.Structure):
    _fields_ = [("precision", _int), ("L_low", _int), ("K", _int), ("form", _int),
                ("item_obs", _i64), ("tile", _int)]


def lib():
    """Load libsrmra.so once; raise if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
            L = ctypes.CDLL(LIB_PATH)
            L.srmra_status_string.restype = ctypes.c_char_p
            L.srmra_status_string.argtypes = [_int]
            L.srmra_version.restype = ctypes.c_char_p
            L.srmra_version.argtypes = []
            L.srmra_em_step_workspace_bytes.restype = _sz
            L.srmra_em_step_workspace_bytes.argtypes = [_i64, _int, _int, _int]
            L.srmra_em_step_passes.restype = _int
            L.srmra_em_step_passes.argtypes = [_i64, _int, _int, _int]
            L.srmra_prepared_bytes.restype = _sz
            L.srmra_prepared_bytes.argtypes = [_i64, _int, _int, _int]
            L.srmra_prepare_observations_ex.restype = _int
            L.srmra_prepare_observations_ex.argtypes = [_vp, _i64, _int, _int, _int, _int, _vp, _sz, _vp]
            L.srmra_prepare_observations.restype = _int
            L.srmra_prepare_observations.argtypes = [_vp, _i64, _int, _int, _int, _vp, _sz, _vp]
            L.srmra_em_step.restype = _int
            L.srmra_em_step.argtypes = [_vp, _i64, _int, _int, _vp, _vp, _f, _vp, _vp, _vp, _int,
                                        _vp, _sz, _vp]
            L.srmra_em_step_noalloc.restype = _int
            L.srmra_em_step_noalloc.argtypes = [_vp, _i64, _int, _int, _vp, _vp, _f, _vp, _vp, _vp,
                                                _int, _vp]
            L.srmra_em_step_prepared.restype = _int
            L.srmra_em_step_prepared.argtypes = [_vp, _vp, _sz, _i64, _int, _int, _vp, _vp, _f,
                                                 _vp, _vp, _vp, _vp, _int, _vp, _sz, _vp]
            L.srmra_em_step_debug.restype = _int
            L.srmra_em_step_debug.argtypes = [_vp, _vp, _sz, _i64, _int, _int, _vp, _vp, _f, _vp,
                                              _vp, _vp, _vp, _vp, _vp, _vp, _int, _vp, _sz, _vp]
            L.srmra_em_step_profiled.restype = _int
            L.srmra_em_step_profiled.argtypes = [_vp, _vp, _sz, _i64, _int, _int, _vp, _vp, _f,
                                                 _vp, _vp, _vp, _vp, _int, _vp, _sz, _vp,
                                                 ctypes.POINTER(_vp)]
            L.srmra_plan_form.restype = _int
            L.srmra_plan_form.argtypes = [_int, _int]
            L.srmra_plan_parity.restype = _int
            L.srmra_plan_parity.argtypes = [_vp]
            L.srmra_plan_create.restype = _int
            L.srmra_plan_create.argtypes = [ctypes.POINTER(srmra_problem), _int, _int,
                                            ctypes.POINTER(_vp), ctypes.POINTER(_sz)]
            L.srmra_plan_create_tuned.restype = _int
            L.srmra_plan_create_tuned.argtypes = [ctypes.POINTER(srmra_problem), _int, _int,
                                                  ctypes.POINTER(srmra_tuning), _int,
                                                  ctypes.POINTER(_vp), ctypes.POINTER(_sz)]
            L.srmra_plan_default_item_obs.restype = _i64
            L.srmra_plan_default_item_obs.argtypes = [_i64, _int, _int, _int]
            L.srmra_plan_set_iterate.restype = _int
            L.srmra_plan_set_iterate.argtypes = [_vp, _int, _vp, _vp, _vp, _vp, _vp]
            L.srmra_plan_upload.restype = _int
            L.srmra_plan_upload.argtypes = [_vp, _vp, _sz, _vp]
            L.srmra_plan_execute.restype = _int
            L.srmra_plan_execute.argtypes = [_vp, _vp, _sz, _vp]
            L.srmra_project_workspace_bytes.restype = _sz
            L.srmra_project_workspace_bytes.argtypes = [_int]
            L.srmra_project_gaussian.restype = _int
            L.srmra_project_gaussian.argtypes = [_vp, _vp, _int, _vp, _f, _vp, _sz, _vp]
            L.srmra_shift_error_workspace_bytes.restype = _sz
            L.srmra_shift_error_workspace_bytes.argtypes = [_int]
            L.srmra_shift_error.restype = _int
            L.srmra_shift_error.argtypes = [_vp, _vp, _int, _vp, _vp, _vp, _sz, _vp]
            L.srmra_moments_workspace_bytes.restype = _sz
            L.srmra_moments_workspace_bytes.argtypes = [_i64, _int]
            L.srmra_moments.restype = _int
            L.srmra_moments.argtypes = [_vp, _i64, _int, _vp, _vp, _vp, _sz, _vp]
            L.srmra_dft2.restype = _int
            L.srmra_dft2.argtypes = [_vp, _i64, _int, _vp, _vp]
            L.srmra_plan_destroy.restype = None
            L.srmra_plan_destroy.argtypes = [_vp]
            _lib = L
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().srmra_status_string(int(status)).decode()
    except RuntimeError:
        return "library not loaded"


def _check(status: int, where: str):
    if status != SRMRA_OK:
        raise SrmraError(status, where)


def _ptr(t: Optional[torch.Tensor], dtype=None) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


# ------------------------------------------------------------------ C-ABI mirrors
def srmra_version() -> str:
    return lib().srmra_version().decode()


def srmra_em_step_workspace_bytes(N: int, L_low: int, K: int, precision) -> int:
    return int(lib().srmra_em_step_workspace_bytes(N, L_low, K, _prec(precision)))


def srmra_em_step_passes(N: int, L_low: int, K: int, precision) -> int:
    r = int(lib().srmra_em_step_passes(N, L_low, K, _prec(precision)))
    _check(r if r < 0 else 0, "srmra_em_step_passes")
    return r


def srmra_prepared_bytes(N: int, L_low: int, K: int, precision) -> int:
    return int(lib().srmra_prepared_bytes(N, L_low, K, _prec(precision)))


def srmra_prepare_observations_ex(y: torch.Tensor, N: int, L_low: int, K: int, precision,
                                  centre: int, prep: torch.Tensor, stream=None) -> None:
    _check(lib().srmra_prepare_observations_ex(_ptr(y, torch.float32), N, L_low, K, _prec(precision),
                                               int(centre), _ptr(prep),
                                               prep.numel() * prep.element_size(), _stream(stream)),
           "srmra_prepare_observations_ex")


def srmra_prepare_observations(y: torch.Tensor, N: int, L_low: int, K: int, precision,
                               prep: torch.Tensor, stream=None) -> None:
    _check(lib().srmra_prepare_observations(_ptr(y, torch.float32), N, L_low, K, _prec(precision),
                                            _ptr(prep), prep.numel() * prep.element_size(),
                                            _stream(stream)), "srmra_prepare_observations")


def srmra_em_step(y, N, L_low, K, x, log_rho, sigma, x_new, rho_new, loglik, precision,
                  workspace, stream=None) -> None:
    _check(lib().srmra_em_step(_ptr(y, torch.float32), N, L_low, K, _ptr(x, torch.float32),
                               _ptr(log_rho, torch.float32), float(sigma),
                               _ptr(x_new, torch.float32), _ptr(rho_new, torch.float32),
                               _ptr(loglik, torch.float64), _prec(precision), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream(stream)),
           "srmra_em_step")


def srmra_em_step_noalloc(y, N, L_low, K, x, log_rho, sigma, x_new, rho_new, loglik, precision,
                          stream=None) -> None:
    _check(lib().srmra_em_step_noalloc(_ptr(y, torch.float32), N, L_low, K, _ptr(x, torch.float32),
                                       _ptr(log_rho, torch.float32), float(sigma),
                                       _ptr(x_new, torch.float32), _ptr(rho_new, torch.float32),
                                       _ptr(loglik, torch.float64), _prec(precision),
                                       _stream(stream)), "srmra_em_step_noalloc")


def srmra_em_step_prepared(y, prep, N, L_low, K, x, log_rho, sigma, x_new, rho_new, log_rho_new,
                           loglik, precision, workspace, stream=None) -> None:
    _check(lib().srmra_em_step_prepared(
        _ptr(y, torch.float32), _ptr(prep), prep.numel() * prep.element_size(), N, L_low, K,
        _ptr(x, torch.float32), _ptr(log_rho, torch.float32), float(sigma),
        _ptr(x_new, torch.float32), _ptr(rho_new, torch.float32),
        _ptr(log_rho_new, torch.float32), _ptr(loglik, torch.float64),
        _prec(precision), _ptr(workspace), workspace.numel() * workspace.element_size(),
        _stream(stream)), "srmra_em_step_prepared")


def srmra_em_step_debug(y, prep, N, L_low, K, x, log_rho, sigma, x_new, rho_new, log_rho_new,
                        loglik, ll_obs, b_out, c_out, precision, workspace, stream=None) -> None:
    _check(lib().srmra_em_step_debug(
        _ptr(y, torch.float32), _ptr(prep), 0 if prep is None else prep.numel() * prep.element_size(),
        N, L_low, K, _ptr(x, torch.float32), _ptr(log_rho, torch.float32), float(sigma),
        _ptr(x_new, torch.float32), _ptr(rho_new, torch.float32),
        _ptr(log_rho_new, torch.float32), _ptr(loglik, torch.float64),
        _ptr(ll_obs, torch.float32), _ptr(b_out, torch.float64), _ptr(c_out, torch.float64),
        _prec(precision), _ptr(workspace), workspace.numel() * workspace.element_size(),
        _stream(stream)), "srmra_em_step_debug")


def srmra_em_step_profiled(y, prep, N, L_low, K, x, log_rho, sigma, x_new, rho_new, log_rho_new,
                           loglik, precision, workspace, events, stream=None) -> None:
    """events: six torch.cuda.Event(enable_timing=True) objects (recorded by the library)."""
    arr = (_vp * 6)(*[ev.cuda_event for ev in events])
    _check(lib().srmra_em_step_profiled(
        _ptr(y, torch.float32), _ptr(prep), prep.numel() * prep.element_size(), N, L_low, K,
        _ptr(x, torch.float32), _ptr(log_rho, torch.float32), float(sigma),
        _ptr(x_new, torch.float32), _ptr(rho_new, torch.float32),
        _ptr(log_rho_new, torch.float32), _ptr(loglik, torch.float64),
        _prec(precision), _ptr(workspace), workspace.numel() * workspace.element_size(),
        _stream(stream), arr), "srmra_em_step_profiled")


# ------------------------------------------------------------------ batched plan
def srmra_plan_form(precision, L_low: int) -> int:
    return int(lib().srmra_plan_form(_prec(precision), int(L_low)))


class Plan:
    """Owner of an srmra_plan* (host object) plus the problem structs."""

    def __init__(self, problems: Sequence[dict], precision, tuning: Optional[Sequence[dict]] = None):
        """tuning: entries {precision, L_low, K, form, item_obs[, tile]} (srmra_tuning)."""
        arr = (srmra_problem * len(problems))()
        for k, pr in enumerate(problems):
            s = arr[k]
            s.y = _ptr(pr["y"], torch.float32)
            s.prep = _ptr(pr["prep"])
            s.prep_bytes = pr["prep"].numel() * pr["prep"].element_size()
            s.N = int(pr["N"]); s.L_low = int(pr["L_low"]); s.K = int(pr["K"])
            s.x = _ptr(pr["x"], torch.float32)
            s.log_rho = _ptr(pr["log_rho"], torch.float32)
            s.sigma = float(pr["sigma"])
            s.x_new = _ptr(pr["x_new"], torch.float32)
            s.rho_new = _ptr(pr["rho_new"], torch.float32)
            s.log_rho_new = _ptr(pr.get("log_rho_new"), torch.float32)
            s.loglik = _ptr(pr["loglik"], torch.float64)
        h = _vp()
        ws = _sz()
        if tuning:
            tab = (srmra_tuning * len(tuning))()
            for k, t in enumerate(tuning):
                tab[k].precision = _prec(t["precision"])
                tab[k].L_low = int(t["L_low"]); tab[k].K = int(t["K"])
                tab[k].form = _prec(t["form"]); tab[k].item_obs = int(t["item_obs"])
                tab[k].tile = int(t.get("tile", 0))
            _check(lib().srmra_plan_create_tuned(arr, len(problems), _prec(precision), tab,
                                                 len(tuning), ctypes.byref(h), ctypes.byref(ws)),
                   "srmra_plan_create_tuned")
        else:
            _check(lib().srmra_plan_create(arr, len(problems), _prec(precision), ctypes.byref(h),
                                           ctypes.byref(ws)), "srmra_plan_create")
        self._h = h
        self.workspace_bytes = int(ws.value)

    def set_iterate(self, index, x, log_rho, x_new, rho_new, log_rho_new=None):
        _check(lib().srmra_plan_set_iterate(self._h, index, _ptr(x), _ptr(log_rho), _ptr(x_new),
                                            _ptr(rho_new), _ptr(log_rho_new)),
               "srmra_plan_set_iterate")

    def upload(self, workspace, stream=None):
        _check(lib().srmra_plan_upload(self._h, _ptr(workspace),
                                       workspace.numel() * workspace.element_size(),
                                       _stream(stream)), "srmra_plan_upload")

    def execute(self, workspace, stream=None):
        _check(lib().srmra_plan_execute(self._h, _ptr(workspace),
                                        workspace.numel() * workspace.element_size(),
                                        _stream(stream)), "srmra_plan_execute")

    def parity(self) -> int:
        return int(lib().srmra_plan_parity(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().srmra_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def srmra_plan_default_item_obs(N: int, L_low: int, K: int, form_precision) -> int:
    r = int(lib().srmra_plan_default_item_obs(N, L_low, K, _prec(form_precision)))
    _check(r if r < 0 else 0, "srmra_plan_default_item_obs")
    return r


def srmra_project_workspace_bytes(L_high: int) -> int:
    return int(lib().srmra_project_workspace_bytes(L_high))


def srmra_project_gaussian(x_in: torch.Tensor, x_out: torch.Tensor, L_high: int,
                           sigma_state: torch.Tensor, decay: float, workspace: torch.Tensor,
                           stream=None) -> None:
    _check(lib().srmra_project_gaussian(_ptr(x_in, torch.float32), _ptr(x_out, torch.float32), L_high,
                                        _ptr(sigma_state, torch.float32), float(decay),
                                        _ptr(workspace), workspace.numel() * workspace.element_size(),
                                        _stream(stream)), "srmra_project_gaussian")


def srmra_dft2(x: torch.Tensor, count: int, L: int, out: torch.Tensor, stream=None) -> None:
    _check(lib().srmra_dft2(_ptr(x, torch.float32), count, L, _ptr(out), _stream(stream)),
           "srmra_dft2")


def srmra_moments_workspace_bytes(N: int, L_low: int) -> int:
    return int(lib().srmra_moments_workspace_bytes(N, L_low))


def srmra_moments(y: torch.Tensor, N: int, L_low: int, m1: torch.Tensor, m2: torch.Tensor,
                  workspace: torch.Tensor, stream=None) -> None:
    _check(lib().srmra_moments(_ptr(y, torch.float32), N, L_low, _ptr(m1, torch.float64),
                               _ptr(m2, torch.float64), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream(stream)),
           "srmra_moments")


def srmra_shift_error_workspace_bytes(L_high: int) -> int:
    return int(lib().srmra_shift_error_workspace_bytes(L_high))


def srmra_shift_error(x_hat: torch.Tensor, x_ref: torch.Tensor, L_high: int, err: torch.Tensor,
                      best_shift: Optional[torch.Tensor], workspace: torch.Tensor, stream=None) -> None:
    _check(lib().srmra_shift_error(_ptr(x_hat, torch.float32), _ptr(x_ref, torch.float32), L_high,
                                   _ptr(err, torch.float64), _ptr(best_shift, torch.int32),
                                   _ptr(workspace), workspace.numel() * workspace.element_size(),
                                   _stream(stream)), "srmra_shift_error")


def empty_bytes(nbytes: int, device="cuda") -> torch.Tensor:
    """A device byte buffer (torch allocations are at least 256-byte aligned)."""
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t
