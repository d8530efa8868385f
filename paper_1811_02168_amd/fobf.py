"""Thin ctypes binding of libfobf.so (argument marshalling only).

Every computation runs inside the library: the float64 fit on the host,
the filter in HIP kernels on the GPU.  torch is used for device memory and
streams only.  There is no fallback: if the library is missing, importing
this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfobf.so")
CHECK_LIB_PATH = os.path.join(HERE, "libfobf_check.so")

KMAX = 32
RMAX = 48

FP32, FP16_STAGE, BF16_STAGE, FP16X2_STAGE = 0, 1, 2, 3
ALGO_AUTO, ALGO_VALU, ALGO_MFMA = 0, 1, 2

OK, WARN_TOL, EBUSY = 0, 1, 2
EINVAL, ENOMEM, EHIP, EINTERNAL, ECANCELED, ETIMEDOUT = -1, -2, -3, -4, -5, -6

_PREC = {"fp32": FP32, "f32": FP32, "fp16": FP16_STAGE, "f16": FP16_STAGE,
         "bf16": BF16_STAGE, "fp16x2": FP16X2_STAGE}
_ALGO = {"auto": ALGO_AUTO, "valu": ALGO_VALU, "mfma": ALGO_MFMA}

EXPORTS = [
    "fobf_fit", "fobf_fit_cache_clear", "fobf_fit_samples", "fobf_filter", "fobf_batch_workspace_size",
    "fobf_filter_batch", "fobf_autotune", "fobf_tune_save", "fobf_tune_load",
    "fobf_tune_reset", "fobf_tune_get", "fobf_serve_create",
    "fobf_serve_submit", "fobf_serve_poll", "fobf_serve_destroy",
    "fobf_serve_get_stats", "fobf_serve_inject_fault", "fobf_last_error",
    "fobf_version", "fobf_peak", "fobf_fit_period", "fobf_lut_create", "fobf_lut_get",
    "fobf_lut_fit", "fobf_lut_save", "fobf_lut_load", "fobf_lut_destroy",
    "fobf_filter_workspace_size", "fobf_filter_ws", "fobf_effective_prec",
    "fobf_filter_ws_static", "fobf_fit_warm", "fobf_serve_cancel",
    "fobf_fit_cache_save", "fobf_fit_cache_load",
]

STATIC_SCRATCH_BYTES = 128 << 20     # FOBF_STATIC_SCRATCH_BYTES


class FobfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class _Coef(C.Structure):
    _fields_ = [("R", C.c_int), ("K", C.c_int), ("T", C.c_int),
                ("Tmax", C.c_int), ("sigma", C.c_double), ("E", C.c_double),
                ("delta", C.c_double), ("c", C.c_double * KMAX)]


class _Job(C.Structure):
    _fields_ = [("d_in", C.c_void_p), ("d_out", C.c_void_p), ("H", C.c_int),
                ("W", C.c_int), ("ld_in", C.c_int), ("ld_out", C.c_int),
                ("theta", C.c_double), ("K", C.c_int), ("T", C.c_int),
                ("prec", C.c_int), ("c", C.c_double * KMAX)]


class _ServeCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_inflight", C.c_int),
                ("max_batch", C.c_int), ("R", C.c_int), ("eps", C.c_double)]


class _Request(C.Structure):
    _fields_ = [("h_in", C.c_void_p), ("h_out", C.c_void_p), ("H", C.c_int),
                ("W", C.c_int), ("ld_in", C.c_int), ("ld_out", C.c_int),
                ("theta", C.c_double), ("sigma", C.c_double),
                ("K", C.c_int), ("prec", C.c_int), ("deadline_s", C.c_double)]


class _ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64),
                ("failed", C.c_uint64), ("batches", C.c_uint64),
                ("peak_bytes_inflight", C.c_size_t), ("peak_inflight", C.c_int),
                ("coef_entries", C.c_int)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double), ("T", C.c_int), ("prec", C.c_int)]


def _load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with "
            "`python paper_1811_02168_amd/build.py` (no CPU fallback exists)")
    lib = C.CDLL(path)
    lib.fobf_fit.argtypes = [C.c_int, C.c_double, C.c_int, C.c_double, C.c_int,
                             C.POINTER(_Coef)]
    lib.fobf_fit_samples.argtypes = [C.c_int, C.POINTER(C.c_double), C.c_int,
                                     C.c_double, C.c_int, C.POINTER(_Coef)]
    lib.fobf_filter.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                C.POINTER(C.c_double), C.c_int, C.c_int,
                                C.c_void_p]
    def bind(name, argtypes, restype=C.c_int):
        if hasattr(lib, name):
            fn = getattr(lib, name)
            fn.argtypes = argtypes
            fn.restype = restype

    bind("fobf_batch_workspace_size", [C.c_int], C.c_size_t)
    bind("fobf_filter_workspace_size", [C.c_int, C.c_int, C.c_double, C.c_int,
                                        C.POINTER(C.c_size_t)])
    bind("fobf_filter_ws", [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                            C.c_double, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_int,
                            C.c_int, C.c_void_p, C.c_size_t, C.c_void_p])
    bind("fobf_effective_prec", [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)])
    bind("fobf_filter_ws_static", [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_double, C.c_int, C.c_int,
                                   C.POINTER(C.c_double), C.c_int, C.c_int, C.c_void_p])
    bind("fobf_filter_batch", [C.POINTER(_Job), C.c_int, C.c_void_p,
                               C.c_size_t, C.c_void_p])
    bind("fobf_serve_create", [C.POINTER(_ServeCfg), C.POINTER(C.c_void_p)])
    bind("fobf_serve_submit", [C.c_void_p, C.POINTER(_Request),
                               C.POINTER(C.c_uint64)])
    bind("fobf_serve_poll", [C.c_void_p, C.c_uint64, C.c_int,
                             C.POINTER(_Result)])
    bind("fobf_serve_destroy", [C.c_void_p])
    bind("fobf_serve_cancel", [C.c_void_p, C.c_uint64])
    bind("fobf_serve_get_stats", [C.c_void_p, C.POINTER(_ServeStats)])
    bind("fobf_serve_inject_fault", [C.c_void_p, C.c_int])
    bind("fobf_autotune", [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p])
    bind("fobf_tune_save", [C.c_char_p])
    bind("fobf_tune_load", [C.c_char_p])
    bind("fobf_tune_reset", [])
    bind("fobf_tune_get", [C.c_int, C.c_double, C.POINTER(C.c_int),
                           C.POINTER(C.c_int)])
    bind("fobf_version", [])
    bind("fobf_fit_cache_clear", [])
    bind("fobf_fit_cache_save", [C.c_char_p])
    bind("fobf_fit_cache_load", [C.c_char_p])
    bind("fobf_peak", [C.c_int, C.c_void_p, C.POINTER(C.c_double)])
    bind("fobf_fit_period", [C.c_int, C.c_double, C.c_int, C.c_int, C.POINTER(_Coef)])
    bind("fobf_fit_warm", [C.c_int, C.c_double, C.c_int, C.c_double, C.c_int, C.c_int,
                           C.POINTER(_Coef)])
    bind("fobf_lut_create", [C.c_int, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double),
                             C.c_int, C.c_int, C.POINTER(C.c_void_p)])
    bind("fobf_lut_get", [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int),
                          C.POINTER(C.c_int)])
    bind("fobf_lut_fit", [C.c_void_p, C.c_double, C.c_double, C.POINTER(_Coef)])
    bind("fobf_lut_save", [C.c_void_p, C.c_char_p])
    bind("fobf_lut_load", [C.c_char_p, C.POINTER(C.c_void_p)])
    bind("fobf_lut_destroy", [C.c_void_p], None)
    bind("fobf_check_take", [C.POINTER(C.c_uint)])
    lib.fobf_last_error.restype = C.c_char_p
    lib.fobf_fit.restype = C.c_int
    lib.fobf_fit_samples.restype = C.c_int
    lib.fobf_filter.restype = C.c_int
    return lib


# libfobf.so links the system ROCm's HIP runtime; PyTorch brings its own
# copy.  Both work in one process when PyTorch's is started first (the
# order every test and the benchmark use); started the other way round,
# PyTorch may find no device.  So PyTorch, where present, is started here,
# before the library is loaded.
try:
    import torch as _torch
    if _torch.cuda.is_available():
        _torch.cuda.init()
except ImportError:   # the C ABI needs no PyTorch
    pass

lib = _load()


def load_check_library():
    """The debug-check build (libfobf_check.so: LDS poisoning and index
    checks), bound like `lib`.  Route this module's calls through it by
    rebinding `lib` (tests do so), and read its violations with
    check_take(that_library)."""
    return _load(CHECK_LIB_PATH)


def check_take(library=None) -> int:
    """Violation bits (FOBF_CHECK_*) recorded by a debug-check library since
    the last call, cleared; waits for the device.  Raises FobfError on the
    release library."""
    L = library or lib
    bits = C.c_uint(0)
    st = L.fobf_check_take(C.byref(bits))
    if st != OK:
        m = L.fobf_last_error()
        raise FobfError(st, m.decode() if m else "")
    return int(bits.value)


CHECK_BITS = {"lds": 0x001, "image": 0x002, "halo_h": 0x004, "halo_v": 0x008,
              "ring": 0x010, "ws": 0x020, "out": 0x040, "tile": 0x080,
              "stage": 0x100}


def last_error() -> str:
    m = lib.fobf_last_error()
    return m.decode() if m else ""


def _check(st, allow=(OK,)):
    if st in allow:
        return st
    raise FobfError(st, last_error())


def _prec(p):
    return _PREC[p] if isinstance(p, str) else int(p)


def _algo(a):
    return _ALGO[a] if isinstance(a, str) else int(a)


def _carr(c, K):
    c = np.asarray(c, dtype=np.float64).ravel()
    if len(c) < K:
        raise ValueError("need K coefficients")
    arr = (C.c_double * KMAX)()
    for k in range(K):
        arr[k] = float(c[k])
    return arr


@dataclass
class Coef:
    """Fitted cosine range kernel of eq. (3): K, T and c[0..K-1]."""
    R: int
    K: int
    T: int
    Tmax: int
    sigma: float
    E: float
    delta: float
    c: np.ndarray = field(repr=False)
    status: int = OK

    @staticmethod
    def _from(s: _Coef, status: int) -> "Coef":
        return Coef(s.R, s.K, s.T, s.Tmax, s.sigma, s.E, s.delta,
                    np.array(s.c[:s.K], dtype=np.float64), status)


def fit(R: int, sigma: float, K: int, eps: float = 0.1, Tmax: int = 0) -> Coef:
    """fobf_fit: K >= 1 fixed order (T scan), K == 0 Algorithm 1."""
    out = _Coef()
    st = lib.fobf_fit(int(R), float(sigma), int(K), float(eps), int(Tmax),
                      C.byref(out))
    _check(st, (OK, WARN_TOL))
    return Coef._from(out, st)


def fit_warm(R: int, sigma: float, K: int, eps: float = 0.1, T0: int = 0,
             Tmax: int = 0) -> Coef:
    """fobf_fit_warm: fixed-order fit with the period found by a local
    search from T0 (0: T0 = R) instead of the full scan."""
    out = _Coef()
    st = lib.fobf_fit_warm(int(R), float(sigma), int(K), float(eps), int(Tmax), int(T0),
                           C.byref(out))
    _check(st, (OK, WARN_TOL))
    return Coef._from(out, st)


def fit_cache_clear() -> int:
    """fobf_fit_cache_clear: drop the host fit cache; returns entries dropped."""
    return int(lib.fobf_fit_cache_clear())


def fit_cache_save(path) -> None:
    """fobf_fit_cache_save: write the host fit cache to a text file."""
    _check(lib.fobf_fit_cache_save(str(path).encode()))


def fit_cache_load(path) -> None:
    """fobf_fit_cache_load: add a saved cache's entries to the fit cache."""
    _check(lib.fobf_fit_cache_load(str(path).encode()))


def fit_period(R: int, sigma: float, K: int, T: int) -> Coef:
    """fobf_fit_period: least squares at one period (T = R: the fixed-period
    filter the paper compares with)."""
    out = _Coef()
    _check(lib.fobf_fit_period(int(R), float(sigma), int(K), int(T), C.byref(out)))
    return Coef._from(out, OK)


class Lut:
    """fobf_lut: (sigma, eps) -> (K*, T*) table with bilinear read-out."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)

    @classmethod
    def create(cls, R, sigmas, eps, Tmax=0):
        s = np.ascontiguousarray(sigmas, dtype=np.float64)
        e = np.ascontiguousarray(eps, dtype=np.float64)
        h = C.c_void_p()
        _check(lib.fobf_lut_create(int(R), s.ctypes.data_as(C.POINTER(C.c_double)), len(s),
                                   e.ctypes.data_as(C.POINTER(C.c_double)), len(e),
                                   int(Tmax), C.byref(h)))
        return cls(h.value)

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        _check(lib.fobf_lut_load(str(path).encode(), C.byref(h)))
        return cls(h.value)

    def get(self, i_sigma, i_eps):
        K, T = C.c_int(), C.c_int()
        _check(lib.fobf_lut_get(self._h, int(i_sigma), int(i_eps), C.byref(K), C.byref(T)))
        return K.value, T.value

    def fit(self, sigma, eps, refine=False) -> Coef:
        """fobf_lut_fit: (K, T) read from the table, c from one solve; with
        ``refine`` the period is then searched locally from the table's T
        (fobf_fit_warm at the table's K)."""
        out = _Coef()
        st = lib.fobf_lut_fit(self._h, float(sigma), float(eps), C.byref(out))
        _check(st, (OK, WARN_TOL))
        if refine:
            return fit_warm(out.R, sigma, out.K, eps, T0=out.T)
        return Coef._from(out, st)

    def save(self, path):
        _check(lib.fobf_lut_save(self._h, str(path).encode()))

    def close(self):
        if self._h:
            lib.fobf_lut_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PEAK_KINDS = {"valu_fma_f32": 0, "valu_sin_f32": 1, "mfma_f32": 2,
              "mfma_f16": 3, "mfma_bf16": 4}


def peak(kind: str, stream=None) -> float:
    """fobf_peak: measured rate of one instruction class (1e12 / s)."""
    out = C.c_double(0.0)
    _check(lib.fobf_peak(PEAK_KINDS[kind], _stream_ptr(stream), C.byref(out)))
    return out.value


def fit_samples(R: int, b, K: int, eps: float = 0.1, Tmax: int = 0) -> Coef:
    """fobf_fit_samples: arbitrary even kernel from samples b[0..R]."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    if b.shape != (R + 1,):
        raise ValueError("b must hold R+1 samples")
    out = _Coef()
    st = lib.fobf_fit_samples(int(R), b.ctypes.data_as(C.POINTER(C.c_double)),
                              int(K), float(eps), int(Tmax), C.byref(out))
    _check(st, (OK, WARN_TOL))
    return Coef._from(out, st)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _check_image(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or t.stride(1) != 1:
        raise TypeError(f"{name} must be 2-D float32 with unit column stride")


def filter_workspace_size(H: int, W: int, theta: float, prec="fp32") -> int:
    """fobf_filter_workspace_size: bytes of device workspace filter(...,
    workspace=...) uses for this image (0: none)."""
    n = C.c_size_t()
    _check(lib.fobf_filter_workspace_size(int(H), int(W), float(theta), _prec(prec),
                                          C.byref(n)))
    return n.value


def effective_prec(prec, K: int, T: int, c) -> int:
    """fobf_effective_prec: the precision the filter calls run for ``prec``
    and the series (K, T, c) (fp16 staging of a series with negative lobes
    runs as two-word fp16)."""
    e = lib.fobf_effective_prec(_prec(prec), int(K), int(T), _carr(c, K))
    if e < 0:
        raise FobfError(EINVAL, "fobf_effective_prec: invalid arguments")
    return e


def filter(img, theta: float, K: int, T: int, c, prec="fp32", algo="auto",
           out=None, stream=None, workspace=None):
    """fobf_filter on a 2-D float32 CUDA tensor; returns the output tensor.
    Enqueued on ``stream`` (default: torch's current stream).  With
    ``workspace`` (a CUDA tensor of at least filter_workspace_size bytes)
    the call goes to fobf_filter_ws.  A WARN_TOL status (fp16 staging run
    as two-word fp16, see effective_prec) is not an error."""
    import torch
    _check_image(img, "img")
    H, W = img.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=img.device)
    _check_image(out, "out")
    if tuple(out.shape) != (H, W):
        raise ValueError("out shape mismatch")
    carr = _carr(c, K)
    if workspace is None:
        st = lib.fobf_filter(C.c_void_p(img.data_ptr()), C.c_void_p(out.data_ptr()),
                             H, W, img.stride(0), out.stride(0), float(theta),
                             int(K), int(T), carr, _prec(prec), _algo(algo),
                             _stream_ptr(stream))
    else:
        if not workspace.is_cuda:
            raise ValueError("workspace must be a CUDA tensor")
        nbytes = workspace.numel() * workspace.element_size()
        st = lib.fobf_filter_ws(C.c_void_p(img.data_ptr()), C.c_void_p(out.data_ptr()),
                                H, W, img.stride(0), out.stride(0), float(theta),
                                int(K), int(T), carr, _prec(prec), _algo(algo),
                                C.c_void_p(workspace.data_ptr()), nbytes,
                                _stream_ptr(stream))
    _check(st, (OK, WARN_TOL))
    return out


def filter_ws_static(img, theta: float, K: int, T: int, c, prec="fp32", algo="auto",
                     out=None, stream=None):
    """fobf_filter_ws_static: fobf_filter_ws with the library's static
    device scratch as the workspace (allocates nothing; images whose
    workspace exceeds STATIC_SCRATCH_BYTES are rejected).  ``out`` must be
    given: this call allocates no device memory, not even for the result."""
    _check_image(img, "img")
    if out is None:
        raise ValueError("filter_ws_static allocates nothing: pass out")
    _check_image(out, "out")
    H, W = img.shape
    if tuple(out.shape) != (H, W):
        raise ValueError("out shape mismatch")
    st = lib.fobf_filter_ws_static(C.c_void_p(img.data_ptr()), C.c_void_p(out.data_ptr()),
                                   H, W, img.stride(0), out.stride(0), float(theta),
                                   int(K), int(T), _carr(c, K), _prec(prec), _algo(algo),
                                   _stream_ptr(stream))
    _check(st, (OK, WARN_TOL))
    return out


def autotune(prec="fp32", H=2048, W=2048, K=8, stream=None):
    """fobf_autotune: time every tile shape for one precision on the device
    and record the fastest per radius class (synchronises the stream)."""
    _check(lib.fobf_autotune(_prec(prec), int(H), int(W), int(K),
                             _stream_ptr(stream)))


def tune_get(prec, theta):
    a, n = C.c_int(), C.c_int()
    _check(lib.fobf_tune_get(_prec(prec), float(theta), C.byref(a), C.byref(n)))
    return a.value, n.value


def tune_save(path):
    _check(lib.fobf_tune_save(str(path).encode()))


def tune_load(path):
    _check(lib.fobf_tune_load(str(path).encode()))


def tune_reset():
    _check(lib.fobf_tune_reset())


def batch_workspace_size(n: int) -> int:
    return int(lib.fobf_batch_workspace_size(int(n)))


def make_job(img, out, theta, K, T, c, prec="fp32") -> _Job:
    """Describe one batch image.  The job keeps references to ``img`` and
    ``out`` so that the device memory stays alive while it is in use."""
    _check_image(img, "img")
    _check_image(out, "out")
    j = _Job()
    j._tensors = (img, out)
    j.d_in = img.data_ptr()
    j.d_out = out.data_ptr()
    j.H, j.W = img.shape
    j.ld_in = img.stride(0)
    j.ld_out = out.stride(0)
    j.theta = float(theta)
    j.K = int(K)
    j.T = int(T)
    j.prec = _prec(prec)
    j.c = _carr(c, K)
    return j


def filter_batch(jobs, workspace=None, stream=None):
    """fobf_filter_batch over a list of _Job (see make_job): one persistent
    launch.  ``workspace`` is a uint8 CUDA tensor of at least
    batch_workspace_size(len(jobs)) bytes (allocated if None)."""
    import torch
    n = len(jobs)
    arr = (_Job * max(1, n))(*jobs)
    # the ctypes array copies the structs; hold the tensors until the call
    # has enqueued (the caller keeps the job objects for the device work)
    keep = [getattr(j, "_tensors", None) for j in jobs]  # noqa: F841
    need = batch_workspace_size(n)
    if workspace is None:
        dev = torch.device("cuda")
        # torch's caching allocator returns blocks aligned to >= 512 bytes
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    st = lib.fobf_filter_batch(arr, n, C.c_void_p(workspace.data_ptr()),
                               workspace.numel(), _stream_ptr(stream))
    _check(st, (OK, WARN_TOL))
    return workspace


class Server:
    """Continuous-batching server (fobf_serve_*) over host images."""

    def __init__(self, hbm_budget_bytes=32 << 30, max_inflight=64,
                 max_batch=16, R=255, eps=0.1):
        cfg = _ServeCfg(int(hbm_budget_bytes), int(max_inflight),
                        int(max_batch), int(R), float(eps))
        h = C.c_void_p()
        _check(lib.fobf_serve_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, img: np.ndarray, out: np.ndarray, theta, sigma, K,
               prec="fp32", deadline_s=0.0) -> int:
        """Queue one host image (2-D float32 with unit column stride; row
        pitch free).  Both arrays must stay alive and unchanged until the
        ticket is polled done; pinned memory makes the copies async.
        ``deadline_s`` > 0: the request completes with ETIMEDOUT if it is
        not admitted to the device within that many seconds."""
        for a, nm in ((img, "img"), (out, "out")):
            if a.dtype != np.float32 or a.ndim != 2 or a.strides[1] != 4:
                raise TypeError(f"{nm} must be 2-D float32 with unit column stride")
        if out.shape != img.shape:
            raise TypeError("out must have img's shape")
        req = _Request(img.ctypes.data, out.ctypes.data, img.shape[0],
                       img.shape[1], img.strides[0] // 4, out.strides[0] // 4,
                       float(theta), float(sigma), int(K), _prec(prec), float(deadline_s))
        t = C.c_uint64()
        _check(lib.fobf_serve_submit(self._h, C.byref(req), C.byref(t)))
        self._keep[t.value] = (img, out)
        return t.value

    def poll(self, ticket: int, wait=True):
        """(status, result) of a ticket: EBUSY while pending, else the
        request's final status (the ticket is then consumed).  Raises for
        a ticket this server does not know."""
        if ticket not in self._keep:
            raise FobfError(EINVAL, "unknown ticket")
        res = _Result()
        st = lib.fobf_serve_poll(self._h, C.c_uint64(ticket), int(bool(wait)),
                                 C.byref(res))
        if st != EBUSY:
            self._keep.pop(ticket, None)
        return st, res

    def cancel(self, ticket: int) -> int:
        """fobf_serve_cancel: OK if the queued request was cancelled (poll
        it to release the ticket), EBUSY if it is already on the device."""
        if ticket not in self._keep:
            raise FobfError(EINVAL, "unknown ticket")
        return _check(lib.fobf_serve_cancel(self._h, C.c_uint64(ticket)), (OK, EBUSY))

    def stats(self):
        st = _ServeStats()
        _check(lib.fobf_serve_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServeStats._fields_}

    def inject_fault(self, count=1):
        _check(lib.fobf_serve_inject_fault(self._h, int(count)))

    def close(self):
        if self._h:
            _check(lib.fobf_serve_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
