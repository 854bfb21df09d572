"""libttsvd: TT-SVD of large dense tensors on AMD Instinct MI355X (gfx950).

Thin Python binding over the C ABI declared in ``include/ttsvd.h``.  The
functions ``ttsvd_tsqr_r``, ``ttsvd_gemm_reshape`` and ``ttsvd_decompose``
only marshal arguments: every step of the decomposition runs in the HIP
kernels of ``libttsvd.so``.  PyTorch provides device memory and streams.

The library is loaded on first use; if it has not been built
(``python -m paper_2102_00104_amd.build``) every call raises -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttsvd.so")

TTSVD_F64, TTSVD_F32, TTSVD_BF16 = 0, 1, 2
TTSVD_OK = 0
MAX_D = 64
ERRORS = {-1: "TTSVD_EINVAL", -2: "TTSVD_ENOMEM", -3: "TTSVD_EHIP",
          -4: "TTSVD_ENONFINITE", -5: "TTSVD_EUNSUPPORTED"}

#: every symbol include/ttsvd.h declares
EXPORTED = ["ttsvd_tsqr_r", "ttsvd_tsqr_workspace_size", "ttsvd_gemm_reshape",
            "ttsvd_decompose", "ttsvd_tt_free", "ttsvd_footprint_bytes",
            "ttsvd_strerror", "ttsvd_last_error", "ttsvd_version",
            "ttsvd_profile_enable", "ttsvd_profile_reset", "ttsvd_profile_read",
            "ttsvd_batch_default_config", "ttsvd_decompose_batch", "ttsvd_batch_autotune",
            "ttsvd_server_default_config", "ttsvd_server_create", "ttsvd_server_submit",
            "ttsvd_server_poll", "ttsvd_server_pending", "ttsvd_server_destroy",
            "ttsvd_server_clock", "ttsvd_thick_bounds_k", "ttsvd_decompose_thick",
            "ttsvd_workspace_size", "ttsvd_cores_size", "ttsvd_decompose_ws",
            "ttsvd_tsqr_r_noalloc", "ttsvd_machine_bench", "ttsvd_decompose_alg1",
            "ttsvd_decompose_two_sided"]


class TTSVDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class TTStruct(ctypes.Structure):
    """ctypes mirror of ``ttsvd_tt``."""
    _fields_ = [
        ("d", ctypes.c_int),
        ("dims", ctypes.c_int64 * MAX_D),
        ("ranks", ctypes.c_int64 * (MAX_D + 1)),
        ("cores", ctypes.c_void_p * MAX_D),
        ("sigma", ctypes.POINTER(ctypes.c_double) * MAX_D),
        ("nsigma", ctypes.c_int64 * MAX_D),
        ("discarded2", ctypes.c_double * MAX_D),
        ("delta", ctypes.c_double),
        ("norm_sigma", ctypes.c_double),
        ("err_bound", ctypes.c_double),
        ("priv", ctypes.c_void_p),
    ]


class KernelStat(ctypes.Structure):
    """ctypes mirror of ``ttsvd_kernel_stat``."""
    _fields_ = [
        ("name", ctypes.c_char * 96),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("bytes", ctypes.c_double),
        ("flops", ctypes.c_double),
    ]


class TensorStruct(ctypes.Structure):
    """ctypes mirror of ``ttsvd_tensor``."""
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("dtype", ctypes.c_int),
        ("ld_last", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
    ]


class BatchConfig(ctypes.Structure):
    """ctypes mirror of ``ttsvd_batch_config``."""
    _fields_ = [
        ("grid", ctypes.c_int),
        ("tile_set", ctypes.c_int),
        ("min_tiles", ctypes.c_int),
        ("max_slices", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    """ctypes mirror of ``ttsvd_server_config``."""
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("workers", ctypes.c_int),
        ("max_batch", ctypes.c_int),
        ("batch_max_elems", ctypes.c_int64),
    ]


class Completion(ctypes.Structure):
    """ctypes mirror of ``ttsvd_completion``."""
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("status", ctypes.c_int),
        ("batch_size", ctypes.c_int),
        ("batched", ctypes.c_int),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("message", ctypes.c_char * 160),
        ("tt", TTStruct),
    ]


_lib = None
_hip = None


def lib() -> ctypes.CDLL:
    """The loaded libttsvd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libttsvd.so is not built (%s); run `python -m paper_2102_00104_amd.build`"
                % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, dp = ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.ttsvd_tsqr_r.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, vp, ctypes.c_size_t, vp]
        L.ttsvd_tsqr_r.restype = ctypes.c_int
        L.ttsvd_tsqr_workspace_size.argtypes = [ctypes.c_int, i64, i64]
        L.ttsvd_tsqr_workspace_size.restype = ctypes.c_size_t
        L.ttsvd_tsqr_r_noalloc.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, vp]
        L.ttsvd_tsqr_r_noalloc.restype = ctypes.c_int
        L.ttsvd_machine_bench.argtypes = [ctypes.c_int, vp, ctypes.c_size_t, ctypes.c_int, vp, dp]
        L.ttsvd_machine_bench.restype = ctypes.c_int
        L.ttsvd_gemm_reshape.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, i64, i64, vp, i64, vp]
        L.ttsvd_gemm_reshape.restype = ctypes.c_int
        L.ttsvd_decompose.argtypes = [ctypes.POINTER(TensorStruct), ctypes.POINTER(i64), ctypes.c_int,
                                      i64, ctypes.c_double, ctypes.POINTER(TTStruct)]
        L.ttsvd_decompose.restype = ctypes.c_int
        L.ttsvd_decompose_alg1.argtypes = [ctypes.POINTER(TensorStruct), ctypes.POINTER(i64),
                                           ctypes.c_int, i64, ctypes.c_double, ctypes.POINTER(TTStruct)]
        L.ttsvd_decompose_alg1.restype = ctypes.c_int
        L.ttsvd_decompose_two_sided.argtypes = [ctypes.POINTER(TensorStruct), ctypes.POINTER(i64),
                                                ctypes.c_int, i64, ctypes.c_double,
                                                ctypes.POINTER(TTStruct)]
        L.ttsvd_decompose_two_sided.restype = ctypes.c_int
        L.ttsvd_workspace_size.argtypes = [ctypes.POINTER(i64), ctypes.c_int, i64, ctypes.c_int]
        L.ttsvd_workspace_size.restype = ctypes.c_size_t
        L.ttsvd_cores_size.argtypes = [ctypes.POINTER(i64), ctypes.c_int, i64]
        L.ttsvd_cores_size.restype = ctypes.c_size_t
        L.ttsvd_decompose_ws.argtypes = [ctypes.POINTER(TensorStruct), ctypes.POINTER(i64),
                                         ctypes.c_int, i64, ctypes.c_double, vp, ctypes.c_size_t,
                                         vp, ctypes.c_size_t, ctypes.POINTER(TTStruct)]
        L.ttsvd_decompose_ws.restype = ctypes.c_int
        L.ttsvd_thick_bounds_k.argtypes = [ctypes.POINTER(i64), ctypes.c_int, i64, ctypes.c_double, i64,
                                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(i64)]
        L.ttsvd_thick_bounds_k.restype = ctypes.c_int
        L.ttsvd_decompose_thick.argtypes = [ctypes.POINTER(TensorStruct), ctypes.POINTER(i64),
                                            ctypes.c_int, i64, ctypes.c_double, i64, ctypes.c_double,
                                            ctypes.POINTER(TTStruct)]
        L.ttsvd_decompose_thick.restype = ctypes.c_int
        L.ttsvd_tt_free.argtypes = [ctypes.POINTER(TTStruct)]
        L.ttsvd_tt_free.restype = None
        L.ttsvd_footprint_bytes.argtypes = [ctypes.POINTER(i64), ctypes.c_int, i64, ctypes.c_int]
        L.ttsvd_footprint_bytes.restype = ctypes.c_size_t
        L.ttsvd_strerror.argtypes = [ctypes.c_int]
        L.ttsvd_strerror.restype = ctypes.c_char_p
        L.ttsvd_last_error.argtypes = []
        L.ttsvd_last_error.restype = ctypes.c_char_p
        L.ttsvd_version.argtypes = []
        L.ttsvd_version.restype = ctypes.c_char_p
        L.ttsvd_profile_enable.argtypes = [ctypes.c_int]
        L.ttsvd_profile_enable.restype = ctypes.c_int
        L.ttsvd_profile_reset.argtypes = []
        L.ttsvd_profile_reset.restype = None
        L.ttsvd_profile_read.argtypes = [ctypes.POINTER(KernelStat), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]
        L.ttsvd_profile_read.restype = ctypes.c_int
        L.ttsvd_batch_default_config.argtypes = [ctypes.POINTER(BatchConfig)]
        L.ttsvd_batch_default_config.restype = ctypes.c_int
        L.ttsvd_decompose_batch.argtypes = [
            ctypes.c_int, ctypes.POINTER(TensorStruct), ctypes.POINTER(ctypes.c_int),
            ctypes.POINTER(i64), ctypes.POINTER(i64), dp, ctypes.POINTER(BatchConfig), vp,
            ctypes.POINTER(TTStruct)]
        L.ttsvd_decompose_batch.restype = ctypes.c_int
        L.ttsvd_batch_autotune.argtypes = [
            ctypes.c_int, ctypes.POINTER(TensorStruct), ctypes.POINTER(ctypes.c_int),
            ctypes.POINTER(i64), ctypes.POINTER(i64), dp, vp, ctypes.POINTER(BatchConfig), dp]
        L.ttsvd_batch_autotune.restype = ctypes.c_int
        L.ttsvd_server_default_config.argtypes = [ctypes.POINTER(ServerConfig)]
        L.ttsvd_server_default_config.restype = ctypes.c_int
        L.ttsvd_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
        L.ttsvd_server_create.restype = ctypes.c_int
        L.ttsvd_server_submit.argtypes = [vp, ctypes.POINTER(TensorStruct), ctypes.POINTER(i64),
                                          ctypes.c_int, i64, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_uint64)]
        L.ttsvd_server_submit.restype = ctypes.c_int
        L.ttsvd_server_poll.argtypes = [vp, ctypes.POINTER(Completion), ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]
        L.ttsvd_server_poll.restype = ctypes.c_int
        L.ttsvd_server_pending.argtypes = [vp]
        L.ttsvd_server_pending.restype = i64
        L.ttsvd_server_destroy.argtypes = [vp]
        L.ttsvd_server_destroy.restype = None
        L.ttsvd_server_clock.argtypes = []
        L.ttsvd_server_clock.restype = ctypes.c_double
        _lib = L
    return _lib


def _hiprt():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int, ctypes.c_void_p]
        _hip.hipMemcpyAsync.restype = ctypes.c_int
    return _hip


def _check(rc: int):
    if rc != TTSVD_OK:
        raise TTSVDError(rc, lib().ttsvd_last_error().decode())


def dtype_code(t) -> int:
    import torch
    return {torch.float64: TTSVD_F64, torch.float32: TTSVD_F32,
            torch.bfloat16: TTSVD_BF16}[t.dtype]


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------------- C-ABI mirror

def ttsvd_tsqr_r(W, dtype: int, rows: int, cols: int, ld: int, R, ldr: int,
                 ws=None, ws_bytes: int = 0, stream=None) -> None:
    """``ttsvd_tsqr_r`` on torch device tensors (raw column-major storage)."""
    _check(lib().ttsvd_tsqr_r(W.data_ptr(), dtype, rows, cols, ld, R.data_ptr(), ldr,
                              ws.data_ptr() if ws is not None else None, ws_bytes,
                              _stream(stream)))


def ttsvd_tsqr_workspace_size(dtype: int, rows: int, cols: int) -> int:
    return int(lib().ttsvd_tsqr_workspace_size(dtype, rows, cols))


def ttsvd_tsqr_r_noalloc(W, dtype: int, rows: int, cols: int, ld: int, R, ldr: int,
                         stream=None) -> None:
    """``ttsvd_tsqr_r_noalloc``: ``ttsvd_tsqr_r`` with the library's fixed
    device scratch instead of a workspace (no device allocation)."""
    _check(lib().ttsvd_tsqr_r_noalloc(W.data_ptr(), dtype, rows, cols, ld, R.data_ptr(), ldr,
                                      _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

MB_LOAD, MB_STORE, MB_COPY, MB_TRIAD, MB_FMA = 0, 1, 2, 3, 4


def ttsvd_machine_bench(kind: int, buf, reps: int = 10, stream=None):
    """``ttsvd_machine_bench``: (ms per launch, bytes or flops per launch)."""
    out = (ctypes.c_double * 2)()
    _check(lib().ttsvd_machine_bench(kind, buf.data_ptr(), buf.numel() * buf.element_size(), reps,
                                     _stream(stream), out))
    return float(out[0]), float(out[1])


def ttsvd_gemm_reshape(W, dtype: int, rows: int, cols: int, ld: int, V, ldv: int, k: int,
                       n_next: int, Y, ld_y: int, stream=None) -> None:
    """``ttsvd_gemm_reshape`` on torch device tensors (raw column-major storage)."""
    _check(lib().ttsvd_gemm_reshape(W.data_ptr(), dtype, rows, cols, ld, V.data_ptr(), ldv, k,
                                    n_next, Y.data_ptr(), ld_y, _stream(stream)))


def ttsvd_profile_enable(on: bool) -> None:
    _check(lib().ttsvd_profile_enable(1 if on else 0))


def ttsvd_profile_reset() -> None:
    lib().ttsvd_profile_reset()


def ttsvd_profile_read() -> list:
    """[{name, launches, total_ms, bytes, flops}] aggregated by kernel."""
    n = ctypes.c_int(0)
    _check(lib().ttsvd_profile_read(None, 0, ctypes.byref(n)))
    arr = (KernelStat * max(1, n.value))()
    _check(lib().ttsvd_profile_read(arr, n.value, ctypes.byref(n)))
    return [dict(name=arr[i].name.decode(), launches=int(arr[i].launches),
                 total_ms=float(arr[i].total_ms), bytes=float(arr[i].bytes),
                 flops=float(arr[i].flops)) for i in range(n.value)]


def ttsvd_footprint_bytes(dims: Sequence[int], r_max: int, dtype: int) -> int:
    arr = (ctypes.c_int64 * len(dims))(*[int(n) for n in dims])
    return int(lib().ttsvd_footprint_bytes(arr, len(dims), r_max, dtype))


@dataclass
class TT:
    """Result of ``ttsvd_decompose`` with the cores copied into torch tensors."""
    dims: List[int]
    ranks: List[int]
    cores: list                 # torch float64 device tensors (r_{j-1}, n_j, r_j), Fortran data
    sigma: List[Optional[list]]
    discarded2: List[float]
    delta: float
    norm_sigma: float
    err_bound: float


def _to_tt(out: TTStruct, device, st: int, fetch: bool = True) -> TT:
    """Copy a filled ``ttsvd_tt`` into a TT (cores only if fetch)."""
    import torch
    d = int(out.d)
    dims = [int(out.dims[j]) for j in range(d)]
    ranks = [int(out.ranks[i]) for i in range(d + 1)]
    cores = []
    if fetch:
        for j in range(d):
            n = ranks[j] * dims[j] * ranks[j + 1]
            t = torch.empty(n, dtype=torch.float64, device=device)
            rc = _hiprt().hipMemcpyAsync(t.data_ptr(), out.cores[j], n * 8, 3, st)
            if rc != 0:
                raise RuntimeError("hipMemcpyAsync failed: %d" % rc)
            cores.append(t)
        torch.cuda.synchronize(device)
    sigma = [None] * d
    for j in range(1, d):
        sigma[j] = [out.sigma[j][i] for i in range(int(out.nsigma[j]))]
    return TT(dims, ranks, cores, sigma, [float(out.discarded2[j]) for j in range(d)],
              float(out.delta), float(out.norm_sigma), float(out.err_bound))


def ttsvd_decompose(X, dims: Sequence[int], r_max: int, tol: float, ld_last: int = 0,
                    stream=None) -> TT:
    """``ttsvd_decompose`` of the Fortran-ordered device tensor X (flat storage)."""
    dims = [int(n) for n in dims]
    d = len(dims)
    st = _stream(stream)
    xs = TensorStruct(X.data_ptr(), dtype_code(X), ld_last, st)
    arr = (ctypes.c_int64 * d)(*dims)
    out = TTStruct()
    _check(lib().ttsvd_decompose(ctypes.byref(xs), arr, d, r_max, float(tol), ctypes.byref(out)))
    try:
        return _to_tt(out, X.device, st)
    finally:
        lib().ttsvd_tt_free(ctypes.byref(out))


def ttsvd_decompose_alg1(X, dims: Sequence[int], r_max: int, tol: float, stream=None) -> TT:
    """``ttsvd_decompose_alg1``: Algorithm 1 (full SVD of every unfolding, no
    QR trick) on the GPU, the comparator for Algorithm 2 (FP64 only)."""
    dims = [int(n) for n in dims]
    d = len(dims)
    st = _stream(stream)
    xs = TensorStruct(X.data_ptr(), dtype_code(X), 0, st)
    arr = (ctypes.c_int64 * d)(*dims)
    out = TTStruct()
    _check(lib().ttsvd_decompose_alg1(ctypes.byref(xs), arr, d, r_max, float(tol),
                                      ctypes.byref(out)))
    try:
        return _to_tt(out, X.device, st)
    finally:
        lib().ttsvd_tt_free(ctypes.byref(out))


def ttsvd_decompose_two_sided(X, dims: Sequence[int], r_max: int, tol: float,
                              stream=None) -> TT:
    """``ttsvd_decompose_two_sided``: Algorithm 4 (steps alternately on the
    right-most and the left-most remaining mode)."""
    dims = [int(n) for n in dims]
    d = len(dims)
    st = _stream(stream)
    xs = TensorStruct(X.data_ptr(), dtype_code(X), 0, st)
    arr = (ctypes.c_int64 * d)(*dims)
    out = TTStruct()
    _check(lib().ttsvd_decompose_two_sided(ctypes.byref(xs), arr, d, r_max, float(tol),
                                           ctypes.byref(out)))
    try:
        return _to_tt(out, X.device, st)
    finally:
        lib().ttsvd_tt_free(ctypes.byref(out))


def ttsvd_workspace_size(dims: Sequence[int], r_max: int, dtype: int) -> int:
    arr = (ctypes.c_int64 * max(1, len(dims)))(*[int(n) for n in dims])
    return int(lib().ttsvd_workspace_size(arr, len(dims), int(r_max), int(dtype)))


def ttsvd_cores_size(dims: Sequence[int], r_max: int) -> int:
    arr = (ctypes.c_int64 * max(1, len(dims)))(*[int(n) for n in dims])
    return int(lib().ttsvd_cores_size(arr, len(dims), int(r_max)))


def ttsvd_decompose_ws(X, dims: Sequence[int], r_max: int, tol: float, ws, cores,
                       ld_last: int = 0, stream=None, fetch: bool = True) -> TT:
    """``ttsvd_decompose_ws``: ``ttsvd_decompose`` with the caller's device
    workspace ``ws`` (a torch tensor of at least ``ttsvd_workspace_size`` bytes)
    and FP64 core buffer ``cores`` (at least ``ttsvd_cores_size`` values); the
    call allocates no device memory.  With fetch=False the cores are not copied
    out (they stay in ``cores``)."""
    dims = [int(n) for n in dims]
    d = len(dims)
    st = _stream(stream)
    xs = TensorStruct(X.data_ptr(), dtype_code(X), ld_last, st)
    arr = (ctypes.c_int64 * d)(*dims)
    out = TTStruct()
    _check(lib().ttsvd_decompose_ws(ctypes.byref(xs), arr, d, r_max, float(tol), ws.data_ptr(),
                                    ws.numel() * ws.element_size(), cores.data_ptr(),
                                    cores.numel() * cores.element_size() // 8, ctypes.byref(out)))
    try:
        return _to_tt(out, X.device, st, fetch)
    finally:
        lib().ttsvd_tt_free(ctypes.byref(out))


def thick_bounds_k(dims: Sequence[int], m_min: int, f1_min: float, r_est: int):
    """``ttsvd_thick_bounds_k``: (k, m) of the thick-bounds variant."""
    dims = [int(n) for n in dims]
    arr = (ctypes.c_int64 * max(1, len(dims)))(*dims)
    k = ctypes.c_int(0)
    m = ctypes.c_int64(0)
    _check(lib().ttsvd_thick_bounds_k(arr, len(dims), int(m_min), float(f1_min), int(r_est),
                                      ctypes.byref(k), ctypes.byref(m)))
    return k.value, m.value


def ttsvd_decompose_thick(X, dims: Sequence[int], r_max: int, tol: float, m_min: int = 16,
                          f1_min: float = 0.5, stream=None) -> TT:
    """``ttsvd_decompose_thick`` (Algorithm 3) of the Fortran-ordered device tensor X."""
    dims = [int(n) for n in dims]
    d = len(dims)
    st = _stream(stream)
    xs = TensorStruct(X.data_ptr(), dtype_code(X), 0, st)
    arr = (ctypes.c_int64 * d)(*dims)
    out = TTStruct()
    _check(lib().ttsvd_decompose_thick(ctypes.byref(xs), arr, d, r_max, float(tol), int(m_min),
                                       float(f1_min), ctypes.byref(out)))
    try:
        return _to_tt(out, X.device, st)
    finally:
        lib().ttsvd_tt_free(ctypes.byref(out))


def _batch_args(Xs, dims_list, r_max, tol, st):
    n = len(Xs)
    if n != len(dims_list):
        raise ValueError("one dims list per tensor")
    r_max = list(r_max) if isinstance(r_max, (list, tuple)) else [int(r_max)] * n
    tol = list(tol) if isinstance(tol, (list, tuple)) else [float(tol)] * n
    xs = (TensorStruct * n)(*[TensorStruct(X.data_ptr(), dtype_code(X), 0, st) for X in Xs])
    d = (ctypes.c_int * n)(*[len(dl) for dl in dims_list])
    flat = [int(v) for dl in dims_list for v in dl]
    dims = (ctypes.c_int64 * max(1, len(flat)))(*flat)
    rm = (ctypes.c_int64 * n)(*[int(r) for r in r_max])
    tl = (ctypes.c_double * n)(*[float(t) for t in tol])
    return n, xs, d, dims, rm, tl


def batch_default_config() -> BatchConfig:
    c = BatchConfig()
    _check(lib().ttsvd_batch_default_config(ctypes.byref(c)))
    return c


def ttsvd_decompose_batch(Xs, dims_list, r_max, tol, cfg: Optional[BatchConfig] = None,
                          stream=None, fetch: bool = True) -> List[TT]:
    """``ttsvd_decompose_batch`` of the Fortran-ordered device tensors Xs (one
    persistent launch); r_max and tol are scalars or per-tensor lists.  With
    fetch=False the cores are not copied out (ranks, sigma and bounds only)."""
    st = _stream(stream)
    n, xs, d, dims, rm, tl = _batch_args(Xs, dims_list, r_max, tol, st)
    outs = (TTStruct * n)()
    _check(lib().ttsvd_decompose_batch(n, xs, d, dims, rm, tl,
                                       ctypes.byref(cfg) if cfg is not None else None, st, outs))
    try:
        return [_to_tt(outs[t], Xs[t].device, st, fetch) for t in range(n)]
    finally:
        for t in range(n):
            lib().ttsvd_tt_free(ctypes.byref(outs[t]))


def ttsvd_batch_autotune(Xs, dims_list, r_max, tol, stream=None):
    """``ttsvd_batch_autotune``: (best BatchConfig, its time in ms)."""
    st = _stream(stream)
    n, xs, d, dims, rm, tl = _batch_args(Xs, dims_list, r_max, tol, st)
    best = BatchConfig()
    ms = ctypes.c_double(0.0)
    _check(lib().ttsvd_batch_autotune(n, xs, d, dims, rm, tl, st, ctypes.byref(best),
                                      ctypes.byref(ms)))
    return best, float(ms.value)


def core_array(t, shape):
    """A Fortran-ordered numpy copy of a flat device core."""
    import numpy as np
    return np.asarray(t.cpu().numpy()).reshape(shape, order="F")


# ----------------------------------------------------------------- serving

def server_default_config() -> ServerConfig:
    c = ServerConfig()
    _check(lib().ttsvd_server_default_config(ctypes.byref(c)))
    return c


def server_clock() -> float:
    """The steady clock (seconds) of the server's timestamps."""
    return float(lib().ttsvd_server_clock())


class Server:
    """``ttsvd_server_*``: queued TT-SVD requests on worker streams.  The
    submitted tensors must stay alive until their completion is polled."""

    def __init__(self, cfg: Optional[ServerConfig] = None):
        self._h = ctypes.c_void_p()
        cfg = cfg if cfg is not None else server_default_config()
        _check(lib().ttsvd_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))

    def submit(self, X, dims: Sequence[int], r_max: int, tol: float, stream=None) -> int:
        """Queue X; its work starts after what was enqueued on ``stream`` (the
        producer's stream, default: torch's current stream) before the call."""
        xs = TensorStruct(X.data_ptr(), dtype_code(X), 0, _stream(stream))
        arr = (ctypes.c_int64 * len(dims))(*[int(n) for n in dims])
        t = ctypes.c_uint64(0)
        _check(lib().ttsvd_server_submit(self._h, ctypes.byref(xs), arr, len(dims), int(r_max),
                                         float(tol), ctypes.byref(t)))
        return int(t.value)

    def poll(self, max_n: int = 256, wait_ms: int = 0, fetch: bool = False, device=None) -> list:
        """Finished requests: dicts with ticket, status, batch_size, the three
        timestamps and the result (a TT; its cores only if fetch)."""
        arr = (Completion * max_n)()
        n = ctypes.c_int(0)
        _check(lib().ttsvd_server_poll(self._h, arr, max_n, int(wait_ms), ctypes.byref(n)))
        out = []
        for i in range(n.value):
            c = arr[i]
            item = dict(ticket=int(c.ticket), status=int(c.status), batch_size=int(c.batch_size),
                        batched=bool(c.batched),
                        t_submit=float(c.t_submit), t_start=float(c.t_start),
                        t_done=float(c.t_done), message=c.message.decode(errors="replace"),
                        result=None)
            if c.status == TTSVD_OK:
                try:
                    item["result"] = _to_tt(c.tt, device, _stream(None), fetch)
                finally:
                    lib().ttsvd_tt_free(ctypes.byref(arr[i].tt))
            out.append(item)
        return out

    def pending(self) -> int:
        return int(lib().ttsvd_server_pending(self._h))

    def close(self) -> None:
        if self._h:
            lib().ttsvd_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
