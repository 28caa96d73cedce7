"""ctypes binding of the C ABI in include/flp.h (argument marshalling only).

Every function here forwards to the HIP library ``libflp.so``; nothing is
computed in Python.  Device buffers are torch CUDA (HIP) tensors; streams
are torch streams.  If the library is not built, the first call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflp.so")

FLP_OK = 0
FLP_E_ARG = -1
FLP_E_INTERVAL = -2
FLP_E_NOTSYM = -3
FLP_E_NOMEM = -4
FLP_E_NOCONV = -5
FLP_E_DEVICE = -6
FLP_E_PENDING = -7
FLP_E_CANCELLED = -8
FLP_PREC_FP64 = 0
FLP_PREC_FP32_FILTER = 1
FLP_FORMAT_AUTO = 0
FLP_FORMAT_CSR = 1
FLP_FORMAT_SELL = 2

EXPORTS = [
    "flp_opts_default", "flp_build_filter", "flp_build_filter_eps", "flp_filter_free",
    "flp_filter_degree", "flp_filter_coeffs", "flp_filter_info", "flp_filter_eval", "flp_filter_divided",
    "flp_filter_apply", "flp_filter_apply_noalloc", "flp_filter_launch_shape", "flp_tile_order", "flp_tune_filter", "flp_set_autotune", "flp_set_filter_shape", "flp_spmm", "flp_block_orth", "flp_block_qr", "flp_estimate_bounds",
    "flp_solve", "flp_solve_sliced", "flp_solve_batch", "flp_result_free", "flp_result_copy_evecs", "flp_host_sym_eig",
    "flp_release_workspace", "flp_set_allocator", "flp_check_symmetric", "flp_last_error", "flp_version",
    "flp_abi_sizes",
    "flp_server_opts_default", "flp_server_create", "flp_server_submit", "flp_server_poll",
    "flp_server_wait", "flp_server_cancel", "flp_server_stats", "flp_server_footprint", "flp_server_destroy",
]


class FlpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"flp error {code}: {msg}")
        self.code = code


class FlpCsrC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p), ("val32", ctypes.c_void_p)]


class FlpTuneInfoC(ctypes.Structure):
    _fields_ = [("group_width", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32),
                ("cols_per_lane", ctypes.c_int32), ("rows_per_wave", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("streaming_loads", ctypes.c_int32),
                ("us_per_step", ctypes.c_double), ("tile_chunk", ctypes.c_int32), ("lds_window", ctypes.c_int32),
                ("window_halo", ctypes.c_int32)]


class FlpOptsC(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("degree", ctypes.c_int32), ("eps", ctypes.c_double),
                ("tol", ctypes.c_double), ("check_every", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("max_basis", ctypes.c_int64), ("k0", ctypes.c_int32),
                ("start", ctypes.c_void_p), ("lmin", ctypes.c_double), ("lmax", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("sym_tol", ctypes.c_double), ("polish_degree", ctypes.c_int32),
                ("unfiltered", ctypes.c_int32), ("format", ctypes.c_int32), ("warm", ctypes.c_void_p),
                ("warm_count", ctypes.c_int32)]


class FlpStatsC(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("mv", ctypes.c_int64), ("basis_cols", ctypes.c_int32),
                ("polish_sweeps", ctypes.c_int32), ("t_pre", ctypes.c_double), ("t_mv", ctypes.c_double),
                ("t_orth", ctypes.c_double), ("t_check", ctypes.c_double), ("t_rr", ctypes.c_double),
                ("t_total", ctypes.c_double), ("filter_bytes", ctypes.c_double), ("orth_bytes", ctypes.c_double),
                ("filter_format", ctypes.c_int32), ("filter_group_width", ctypes.c_int32),
                ("filter_lanes_per_row", ctypes.c_int32), ("filter_cols_per_lane", ctypes.c_int32),
                ("filter_streaming_loads", ctypes.c_int32), ("filter_tile_chunk", ctypes.c_int32),
                ("polish_bytes", ctypes.c_double),
                ("t_polish", ctypes.c_double), ("warm_status", ctypes.c_int32), ("warm_sweeps", ctypes.c_int32),
                ("filter_lds_window", ctypes.c_int32), ("filter_window_halo", ctypes.c_int32),
                ("separations", ctypes.c_int32), ("candidates", ctypes.c_int32), ("guards", ctypes.c_int32)]


class FlpBatchStatsC(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_int32), ("block_steps", ctypes.c_int32), ("filter_launches", ctypes.c_int32),
                ("graph_captures", ctypes.c_int32), ("graph_replays", ctypes.c_int32),
                ("t_total", ctypes.c_double), ("t_setup", ctypes.c_double), ("t_filter", ctypes.c_double),
                ("t_orth_check", ctypes.c_double), ("t_finish", ctypes.c_double),
                ("filter_bytes", ctypes.c_double), ("t_orth", ctypes.c_double), ("orth_bytes", ctypes.c_double),
                ("peak_active", ctypes.c_int32), ("admission_waits", ctypes.c_int32),
                ("finish_waits", ctypes.c_int32), ("mem_budget", ctypes.c_double),
                ("peak_mem_reserved", ctypes.c_double)]


class FlpServerOptsC(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("prec", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("max_basis", ctypes.c_int64), ("mem_budget", ctypes.c_double), ("use_graph", ctypes.c_int32)]


class FlpResultC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("count", ctypes.c_int32), ("evals", ctypes.POINTER(ctypes.c_double)),
                ("resid", ctypes.POINTER(ctypes.c_double)), ("evecs", ctypes.c_void_p),
                ("lmin", ctypes.c_double), ("lmax", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("degree", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("stats", FlpStatsC)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libflp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run python -m paper_2409_15053_amd.build)")
    lib = ctypes.CDLL(path)
    P, I32, I64, F64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "flp_opts_default": (None, [ctypes.POINTER(FlpOptsC)]),
        "flp_build_filter": (ctypes.c_int, [F64, F64, I32, F64, F64, PP]),
        "flp_build_filter_eps": (ctypes.c_int, [F64, F64, I32, F64, F64, F64, PP]),
        "flp_filter_free": (None, [P]),
        "flp_filter_degree": (I32, [P]),
        "flp_filter_coeffs": (I32, [P, P, I32]),
        "flp_filter_info": (ctypes.c_int, [P, P]),
        "flp_filter_eval": (ctypes.c_int, [P, P, P, I32]),
        "flp_filter_divided": (I32, [P, F64, P, I32]),
        "flp_filter_apply": (ctypes.c_int, [P, ctypes.POINTER(FlpCsrC), P, I64, P, I64, I32, I32, I32, P]),
        "flp_filter_apply_noalloc": (ctypes.c_int, [P, ctypes.POINTER(FlpCsrC), P, I64, P, I64, I32, I32, P]),
        "flp_filter_launch_shape": (ctypes.c_int, [I32, I32, I32, ctypes.POINTER(FlpTuneInfoC)]),
        "flp_tile_order": (ctypes.c_int, [I32, I32, I32, P]),
        "flp_tune_filter": (ctypes.c_int, [ctypes.POINTER(FlpCsrC), I32, I32, I32, P,
                                           ctypes.POINTER(FlpTuneInfoC)]),
        "flp_set_autotune": (None, [I32]),
        "flp_set_filter_shape": (None, [I32, I32, I32, I32, I32, I32]),
        "flp_spmm": (ctypes.c_int, [ctypes.POINTER(FlpCsrC), P, I32, P, I32, I32, P]),
        "flp_block_orth": (ctypes.c_int, [P, I64, I32, I32, P, I32, P, P]),
        "flp_block_qr": (ctypes.c_int, [P, I32, I32, P, P]),
        "flp_estimate_bounds": (ctypes.c_int, [ctypes.POINTER(FlpCsrC), I32, U64, P, P, P]),
        "flp_solve": (ctypes.c_int, [ctypes.POINTER(FlpCsrC), F64, F64, ctypes.POINTER(FlpOptsC),
                                     ctypes.POINTER(ctypes.POINTER(FlpResultC))]),
        "flp_solve_sliced": (ctypes.c_int, [ctypes.POINTER(FlpCsrC), F64, F64, I32, ctypes.POINTER(FlpOptsC),
                                            ctypes.POINTER(ctypes.POINTER(FlpResultC))]),
        "flp_solve_batch": (ctypes.c_int, [I32, P, P, P, P, I32, P, P, ctypes.POINTER(FlpBatchStatsC)]),
        "flp_result_free": (None, [ctypes.POINTER(FlpResultC)]),
        "flp_result_copy_evecs": (ctypes.c_int, [ctypes.POINTER(FlpResultC), P, P]),
        "flp_host_sym_eig": (ctypes.c_int, [I32, I32, P, P, P]),
        "flp_release_workspace": (None, []),
        "flp_set_allocator": (None, [P, P, P]),
        "flp_check_symmetric": (ctypes.c_int, [ctypes.POINTER(FlpCsrC), F64, P]),
        "flp_server_cancel": (ctypes.c_int, [P, U64]),
        "flp_server_opts_default": (None, [ctypes.POINTER(FlpServerOptsC)]),
        "flp_server_create": (ctypes.c_int, [ctypes.POINTER(FlpServerOptsC), PP]),
        "flp_server_submit": (ctypes.c_int, [P, ctypes.POINTER(FlpCsrC), F64, F64, ctypes.POINTER(FlpOptsC),
                                             ctypes.POINTER(ctypes.c_uint64)]),
        "flp_server_poll": (ctypes.c_int, [P, U64, ctypes.POINTER(ctypes.POINTER(FlpResultC))]),
        "flp_server_wait": (ctypes.c_int, [P, U64, ctypes.POINTER(ctypes.POINTER(FlpResultC))]),
        "flp_server_stats": (ctypes.c_int, [P, ctypes.POINTER(FlpBatchStatsC)]),
        "flp_server_footprint": (ctypes.c_int, [P, ctypes.POINTER(FlpCsrC), ctypes.POINTER(FlpOptsC),
                                                ctypes.POINTER(ctypes.c_double)]),
        "flp_server_destroy": (ctypes.c_int, [P]),
        "flp_last_error": (ctypes.c_char_p, []),
        "flp_version": (ctypes.c_char_p, []),
        "flp_abi_sizes": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, allow=()):
    if rc != FLP_OK and rc not in allow:
        raise FlpError(rc, load().flp_last_error().decode())
    return rc


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ matrices

class DeviceCsr:
    """A CSR matrix resident in device memory (torch tensors kept alive here)."""

    def __init__(self, n, rowptr, colind, val, val32=None):
        self.n = int(n)
        self.rowptr, self.colind, self.val, self.val32 = rowptr, colind, val, val32
        self.nnz = int(colind.numel())
        self.c = FlpCsrC(self.n, self.nnz, rowptr.data_ptr(), colind.data_ptr(), val.data_ptr(),
                         val32.data_ptr() if val32 is not None else None)

    @classmethod
    def from_host(cls, A, device="cuda:0", with_fp32: bool = False):
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(A.rowptr, dtype=np.int32)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(A.colind, dtype=np.int32)).to(device)
        va = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(device)
        v32 = va.float() if with_fp32 else None
        return cls(A.n, rp, ci, va, v32)


# ------------------------------------------------------------------ filter

class Filter:
    """Owner of an flp_filter handle."""

    def __init__(self, handle):
        self.h = handle

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.flp_filter_free(self.h)
            self.h = None

    @property
    def degree(self) -> int:
        return int(load().flp_filter_degree(self.h))

    def coeffs(self) -> np.ndarray:
        m1 = load().flp_filter_coeffs(self.h, None, 0)
        out = np.zeros(m1)
        _check(0 if load().flp_filter_coeffs(self.h, _np_ptr(out), m1) == m1 else -1)
        return out

    def info(self) -> dict:
        o = np.zeros(6)
        _check(load().flp_filter_info(self.h, _np_ptr(o)))
        return dict(lmin=o[0], lmax=o[1], c=o[2], e=o[3], alpha=o[4], beta=o[5])

    def eval(self, z) -> np.ndarray:
        z = np.ascontiguousarray(np.atleast_1d(z), dtype=np.float64)
        out = np.zeros_like(z)
        _check(load().flp_filter_eval(self.h, _np_ptr(z), _np_ptr(out), z.size))
        return out

    def divided(self, t: float) -> np.ndarray:
        """Chebyshev coefficients of (p(z) - p(t)) / (z - t)."""
        m = max(self.degree, 1)
        out = np.zeros(m)
        got = load().flp_filter_divided(self.h, float(t), _np_ptr(out), m)
        _check(0 if got == m else (got if got < 0 else -1))
        return out


def flp_build_filter(alpha: float, beta: float, degree: int, lmin: float, lmax: float,
                     eps: float | None = None) -> Filter:
    lib = load()
    h = ctypes.c_void_p()
    if eps is None:
        _check(lib.flp_build_filter(alpha, beta, degree, lmin, lmax, ctypes.byref(h)))
    else:
        _check(lib.flp_build_filter_eps(alpha, beta, degree, lmin, lmax, eps, ctypes.byref(h)))
    return Filter(h)


def flp_filter_apply(filt: Filter, A: DeviceCsr, V, W, prec: int = FLP_PREC_FP64, stream=None,
                     format: int = FLP_FORMAT_CSR):
    """W = p(Ahat) V on the device.  V, W: float64 n x r tensors (or
    vectors) whose rows may be strided (stride(1) == 1); their row strides
    are passed as the leading dimensions.  ``format`` selects the storage
    the products read A in (FLP_FORMAT_CSR, FLP_FORMAT_SELL, FLP_FORMAT_AUTO)."""
    assert V.dtype == W.dtype
    r = 1 if V.dim() == 1 else V.shape[1]
    if V.dim() == 1:
        assert V.is_contiguous() and W.is_contiguous()
        ldv = ldw = 1
    else:
        assert V.stride(1) == 1 and W.stride(1) == 1
        ldv, ldw = V.stride(0), W.stride(0)
    _check(load().flp_filter_apply(filt.h, ctypes.byref(A.c), V.data_ptr(), ldv, W.data_ptr(), ldw, r, prec,
                                   format, _stream_ptr(stream)))


def flp_filter_apply_noalloc(filt: Filter, A: DeviceCsr, V, W, prec: int = FLP_PREC_FP64, stream=None):
    """W = p(Ahat) V on the device without allocating device memory (CSR
    storage, the library's fixed scratch array; n * r <= 2^20).  V, W as
    for flp_filter_apply."""
    assert V.dtype == W.dtype
    r = 1 if V.dim() == 1 else V.shape[1]
    if V.dim() == 1:
        assert V.is_contiguous() and W.is_contiguous()
        ldv = ldw = 1
    else:
        assert V.stride(1) == 1 and W.stride(1) == 1
        ldv, ldw = V.stride(0), W.stride(0)
    _check(load().flp_filter_apply_noalloc(filt.h, ctypes.byref(A.c), V.data_ptr(), ldv, W.data_ptr(), ldw, r,
                                           prec, _stream_ptr(stream)))


def flp_filter_launch_shape(r: int, prec: int = FLP_PREC_FP64, segmented: bool = False) -> dict:
    """The untuned launch shape of a filter step over r columns (host only)."""
    info = FlpTuneInfoC()
    _check(load().flp_filter_launch_shape(r, prec, 1 if segmented else 0, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in FlpTuneInfoC._fields_}


def flp_tile_order(tiles: int, tile_chunk: int, rows_per_tile: int) -> np.ndarray:
    """Row tile processed by each workgroup of a filter launch (host only)."""
    out = np.zeros(max(0, tiles), dtype=np.int32)
    _check(load().flp_tile_order(tiles, tile_chunk, rows_per_tile, _np_ptr(out)))
    return out


def flp_tune_filter(A: DeviceCsr, r: int, prec: int = FLP_PREC_FP64, stream=None,
                    format: int = FLP_FORMAT_CSR) -> dict:
    """The filter launch configuration for r columns of A read in storage
    ``format`` (tuned on first use)."""
    info = FlpTuneInfoC()
    _check(load().flp_tune_filter(ctypes.byref(A.c), r, prec, format, _stream_ptr(stream), ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in FlpTuneInfoC._fields_}


def flp_set_autotune(on: bool):
    load().flp_set_autotune(1 if on else 0)


FLP_TILE_CHUNK_TUNED = -(1 << 31)


def flp_set_filter_shape(lanes_per_row: int = 0, cols_per_lane: int = 0, group_width: int = 0,
                         streaming_loads: bool = False, tile_chunk: int = FLP_TILE_CHUNK_TUNED,
                         lds_window: int = 0):
    """Force one filter launch configuration (all zeros and tile_chunk =
    FLP_TILE_CHUNK_TUNED: back to tuning).  Any other tile_chunk forces the
    tile-to-XCD mapping (< 0: the pencil walk over planes of -tile_chunk rows).
    lds_window: 0 none, 1 the fixed +-8-row window, 2 the sliding window
    fitted to each matrix."""
    load().flp_set_filter_shape(lanes_per_row, cols_per_lane, group_width, 1 if streaming_loads else 0,
                                tile_chunk, int(lds_window))


def flp_spmm(A: DeviceCsr, X, Y, stream=None):
    r = 1 if X.dim() == 1 else X.shape[1]
    ldx = r if X.dim() == 1 else X.stride(0)
    ldy = r if Y.dim() == 1 else Y.stride(0)
    _check(load().flp_spmm(ctypes.byref(A.c), X.data_ptr(), ldx, Y.data_ptr(), ldy, r, _stream_ptr(stream)))


def flp_block_orth(Q, k: int, W, stream=None) -> np.ndarray:
    """CGS2 of W (n x r) against the first k columns of Q (n x ldq); returns H (k x r)."""
    n, r = W.shape
    H = np.zeros((k, r))
    _check(load().flp_block_orth(Q.data_ptr(), Q.stride(0), k, n, W.data_ptr(), r, _np_ptr(H),
                                 _stream_ptr(stream)))
    return H


def flp_block_qr(W, stream=None) -> np.ndarray:
    n, r = W.shape
    S = np.zeros((r, r))
    _check(load().flp_block_qr(W.data_ptr(), n, r, _np_ptr(S), _stream_ptr(stream)))
    return S


def flp_estimate_bounds(A: DeviceCsr, k0: int = 40, seed: int = 0, stream=None):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(load().flp_estimate_bounds(ctypes.byref(A.c), k0, seed, ctypes.byref(lo), ctypes.byref(hi),
                                      _stream_ptr(stream)))
    return lo.value, hi.value


def flp_host_sym_eig(M: np.ndarray, bw: int | None = None, vectors: bool = True):
    M = np.ascontiguousarray(M, dtype=np.float64)
    N = M.shape[0]
    ev = np.zeros(N)
    Z = np.zeros((N, N)) if vectors else None
    _check(load().flp_host_sym_eig(N, N - 1 if bw is None else bw, _np_ptr(M), _np_ptr(ev),
                                   _np_ptr(Z) if vectors else None))
    return (ev, Z) if vectors else ev


def default_opts() -> FlpOptsC:
    o = FlpOptsC()
    load().flp_opts_default(ctypes.byref(o))
    return o


def flp_solve(A: DeviceCsr, alpha: float, beta: float, block: int = 1, degree: int = 0, seed: int = 0,
              prec: int = FLP_PREC_FP64, start: np.ndarray | None = None, bounds=None, max_basis: int = 0,
              check_every: int = 0, eps: float = 0.0, k0: int = 0, want_vectors: bool = True,
              stream=None, sym_tol: float = -1.0, polish_degree: int = 0, unfiltered: bool = False,
              format: int = 0, warm=None) -> dict:
    """Every eigenpair of A in [alpha, beta].  Returns a dict with numpy
    ``evals``/``resid``, a torch ``evecs`` (n x count, float64, on A's
    device) and the solve statistics.  ``sym_tol >= 0`` checks A for
    symmetry first (FLP_E_NOTSYM if it is not).  ``unfiltered=True`` runs
    plain block Lanczos with the mapped matrix in place of the filter (FP64
    only).  ``format`` picks the storage the filter reads A in
    (FLP_FORMAT_AUTO, FLP_FORMAT_CSR or FLP_FORMAT_SELL, a sliced ELL copy);
    ``stats["filter_format"]`` reports the one used.  ``warm``: a float64
    n x k device tensor with unit column stride or column-major layout
    (e.g. a previous result's ``evecs``) to warm-start from."""
    import torch
    lib = load()
    o = default_opts()
    o.block = block
    o.degree = degree
    o.seed = seed
    o.prec = prec
    o.max_basis = max_basis
    if check_every:
        o.check_every = check_every
    if eps:
        o.eps = eps
    if k0:
        o.k0 = k0
    keep = None
    if start is not None:
        keep = np.ascontiguousarray(start, dtype=np.float64)
        o.start = _np_ptr(keep)
    if bounds is not None:
        o.lmin, o.lmax = bounds
    o.stream = _stream_ptr(stream)
    o.sym_tol = sym_tol
    o.polish_degree = polish_degree
    o.unfiltered = 1 if unfiltered else 0
    o.format = format
    if warm is not None:
        # column-major n x k: column j at data_ptr + j * n
        assert warm.dtype == torch.float64 and warm.shape[0] == A.n
        if warm.dim() == 1:
            warm = warm[:, None]
        if not (warm.stride(0) == 1 and warm.stride(1) == A.n):
            warm = warm.t().contiguous().t()
        o.warm = warm.data_ptr()
        o.warm_count = warm.shape[1]
    res = ctypes.POINTER(FlpResultC)()
    rc = lib.flp_solve(ctypes.byref(A.c), alpha, beta, ctypes.byref(o), ctypes.byref(res))
    _check(rc, allow=(FLP_E_NOCONV,))
    try:
        r = res.contents
        cnt = r.count
        evals = np.array([r.evals[i] for i in range(cnt)], dtype=np.float64)
        resid = np.array([r.resid[i] for i in range(cnt)], dtype=np.float64)
        evecs = None
        if want_vectors:
            evecs_t = torch.empty((cnt, A.n), dtype=torch.float64, device=A.val.device)
            if cnt:
                _check(lib.flp_result_copy_evecs(res, evecs_t.data_ptr(), _stream_ptr(stream)))
            evecs = evecs_t.t()
        st = r.stats
        stats = {f: getattr(st, f) for f, _ in FlpStatsC._fields_}
        out = dict(evals=evals, resid=resid, evecs=evecs, count=cnt, lmin=r.lmin, lmax=r.lmax,
                   degree=r.degree, converged=bool(r.converged), rc=rc, stats=stats)
    finally:
        lib.flp_result_free(res)
    return out


def flp_solve_sliced(A: DeviceCsr, alpha: float, beta: float, nslices: int, block: int = 8, degree: int = 0,
                     seed: int = 0, prec: int = FLP_PREC_FP64, bounds=None, max_basis: int = 0,
                     check_every: int = 0, eps: float = 0.0, k0: int = 0, want_vectors: bool = True,
                     stream=None, polish_degree: int = 0) -> dict:
    """Every eigenpair of A in [alpha, beta] by nslices slices solved as one
    batch (same return value as flp_solve)."""
    lib = load()
    o = _make_opts(block, degree, seed, prec, max_basis, check_every, eps, k0, bounds, stream,
                   polish_degree=polish_degree)
    res = ctypes.POINTER(FlpResultC)()
    rc = lib.flp_solve_sliced(ctypes.byref(A.c), alpha, beta, nslices, ctypes.byref(o), ctypes.byref(res))
    _check(rc, allow=(FLP_E_NOCONV,))
    try:
        out = _collect(res, A.n, A.val.device, want_vectors, stream)
        out["rc"] = rc
    finally:
        lib.flp_result_free(res)
    return out


def _make_opts(block, degree, seed, prec, max_basis, check_every, eps, k0, bounds, stream, start=None,
               polish_degree=0, format=FLP_FORMAT_AUTO):
    o = default_opts()
    o.polish_degree = polish_degree
    o.format = format
    o.block = block
    o.degree = degree
    o.seed = seed
    o.prec = prec
    o.max_basis = max_basis
    if check_every:
        o.check_every = check_every
    if eps:
        o.eps = eps
    if k0:
        o.k0 = k0
    if bounds is not None:
        o.lmin, o.lmax = bounds
    o.stream = _stream_ptr(stream)
    return o


def _collect(res_ptr, n, device, want_vectors, stream):
    import torch
    lib = load()
    r = res_ptr.contents
    cnt = r.count
    evals = np.array([r.evals[i] for i in range(cnt)], dtype=np.float64)
    resid = np.array([r.resid[i] for i in range(cnt)], dtype=np.float64)
    evecs = None
    if want_vectors:
        evecs_t = torch.empty((cnt, n), dtype=torch.float64, device=device)
        if cnt:
            _check(lib.flp_result_copy_evecs(res_ptr, evecs_t.data_ptr(), _stream_ptr(stream)))
        evecs = evecs_t.t()
    st = r.stats
    stats = {f: getattr(st, f) for f, _ in FlpStatsC._fields_}
    return dict(evals=evals, resid=resid, evecs=evecs, count=cnt, lmin=r.lmin, lmax=r.lmax,
                degree=r.degree, converged=bool(r.converged), stats=stats)


def flp_solve_batch(As, alphas, betas, block: int = 8, degree=0, seeds=None, prec: int = FLP_PREC_FP64,
                    use_graph: bool = True, max_basis: int = 0, check_every: int = 0, eps: float = 0.0,
                    k0: int = 0, want_vectors: bool = True, stream=None, polish_degree: int = 0,
                    format: int = FLP_FORMAT_AUTO):
    """Solve len(As) independent problems together (segmented filter
    launches).  Returns (list of per-solve dicts like flp_solve, batch stats)."""
    import torch
    lib = load()
    cnt = len(As)
    if seeds is None:
        seeds = list(range(cnt))
    degrees = degree if isinstance(degree, (list, tuple)) else [degree] * cnt
    opts = (FlpOptsC * cnt)()
    for i in range(cnt):
        opts[i] = _make_opts(block, degrees[i], seeds[i], prec, max_basis, check_every, eps, k0, None, stream,
                             polish_degree=polish_degree, format=format)
    arr = (ctypes.POINTER(FlpCsrC) * cnt)(*[ctypes.pointer(A.c) for A in As])
    al = np.ascontiguousarray(alphas, dtype=np.float64)
    be = np.ascontiguousarray(betas, dtype=np.float64)
    res = (ctypes.POINTER(FlpResultC) * cnt)()
    codes = np.zeros(cnt, dtype=np.int32)
    bst = FlpBatchStatsC()
    rc = lib.flp_solve_batch(cnt, ctypes.cast(arr, ctypes.c_void_p), _np_ptr(al), _np_ptr(be),
                             ctypes.cast(opts, ctypes.c_void_p), 1 if use_graph else 0,
                             ctypes.cast(res, ctypes.c_void_p), _np_ptr(codes), ctypes.byref(bst))
    out = []
    try:
        _check(rc, allow=(FLP_E_NOCONV,))
        for i in range(cnt):
            _check(int(codes[i]), allow=(FLP_E_NOCONV,))
            d = _collect(res[i], As[i].n, As[i].val.device, want_vectors, stream)
            d["rc"] = int(codes[i])
            out.append(d)
    finally:
        for i in range(cnt):
            if res[i]:
                lib.flp_result_free(res[i])
    return out, {f: getattr(bst, f) for f, _ in FlpBatchStatsC._fields_}


class Server:
    """Continuous-batching server (flp_server_*): submit requests from any
    thread, collect results with poll/wait."""

    def __init__(self, block: int = 8, prec: int = FLP_PREC_FP32_FILTER, max_active: int = 64,
                 max_basis: int = 1024, mem_budget: float = 0.0, use_graph: bool = True):
        lib = load()
        o = FlpServerOptsC()
        lib.flp_server_opts_default(ctypes.byref(o))
        o.block, o.prec, o.max_active, o.max_basis = block, prec, max_active, max_basis
        o.mem_budget, o.use_graph = mem_budget, 1 if use_graph else 0
        h = ctypes.c_void_p()
        _check(lib.flp_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, A: DeviceCsr, alpha: float, beta: float, seed: int = 0, degree: int = 0,
               max_basis: int = 0, check_every: int = 0, polish_degree: int = 0) -> int:
        import torch
        o = _make_opts(1, degree, seed, 0, max_basis, check_every, 0.0, 0, None, None, polish_degree=polish_degree)
        # the server reads A after the work queued so far on torch's current
        # stream (where from_host wrote it)
        o.stream = _stream_ptr(torch.cuda.current_stream(A.val.device))
        t = ctypes.c_uint64()
        _check(load().flp_server_submit(self.h, ctypes.byref(A.c), alpha, beta, ctypes.byref(o), ctypes.byref(t)))
        self._keep[t.value] = A  # the matrix must outlive the request
        return t.value

    def cancel(self, ticket: int):
        """Cancel a request that has not completed (wait/poll then raise
        FlpError with code FLP_E_CANCELLED)."""
        _check(load().flp_server_cancel(self.h, ticket))

    def _finish(self, ticket, rc, res, want_vectors):
        A = self._keep.pop(ticket, None)
        try:
            _check(rc, allow=(FLP_E_NOCONV,))
            d = _collect(res, A.n, A.val.device, want_vectors, None)
            d["rc"] = rc
            return d
        finally:
            if res:
                load().flp_result_free(res)

    def poll(self, ticket: int, want_vectors: bool = False):
        res = ctypes.POINTER(FlpResultC)()
        rc = load().flp_server_poll(self.h, ticket, ctypes.byref(res))
        if rc == FLP_E_PENDING:
            return None
        return self._finish(ticket, rc, res, want_vectors)

    def wait(self, ticket: int, want_vectors: bool = False):
        res = ctypes.POINTER(FlpResultC)()
        rc = load().flp_server_wait(self.h, ticket, ctypes.byref(res))
        return self._finish(ticket, rc, res, want_vectors)

    def footprint(self, A: DeviceCsr, max_basis: int = 0) -> float:
        """Device bytes a request for A reserves at admission."""
        o = _make_opts(1, 0, 0, 0, max_basis, 0, 0.0, 0, None, None)
        o.stream = None
        b = ctypes.c_double()
        _check(load().flp_server_footprint(self.h, ctypes.byref(A.c), ctypes.byref(o), ctypes.byref(b)))
        return b.value

    def stats(self) -> dict:
        st = FlpBatchStatsC()
        _check(load().flp_server_stats(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in FlpBatchStatsC._fields_}

    def close(self):
        if getattr(self, "h", None):
            rc = load().flp_server_destroy(self.h)
            self.h = None
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocators = []  # every registered pair stays alive: memory returns to the pair that made it


def flp_set_allocator(alloc=None, free=None):
    """Route the library's device allocations through alloc(nbytes) -> int
    address (0 on failure) and free(address); no arguments restores
    hipMalloc/hipFree."""
    lib = load()
    if alloc is None or free is None:
        lib.flp_set_allocator(None, None, None)
        return
    a = _ALLOC_FN(lambda nbytes, ctx: int(alloc(int(nbytes)) or 0))
    f = _FREE_FN(lambda ptr, ctx: free(int(ptr)))
    _allocators.append((a, f))
    lib.flp_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p), None)


def torch_allocator():
    """(alloc, free) backed by torch's caching allocator on the current device."""
    import torch
    dev = torch.cuda.current_device()
    live = {}

    def alloc(nbytes):
        t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=f"cuda:{dev}")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr):
        live.pop(ptr, None)

    return alloc, free


def flp_check_symmetric(A: "DeviceCsr", tol: float = 0.0, stream=None) -> bool:
    """True when every stored a_ij has a stored a_ji within tol (relative)."""
    rc = load().flp_check_symmetric(ctypes.byref(A.c), tol, _stream_ptr(stream))
    if rc == FLP_E_NOTSYM:
        return False
    _check(rc)
    return True


def flp_release_workspace():
    load().flp_release_workspace()


def flp_version() -> str:
    return load().flp_version().decode()
