"""ctypes binding to libgmres_hip.so (C ABI in include/gmres.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels. The functions carry the C names; ``GmresSolver`` bundles a context
with the torch tensors (CSR arrays, workspace) it borrows. There is no CPU
fallback: if the library is not built, loading it raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmres_hip.so")

GMRES_MGS, GMRES_MGS_1R, GMRES_CGS2, GMRES_MGS_1R_IR32, GMRES_MGS_1R_IR16 = 0, 1, 2, 3, 4
GMRES_CGS2_3R, GMRES_TWO_SYNCH = 5, 6
SCHEMES = {"mgs": GMRES_MGS, "mgs1r": GMRES_MGS_1R, "cgs2": GMRES_CGS2,
           "mgs1r_ir32": GMRES_MGS_1R_IR32, "mgs1r_ir16": GMRES_MGS_1R_IR16,
           "cgs2_3r": GMRES_CGS2_3R, "two_synch": GMRES_TWO_SYNCH}
GMRES_OK, GMRES_ERR_ARG, GMRES_ERR_HIP, GMRES_ERR_NONFINITE, GMRES_ERR_WORKSPACE = 0, -1, -2, -3, -4
GMRES_ERR_TOO_LARGE = -5
GMRES_MAX_RESTART = 256
GMRES_NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTED = ["gmres_workspace_bytes", "gmres_create", "gmres_solve", "gmres_destroy",
            "gmres_status_string", "gmres_spmv", "gmres_last_cycle", "gmres_basis",
            "gmres_set_timing", "gmres_get_timing", "gmres_refresh_matrix", "gmres_get_format",
            "gmres_matrix_storage_bytes", "gmres_set_matrix_storage",
            "gmres_batch_workspace_bytes", "gmres_batch_create", "gmres_batch_destroy",
            "gmres_batch_set_stream", "gmres_batch_solve_async", "gmres_batch_solve",
            "gmres_batch_read_info", "gmres_batch_set_config", "gmres_batch_get_config",
            "gmres_batch_autotune", "gmres_batch_capture", "gmres_batch_replay",
            "gmres_solve_noalloc", "gmres_options_init", "gmres_workspace_bytes_ex",
            "gmres_create_ex", "gmres_batch_set_wait_limit", "gmres_batch_set_loads",
            "gmres_batch_get_loads", "gmres_batch_matrix_storage_bytes",
            "gmres_batch_set_matrix_storage", "gmres_batch_get_format"]
GMRES_BATCH_ORDER_NATURAL, GMRES_BATCH_ORDER_LARGEST_FIRST = 0, 1
GMRES_BATCH_LOADS_AUTO, GMRES_BATCH_LOADS_CACHED, GMRES_BATCH_LOADS_STREAMED = 0, 1, 2
BATCH_LOADS = {"auto": 0, "cached": 1, "streamed": 2}
GMRES_FORMAT_CSR, GMRES_FORMAT_SELL64, GMRES_FORMAT_SELL64_D16, GMRES_FORMAT_SELL64_DIAG = 0, 1, 2, 3
GMRES_KSTAT_STEP, GMRES_KSTAT_MAXPY, GMRES_KSTAT_SPMV, GMRES_KSTAT_COUNT = 0, 1, 2, 3
GMRES_OPT_FORMAT_AUTO, GMRES_OPT_FORMAT_CSR, GMRES_OPT_FORMAT_SELL64 = 0, 1, 2
GMRES_OPT_FORMAT_SELL64_D16, GMRES_OPT_FORMAT_SELL64_DIAG = 3, 4
OPT_FORMATS = {None: GMRES_OPT_FORMAT_AUTO, "auto": GMRES_OPT_FORMAT_AUTO,
               "csr": GMRES_OPT_FORMAT_CSR, "sell": GMRES_OPT_FORMAT_SELL64,
               "sell64": GMRES_OPT_FORMAT_SELL64, "sell_d16": GMRES_OPT_FORMAT_SELL64_D16,
               "sell64_d16": GMRES_OPT_FORMAT_SELL64_D16, "sell_diag": GMRES_OPT_FORMAT_SELL64_DIAG,
               "sell64_diag": GMRES_OPT_FORMAT_SELL64_DIAG}
FORMAT_NAMES = {GMRES_FORMAT_CSR: "csr", GMRES_FORMAT_SELL64: "sell64",
                GMRES_FORMAT_SELL64_D16: "sell64_d16", GMRES_FORMAT_SELL64_DIAG: "sell64_diag"}
GMRES_BATCH_WAIT_LIMIT = 1 << 23


class GmresOptions(ctypes.Structure):
    """gmres_options: zero fields take the library's choices."""
    _fields_ = [("format", ctypes.c_int32), ("rows_per_lane", ctypes.c_int32),
                ("csr_spmv_shape", ctypes.c_int32), ("split_spmv", ctypes.c_int32),
                ("pipeline_depth", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


def make_options(format=None, rows_per_lane: int = 0, csr_spmv_shape: int = 0,
                 split_spmv: bool = False, pipeline_depth: int = 0) -> GmresOptions:
    """A gmres_options from keyword values (format: None/"auto", "csr", "sell",
    "sell_d16" or "sell_diag")."""
    o = GmresOptions()
    o.format = OPT_FORMATS[format] if format in OPT_FORMATS else int(format)
    o.rows_per_lane = int(rows_per_lane)
    o.csr_spmv_shape = int(csr_spmv_shape)
    o.split_spmv = 1 if split_spmv else 0
    o.pipeline_depth = int(pipeline_depth)
    return o


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("cycles", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("breakdown", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("rel_res_true", ctypes.c_double),
                ("rel_res_est", ctypes.c_double), ("reductions", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class GmresKernelStat(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("bytes", ctypes.c_double), ("launches", ctypes.c_int64)]


class GmresBatchInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("cycles", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("status", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("rel_res_true", ctypes.c_double)]


class GmresBatchTrial(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("order", ctypes.c_int32), ("ms", ctypes.c_float), ("part_rows", ctypes.c_int64),
                ("streamed", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1809_05805_amd.build_native "
                           "(or __graft_entry__.build()); there is no fallback path")
    # This binding hands torch's device pointers to the library, so torch's
    # HIP runtime is loaded first and the library binds to that same one:
    # torch ships its own libamdhip64, and a library loaded before it would
    # bring in the system's copy, a second runtime that knows nothing of
    # torch's allocations (every pointer check then fails).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.gmres_workspace_bytes.restype = SZ
    lib.gmres_workspace_bytes.argtypes = [I64, I32, I32]
    lib.gmres_create.restype = ctypes.c_int
    lib.gmres_create.argtypes = [ctypes.POINTER(P), I64, I64, P, P, P, I32, I32, P, SZ, P]
    lib.gmres_solve.restype = ctypes.c_int
    lib.gmres_solve.argtypes = [P, P, P, D, I64, ctypes.POINTER(GmresInfo), P, P]
    lib.gmres_destroy.restype = ctypes.c_int
    lib.gmres_destroy.argtypes = [P]
    lib.gmres_status_string.restype = ctypes.c_char_p
    lib.gmres_status_string.argtypes = [ctypes.c_int]
    lib.gmres_spmv.restype = ctypes.c_int
    lib.gmres_spmv.argtypes = [P, P, P]
    lib.gmres_last_cycle.restype = ctypes.c_int
    lib.gmres_last_cycle.argtypes = [P, P, P, P, ctypes.POINTER(I32)]
    lib.gmres_basis.restype = ctypes.c_int
    lib.gmres_basis.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(I64)]
    lib.gmres_set_timing.restype = ctypes.c_int
    lib.gmres_set_timing.argtypes = [P, ctypes.c_int]
    lib.gmres_get_timing.restype = ctypes.c_int
    lib.gmres_get_timing.argtypes = [P, ctypes.POINTER(GmresKernelStat)]
    lib.gmres_refresh_matrix.restype = ctypes.c_int
    lib.gmres_refresh_matrix.argtypes = [P]
    lib.gmres_get_format.restype = ctypes.c_int
    lib.gmres_get_format.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I64)]
    lib.gmres_matrix_storage_bytes.restype = ctypes.c_int
    lib.gmres_matrix_storage_bytes.argtypes = [P, ctypes.POINTER(SZ)]
    lib.gmres_set_matrix_storage.restype = ctypes.c_int
    lib.gmres_set_matrix_storage.argtypes = [P, P, SZ]
    lib.gmres_batch_workspace_bytes.restype = SZ
    lib.gmres_batch_workspace_bytes.argtypes = [I32, P, I32, I32]
    lib.gmres_batch_create.restype = ctypes.c_int
    lib.gmres_batch_create.argtypes = [ctypes.POINTER(P), I32, P, I64, P, P, P, I32, I32, P, SZ, P]
    for name, args in (("gmres_batch_destroy", [P]), ("gmres_batch_set_stream", [P, P]),
                       ("gmres_batch_solve_async", [P, P, P, D, I64, P]),
                       ("gmres_batch_solve", [P, P, P, D, I64, P]),
                       ("gmres_batch_read_info", [P, P]),
                       ("gmres_batch_set_config", [P, I32, I32, I32, I64]),
                       ("gmres_batch_get_config", [P, ctypes.POINTER(I32), ctypes.POINTER(I32),
                                                   ctypes.POINTER(I32), ctypes.POINTER(I64),
                                                   ctypes.POINTER(I32)]),
                       ("gmres_batch_autotune", [P, P, P, D, I64, P, I32, ctypes.POINTER(I32)]),
                       ("gmres_batch_capture", [P, P, P, D, I64]),
                       ("gmres_batch_set_loads", [P, I32]),
                       ("gmres_batch_get_loads", [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
                       ("gmres_batch_matrix_storage_bytes", [P, ctypes.POINTER(ctypes.c_size_t)]),
                       ("gmres_batch_set_matrix_storage", [P, P, ctypes.c_size_t]),
                       ("gmres_batch_get_format", [P, ctypes.POINTER(I32), ctypes.POINTER(I64)]),
                       ("gmres_batch_replay", [P])):
        getattr(lib, name).restype = ctypes.c_int
        getattr(lib, name).argtypes = args
    lib.gmres_options_init.restype = None
    lib.gmres_options_init.argtypes = [ctypes.POINTER(GmresOptions)]
    lib.gmres_workspace_bytes_ex.restype = SZ
    lib.gmres_workspace_bytes_ex.argtypes = [I64, I32, I32, ctypes.POINTER(GmresOptions)]
    lib.gmres_create_ex.restype = ctypes.c_int
    lib.gmres_create_ex.argtypes = [ctypes.POINTER(P), I64, I64, P, P, P, I32, I32, P, SZ, P,
                                    ctypes.POINTER(GmresOptions)]
    lib.gmres_batch_set_wait_limit.restype = ctypes.c_int
    lib.gmres_batch_set_wait_limit.argtypes = [P, ctypes.c_uint32]
    lib.gmres_solve_noalloc.restype = ctypes.c_int
    lib.gmres_solve_noalloc.argtypes = [I64, I64, P, P, P, I32, I32, P, P, D, I64,
                                        ctypes.POINTER(GmresInfo), P, P]
    _lib = lib
    return lib


# ---------------------------------------------------------- C-named wrappers

def gmres_workspace_bytes(n: int, m: int, scheme: int) -> int:
    return int(load().gmres_workspace_bytes(n, m, scheme))


def gmres_workspace_bytes_ex(n: int, m: int, scheme: int, opt: GmresOptions | None) -> int:
    return int(load().gmres_workspace_bytes_ex(n, m, scheme, None if opt is None else ctypes.byref(opt)))


def gmres_options_init() -> GmresOptions:
    o = GmresOptions()
    load().gmres_options_init(ctypes.byref(o))
    return o


def gmres_create_ex(n, nnz, row_ptr_ptr, col_idx_ptr, vals_ptr, m, scheme, ws_ptr, ws_bytes,
                    stream_ptr, opt: GmresOptions | None) -> tuple[int, int | None]:
    ctx = ctypes.c_void_p()
    rc = load().gmres_create_ex(ctypes.byref(ctx), n, nnz, row_ptr_ptr, col_idx_ptr, vals_ptr, m,
                                scheme, ws_ptr, ws_bytes, stream_ptr,
                                None if opt is None else ctypes.byref(opt))
    return rc, (ctx.value if rc == GMRES_OK else None)


def gmres_batch_set_wait_limit(ctx, polls: int) -> int:
    return load().gmres_batch_set_wait_limit(ctx, polls)


def gmres_status_string(status: int) -> str:
    return load().gmres_status_string(status).decode()


def gmres_create(n, nnz, row_ptr_ptr, col_idx_ptr, vals_ptr, m, scheme, ws_ptr, ws_bytes,
                 stream_ptr) -> tuple[int, int | None]:
    ctx = ctypes.c_void_p()
    rc = load().gmres_create(ctypes.byref(ctx), n, nnz, row_ptr_ptr, col_idx_ptr, vals_ptr, m,
                             scheme, ws_ptr, ws_bytes, stream_ptr)
    return rc, (ctx.value if rc == GMRES_OK else None)


def gmres_solve(ctx, b_ptr, x_ptr, rtol, max_iters, hist: np.ndarray | None = None,
                orth: np.ndarray | None = None):
    info = GmresInfo()
    hp = None if hist is None else hist.ctypes.data_as(ctypes.c_void_p)
    op = None if orth is None else orth.ctypes.data_as(ctypes.c_void_p)
    rc = load().gmres_solve(ctx, b_ptr, x_ptr, float(rtol), int(max_iters), ctypes.byref(info), hp, op)
    return rc, info


def gmres_destroy(ctx) -> int:
    return load().gmres_destroy(ctx)


def gmres_spmv(ctx, x_ptr, y_ptr) -> int:
    return load().gmres_spmv(ctx, x_ptr, y_ptr)


def gmres_refresh_matrix(ctx) -> int:
    return load().gmres_refresh_matrix(ctx)


def gmres_matrix_storage_bytes(ctx):
    nb = ctypes.c_size_t()
    rc = load().gmres_matrix_storage_bytes(ctx, ctypes.byref(nb))
    return rc, nb.value


def gmres_set_matrix_storage(ctx, ptr, nbytes: int) -> int:
    return load().gmres_set_matrix_storage(ctx, ptr, nbytes)


def gmres_get_format(ctx):
    fmt, stored = ctypes.c_int32(), ctypes.c_int64()
    rc = load().gmres_get_format(ctx, ctypes.byref(fmt), ctypes.byref(stored))
    return rc, fmt.value, stored.value


def gmres_last_cycle(ctx, m: int):
    H = np.zeros((m, m + 1))
    T = np.zeros((m + 2, m + 2))
    g = np.zeros(m + 2)
    j = ctypes.c_int32(0)
    rc = load().gmres_last_cycle(ctx, H.ctypes.data_as(ctypes.c_void_p),
                                 T.ctypes.data_as(ctypes.c_void_p),
                                 g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(j))
    return rc, H.T, T.T, g, j.value     # column-major buffers read as their transposes


def gmres_basis(ctx):
    V = ctypes.c_void_p()
    ld = ctypes.c_int64()
    rc = load().gmres_basis(ctx, ctypes.byref(V), ctypes.byref(ld))
    return rc, V.value, ld.value


def gmres_set_timing(ctx, enable: bool) -> int:
    return load().gmres_set_timing(ctx, 1 if enable else 0)


def gmres_get_timing(ctx):
    arr = (GmresKernelStat * GMRES_KSTAT_COUNT)()
    rc = load().gmres_get_timing(ctx, arr)
    return rc, [{"ms": a.ms, "bytes": a.bytes, "launches": a.launches} for a in arr]


def gmres_batch_workspace_bytes(row_off: np.ndarray, m: int, scheme: int) -> int:
    ro = np.ascontiguousarray(row_off, dtype=np.int64)
    return int(load().gmres_batch_workspace_bytes(len(ro) - 1, ro.ctypes.data, m, scheme))


def gmres_batch_create(row_off: np.ndarray, nnz, row_ptr_ptr, col_idx_ptr, vals_ptr, m, scheme,
                       ws_ptr, ws_bytes, stream_ptr) -> tuple[int, int | None]:
    ro = np.ascontiguousarray(row_off, dtype=np.int64)
    ctx = ctypes.c_void_p()
    rc = load().gmres_batch_create(ctypes.byref(ctx), len(ro) - 1, ro.ctypes.data, nnz, row_ptr_ptr,
                                   col_idx_ptr, vals_ptr, m, scheme, ws_ptr, ws_bytes, stream_ptr)
    return rc, (ctx.value if rc == GMRES_OK else None)


def gmres_batch_destroy(ctx) -> int:
    return load().gmres_batch_destroy(ctx)


def gmres_batch_set_stream(ctx, stream_ptr) -> int:
    return load().gmres_batch_set_stream(ctx, stream_ptr)


def gmres_batch_solve_async(ctx, b_ptr, x_ptr, rtol, max_iters, info_ptr=None) -> int:
    return load().gmres_batch_solve_async(ctx, b_ptr, x_ptr, float(rtol), int(max_iters), info_ptr)


def gmres_batch_solve(ctx, b_ptr, x_ptr, rtol, max_iters, nsys: int):
    info = (GmresBatchInfo * nsys)()
    rc = load().gmres_batch_solve(ctx, b_ptr, x_ptr, float(rtol), int(max_iters), info)
    return rc, info


def gmres_batch_read_info(ctx, nsys: int):
    info = (GmresBatchInfo * nsys)()
    rc = load().gmres_batch_read_info(ctx, info)
    return rc, info


def gmres_batch_set_config(ctx, block_size: int, grid: int, order: int, part_rows: int) -> int:
    return load().gmres_batch_set_config(ctx, block_size, grid, order, part_rows)


def gmres_batch_get_config(ctx):
    a, b, c, mp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    pr = ctypes.c_int64()
    rc = load().gmres_batch_get_config(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                       ctypes.byref(pr), ctypes.byref(mp))
    return rc, a.value, b.value, c.value, pr.value, mp.value


def gmres_batch_autotune(ctx, b_ptr, x_ptr, rtol, max_iters, max_trials: int = 32):
    trials = (GmresBatchTrial * max(max_trials, 1))()
    nt = ctypes.c_int32()
    rc = load().gmres_batch_autotune(ctx, b_ptr, x_ptr, float(rtol), int(max_iters), trials,
                                     max_trials, ctypes.byref(nt))
    return rc, [(t.block_size, t.grid, t.order, t.ms, t.part_rows, t.streamed)
                for t in trials[: nt.value]]


def gmres_batch_set_loads(ctx, mode: int) -> int:
    return load().gmres_batch_set_loads(ctx, mode)


def gmres_batch_get_loads(ctx):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    rc = load().gmres_batch_get_loads(ctx, ctypes.byref(a), ctypes.byref(b))
    return rc, a.value, b.value


def gmres_batch_matrix_storage_bytes(ctx):
    nb = ctypes.c_size_t(0)
    rc = load().gmres_batch_matrix_storage_bytes(ctx, ctypes.byref(nb))
    return rc, nb.value


def gmres_batch_set_matrix_storage(ctx, ptr, nbytes: int) -> int:
    return load().gmres_batch_set_matrix_storage(ctx, ptr, nbytes)


def gmres_batch_get_format(ctx):
    fmt, stored = ctypes.c_int32(), ctypes.c_int64()
    rc = load().gmres_batch_get_format(ctx, ctypes.byref(fmt), ctypes.byref(stored))
    return rc, fmt.value, stored.value


def gmres_batch_capture(ctx, b_ptr, x_ptr, rtol, max_iters) -> int:
    return load().gmres_batch_capture(ctx, b_ptr, x_ptr, float(rtol), int(max_iters))


def gmres_batch_replay(ctx) -> int:
    return load().gmres_batch_replay(ctx)


# ----------------------------------------------------------- torch front end

def gmres_solve_noalloc(n, nnz, row_ptr_ptr, col_idx_ptr, vals_ptr, m, scheme, b_ptr, x_ptr,
                        rtol, max_iters, hist: np.ndarray | None = None, stream_ptr=None):
    """One whole solve in the library's fixed device scratch (no allocation)."""
    lib = load()
    info = GmresInfo()
    hp = hist.ctypes.data_as(ctypes.c_void_p) if hist is not None else None
    rc = lib.gmres_solve_noalloc(n, nnz, row_ptr_ptr, col_idx_ptr, vals_ptr, m, scheme, b_ptr,
                                 x_ptr, float(rtol), int(max_iters), ctypes.byref(info), hp,
                                 stream_ptr)
    return rc, info


class GmresError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"{what}: {gmres_status_string(rc)} ({rc})")
        self.rc = rc


@dataclass
class SolveResult:
    status: int
    iters: int
    cycles: int
    converged: bool
    breakdown: bool
    rel_res_true: float
    rel_res_est: float
    reductions: int
    hist: np.ndarray | None
    orth: np.ndarray | None = None


class GmresSolver:
    """A context bound to CSR tensors on a GPU and a workspace it allocates with torch.

    Keyword options go to gmres_create_ex (see make_options): format (None,
    "csr" or "sell"), rows_per_lane, csr_spmv_shape, split_spmv, pipeline_depth.
    """

    def __init__(self, row_ptr, col_idx, vals, m: int, scheme: str = "mgs1r", stream=None,
                 **options):
        import torch

        if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32 or vals.dtype != torch.float64:
            raise TypeError("CSR arrays must be int32, int32, float64")
        for t in (row_ptr, col_idx, vals):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous device tensors")
        self.n = int(row_ptr.numel() - 1)
        self.nnz = int(col_idx.numel())
        self.m = int(m)
        self.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        self.device = row_ptr.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._keep = (row_ptr, col_idx, vals)
        self.options = make_options(**options) if options else None
        nbytes = gmres_workspace_bytes_ex(self.n, self.m, self.scheme, self.options)
        if nbytes == 0:
            raise GmresError(GMRES_ERR_ARG, "gmres_workspace_bytes_ex")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = self.ws.data_ptr() + off
        self.ws_bytes = nbytes
        rc, ctx = gmres_create_ex(self.n, self.nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                  vals.data_ptr() if self.nnz else None, self.m, self.scheme,
                                  self.ws_ptr, nbytes, self.stream.cuda_stream, self.options)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_create_ex")
        self.ctx = ctx
        # the sliced copy of A, when the library plans one, lives in a tensor of ours
        rc, mbytes = gmres_matrix_storage_bytes(ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_matrix_storage_bytes")
        self.mat = None
        if mbytes:
            self.mat = torch.empty(mbytes + 256, dtype=torch.uint8, device=self.device)
            moff = (-self.mat.data_ptr()) % 256
            rc = gmres_set_matrix_storage(ctx, self.mat.data_ptr() + moff, mbytes)
            if rc != GMRES_OK:
                raise GmresError(rc, "gmres_set_matrix_storage")

    def close(self):
        if getattr(self, "ctx", None):
            gmres_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x, rtol: float, max_iters: int, hist: bool = False,
              check: bool = True, orth: bool = False) -> SolveResult:
        import torch

        for t in (b, x):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != self.n:
                raise ValueError("b and x must be contiguous float64 device tensors of length n")
        h = np.full(max(int(max_iters), 1), np.nan) if hist else None
        o = np.full(max(int(max_iters), 1), np.nan) if orth else None
        rc, info = gmres_solve(self.ctx, b.data_ptr(), x.data_ptr(), rtol, max_iters, h, o)
        if check and rc not in (GMRES_OK, GMRES_ERR_NONFINITE):
            raise GmresError(rc, "gmres_solve")
        return SolveResult(rc, info.iters, info.cycles, bool(info.converged), bool(info.breakdown),
                           info.rel_res_true, info.rel_res_est, info.reductions,
                           None if h is None else h[: info.iters].copy(),
                           None if o is None else o[: info.iters].copy())

    def spmv(self, x, y):
        rc = gmres_spmv(self.ctx, x.data_ptr(), y.data_ptr())
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_spmv")

    def refresh_matrix(self):
        """Re-read A's values after they were changed in place (same structure)."""
        rc = gmres_refresh_matrix(self.ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_refresh_matrix")

    def format(self):
        """("csr" | "sell64" | "sell64_d16" | "sell64_diag", stored entries) of the context's SpMV."""
        rc, fmt, stored = gmres_get_format(self.ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_get_format")
        return FORMAT_NAMES[fmt], stored

    def last_cycle(self):
        rc, H, T, g, j = gmres_last_cycle(self.ctx, self.m)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_last_cycle")
        return H, T, g, j

    def set_timing(self, enable: bool):
        rc = gmres_set_timing(self.ctx, enable)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_set_timing")

    def timing(self) -> dict:
        rc, st = gmres_get_timing(self.ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_get_timing")
        return {"step": st[GMRES_KSTAT_STEP], "maxpy": st[GMRES_KSTAT_MAXPY],
                "spmv": st[GMRES_KSTAT_SPMV]}

    def basis(self):
        """V (n x (m+2)) as a view into the workspace tensor."""
        import torch

        rc, vptr, ld = gmres_basis(self.ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_basis")
        off = vptr - self.ws.data_ptr()
        cols = self.m + 2
        flat = self.ws[off: off + ld * cols * 8].view(torch.float64)
        return flat.view(cols, ld)[:, : self.n].t()


def batch_info_arrays(info) -> dict:
    """Per-system fields of a gmres_batch_info array as numpy arrays."""
    return {k: np.array([getattr(o, k) for o in info]) for k, _ in GmresBatchInfo._fields_}


class BatchSolver:
    """A batch context over a block-diagonal CSR matrix on a GPU, workspace allocated with torch.

    row_off: host int64[nsys+1] system boundaries. scheme "mgs1r" or "mgs1r_ir32".
    format: None or "auto" (the copy of A by diagonals when the library plans
    one, in a torch buffer), or "csr" (always the CSR arrays).
    """

    def __init__(self, row_off, row_ptr, col_idx, vals, m: int, scheme: str = "mgs1r", stream=None,
                 format: str | None = None):
        import torch

        if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32 or vals.dtype != torch.float64:
            raise TypeError("CSR arrays must be int32, int32, float64")
        for t in (row_ptr, col_idx, vals):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous device tensors")
        self.row_off = np.ascontiguousarray(row_off, dtype=np.int64)
        self.nsys = len(self.row_off) - 1
        self.n = int(row_ptr.numel() - 1)
        self.m = int(m)
        self.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        self.device = row_ptr.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._keep = (row_ptr, col_idx, vals)
        nbytes = gmres_batch_workspace_bytes(self.row_off, self.m, self.scheme)
        if nbytes == 0:
            raise GmresError(GMRES_ERR_ARG, "gmres_batch_workspace_bytes")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        self.ws_bytes = nbytes
        nnz = int(col_idx.numel())
        rc, ctx = gmres_batch_create(self.row_off, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
                                     vals.data_ptr() if nnz else None, self.m, self.scheme,
                                     self.ws_ptr, nbytes, self.stream.cuda_stream)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_create")
        self.ctx = ctx
        self.storage = None
        if format not in (None, "auto", "csr"):
            raise ValueError(format)
        rc, sbytes = gmres_batch_matrix_storage_bytes(ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_matrix_storage_bytes")
        if sbytes and format != "csr":
            self.storage = torch.empty(sbytes + 256, dtype=torch.uint8, device=self.device)
            sp = self.storage.data_ptr() + (-self.storage.data_ptr()) % 256
            rc = gmres_batch_set_matrix_storage(ctx, sp, sbytes)
            if rc != GMRES_OK:
                raise GmresError(rc, "gmres_batch_set_matrix_storage")

    def format(self):
        """("csr" | "sell64_diag", stored entries) of the batched SpMV."""
        rc, fmt, stored = gmres_batch_get_format(self.ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_get_format")
        return FORMAT_NAMES[fmt], stored

    def close(self):
        if getattr(self, "ctx", None):
            gmres_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, b, x):
        import torch

        for t in (b, x):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != self.n:
                raise ValueError("b and x must be contiguous float64 device tensors of length n")

    def solve(self, b, x, rtol: float, max_iters: int, check: bool = True):
        """Solve every system; returns (status, dict of per-system numpy arrays)."""
        self._check(b, x)
        rc, info = gmres_batch_solve(self.ctx, b.data_ptr(), x.data_ptr(), rtol, max_iters, self.nsys)
        if check and rc not in (GMRES_OK, GMRES_ERR_NONFINITE):
            raise GmresError(rc, "gmres_batch_solve")
        return rc, batch_info_arrays(info)

    def solve_async(self, b, x, rtol: float, max_iters: int, info=None):
        self._check(b, x)
        rc = gmres_batch_solve_async(self.ctx, b.data_ptr(), x.data_ptr(), rtol, max_iters,
                                     None if info is None else info.data_ptr())
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_solve_async")

    def read_info(self) -> dict:
        rc, info = gmres_batch_read_info(self.ctx, self.nsys)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_read_info")
        return batch_info_arrays(info)

    def set_config(self, block_size: int = 256, grid: int = 0,
                   order: int = GMRES_BATCH_ORDER_LARGEST_FIRST, part_rows: int = 8192):
        rc = gmres_batch_set_config(self.ctx, block_size, grid, order, part_rows)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_set_config")

    def set_wait_limit(self, polls: int):
        """Polls a part makes at a team barrier before its system gives up."""
        rc = gmres_batch_set_wait_limit(self.ctx, polls)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_set_wait_limit")

    def set_loads(self, mode: str):
        """How basis columns are loaded: "auto", "cached" or "streamed"."""
        rc = gmres_batch_set_loads(self.ctx, BATCH_LOADS[mode])
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_set_loads")

    def config(self):
        rc, bs, grid, order, pr, mp = gmres_batch_get_config(self.ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_get_config")
        rc, mode, streamed = gmres_batch_get_loads(self.ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_get_loads")
        names = {v: k for k, v in BATCH_LOADS.items()}
        return {"block_size": bs, "grid": grid, "order": order, "part_rows": pr, "max_parts": mp,
                "loads": names[mode], "streamed": bool(streamed)}

    def autotune(self, b, x, rtol: float, max_iters: int):
        self._check(b, x)
        rc, trials = gmres_batch_autotune(self.ctx, b.data_ptr(), x.data_ptr(), rtol, max_iters)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_autotune")
        return trials

    def capture(self, b, x, rtol: float, max_iters: int):
        self._check(b, x)
        rc = gmres_batch_capture(self.ctx, b.data_ptr(), x.data_ptr(), rtol, max_iters)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_capture")

    def replay(self):
        rc = gmres_batch_replay(self.ctx)
        if rc != GMRES_OK:
            raise GmresError(rc, "gmres_batch_replay")
