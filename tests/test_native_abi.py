"""The C-ABI library builds, loads without a GPU and exports what include/gmres.h declares.

No compute call is made here: only the pure host functions (workspace sizing,
status strings) run.
"""

import ctypes
import os
import re

import pytest

from paper_1809_05805_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gmres.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmres_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(native.LIB_PATH):
        from paper_1809_05805_amd import build_native
        build_native.build()
    return native.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert set(names) == set(native.EXPORTED)
    for name in names:
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr), name


def declared_constants():
    """Every GMRES_* enumerator of include/gmres.h with its value."""
    src = open(os.path.join(ROOT, "include", "gmres.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for body in re.findall(r"enum\s*\w*\s*\{(.*?)\}", src, flags=re.S):
        for name, val in re.findall(r"\b(GMRES_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            out[name] = int(val)
    return out


def test_binding_constants_match_header():
    """The binding's copies of the header's enumerators (formats, options,
    schemes, statuses, batch load forms) carry the header's values."""
    consts = declared_constants()
    assert "GMRES_FORMAT_SELL64_DIAG" in consts and "GMRES_OPT_FORMAT_SELL64_DIAG" in consts
    checked = 0
    for name, val in consts.items():
        if hasattr(native, name):
            assert getattr(native, name) == val, name
            checked += 1
    assert checked >= 10
    for prefix in ("GMRES_FORMAT_", "GMRES_OPT_FORMAT_"):
        for name in consts:
            if name.startswith(prefix):
                assert hasattr(native, name), name


def test_workspace_sizing(lib):
    assert native.gmres_workspace_bytes(0, 30, 1) == 0
    assert native.gmres_workspace_bytes(100, 0, 1) == 0
    assert native.gmres_workspace_bytes(100, native.GMRES_MAX_RESTART + 1, 1) == 0
    # the FP32-basis scheme: a float32 basis and SpMV output plus a float64 residual
    f64 = native.gmres_workspace_bytes(2_097_152, 50, 1)
    f32 = native.gmres_workspace_bytes(2_097_152, 50, native.GMRES_MGS_1R_IR32)
    assert 2_097_152 * 53 * 4 + 2_097_152 * 8 <= f32 < 0.6 * f64
    # the bfloat16 experiment: a 2-byte basis and SpMV output plus the float64 residual
    f16 = native.gmres_workspace_bytes(2_097_152, 50, native.GMRES_MGS_1R_IR16)
    assert 2_097_152 * 53 * 2 + 2_097_152 * 8 <= f16 < 0.6 * f32
    assert native.gmres_workspace_bytes(100, 30, 7) == 0
    small = native.gmres_workspace_bytes(4096, 30, 1)
    # the basis alone: n x (m+2) doubles
    assert small >= 4096 * 32 * 8
    assert native.gmres_workspace_bytes(2 * 4096, 30, 1) > small
    assert native.gmres_workspace_bytes(4096, 60, 1) > small
    big = native.gmres_workspace_bytes(2_097_152, 50, 1)
    assert 2_097_152 * 52 * 8 <= big <= 2_097_152 * 52 * 8 * 1.1
    assert native.gmres_workspace_bytes(4096, 30, 0) == native.gmres_workspace_bytes(4096, 30, 2)


def test_status_strings(lib):
    assert native.gmres_status_string(0) == "ok"
    for rc in (-1, -2, -3, -4):
        assert native.gmres_status_string(rc) not in ("ok", "unknown status")
    assert native.gmres_status_string(7) == "unknown status"


def test_header_constants_match_binding():
    src = open(os.path.join(ROOT, "include", "gmres.h")).read()
    assert int(re.search(r"GMRES_MAX_RESTART (\d+)", src).group(1)) == native.GMRES_MAX_RESTART
    for name, val in (("GMRES_MGS", 0), ("GMRES_MGS_1R", 1), ("GMRES_CGS2", 2), ("GMRES_MGS_1R_IR32", 3),
                      ("GMRES_MGS_1R_IR16", 4), ("GMRES_CGS2_3R", 5), ("GMRES_TWO_SYNCH", 6),
                      ("GMRES_ERR_ARG", -1), ("GMRES_ERR_HIP", -2), ("GMRES_ERR_NONFINITE", -3),
                      ("GMRES_ERR_WORKSPACE", -4)):
        assert re.search(rf"{name} = {val}\b", src), name


def test_batch_workspace_sizing(lib):
    import numpy as np

    ro = np.array([0, 1000, 1100, 5196], dtype=np.int64)
    m = 30
    f64 = native.gmres_batch_workspace_bytes(ro, m, native.GMRES_MGS_1R)
    f32 = native.gmres_batch_workspace_bytes(ro, m, native.GMRES_MGS_1R_IR32)
    # bases: (m+1) columns of n_i rounded up to 64
    ld = [1024, 128, 4096]
    basis = sum(ld) * (m + 1)
    # one slot per possible part of a team: ceil(n_i / 256) parts, at most 16
    slots = 4 + 1 + 16
    small = 2 * (m + 1) * m + 2 * (m + 2) ** 2 + 7 * (m + 2)
    per_slot = 8 * small + 8 * 4 * (m + 2) + 16 + 128      # small arrays, partials, ticket, state
    assert f64 >= 8 * basis + slots * (8 * small + 8 * 4 * (m + 2)) + 8 * 5196 * 2
    assert f64 <= 8 * basis + slots * per_slot + 8 * 5196 * 2 + 3 * 64 + 14 * 256
    assert f32 >= 4 * basis + slots * (8 * small) + 4 * 5196 + 2 * 8 * 5196
    assert f32 < f64
    # refusals: empty systems, a bad first offset, the schemes with no batched form, m out of range
    assert native.gmres_batch_workspace_bytes(np.array([0, 10, 10]), m, 1) == 0
    assert native.gmres_batch_workspace_bytes(np.array([1, 10]), m, 1) == 0
    assert native.gmres_batch_workspace_bytes(ro, m, native.GMRES_MGS) == 0
    assert native.gmres_batch_workspace_bytes(ro, m, native.GMRES_CGS2) == 0
    assert native.gmres_batch_workspace_bytes(ro, 0, 1) == 0
    assert native.gmres_batch_workspace_bytes(ro, native.GMRES_MAX_RESTART + 1, 1) == 0
    assert native.gmres_batch_workspace_bytes(np.array([0, 2**28]), m, 1) == 0
    assert native.gmres_batch_workspace_bytes(np.array([0, 2**28 - 1]), m, 1) > 0


def test_batch_info_layout():
    assert ctypes.sizeof(native.GmresBatchInfo) == 32
    assert native.GmresBatchInfo.rel_res_true.offset == 24
    src = open(os.path.join(ROOT, "include", "gmres.h")).read()
    for name, val in (("GMRES_BATCH_ORDER_NATURAL", 0), ("GMRES_BATCH_ORDER_LARGEST_FIRST", 1)):
        assert re.search(rf"{name} = {val}\b", src), name


def test_options_sizing_and_refusals(lib):
    """gmres_options: zeros are the defaults, rows_per_lane changes the tiling
    (and so the reduction scratch in the workspace), out-of-range fields and a
    pipeline depth on a non-lagged scheme are refused."""
    n, m = 2_097_152, 50
    base = native.gmres_workspace_bytes(n, m, native.GMRES_MGS_1R)
    assert native.gmres_workspace_bytes_ex(n, m, native.GMRES_MGS_1R, None) == base
    assert native.gmres_workspace_bytes_ex(n, m, native.GMRES_MGS_1R, native.gmres_options_init()) == base
    assert ctypes.sizeof(native.GmresOptions) == 32
    o = native.gmres_options_init()
    assert all(getattr(o, f) == 0 for f in ("format", "rows_per_lane", "csr_spmv_shape",
                                              "split_spmv", "pipeline_depth"))
    # one row per lane: 8x the tiles of the default 8 rows per lane at 128^3
    one = native.gmres_workspace_bytes_ex(n, m, native.GMRES_MGS_1R, native.make_options(rows_per_lane=1))
    assert one > base
    ok = [dict(format="csr"), dict(format="sell"), dict(format="sell_d16"), dict(format="sell_diag"),
          dict(rows_per_lane=2), dict(csr_spmv_shape=804),
          dict(split_spmv=True), dict(pipeline_depth=2), dict(pipeline_depth=1)]
    for kw in ok:
        assert native.gmres_workspace_bytes_ex(4096, 30, native.GMRES_MGS_1R, native.make_options(**kw)) > 0, kw
    bad = [dict(format=5), dict(format=-1), dict(rows_per_lane=3), dict(rows_per_lane=16), dict(csr_spmv_shape=107),
           dict(pipeline_depth=-1), dict(pipeline_depth=native.GMRES_MAX_RESTART + 1)]
    for kw in bad:
        assert native.gmres_workspace_bytes_ex(4096, 30, native.GMRES_MGS_1R, native.make_options(**kw)) == 0, kw
    o = native.make_options(split_spmv=True)
    o.split_spmv = 2
    assert native.gmres_workspace_bytes_ex(4096, 30, native.GMRES_MGS_1R, o) == 0
    o = native.gmres_options_init()
    o.reserved[1] = 1
    assert native.gmres_workspace_bytes_ex(4096, 30, native.GMRES_MGS_1R, o) == 0
    # a pipeline depth only for the lagged schemes
    for scheme in (native.GMRES_MGS_1R, native.GMRES_CGS2, native.GMRES_MGS_1R_IR32, native.GMRES_MGS_1R_IR16):
        assert native.gmres_workspace_bytes_ex(4096, 30, scheme, native.make_options(pipeline_depth=3)) > 0
    for scheme in (native.GMRES_MGS, native.GMRES_CGS2_3R, native.GMRES_TWO_SYNCH):
        assert native.gmres_workspace_bytes_ex(4096, 30, scheme, native.make_options(pipeline_depth=2)) == 0
        assert native.gmres_workspace_bytes_ex(4096, 30, scheme, native.make_options(pipeline_depth=1)) > 0


def test_no_environment_knobs_in_the_library():
    """Every launch and format choice goes through the C ABI (gmres_options,
    gmres_batch_set_wait_limit): the library reads no environment variables."""
    csrc = os.path.join(ROOT, "paper_1809_05805_amd", "csrc")
    for name in os.listdir(csrc):
        src = open(os.path.join(csrc, name)).read()
        assert "getenv" not in src, name


def test_probe_library_exports_its_header():
    from paper_1809_05805_amd import build_native

    if not os.path.exists(build_native.PROBE_LIB):
        build_native.build()
    src = open(os.path.join(ROOT, "include", "gmres_probe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(gmres_[a-z_]+)\s*\(", src)))
    assert names == ["gmres_probe_bandwidth"]
    lib = ctypes.CDLL(build_native.PROBE_LIB)
    for name in names:
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr), name
    # argument checks run on the host before any device call
    ms = ctypes.c_float()
    f = lib.gmres_probe_bandwidth
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]
    assert f(9, 16, 16, 1024, 1, 1, None, ctypes.byref(ms)) == -1
    assert f(0, 16, 16, 1000, 1, 1, None, ctypes.byref(ms)) == -1
    assert f(0, None, 16, 1024, 1, 1, None, ctypes.byref(ms)) == -1


def test_column_stride_padding(lib):
    """Basis columns are n rounded up to 64 apart, plus 17 x 64 = 1088 elements
    when that is a multiple of 1024 (a large power-of-two stride). The float64
    one-reduce workspace holds m + 2 basis columns and w at that stride, so
    between n = 4032 and n = 4096 it grows by (m + 3) x (64 + 1088) x 8 bytes,
    and between n = 4096 and n = 5120 (both padded) by (m + 3) x 1024 x 8, up
    to the 256-byte rounding of each part."""
    m = 16
    f = lambda n: native.gmres_workspace_bytes(n, m, native.GMRES_MGS_1R)
    cols = m + 3
    slack = 16 * 256
    assert abs((f(4032) - f(3968)) - cols * 64 * 8) <= slack
    assert abs((f(4096) - f(4032)) - cols * (64 + 1088) * 8) <= slack
    assert abs((f(5120) - f(4096)) - cols * 1024 * 8) <= slack
