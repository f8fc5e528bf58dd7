"""The library's SpMV format: which one it picks, and its sliced copy of A.

A context keeps a sliced-ELL copy of A (64 rows per slice, each row padded to
its slice's longest row) when that costs at most a quarter more entries, and
otherwise reads the CSR arrays. The copy's column indices are 16-bit deltas
from a base per slice column when every slice column's col - row values span
at most 65535, else int32. These tests check the choice on regular,
wide-banded and irregular matrices, the stored-entry count against a count
made here from the row lengths, the storage layout, and that
gmres_refresh_matrix picks up new values (the solve then matches the oracle on
the changed matrix) and refuses a structure that no longer fits the copy.
"""

import numpy as np
import pytest

from paper_1809_05805_amd import problems as P
from tests.gpu_util import gpu_run, log, oracle_run, rel

pytestmark = pytest.mark.gpu


def padded_entries(p):
    """Entries of the 64-row sliced layout: per slice 64 x max(1, longest row)."""
    lens = np.diff(p.row_ptr)
    ns = (p.n + 63) // 64
    pad = np.zeros(ns * 64, dtype=np.int64)
    pad[: p.n] = lens
    return int(64 * np.maximum(pad.reshape(ns, 64).max(axis=1), 1).sum())


def solver(p, m=10, scheme="mgs1r", fmt=None):
    import torch

    from paper_1809_05805_amd.native import GmresSolver

    rp, ci, va = (torch.from_numpy(np.array(a)).cuda() for a in (p.row_ptr, p.col_idx, p.vals))
    s = GmresSolver(rp, ci, va, m, scheme, **({"format": fmt} if fmt else {}))
    return s, (rp, ci, va)


def wide_band(n=140_000, far=70_000):
    """Tridiagonal plus couplings `far` rows away: in the slice where rows start
    to have the far lower coupling, entry 0 of a row is col - row = -1 or
    -far, a spread beyond 16 bits."""
    import scipy.sparse as sp

    A = sp.diags([np.full(n - far, -0.1), np.full(n - 1, -1.0), np.full(n, 4.0), np.full(n - 1, -1.0),
                  np.full(n - far, -0.1)], [-far, -1, 0, 1, far], format="csr")
    rp, ci, va = P.csr_from_scipy(A)
    return P.Problem("wide_band", rp, ci, va, np.ones(n), np.zeros(n), None, 10, 0.0)


def test_format_choice():
    import scipy.sparse as sp

    cases = {
        "convdiff2d": (P.make_config("convdiff2d"), "sell64_d16"),              # 5-point rows
        "convdiff3d_24": (P.make_config("convdiff3d", N=24), "sell64_d16"),     # 7-point rows
        "stencil27_12": (P.make_config("stencil27", N=12), "sell64_d16"),     # 27-point rows
        "wide_band": (wide_band(), "sell64"),                       # col - row spread > 65535
        "dense50": (P.random_dense(50, seed=3), "csr"),             # one slice, 14 padding rows
    }
    A = sp.csr_matrix(sp.random(3000, 3000, density=0.003, random_state=4) + sp.identity(3000))
    rp, ci, va = P.csr_from_scipy(A)
    cases["irregular"] = (P.Problem("irregular", rp, ci, va, np.ones(3000), np.zeros(3000), None,
                                    10, 0.0), "csr")
    for name, (p, want) in cases.items():
        s, _ = solver(p)
        fmt, stored = s.format()
        log(f"format {name}: {fmt} stored={stored} nnz={p.nnz} padded={padded_entries(p)}")
        assert fmt == want, name
        assert stored == (padded_entries(p) if fmt.startswith("sell") else p.nnz)
        s.close()
    # forced: int32 indices on a stencil; deltas where they do not fit fall back to int32
    s, _ = solver(cases["convdiff2d"][0], fmt="sell")
    assert s.format()[0] == "sell64"
    s, _ = solver(cases["wide_band"][0], fmt="sell_d16")
    assert s.format()[0] == "sell64"
    s, _ = solver(cases["dense50"][0], fmt="sell_d16")
    assert s.format()[0] == "sell64_d16"


def test_wide_band_solve_matches_oracle():
    """The int32 copy chosen for the wide band gives the oracle's cycle."""
    p = wide_band(n=70_000 + 3000, far=70_000)
    g = gpu_run(p, "mgs1r", m=10, rtol=0.0, max_iters=10)
    assert g["solver"].format()[0] == "sell64"
    o = oracle_run(p, "mgs1r", m=10, rtol=0.0, max_iters=10)
    assert rel(g["x"], o.x) <= 1e-10


@pytest.mark.parametrize("fmt", ["csr", "sell", "sell_d16"])
def test_refresh_matrix(fmt):
    """Scale two rows' values in place: after refresh the solve is the one on the new matrix."""
    import torch

    p = P.make_config("convdiff2d", N=40)
    s, (rp, ci, va) = solver(p, m=20, fmt=fmt)
    log(f"refresh {fmt}")
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    s.solve(b, x, 0.0, 20)
    vals2 = p.vals.copy()
    for r in (3, p.n - 2):
        vals2[p.row_ptr[r]:p.row_ptr[r + 1]] *= 3.0
    va.copy_(torch.from_numpy(vals2))
    s.refresh_matrix()
    x.zero_()
    r = s.solve(b, x, 0.0, 20)
    q = P.Problem("scaled", p.row_ptr, p.col_idx, vals2, p.b, p.x0, None, 20, 0.0)
    o = oracle_run(q, "mgs1r", m=20, rtol=0.0, max_iters=20, dump=False)
    assert r.iters == o.iters == 20
    assert rel(x.cpu().numpy(), o.x) <= 1e-10


@pytest.mark.parametrize("fmt", ["sell", "sell_d16"])
def test_refresh_refuses_bad_structure(fmt):
    import torch

    from paper_1809_05805_amd import native
    from paper_1809_05805_amd.native import GmresError

    p = P.make_config("convdiff2d", N=40)
    s, (rp, ci, va) = solver(p, fmt=fmt)
    log("refresh bad structure")
    bad = p.col_idx.copy()
    bad[9] = p.n
    ci.copy_(torch.from_numpy(bad))
    with pytest.raises(GmresError) as e:
        s.refresh_matrix()
    assert e.value.rc == native.GMRES_ERR_ARG
    # the context refuses to run on the refused matrix ...
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    with pytest.raises(GmresError) as e:
        s.solve(b, x, 1e-8, 10)
    assert e.value.rc == native.GMRES_ERR_ARG
    # ... until the structure is restored and refreshed
    ci.copy_(torch.from_numpy(p.col_idx))
    s.refresh_matrix()
    r = s.solve(b, x, 0.0, 10)
    assert r.iters == 10
    s.close()


@pytest.mark.parametrize("fmt", ["sell", "sell_d16"])
@pytest.mark.parametrize("scheme", ["mgs1r", "cgs2"])
def test_sell_small_and_one_row(scheme, fmt):
    """The sliced copy on sizes that leave most of the one slice as padding."""
    import scipy.sparse as sp

    name = {"sell": "sell64", "sell_d16": "sell64_d16"}[fmt]
    rp, ci, va = P.csr_from_scipy(sp.csr_matrix(np.array([[3.0]])))
    p = P.Problem("one", rp, ci, va, np.array([6.0]), np.zeros(1), np.array([2.0]), m=1, rtol=1e-12)
    g = gpu_run(p, scheme, fmt=fmt)
    assert g["solver"].format()[0] == name
    assert g["res"].converged and abs(g["x"][0] - 2.0) <= 1e-15
    p = P.make_config("convdiff2d", N=5)  # n = 25
    g = gpu_run(p, scheme, m=10, rtol=0.0, max_iters=10, fmt=fmt)
    assert g["solver"].format()[0] == name
    o = oracle_run(p, scheme, m=10, rtol=0.0, max_iters=10)
    assert g["res"].iters == o.iters
    assert rel(g["x"], o.x) <= 1e-10


def test_storage_calls():
    """The raw entry points: the planned size, CSR until storage is given, and refusals."""
    import torch

    from paper_1809_05805_amd import native

    p = P.make_config("convdiff2d", N=33)  # n = 1089: 18 slices, the last one ragged
    rp, ci, va = (torch.from_numpy(a).cuda() for a in (p.row_ptr, p.col_idx, p.vals))
    m = 10
    need = native.gmres_workspace_bytes(p.n, m, native.GMRES_MGS_1R)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    wp = ws.data_ptr() + (-ws.data_ptr()) % 256
    stream = torch.cuda.current_stream().cuda_stream
    rc, ctx = native.gmres_create(p.n, p.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), m,
                                  native.GMRES_MGS_1R, wp, need, stream)
    assert rc == native.GMRES_OK
    try:
        rc, nb = native.gmres_matrix_storage_bytes(ctx)
        ns = (p.n + 63) // 64
        total = padded_entries(p)
        up = lambda v: (v + 255) // 256 * 256
        # the default for a stencil: offsets, a base per slice column, 16-bit deltas, values
        o_cb = up(8 * (ns + 1))
        o_cd = up(o_cb + 4 * (total // 64))
        o_va = up(o_cd + 2 * total)
        assert rc == native.GMRES_OK and nb == o_va + 8 * total
        assert native.gmres_get_format(ctx)[1] == native.GMRES_FORMAT_CSR
        buf = torch.empty(nb + 512, dtype=torch.uint8, device="cuda")
        bp = buf.data_ptr() + (-buf.data_ptr()) % 256
        assert native.gmres_set_matrix_storage(ctx, bp, nb - 8) == native.GMRES_ERR_ARG
        assert native.gmres_set_matrix_storage(ctx, bp + 8, nb) == native.GMRES_ERR_ARG
        host = np.zeros(nb // 8 + 64)
        assert native.gmres_set_matrix_storage(ctx, host.ctypes.data, nb) == native.GMRES_ERR_ARG
        assert native.gmres_set_matrix_storage(ctx, bp, nb) == native.GMRES_OK
        rc, fmt, stored = native.gmres_get_format(ctx)
        assert fmt == native.GMRES_FORMAT_SELL64_D16 and stored == total
        # the copy gives the same product as the CSR arrays
        x = torch.from_numpy(P.rng(5, 1).standard_normal(p.n)).cuda()
        y1 = torch.empty_like(x)
        y0 = torch.empty_like(x)
        assert native.gmres_spmv(ctx, x.data_ptr(), y1.data_ptr()) == native.GMRES_OK
        assert native.gmres_set_matrix_storage(ctx, None, 0) == native.GMRES_OK
        assert native.gmres_get_format(ctx)[1] == native.GMRES_FORMAT_CSR
        assert native.gmres_spmv(ctx, x.data_ptr(), y0.data_ptr()) == native.GMRES_OK
        torch.cuda.synchronize()
        absA = p.scipy().copy()
        absA.data = np.abs(absA.data)
        bound = 8 * np.finfo(float).eps * (absA @ np.abs(x.cpu().numpy()))
        assert np.all(np.abs((y0 - y1).cpu().numpy()) <= bound)
    finally:
        native.gmres_destroy(ctx)


def test_storage_layout_int32_indices():
    """With the int32 copy forced through the options: offsets, indices, values."""
    import torch

    from paper_1809_05805_amd import native

    p = P.make_config("convdiff2d", N=33)
    rp, ci, va = (torch.from_numpy(a).cuda() for a in (p.row_ptr, p.col_idx, p.vals))
    m = 10
    opt = native.make_options(format="sell")
    need = native.gmres_workspace_bytes_ex(p.n, m, native.GMRES_MGS_1R, opt)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    wp = ws.data_ptr() + (-ws.data_ptr()) % 256
    stream = torch.cuda.current_stream().cuda_stream
    rc, ctx = native.gmres_create_ex(p.n, p.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), m,
                                     native.GMRES_MGS_1R, wp, need, stream, opt)
    assert rc == native.GMRES_OK
    try:
        rc, nb = native.gmres_matrix_storage_bytes(ctx)
        ns = (p.n + 63) // 64
        total = padded_entries(p)
        up = lambda v: (v + 255) // 256 * 256
        o_ci = up(8 * (ns + 1))
        o_va = up(o_ci + 4 * total)
        assert rc == native.GMRES_OK and nb == o_va + 8 * total
        buf = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        bp = buf.data_ptr() + (-buf.data_ptr()) % 256
        assert native.gmres_set_matrix_storage(ctx, bp, nb) == native.GMRES_OK
        rc, fmt, stored = native.gmres_get_format(ctx)
        assert fmt == native.GMRES_FORMAT_SELL64 and stored == total
    finally:
        native.gmres_destroy(ctx)
