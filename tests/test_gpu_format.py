"""The library's SpMV format: which one it picks, and its sliced copy of A.

A context keeps a sliced-ELL copy of A (64 rows per slice). Stored by
diagonals (a slice column per distinct col - row value among the slice's
rows, no per-entry column index) when every row's columns are strictly
increasing and that costs at most a quarter more entries than nnz; else by
rows (each row padded to its slice's longest) when that costs at most a
quarter more, with column indices as 16-bit deltas from a base per slice
column when every slice column's col - row values span at most 65535, else
int32; else the SpMV reads the CSR arrays. These tests check the choice on
stencil, banded, scattered, unsorted and irregular matrices, the stored-entry
counts against counts made here from the CSR arrays, the storage layouts, that
the three sliced forms give bitwise the same solve, and that
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


def diag_entries(p):
    """Entries of the sliced layout by diagonals: per slice 64 x max(1, distinct col - row)."""
    n = p.n
    rows = np.repeat(np.arange(n), np.diff(p.row_ptr))
    d = p.col_idx.astype(np.int64) - rows
    sl = rows // 64
    ns = (n + 63) // 64
    counts = np.zeros(ns, dtype=np.int64)
    if d.size:
        pairs = np.unique(np.stack([sl, d]), axis=1)
        counts += np.bincount(pairs[0], minlength=ns)
    return int(64 * np.maximum(counts, 1).sum())


def scattered(n, reach, seed):
    """The diagonal plus two columns per row drawn within `reach` of it (or
    anywhere when reach is None): every row 3 long, so the copy by rows is
    cheap, but a slice's rows share few diagonals."""
    import scipy.sparse as sp

    g = P.rng(seed, 2)
    r = np.arange(n)
    if reach is None:
        c1, c2 = g.integers(0, n, n), g.integers(0, n, n)
    else:
        c1 = np.clip(r + g.integers(-reach, reach + 1, n), 0, n - 1)
        c2 = np.clip(r + g.integers(-reach, reach + 1, n), 0, n - 1)
    rr = np.concatenate([r, r, r])
    cc = np.concatenate([r, c1, c2])
    vv = np.concatenate([np.full(n, 8.0), np.full(n, -1.0), np.full(n, -1.0)])
    A = sp.csr_matrix((vv, (rr, cc)), shape=(n, n))
    rp, ci, va = P.csr_from_scipy(A)
    name = f"scattered_{reach}"
    return P.Problem(name, rp, ci, va, np.ones(n), np.zeros(n), None, 10, 0.0)


def reversed_rows(p):
    """The same matrix with each row's entries stored in decreasing column order."""
    ci = p.col_idx.copy()
    va = p.vals.copy()
    for r in range(p.n):
        a, b = p.row_ptr[r], p.row_ptr[r + 1]
        ci[a:b] = ci[a:b][::-1]
        va[a:b] = va[a:b][::-1]
    return P.Problem(p.name + "_rev", p.row_ptr, ci, va, p.b, p.x0, p.x_true, p.m, p.rtol)


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
        "convdiff2d": (P.make_config("convdiff2d"), "sell64_diag"),             # 5-point rows
        "convdiff3d_24": (P.make_config("convdiff3d", N=24), "sell64_diag"),    # 7-point rows
        "stencil27_12": (P.make_config("stencil27", N=12), "sell64_diag"),      # 27-point rows
        "wide_band": (wide_band(), "sell64_diag"),                  # 4 diagonals per slice
        "near": (scattered(20_000, 1000, 1), "sell64_d16"),         # deltas span < 65536
        "far": (scattered(140_000, None, 2), "sell64"),             # col - row spread > 65535
        "dense50": (P.random_dense(50, seed=3), "csr"),             # one slice, 14 padding rows
        "convdiff2d_rev": (reversed_rows(P.make_config("convdiff2d", N=24)), "sell64_d16"),
    }
    A = sp.csr_matrix(sp.random(3000, 3000, density=0.003, random_state=4) + sp.identity(3000))
    rp, ci, va = P.csr_from_scipy(A)
    cases["irregular"] = (P.Problem("irregular", rp, ci, va, np.ones(3000), np.zeros(3000), None,
                                    10, 0.0), "csr")
    for name, (p, want) in cases.items():
        s, _ = solver(p)
        fmt, stored = s.format()
        log(f"format {name}: {fmt} stored={stored} nnz={p.nnz} padded={padded_entries(p)} "
            f"diag={diag_entries(p)}")
        assert fmt == want, name
        expect = {"sell64_diag": diag_entries, "sell64_d16": padded_entries,
                  "sell64": padded_entries}.get(fmt, lambda q: q.nnz)(p)
        assert stored == expect, name
        s.close()
    # forced: int32 indices or deltas on a stencil; deltas where they do not fit
    # fall back to int32; diagonals on unsorted rows fall back to deltas;
    # diagonals and deltas whatever the padding
    for name, fmt, want in [("convdiff2d", "sell", "sell64"), ("convdiff2d", "sell_d16", "sell64_d16"),
                            ("wide_band", "sell_d16", "sell64"), ("dense50", "sell_d16", "sell64_d16"),
                            ("convdiff2d_rev", "sell_diag", "sell64_d16"),
                            ("dense50", "sell_diag", "sell64_diag"), ("far", "sell_diag", "sell64_diag")]:
        s, _ = solver(cases[name][0], fmt=fmt)
        got, stored = s.format()
        assert got == want, (name, fmt)
        if got == "sell64_diag":
            assert stored == diag_entries(cases[name][0])
        s.close()


@pytest.mark.parametrize("name", ["convdiff3d", "stencil27", "wide_band", "far", "convdiff2d_rev"])
def test_sliced_forms_bitwise(name):
    """The sliced forms sum each row's products in the same order (padding adds
    exact zeros), so a fixed-budget cycle gives the same bits in each, and the
    oracle's iterate to 1e-10. Rows stored in decreasing column order keep that
    order (the diagonal form is then refused and falls back to deltas)."""
    p = {"convdiff3d": lambda: P.make_config("convdiff3d", N=20),
         "stencil27": lambda: P.make_config("stencil27", N=14),
         "wide_band": lambda: wide_band(n=70_000 + 3000, far=70_000),
         "far": lambda: scattered(70_000, None, 5),
         "convdiff2d_rev": lambda: reversed_rows(P.make_config("convdiff2d", N=30))}[name]()
    log(f"forms {name} n={p.n}")
    runs = {}
    for fmt in ("sell", "sell_d16", "sell_diag"):
        g = gpu_run(p, "mgs1r", m=12, rtol=0.0, max_iters=18, fmt=fmt)
        runs[g["solver"].format()[0]] = g
    o = oracle_run(p, "mgs1r", m=12, rtol=0.0, max_iters=18, dump=False)
    ref = runs["sell64"]
    for f, g in runs.items():
        assert g["res"].iters == o.iters == 18, f
        assert np.array_equal(g["x"], ref["x"]), f
        assert rel(g["x"], o.x) <= 1e-10, f


def test_wide_band_solve_matches_oracle():
    """On the wide band (couplings 70,000 rows away), the copy by diagonals the
    library picks and the int32 copy that deltas fall back to both give the
    oracle's cycle."""
    p = wide_band(n=70_000 + 3000, far=70_000)
    o = oracle_run(p, "mgs1r", m=10, rtol=0.0, max_iters=10)
    for fmt, want in ((None, "sell64_diag"), ("sell_d16", "sell64")):
        g = gpu_run(p, "mgs1r", m=10, rtol=0.0, max_iters=10, fmt=fmt)
        assert g["solver"].format()[0] == want
        assert rel(g["x"], o.x) <= 1e-10


@pytest.mark.parametrize("fmt", ["csr", "sell", "sell_d16", "sell_diag"])
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


@pytest.mark.parametrize("fmt", ["sell", "sell_d16", "sell_diag"])
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


@pytest.mark.parametrize("fmt", ["sell", "sell_d16", "sell_diag"])
@pytest.mark.parametrize("scheme", ["mgs1r", "cgs2"])
def test_sell_small_and_one_row(scheme, fmt):
    """The sliced copy on sizes that leave most of the one slice as padding."""
    import scipy.sparse as sp

    name = {"sell": "sell64", "sell_d16": "sell64_d16", "sell_diag": "sell64_diag"}[fmt]
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
        total = diag_entries(p)
        up = lambda v: (v + 255) // 256 * 256
        # the default for a stencil: offsets, a diagonal per slice column, values
        o_cb = up(8 * (ns + 1))
        o_va = up(o_cb + 4 * (total // 64))
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
        assert fmt == native.GMRES_FORMAT_SELL64_DIAG and stored == total
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


@pytest.mark.parametrize("form", ["sell", "sell_d16"])
def test_storage_layout_by_rows(form):
    """With the copy by rows forced through the options: offsets, then int32
    indices, or a base per slice column and 16-bit deltas; then values."""
    import torch

    from paper_1809_05805_amd import native

    p = P.make_config("convdiff2d", N=33)
    rp, ci, va = (torch.from_numpy(a).cuda() for a in (p.row_ptr, p.col_idx, p.vals))
    m = 10
    opt = native.make_options(format=form)
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
        if form == "sell":
            o_va = up(up(8 * (ns + 1)) + 4 * total)
        else:
            o_va = up(up(up(8 * (ns + 1)) + 4 * (total // 64)) + 2 * total)
        assert rc == native.GMRES_OK and nb == o_va + 8 * total
        buf = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        bp = buf.data_ptr() + (-buf.data_ptr()) % 256
        assert native.gmres_set_matrix_storage(ctx, bp, nb) == native.GMRES_OK
        rc, fmt, stored = native.gmres_get_format(ctx)
        want = native.GMRES_FORMAT_SELL64 if form == "sell" else native.GMRES_FORMAT_SELL64_D16
        assert fmt == want and stored == total
    finally:
        native.gmres_destroy(ctx)


@pytest.mark.parametrize("scheme", ["mgs1r_ir32", "mgs1r_ir16"])
def test_refinement_copy_float64_values(scheme):
    """The refinement schemes' copy holds float32 values (their inner cycles)
    followed by float64 values: its size is laid out so, and the float64
    SpMV (gmres_spmv, the restart residual) reads the float64 values and gives
    the CSR arrays' product to rounding."""
    import torch

    from paper_1809_05805_amd import native

    p = P.make_config("convdiff2d", N=33)  # n = 1089: 18 slices, the last one ragged
    s, _ = solver(p, scheme=scheme)
    log(f"refinement copy {scheme}")
    assert s.format()[0] == "sell64_diag"
    rc, nb = native.gmres_matrix_storage_bytes(s.ctx)
    ns, total = (p.n + 63) // 64, diag_entries(p)
    up = lambda v: (v + 255) // 256 * 256
    o_va = up(up(8 * (ns + 1)) + 4 * (total // 64))
    assert rc == 0 and nb == up(o_va + 4 * total) + 8 * total
    x = torch.from_numpy(P.rng(5, 2).standard_normal(p.n)).cuda()
    y = torch.empty_like(x)
    s.spmv(x, y)
    c, _ = solver(p, scheme=scheme, fmt="csr")
    y0 = torch.empty_like(x)
    c.spmv(x, y0)
    torch.cuda.synchronize()
    absA = p.scipy().copy()
    absA.data = np.abs(absA.data)
    bound = 8 * np.finfo(float).eps * (absA @ np.abs(x.cpu().numpy()))
    assert np.all(np.abs((y - y0).cpu().numpy()) <= bound)
    assert np.abs(y.cpu().numpy() - p.scipy() @ x.cpu().numpy()).max() <= bound.max()
