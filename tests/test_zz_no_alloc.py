"""gmres_solve_noalloc (one solve in the library's fixed device scratch) against
gmres_create + gmres_solve with a caller workspace and the CSR format, through
the C ABI, on two calls in a row whose second input is smaller.

Bar: the same kernels run in the same order on the same inputs, so the
iterate must match to 1e-10 relative (FP64) and every integer outcome
(iterations, cycles, reductions, flags) must be equal; the residual history
too, to 1e-10 relative.
"""

import numpy as np
import pytest

from paper_1809_05805_amd import native as N
from paper_1809_05805_amd import problems as P
from tests.gpu_util import log, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _dev(p):
    import torch

    return (torch.from_numpy(p.row_ptr).cuda(), torch.from_numpy(p.col_idx).cuda(),
            torch.from_numpy(p.vals).cuda(), torch.from_numpy(p.b).cuda())


def _with_workspace(p, scheme, m, rtol, max_iters):
    """gmres_create (caller workspace, no sliced copy: CSR) + gmres_solve + gmres_destroy."""
    import torch

    rp, ci, va, b = _dev(p)
    nbytes = N.gmres_workspace_bytes(p.n, m, scheme)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    wp = ws.data_ptr() + (-ws.data_ptr()) % 256
    stream = torch.cuda.current_stream().cuda_stream
    rc, ctx = N.gmres_create(p.n, p.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), m, scheme,
                             wp, nbytes, stream)
    assert rc == N.GMRES_OK, N.gmres_status_string(rc)
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    hist = np.full(max_iters, np.nan)
    rc, info = N.gmres_solve(ctx, b.data_ptr(), x.data_ptr(), rtol, max_iters, hist)
    assert rc == N.GMRES_OK, N.gmres_status_string(rc)
    assert N.gmres_destroy(ctx) == N.GMRES_OK
    return x.cpu().numpy(), info, hist[: info.iters]


def _noalloc(p, scheme, m, rtol, max_iters):
    import torch

    rp, ci, va, b = _dev(p)
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    hist = np.full(max_iters, np.nan)
    stream = torch.cuda.current_stream().cuda_stream
    rc, info = N.gmres_solve_noalloc(p.n, p.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), m,
                                     scheme, b.data_ptr(), x.data_ptr(), rtol, max_iters, hist,
                                     stream)
    assert rc == N.GMRES_OK, N.gmres_status_string(rc)
    return x.cpu().numpy(), info, hist[: info.iters]


@pytest.mark.parametrize("scheme", ["mgs1r", "mgs", "cgs2", "two_synch", "mgs1r_ir32"])
def test_noalloc_matches_workspace_path(scheme):
    import torch

    assert torch.cuda.is_available()
    sc = N.SCHEMES[scheme]
    # the second call is smaller (and has a ragged last tile): it runs on
    # whatever the first left in the scratch
    for p, m in ((P.make_config("convdiff2d"), 30), (P.make_config("convdiff2d", N=37), 20)):
        max_iters = 400
        log(f"noalloc: scheme={scheme} n={p.n} m={m}")
        xr, ir, hr = _with_workspace(p, sc, m, p.rtol, max_iters)
        xn, inn, hn = _noalloc(p, sc, m, p.rtol, max_iters)
        e = rel(xn, xr)
        log(f"  iters {inn.iters}/{ir.iters} reductions {inn.reductions}/{ir.reductions} "
            f"|x-x_ref|/|x_ref|={e:.2e} rel_res={inn.rel_res_true:.3e}")
        assert (inn.iters, inn.cycles, inn.converged, inn.breakdown, inn.reductions) == \
            (ir.iters, ir.cycles, ir.converged, ir.breakdown, ir.reductions)
        assert ir.converged == 1
        assert e <= TOL
        assert abs(inn.rel_res_true - ir.rel_res_true) <= TOL * ir.rel_res_true
        assert np.all(np.abs(hn - hr) <= TOL * np.maximum(np.abs(hr), 1e-300))


def test_noalloc_rejects_oversize_and_bad_args():
    import torch

    rp = torch.zeros(2, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    va = torch.ones(1, dtype=torch.float64, device="cuda")
    b = torch.ones(1, dtype=torch.float64, device="cuda")
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    # a workspace beyond the fixed scratch is refused before any pointer is used
    n_big = 1 << 20
    assert N.gmres_workspace_bytes(n_big, 30, N.GMRES_MGS_1R) > N.GMRES_NOALLOC_SCRATCH_BYTES
    rc, _ = N.gmres_solve_noalloc(n_big, 1, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), 30,
                                  N.GMRES_MGS_1R, b.data_ptr(), x.data_ptr(), 1e-8, 10)
    assert rc == N.GMRES_ERR_TOO_LARGE
    assert "GMRES_NOALLOC_SCRATCH_BYTES" in N.gmres_status_string(rc)
    # invalid scalars
    rc, _ = N.gmres_solve_noalloc(1, 1, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), 0,
                                  N.GMRES_MGS_1R, b.data_ptr(), x.data_ptr(), 1e-8, 10)
    assert rc == N.GMRES_ERR_ARG
    # a malformed matrix (row_ptr[n] != nnz) is found on the device
    rc, _ = N.gmres_solve_noalloc(1, 1, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), 5,
                                  N.GMRES_MGS_1R, b.data_ptr(), x.data_ptr(), 1e-8, 10)
    assert rc == N.GMRES_ERR_ARG
    # a well-formed 1 x 1 system then solves in one step
    rp[1] = 1
    b.fill_(3.0)
    va.fill_(2.0)
    rc, info = N.gmres_solve_noalloc(1, 1, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), 5,
                                     N.GMRES_MGS_1R, b.data_ptr(), x.data_ptr(), 1e-12, 10)
    assert rc == N.GMRES_OK and info.converged == 1
    assert abs(float(x[0]) - 1.5) <= 1e-15
