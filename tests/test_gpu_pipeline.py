"""Pipeline depth of the rotations and the launch options, through the C ABI.

Depth L (Section III, the depth-L pipeline; the paper's listing has L = 2):
the Givens rotations and the stopping test of the lagged schemes run every L
steps, on the columns finished since. They feed nothing back into the
Arnoldi recurrence, so on the GPU the iterate, the Hessenberg matrix and the
residual history are bitwise those of depth 1, and a cycle stops at the same
column count, noticed up to L - 1 steps later; the reductions of the steps
run in between are counted, exactly as in the oracle's depth-L form. Both
depths are also held to the oracle at its own depth (1e-10).

Options: every rows-per-lane tiling, the separate SpMV launch and the CSR
SpMV shapes give the oracle's results to the parity tolerance; tilings differ
from one another only by the order of the device-wide sums.
"""

import numpy as np
import pytest

import oracle
from paper_1809_05805_amd import problems as P
from tests.gpu_util import gpu_run, log, oracle_run, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10
LAGGED = ["mgs1r", "cgs2"]


@pytest.fixture(scope="module", autouse=True)
def _torch_cuda():
    import torch

    assert torch.cuda.is_available()
    from paper_1809_05805_amd import native
    native.load()
    yield


def oracle_depth(p, scheme, m, rtol, max_iters, depth):
    return oracle.solve(p.row_ptr, p.col_idx, p.vals, p.b, p.x0, m, scheme, rtol, max_iters,
                        dump=True, depth=depth)


@pytest.mark.parametrize("depth", [2, 3, 7])
@pytest.mark.parametrize("scheme", LAGGED + ["mgs1r_ir32"])
def test_fixed_budget_depth_is_depth_one(scheme, depth):
    """No early stop: every output bitwise equal to depth 1, one reduction per
    step (two for CGS2) as at depth 1."""
    p = P.make_config("convdiff3d", N=24)
    m = 30
    log(f"depth {depth} fixed budget {scheme} n={p.n} m={m}")
    a = gpu_run(p, scheme, m=m, rtol=0.0, max_iters=m)
    b = gpu_run(p, scheme, m=m, rtol=0.0, max_iters=m, pipeline_depth=depth)
    ra, rb = a["res"], b["res"]
    assert rb.status == 0 and rb.iters == ra.iters == m and b["j"] == a["j"] == m
    assert rb.reductions == ra.reductions
    assert np.array_equal(b["x"], a["x"])
    assert np.array_equal(b["H"], a["H"])
    assert np.array_equal(b["T"], a["T"])
    assert np.array_equal(rb.hist, ra.hist)
    assert rb.rel_res_est == ra.rel_res_est
    if scheme in LAGGED:
        o = oracle_depth(p, scheme, m, 0.0, m, depth)
        assert o.reductions == rb.reductions
        assert rel(b["x"], o.x) <= TOL
        assert np.max(np.abs(rb.hist - o.hist)) <= TOL


# restarted solves that converge in several cycles: (config, N, m, rtol)
DEPTH_CASES = {"convdiff2d_64": ("convdiff2d", 64, 30, 1e-8), "convdiff2d_48": ("convdiff2d", 48, 12, 1e-9),
               "convdiff3d_16": ("convdiff3d", 16, 20, 1e-10)}


@pytest.mark.parametrize("depth", [2, 3, 5])
@pytest.mark.parametrize("scheme", LAGGED)
@pytest.mark.parametrize("case", list(DEPTH_CASES))
def test_to_tolerance_depth(case, scheme, depth):
    """Restarted solves to rtol: the same iterations, cycles and iterate as
    depth 1 (bitwise), and the oracle's depth-L reduction count exactly (the
    steps between the met tolerance and the next multiple of L)."""
    name, N, m, rtol = DEPTH_CASES[case]
    p = P.make_config(name, N=N)
    log(f"depth {depth} to tolerance {scheme} {case} m={m} rtol={rtol}")
    a = gpu_run(p, scheme, m=m, rtol=rtol, max_iters=20000)
    b = gpu_run(p, scheme, m=m, rtol=rtol, max_iters=20000, pipeline_depth=depth)
    ra, rb = a["res"], b["res"]
    assert ra.converged and rb.converged
    assert rb.iters == ra.iters and rb.cycles == ra.cycles
    assert np.array_equal(b["x"], a["x"])
    assert np.array_equal(rb.hist, ra.hist)
    assert rb.rel_res_est == ra.rel_res_est
    o1 = oracle_depth(p, scheme, m, rtol, 20000, 1)
    oL = oracle_depth(p, scheme, m, rtol, 20000, depth)
    assert oL.iters == o1.iters
    log(f"  reductions: gpu {ra.reductions} -> {rb.reductions}, oracle {o1.reductions} -> {oL.reductions}")
    assert rb.reductions - ra.reductions == oL.reductions - o1.reductions
    if ra.iters == o1.iters:
        assert rb.reductions == oL.reductions
    assert rel(b["x"], oL.x) <= 10 * rtol


def test_depth_refused_for_normalized_schemes():
    import torch

    from paper_1809_05805_amd.native import GmresError, GmresSolver

    p = P.make_config("convdiff2d", N=16)
    rp, ci, va = (torch.from_numpy(a).cuda() for a in (p.row_ptr, p.col_idx, p.vals))
    for scheme in ("mgs", "cgs2_3r", "two_synch"):
        with pytest.raises(GmresError):
            GmresSolver(rp, ci, va, 10, scheme, pipeline_depth=2)
        GmresSolver(rp, ci, va, 10, scheme, pipeline_depth=1).close()


@pytest.mark.parametrize("scheme", ["mgs1r", "cgs2", "mgs", "two_synch"])
def test_rows_per_lane_option(scheme):
    """Every tiling (1, 2, 4, 8 rows per lane; the last tile ragged) matches
    the oracle; the tilings agree with one another to rounding."""
    p = P.make_config("convdiff3d", N=23)  # n = 12167
    m = 20
    o = oracle_run(p, scheme, m=m, rtol=0.0, max_iters=m)
    xs = []
    for rpt in (1, 2, 4, 8):
        log(f"rows per lane {rpt} {scheme} n={p.n}")
        g = gpu_run(p, scheme, m=m, rtol=0.0, max_iters=m, rows_per_lane=rpt)
        r = g["res"]
        assert r.status == 0 and r.iters == m and r.reductions == o.reductions
        assert rel(g["x"], o.x) <= TOL
        assert np.max(np.abs(r.hist - o.hist)) <= TOL
        xs.append(g["x"])
    for x in xs[1:]:
        assert rel(x, xs[0]) <= 1e-12


@pytest.mark.parametrize("shape", [108, 208, 408, 804, 808, 6401])
def test_csr_spmv_shape_option(shape):
    """Each CSR SpMV shape gives the oracle's product within 64 eps |A||x| and
    a fixed-budget cycle within the parity tolerance."""
    import torch

    from paper_1809_05805_amd.native import GmresSolver

    p = P.make_config("stencil27", N=11)
    rp, ci, va = (torch.from_numpy(a).cuda() for a in (p.row_ptr, p.col_idx, p.vals))
    s = GmresSolver(rp, ci, va, 4, "mgs1r", format="csr", csr_spmv_shape=shape)
    assert s.format()[0] == "csr"
    x = P.rng(78, 0).standard_normal(p.n)
    y = torch.empty(p.n, dtype=torch.float64, device="cuda")
    s.spmv(torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    ref = oracle.spmv(p.row_ptr, p.col_idx, p.vals, x)
    absA = p.scipy().copy()
    absA.data = np.abs(absA.data)
    bound = 64 * np.finfo(float).eps * (absA @ np.abs(x))
    assert np.all(np.abs(y.cpu().numpy() - ref) <= bound + 1e-300)
    g = gpu_run(p, "mgs1r", m=20, rtol=0.0, max_iters=20, fmt="csr", csr_spmv_shape=shape)
    o = oracle_run(p, "mgs1r", m=20, rtol=0.0, max_iters=20)
    assert rel(g["x"], o.x) <= TOL


@pytest.mark.parametrize("fmt", ["csr", "sell"])
def test_split_spmv_option(fmt):
    """The SpMV in a launch of its own (the step kernel reads w back): the
    oracle's cycle to the parity tolerance, and the same reduction count."""
    p = P.make_config("convdiff3d", N=24)
    m = 30
    g = gpu_run(p, "mgs1r", m=m, rtol=0.0, max_iters=m, fmt=fmt, split_spmv=True)
    f = gpu_run(p, "mgs1r", m=m, rtol=0.0, max_iters=m, fmt=fmt)
    o = oracle_run(p, "mgs1r", m=m, rtol=0.0, max_iters=m)
    assert g["res"].reductions == o.reductions
    assert rel(g["x"], o.x) <= TOL
    assert np.max(np.abs(g["res"].hist - o.hist)) <= TOL
    # the fused and separate SpMV compute the same row sums in the same order
    assert rel(g["x"], f["x"]) <= 1e-13
