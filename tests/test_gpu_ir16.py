"""The bfloat16-basis experiment (GMRES_MGS_1R_IR16): the one-reduce step on a
basis stored in bfloat16 (float32 arithmetic) inside float64 refinement.

The stopping test is the float64 true residual, so a converged solve meets
1e-10 like the float64 schemes; what the 8-bit significand changes is how
much each refinement cycle gains, so the iteration counts are logged against
the float64 and float32-basis ones. Each result states its error against the
float64 oracle:

* to tolerance: ||b - A x|| / ||b|| recomputed here in float64 <= rtol, and
  ||x - x_oracle|| / ||x_oracle|| within 10 kappa_est rtol (kappa_est as in
  the float32-basis tests);
* one cycle (no refinement yet): x and |g_k| against the float64 oracle's
  cycle within 1e4 eps_bf16 (eps_bf16 = 2^-8), the float32-basis bound with
  the bfloat16 epsilon;
* bitwise reproducibility, both SpMV formats, the error paths.
"""

import numpy as np
import pytest

from paper_1809_05805_amd import problems as P
from tests.gpu_util import gpu_run, log, oracle_run, rel

pytestmark = pytest.mark.gpu

EPS16 = 2.0 ** -8


@pytest.fixture(scope="module", autouse=True)
def _torch_cuda():
    import torch

    assert torch.cuda.is_available()
    from paper_1809_05805_amd import native
    native.load()
    yield


CASES = {
    "convdiff2d": P.make_config("convdiff2d"),
    "convdiff2d_ragged": P.make_config("convdiff2d", N=37),
    "convdiff3d_24": P.make_config("convdiff3d", N=24),
}


def true_rel_res(p, x):
    return float(np.linalg.norm(p.b - p.scipy() @ x) / np.linalg.norm(p.b))


@pytest.mark.parametrize("fmt", ["sell", "csr"])
@pytest.mark.parametrize("case", ["convdiff2d", "convdiff2d_ragged", "convdiff3d_24"])
def test_ir16_to_tolerance(case, fmt):
    p = CASES[case]
    rtol = 1e-10
    m = min(p.m, 40)
    log(f"ir16 {case} {fmt}")
    g = gpu_run(p, "mgs1r_ir16", m=m, rtol=rtol, fmt=fmt)
    r = g["res"]
    f64 = gpu_run(p, "mgs1r", m=m, rtol=rtol)["res"]
    f32 = gpu_run(p, "mgs1r_ir32", m=m, rtol=rtol, fmt=fmt)["res"]
    o = oracle_run(p, "mgs1r", m=m, rtol=rtol, dump=False)
    res = true_rel_res(p, g["x"])
    ex = rel(g["x"], o.x)
    kappa = max(rel(o.x, p.x_true) / rtol, 1.0)
    log(f"  iters {r.iters} (fp32 basis {f32.iters}, fp64 {f64.iters}, oracle {o.iters}), cycles "
        f"{r.cycles}, rel_res {res:.2e}, |x-x_oracle|/|x_oracle| {ex:.2e}, kappa_est {kappa:.1e}")
    assert r.status == 0 and r.converged
    assert res <= rtol * (1 + 1e-6)
    assert abs(r.rel_res_true - res) <= 1e-3 * res + 1e-16
    assert ex <= 10 * kappa * rtol
    assert r.iters <= 3 * f64.iters + m


@pytest.mark.parametrize("case", ["convdiff2d", "convdiff3d_24"])
def test_ir16_one_cycle_vs_fp64_oracle(case):
    p = CASES[case]
    m = min(p.m, 40)
    log(f"ir16 one cycle {case}")
    g = gpu_run(p, "mgs1r_ir16", m=m, rtol=0.0, max_iters=m)
    o = oracle_run(p, "mgs1r", m=m, rtol=0.0, max_iters=m)
    r = g["res"]
    assert r.iters == o.iters == m and g["j"] == o.j == m
    ex = rel(g["x"], o.x)
    eh = np.max(np.abs(r.hist - o.hist) / np.maximum(o.hist, 1e-300))
    log(f"  |x-x_o|/|x_o| {ex:.2e}, max rel |g_k| diff {eh:.2e}")
    assert ex <= 1e4 * EPS16
    assert eh <= 1e4 * EPS16


def test_ir16_deterministic():
    p = CASES["convdiff3d_24"]
    a = gpu_run(p, "mgs1r_ir16", m=30, rtol=1e-10)
    b = gpu_run(p, "mgs1r_ir16", m=30, rtol=1e-10)
    assert a["res"].iters == b["res"].iters
    assert np.array_equal(a["x"], b["x"])


def test_ir16_errors_and_edges():
    import scipy.sparse as sp

    from paper_1809_05805_amd import native
    from paper_1809_05805_amd.native import GmresError

    p = P.make_config("convdiff2d", N=16)
    b = p.b.copy()
    b[3] = np.nan
    g = gpu_run(p, "mgs1r_ir16", b=b)
    assert g["res"].status == native.GMRES_ERR_NONFINITE
    g = gpu_run(p, "mgs1r_ir16", b=np.zeros(p.n), x0=np.ones(p.n))
    assert g["res"].converged and g["res"].iters == 0 and np.all(g["x"] == 0.0)
    g = gpu_run(p, "mgs1r_ir16", max_iters=0)
    assert g["res"].iters == 0 and abs(g["res"].rel_res_true - 1.0) <= 1e-15
    rp, ci, va = P.csr_from_scipy(sp.csr_matrix(np.array([[4.0]])))
    one = P.Problem("one", rp, ci, va, np.array([2.0]), np.zeros(1), np.array([0.5]), m=1, rtol=1e-12)
    g = gpu_run(one, "mgs1r_ir16")
    assert g["res"].converged and abs(g["x"][0] - 0.5) <= 1e-15
    with pytest.raises(GmresError):
        g["solver"].basis()
