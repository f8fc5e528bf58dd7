"""Batched persistent solver (gmres_batch_*) against the oracle, system by system.

Every system of a batch is an independent restarted one-reduce GMRES(m)
solve, so each is compared with the oracle's GMRES_MGS_1R solve of that
system alone, with the tolerances of the single-system parity tests: after a
fixed budget (no early exit) the iterate within 1e-10 relative; to tolerance,
equal iteration counts up to one and both truly converged. The float32-basis
batch is held to the float64 stopping test and its iterate compared with the
float64 oracle within 10 kappa_est rtol (as for the single-system float32
scheme). Systems split over a team of workgroups (parts of 256 rows here, so
that the small systems form teams of up to 6) are held to the same bounds.
Results must not depend on the grid or the queue order, and a captured graph
must reproduce the eager solve bit for bit on every replay. The batched SpMV
reads a copy of the block-diagonal matrix by diagonals when the library plans
one (stencil systems, so by default here), else the CSR arrays; both forms
accumulate each row's products in the same order and give the same bits.
"""

import numpy as np
import pytest

from paper_1809_05805_amd import problems as P
from tests.gpu_util import log, oracle_run, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _torch_cuda():
    import torch

    assert torch.cuda.is_available()
    from paper_1809_05805_amd import native
    native.load()
    yield


def small_batch(nsys=24, seed=1, lo=6, hi=40):
    # sides 6..40: n from 36 (most of a 256-thread workgroup idle) to 1600
    # (several row blocks of 2048 and a ragged last one)
    return P.make_batch(nsys=nsys, seed=seed, side_lo=lo, side_hi=hi, m=30, rtol=TOL)


SMALL = small_batch()


def tensors(bp):
    import torch

    return (torch.from_numpy(bp.row_ptr).cuda(), torch.from_numpy(bp.col_idx).cuda(),
            torch.from_numpy(bp.vals).cuda())


def solver(bp, scheme="mgs1r", m=None, stream=None, fmt=None):
    from paper_1809_05805_amd.native import BatchSolver

    rp, ci, va = tensors(bp)
    return BatchSolver(bp.row_off, rp, ci, va, bp.m if m is None else m, scheme, stream=stream,
                       format=fmt)


def run(bp, scheme="mgs1r", rtol=TOL, max_iters=20000, b=None, x0=None, config=None, m=None,
        fmt=None):
    import torch

    s = solver(bp, scheme, m, fmt=fmt)
    if config:
        s.set_config(*config)
    bt = torch.from_numpy(np.ascontiguousarray(bp.b if b is None else b)).cuda()
    xt = torch.from_numpy(np.array(bp.x0 if x0 is None else x0, dtype=np.float64)).cuda()
    rc, info = s.solve(bt, xt, rtol, max_iters)
    torch.cuda.synchronize()
    return rc, info, xt.cpu().numpy(), s


def true_rel(bp, i, x):
    p = bp.system(i)
    nb = np.linalg.norm(p.b)
    return float(np.linalg.norm(p.b - p.scipy() @ x[bp.row_off[i]: bp.row_off[i + 1]]) / nb)


@pytest.mark.parametrize("bs,part_rows", [(256, 0), (512, 0), (1024, 0), (256, 256), (1024, 256)])
def test_fixed_budget_parity(bs, part_rows):
    """45 Arnoldi steps per system (one full cycle and half of the next), rtol 0."""
    bp = SMALL
    log(f"batch fixed budget bs={bs} part_rows={part_rows}")
    rc, info, x, s = run(bp, rtol=0.0, max_iters=45, config=(bs, 0, 1, part_rows))
    if part_rows:
        assert s.config()["max_parts"] == 6
    assert rc == 0
    worst = 0.0
    for i in range(bp.nsys):
        p = bp.system(i)
        o = oracle_run(p, "mgs1r", m=30, rtol=0.0, max_iters=45, dump=False)
        xi = x[bp.row_off[i]: bp.row_off[i + 1]]
        assert info["iters"][i] == o.iters, i
        assert info["cycles"][i] == o.cycles, i
        assert info["status"][i] == 0
        e = rel(xi, o.x)
        worst = max(worst, e)
        assert e <= TOL, (i, p.n, e)
        assert abs(info["rel_res_true"][i] - o.rel_res_true) <= TOL * max(o.rel_res_true, 1e-3)
    log(f"  worst |x - x_oracle| / |x_oracle| = {worst:.2e}")


@pytest.mark.parametrize("part_rows", [0, 256])
def test_to_tolerance_parity(part_rows):
    bp = SMALL
    log(f"batch to tolerance fp64 part_rows={part_rows}")
    rc, info, x, _ = run(bp, config=(256, 0, 1, part_rows))
    assert rc == 0
    for i in range(bp.nsys):
        p = bp.system(i)
        o = oracle_run(p, "mgs1r", m=30, rtol=TOL, dump=False)
        xi = x[bp.row_off[i]: bp.row_off[i + 1]]
        assert o.converged and info["converged"][i] == 1, i
        assert abs(int(info["iters"][i]) - o.iters) <= 1, (i, info["iters"][i], o.iters)
        r = true_rel(bp, i, x)
        assert r <= TOL * (1 + 1e-6), (i, r)
        assert abs(info["rel_res_true"][i] - r) <= 1e-3 * r + 1e-16
        assert rel(xi, o.x) <= 10 * 1e4 * TOL


@pytest.mark.parametrize("part_rows", [0, 256])
def test_fp32_basis_to_tolerance(part_rows):
    bp = SMALL
    log(f"batch to tolerance fp32 basis part_rows={part_rows}")
    rc, info, x, _ = run(bp, "mgs1r_ir32", config=(256, 0, 1, part_rows))
    _, info64, x64, _ = run(bp, config=(256, 0, 1, part_rows))
    assert rc == 0
    errs = []
    for i in range(bp.nsys):
        p = bp.system(i)
        o = oracle_run(p, "mgs1r", m=30, rtol=TOL, dump=False)
        xi = x[bp.row_off[i]: bp.row_off[i + 1]]
        assert info["converged"][i] == 1 and info["status"][i] == 0, i
        r = true_rel(bp, i, x)
        assert r <= TOL * (1 + 1e-6), (i, r)
        kappa = max(rel(o.x, p.x_true) / TOL, 1.0)
        e = rel(xi, o.x)
        errs.append(e)
        assert e <= 10 * kappa * TOL, (i, e, kappa)
        assert info["iters"][i] <= int(np.ceil(1.34 * info64["iters"][i])) + 30
    log(f"  fp32 basis: iters {int(info['iters'].sum())} (fp64 {int(info64['iters'].sum())}), "
        f"max |x - x_oracle| / |x_oracle| {max(errs):.2e}")


@pytest.mark.parametrize("part_rows", [0, 256])
def test_config_invariance(part_rows):
    """Grid and queue order change the schedule, not the arithmetic (grids of at
    least the largest team, 6 parts, keep every team whole)."""
    bp = SMALL
    log(f"batch config invariance part_rows={part_rows}")
    _, i0, x0, _ = run(bp, rtol=TOL, config=(256, 0, 1, part_rows))
    grids = [(6, 1), (9, 0), (1000, 0)] + ([(1, 1)] if part_rows == 0 else [])
    for grid, order in grids:
        _, i1, x1, _ = run(bp, rtol=TOL, config=(256, grid, order, part_rows))
        assert np.array_equal(x0, x1), (grid, order)
        assert np.array_equal(i0["iters"], i1["iters"])


def test_graph_replay():
    """Capture once, replay three times with eager work in between: every replay equals eager."""
    import torch

    bp = SMALL
    log("batch graph capture")
    stream = torch.cuda.Stream()
    s = solver(bp, stream=stream)
    bt = torch.from_numpy(bp.b).cuda()
    x_e = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        rc, info_e = s.solve(bt, x_e, TOL, 20000)
    torch.cuda.synchronize()
    x = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.capture(bt, x, TOL, 20000)
    for rep in range(3):
        with torch.cuda.stream(stream):
            x.zero_()
            s.replay()
        stream.synchronize()
        info = s.read_info()
        assert torch.equal(x, x_e), rep
        assert np.array_equal(info["iters"], info_e["iters"])
        # eager work between replays
        y = (x_e * 2.0).sum().item()
        assert np.isfinite(y)


def test_graph_dropped_on_config_change():
    """A configuration change discards the captured graph (it holds the old grid,
    block size and queue): replay is refused until the next capture, whose
    replays then equal the eager solve under the new configuration bit for bit."""
    import torch

    from paper_1809_05805_amd import native

    bp = SMALL
    log("batch graph dropped on set_config")
    stream = torch.cuda.Stream()
    s = solver(bp, stream=stream)
    bt = torch.from_numpy(bp.b).cuda()
    x = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.capture(bt, x, TOL, 20000)
    s.set_config(512, 0, 1, 256)  # another block size and teams of 256-row parts
    assert native.gmres_batch_replay(s.ctx) == native.GMRES_ERR_ARG
    x_e = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        rc, info_e = s.solve(bt, x_e, TOL, 20000)
    torch.cuda.synchronize()
    assert rc == 0 and np.all(info_e["converged"] == 1)
    s.capture(bt, x, TOL, 20000)
    for rep in range(2):
        with torch.cuda.stream(stream):
            x.zero_()
            s.replay()
        stream.synchronize()
        info = s.read_info()
        assert torch.equal(x, x_e), rep
        assert np.array_equal(info["iters"], info_e["iters"])


def test_autotune():
    import torch

    bp = SMALL
    log("batch autotune")
    s = solver(bp)
    bt = torch.from_numpy(bp.b).cuda()
    x = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
    trials = s.autotune(bt, x, TOL, 20000)
    assert len(trials) >= 6 and all(t[3] > 0 for t in trials)
    best = min(trials, key=lambda t: t[3])
    cfg = s.config()
    assert (cfg["block_size"], cfg["grid"], cfg["order"], cfg["part_rows"]) == (*best[:3], best[4])
    assert cfg["streamed"] == bool(best[5])
    assert len({t[5] for t in trials}) == 2  # both load forms were timed
    assert torch.count_nonzero(x).item() == 0  # x restored
    rc, info = s.solve(bt, x, TOL, 20000)
    assert rc == 0 and np.all(info["converged"] == 1)
    log("  trials: " + ", ".join(f"{t[0]}/{t[1]}/{t[2]}/{t[4]}/{t[5]}:{t[3]:.2f}ms" for t in trials))


@pytest.mark.parametrize("config", [(256, 0, 1, 256), (1024, 0, 1, 0), (1024, 0, 1, 512)])
def test_load_forms_bitwise(config):
    """Streamed (non-temporal) and cached loads of the basis give bitwise the
    same iterates and iteration counts, with and without teams."""
    import torch

    bp = SMALL
    log(f"batch load forms {config}")
    outs = []
    for mode in ("cached", "streamed"):
        s = solver(bp)
        s.set_config(*config)
        s.set_loads(mode)
        cfg = s.config()
        assert cfg["loads"] == mode and cfg["streamed"] == (mode == "streamed")
        bt = torch.from_numpy(bp.b).cuda()
        x = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
        rc, info = s.solve(bt, x, TOL, 20000)
        torch.cuda.synchronize()
        assert rc == 0 and np.all(info["converged"] == 1)
        outs.append((x.cpu().numpy(), info["iters"].copy()))
        s.close()
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][0], outs[1][0])
    from paper_1809_05805_amd import native
    s = solver(bp)
    with pytest.raises(native.GmresError):
        native_rc = native.gmres_batch_set_loads(s.ctx, 3)
        if native_rc != 0:
            raise native.GmresError(native_rc, "gmres_batch_set_loads")
    s.close()


def test_edges():
    """Zero right-hand side, a NaN in one system, max_iters 0, one-row systems."""
    import scipy.sparse as sp

    from paper_1809_05805_amd import native

    bp = small_batch(nsys=6, seed=3, lo=3, hi=12)
    log("batch edges")
    b = bp.b.copy()
    b[bp.row_off[1]: bp.row_off[2]] = 0.0
    b[bp.row_off[3] + 2] = np.nan
    x0 = np.ones(bp.n)
    rc, info, x, _ = run(bp, b=b, x0=x0)
    assert rc == native.GMRES_ERR_NONFINITE
    assert info["status"][3] == native.GMRES_ERR_NONFINITE
    assert info["converged"][1] == 1 and info["iters"][1] == 0
    assert np.all(x[bp.row_off[1]: bp.row_off[2]] == 0.0)
    for i in (0, 2, 4, 5):
        assert info["status"][i] == 0 and info["converged"][i] == 1
        assert true_rel(bp, i, x) <= TOL * (1 + 1e-6)
    rc, info, x, _ = run(bp, max_iters=0)
    assert np.all(info["iters"] == 0) and np.all(np.abs(info["rel_res_true"] - 1.0) <= 1e-15)
    # one-row systems next to a larger one
    blocks = [sp.csr_matrix(np.array([[4.0]])), sp.csr_matrix(np.array([[2.0]])),
              P.convdiff(9, 2, (1.0, 0.0), 5.0)]
    A = sp.block_diag(blocks, format="csr")
    rp, ci, va = P.csr_from_scipy(A)
    n = A.shape[0]
    xt = np.linspace(-1.0, 1.0, n)
    one = P.BatchProblem("ones", np.array([0, 1, 2, n]), rp, ci, va, A @ xt, np.zeros(n), xt, 5,
                         1e-12, np.array([1, 1, 9]), np.ones(3), np.zeros(3))
    rc, info, x, _ = run(one, rtol=1e-12)
    assert rc == 0 and np.all(info["converged"] == 1)
    assert abs(x[0] - xt[0]) <= 1e-15 and abs(x[1] - xt[1]) <= 1e-15
    assert rel(x[2:], xt[2:]) <= 1e-8


def test_create_refusals():
    import torch

    from paper_1809_05805_amd import native
    from paper_1809_05805_amd.native import BatchSolver, GmresError

    bp = small_batch(nsys=4, seed=2, lo=4, hi=8)
    rp, ci, va = tensors(bp)
    log("batch create refusals")
    # a column of system 1 pointing into system 0
    bad = bp.col_idx.copy()
    bad[bp.row_ptr[bp.row_off[1]]] = 0
    with pytest.raises(GmresError) as e:
        BatchSolver(bp.row_off, rp, torch.from_numpy(bad).cuda(), va, 10)
    assert e.value.rc == native.GMRES_ERR_ARG
    # row offsets that do not increase, and the schemes without a batched form
    ro = bp.row_off.copy()
    ro[2] = ro[1]
    with pytest.raises(GmresError):
        BatchSolver(ro, rp, ci, va, 10)
    for scheme in ("mgs", "cgs2"):
        with pytest.raises(GmresError):
            BatchSolver(bp.row_off, rp, ci, va, 10, scheme)
    s = BatchSolver(bp.row_off, rp, ci, va, 10)
    with pytest.raises(GmresError):
        s.set_config(128, 0, 0)
    with pytest.raises(GmresError):
        s.set_config(256, -1, 0)
    with pytest.raises(GmresError):
        s.set_config(256, 0, 0, -1)
    with pytest.raises(GmresError):
        s.set_config(256, 0, 2)


@pytest.mark.parametrize("scheme", ["mgs1r", "mgs1r_ir32"])
def test_full_batch(scheme):
    """512 systems, sides 32..256, Peclet 1..100, m=30, rtol 1e-10: every system truly
    converged (residuals recomputed here), the three smallest against the oracle."""
    bp = P.make_batch()
    log(f"full batch {scheme}: n={bp.n} nnz={bp.nnz}")
    rc, info, x, s = run(bp, scheme)
    assert s.config()["loads"] == "auto"
    assert rc == 0
    assert np.all(info["status"] == 0) and np.all(info["converged"] == 1)
    A = None
    worst = 0.0
    for i in range(bp.nsys):
        r = true_rel(bp, i, x)
        worst = max(worst, r)
        assert r <= TOL * (1 + 1e-6), (i, r)
    log(f"  iters total {int(info['iters'].sum())}, max {int(info['iters'].max())}, "
        f"worst true rel res {worst:.2e}")
    for i in np.argsort(bp.row_off[1:] - bp.row_off[:-1], kind="stable")[:3]:
        p = bp.system(int(i))
        o = oracle_run(p, "mgs1r", m=30, rtol=TOL, dump=False)
        xi = x[bp.row_off[i]: bp.row_off[i + 1]]
        if scheme == "mgs1r":
            assert abs(int(info["iters"][i]) - o.iters) <= 1
        assert rel(xi, o.x) <= 10 * 1e4 * TOL
    del A


def test_load_form_auto_choice():
    """Under the default mode the kernel streams the basis exactly when the
    bases in use at once exceed 384 MiB: the 512-system 2D batch at 1024
    threads and parts of 4096 rows keeps about 240 MB in use (cached); the 3D
    batch keeps about 900 MB (streamed)."""
    for bp, want in ((P.make_batch(), False), (P.make_batch3d(), True)):
        s = solver(bp)
        s.set_config(1024, 0, 1, 4096)
        cfg = s.config()
        log(f"{bp.name}: grid {cfg['grid']} streamed {cfg['streamed']}")
        assert cfg["loads"] == "auto" and cfg["streamed"] == want
        s.close()


def test_full_batch_repeat_bitwise():
    """The team barrier and the per-system reductions sum in a fixed order: the
    whole 512-system batch, solved twice on one context with teams of parts
    (the configuration the autotuner picks), gives bitwise equal iterates and
    iteration counts, and so does a second context."""
    import torch

    bp = P.make_batch()
    log(f"full batch repeat: n={bp.n}")
    outs = []
    for _ in range(2):
        s = solver(bp)
        s.set_config(1024, 0, 1, 4096)
        bt = torch.from_numpy(bp.b).cuda()
        for _ in range(2):
            xt = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
            rc, info = s.solve(bt, xt, TOL, 20000)
            torch.cuda.synchronize()
            assert rc == 0 and np.all(info["converged"] == 1)
            outs.append((xt.cpu().numpy(), info["iters"].copy()))
        s.close()
    for x, it in outs[1:]:
        assert np.array_equal(it, outs[0][1])
        assert np.array_equal(x, outs[0][0])


def test_team_wait_limit():
    """A team whose parts stop waiting gives up with GMRES_ERR_HIP for that
    system, and every kernel still ends. The wait limit is set to zero polls
    through the C ABI (gmres_batch_set_wait_limit), so a part that arrives
    before its partners gives up at once; one-part systems are not affected."""
    import torch

    from paper_1809_05805_amd import native

    bp = SMALL
    log("batch team wait limit")
    s = solver(bp)
    s.set_wait_limit(0)
    with pytest.raises(native.GmresError):
        s.set_wait_limit(native.GMRES_BATCH_WAIT_LIMIT + 1)
    s.set_config(256, 0, 1, 256)
    bt = torch.from_numpy(bp.b).cuda()
    x = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
    rc, info = s.solve(bt, x, TOL, 20000, check=False)
    torch.cuda.synchronize()
    assert rc == native.GMRES_ERR_HIP
    sizes = np.diff(bp.row_off)
    teams = sizes > 256
    assert np.all(np.isin(info["status"][teams], (0, native.GMRES_ERR_HIP)))
    assert np.any(info["status"][teams] == native.GMRES_ERR_HIP)
    xs = x.cpu().numpy()
    for i in np.nonzero(~teams)[0]:
        assert info["status"][i] == 0 and info["converged"][i] == 1
        assert true_rel(bp, i, xs) <= TOL * (1 + 1e-6)
    # the default limit: the same context shape solves normally
    rc, info = run(bp, config=(256, 0, 1, 256))[:2]
    assert rc == 0 and np.all(info["converged"] == 1)


@pytest.mark.parametrize("m,side_lo,steps", [(100, 12, 120), (150, 17, 170)])
@pytest.mark.parametrize("bs", [256, 1024])
def test_long_restart(bs, m, side_lo, steps):
    """Long restarts, one-part systems and teams, against the oracle after a
    cycle and part of the next: m = 100 keeps T in LDS, m = 150 in global
    memory (beyond 128); the per-wavefront sums and the small dense arrays
    are at their largest in these tests."""
    bp = P.make_batch(nsys=6, seed=7, side_lo=side_lo, side_hi=30, m=m, rtol=TOL)
    log(f"batch long restart bs={bs} m={m}")
    for part_rows in (0, 256):
        rc, info, x, _ = run(bp, rtol=0.0, max_iters=steps, config=(bs, 0, 1, part_rows), m=m)
        assert rc == 0
        for i in range(bp.nsys):
            p = bp.system(i)
            o = oracle_run(p, "mgs1r", m=m, rtol=0.0, max_iters=steps, dump=False)
            assert info["iters"][i] == o.iters == steps
            assert rel(x[bp.row_off[i]: bp.row_off[i + 1]], o.x) <= TOL, (i, part_rows)


@pytest.mark.parametrize("bs,part_rows", [(256, 0), (1024, 0), (256, 1024), (1024, 512)])
def test_batch3d_fixed_budget_parity(bs, part_rows):
    """3D 7-point systems (sides 8..24, m = 50): every system against the
    oracle's solve of that system alone after 70 steps, with and without teams."""
    bp = P.make_batch3d(nsys=6, seed=3, side_lo=8, side_hi=24, m=50)
    log(f"3D batch fixed budget bs={bs} part_rows={part_rows} n={bp.n}")
    rc, info, x, s = run(bp, rtol=0.0, max_iters=70, config=(bs, 0, 1, part_rows))
    assert rc == 0
    for i in range(bp.nsys):
        p = bp.system(i)
        o = oracle_run(p, "mgs1r", m=50, rtol=0.0, max_iters=70, dump=False)
        assert info["iters"][i] == o.iters == 70 and info["cycles"][i] == o.cycles, i
        assert rel(x[bp.row_off[i]: bp.row_off[i + 1]], o.x) <= TOL, (i, p.n)


@pytest.mark.parametrize("scheme", ["mgs1r", "mgs1r_ir32"])
def test_full_batch3d(scheme):
    """The 64-system 3D batch (sides 32..64, m = 50, about 3 GB of float64
    basis): every system truly converged to 1e-10 (residuals recomputed here),
    the two smallest against the oracle."""
    bp = P.make_batch3d()
    log(f"full 3D batch {scheme}: n={bp.n} nnz={bp.nnz}")
    rc, info, x, s = run(bp, scheme, config=(1024, 0, 1, 4096))
    assert s.config()["streamed"]  # its bases in use at once exceed the last-level cache
    assert rc == 0
    assert np.all(info["status"] == 0) and np.all(info["converged"] == 1)
    worst = 0.0
    for i in range(bp.nsys):
        r = true_rel(bp, i, x)
        worst = max(worst, r)
        assert r <= TOL * (1 + 1e-6), (i, r)
    log(f"  iters total {int(info['iters'].sum())}, max {int(info['iters'].max())}, "
        f"worst true rel res {worst:.2e}")
    for i in np.argsort(np.diff(bp.row_off), kind="stable")[:2]:
        p = bp.system(int(i))
        o = oracle_run(p, "mgs1r", m=50, rtol=TOL, dump=False)
        if scheme == "mgs1r":
            assert abs(int(info["iters"][i]) - o.iters) <= 1
        assert rel(x[bp.row_off[i]: bp.row_off[i + 1]], o.x) <= 10 * 1e4 * TOL


def batch_diag_entries(bp):
    """Entries of the block-diagonal matrix's copy by diagonals: per 64-row
    slice of global rows, 64 x max(1, distinct col - row)."""
    n = int(bp.row_ptr.shape[0] - 1)
    rows = np.repeat(np.arange(n), np.diff(bp.row_ptr))
    d = bp.col_idx.astype(np.int64) - rows
    ns = (n + 63) // 64
    pairs = np.unique(np.stack([rows // 64, d]), axis=1)
    return int(64 * np.maximum(np.bincount(pairs[0], minlength=ns), 1).sum())


def test_batch_format_choice():
    """Stencil systems get the copy by diagonals (its entry count as counted
    here); format "csr" keeps the CSR arrays; rows stored out of column order
    rule the copy out."""
    import torch

    from paper_1809_05805_amd.native import BatchSolver

    bp = SMALL
    log("batch format choice")
    s = solver(bp)
    fmt, stored = s.format()
    assert fmt == "sell64_diag" and stored == batch_diag_entries(bp)
    assert solver(bp, fmt="csr").format() == ("csr", int(bp.col_idx.shape[0]))
    # reverse the entries of one row of system 3
    ci, va = bp.col_idx.copy(), bp.vals.copy()
    r = int(bp.row_off[3]) + 5
    a, b = bp.row_ptr[r], bp.row_ptr[r + 1]
    ci[a:b], va[a:b] = ci[a:b][::-1].copy(), va[a:b][::-1].copy()
    t = BatchSolver(bp.row_off, torch.from_numpy(bp.row_ptr).cuda(), torch.from_numpy(ci).cuda(),
                    torch.from_numpy(va).cuda(), bp.m)
    assert t.format()[0] == "csr"


@pytest.mark.parametrize("scheme,config", [("mgs1r", (256, 0, 1, 0)), ("mgs1r", (1024, 0, 1, 256)),
                                           ("mgs1r_ir32", (512, 0, 1, 256))])
def test_batch_formats_bitwise(scheme, config):
    """The copy by diagonals and the CSR arrays give the same bits: iterates
    and iteration counts of a whole batch solved to tolerance, with one-part
    systems and with teams (whose parts gather across part boundaries)."""
    log(f"batch formats {scheme} {config}")
    outs = []
    for fmt in ("csr", None):
        rc, info, x, s = run(SMALL, scheme, config=config, fmt=fmt)
        assert rc == 0 and np.all(info["converged"] == 1)
        outs.append((x, info["iters"], s.format()[0]))
    assert outs[0][2] == "csr" and outs[1][2] == "sell64_diag"
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][0], outs[1][0])


def test_batch_storage_calls():
    """The raw entry points: the planned size, refusals, going back to the CSR
    arrays, and a captured graph discarded by either call."""
    import torch

    from paper_1809_05805_amd import native

    bp = SMALL
    log("batch storage calls")
    stream = torch.cuda.Stream()  # a graph is captured from a stream of its own
    s = solver(bp, stream=stream, fmt="csr")
    rc, nb = native.gmres_batch_matrix_storage_bytes(s.ctx)
    total = batch_diag_entries(bp)
    ns = (bp.n + 63) // 64
    up = lambda v: (v + 255) // 256 * 256
    assert rc == 0 and nb == up(up(8 * (ns + 1)) + 4 * (total // 64)) + 8 * total
    buf = torch.empty(nb + 512, dtype=torch.uint8, device="cuda")
    bp_ = buf.data_ptr() + (-buf.data_ptr()) % 256
    assert native.gmres_batch_set_matrix_storage(s.ctx, bp_, nb - 8) == native.GMRES_ERR_ARG
    assert native.gmres_batch_set_matrix_storage(s.ctx, bp_ + 8, nb) == native.GMRES_ERR_ARG
    host = np.zeros(nb // 8 + 64)
    assert native.gmres_batch_set_matrix_storage(s.ctx, host.ctypes.data, nb) == native.GMRES_ERR_ARG
    assert s.format()[0] == "csr"
    bt = torch.from_numpy(bp.b).cuda()
    x = torch.zeros(bp.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.capture(bt, x, TOL, 20000)
    assert native.gmres_batch_set_matrix_storage(s.ctx, bp_, nb) == native.GMRES_OK
    assert native.gmres_batch_replay(s.ctx) == native.GMRES_ERR_ARG
    assert s.format() == ("sell64_diag", total)
    with torch.cuda.stream(stream):
        rc, info = s.solve(bt, x, TOL, 20000)
    torch.cuda.synchronize()
    assert rc == 0 and np.all(info["converged"] == 1)
    assert native.gmres_batch_set_matrix_storage(s.ctx, None, 0) == native.GMRES_OK
    assert s.format()[0] == "csr"
