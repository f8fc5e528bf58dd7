#!/usr/bin/env python3
"""Benchmark: one-reduce MGS-GMRES vs level-1 MGS-GMRES (and CGS2) on one MI355X.

A step is one complete restarted GMRES(50) solve of the 3D 7-point upwind
convection-diffusion system on a 128^3 grid (n = 2,097,152, 14,581,760
nonzeros, wind (1, 0.5, 0.25), Peclet 50) from x0 = 0 to a true relative
residual of 1e-10: restart residuals, every Arnoldi step (SpMV, projection with
its device-wide reduction, small dense step, MAXPY), convergence checks and
cycle-end solution updates all run in the HIP library. Inputs are synthetic
and seeded and sit in HBM before timing starts.

Prints one JSON line. value = Arnoldi iterations per second of the one-reduce
solve. The roofline object covers the dominant kernel (by summed time), timed
with HIP events attached to its dispatches on the library's stream during the
last solve of the timed region; its bytes are the method's algorithmic bytes
per launch (the CSR arrays, the SpMV's u and w, the projection's basis
columns). Beside the headline the same JSON line reports, on this GPU:
- the same solve with the rotations batched two steps at a time (depth 2);
- the plain MGS, CGS2, re-orthogonalized CGS and two-synchronization CGS
  solves of the same system;
- the float32- and bfloat16-basis refinement on this system and on the 3D
  7-point 256^3 precision workload (GMRES(40) to 1e-10);
- the loss-of-orthogonality study on the row-scaled 27-point 100^3 system
  (every scheme, ||I - V^T V|| and Paige's ||S|| per iteration);
- the latency-bound 2D 64^2 system (microseconds per step);
- the batched solver on 512 uneven 2D systems;
- achievable read and copy rates from the project's own probe kernels;
- the CPU oracle on the host's cores (OpenMP timing build) and on one.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
WORKLOAD = "3D 7-point upwind convection-diffusion 128^3 (wind (1,0.5,0.25), Peclet 50), GMRES(50) to 1e-10"


KERNEL_NAMES = {"step": "k_fused", "maxpy": "k_maxpy", "spmv": "k_spmv"}
KERNEL_LABELS = {"step": "k_fused (projection + device-wide reduction + small dense step, SpMV "
                         "fused unless launched on its own)",
                 "maxpy": "k_maxpy", "spmv": "k_spmv (CSR SpMV launched on its own)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counted_traffic(kernel: str):
    """HBM bytes per launch from the committed counter summary, or None once the
    kernel source differs from the one the counters were taken on."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "k_fused_convdiff128_hbm_counters.md")
    src = os.path.join(ROOT, "paper_1809_05805_amd", "csrc", "gmres_device.hip")
    try:
        text = open(path).read()
        now = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    m = re.search(r"kernel_sha256_16 = ([0-9a-f]{16})", text)
    v = re.search(rf"{kernel}_traffic_bytes_per_launch = (\d+)", text)
    if not m or not v or m.group(1) != now:
        return None
    return int(v.group(1))


def time_solves(solver, b, x, rtol, max_iters, steps, warmup, timing=False, timed_runs=3):
    """Time `steps` solves after `warmup` untimed ones, with no per-launch
    events. With timing, `timed_runs` further solves carry HIP events attached
    to each step-kernel dispatch (they add a few microseconds per launch, and
    now and then a solve's step kernels read several microseconds long); the
    per-kernel figures of the solve with the median event total are returned."""
    import torch

    res = None
    for _ in range(warmup):
        x.zero_()
        res = solver.solve(b, x, rtol, max_iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for i in range(steps):
        x.zero_()
        res = solver.solve(b, x, rtol, max_iters)
        iters += res.iters
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = None
    if timing:
        runs = []
        for _ in range(timed_runs):
            solver.set_timing(True)
            x.zero_()
            solver.solve(b, x, rtol, max_iters)
            runs.append(solver.timing())
            solver.set_timing(False)
        runs.sort(key=lambda t: sum(v["ms"] for v in t.values()))
        kt = runs[len(runs) // 2]
    return dt, iters, res, kt


PROBE_KINDS = {"read": 0, "read_nt": 1, "copy": 2, "copy_nt": 3, "read_tiled": 4, "read_tiled_nt": 5,
               "copy_tiled": 6, "copy_tiled_nt": 7}


def measured_ceilings(dev, mib=2048, reps=5):
    """Achievable HBM rates of this GPU from the project's own probe kernels
    (libgmres_probe.so): streaming 16-byte reads of a `mib` MiB buffer, and
    copies of half of it into a second buffer, each buffer at least 4x the
    256 MB last-level cache; the best over launch sizes and plain or
    non-temporal loads (stores), reported beside the 8 TB/s peak."""
    import ctypes

    import torch

    from paper_1809_05805_amd import build_native

    lib = ctypes.CDLL(build_native.PROBE_LIB)
    f = lib.gmres_probe_bandwidth
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]
    nbytes = mib * 2**20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty(nbytes // 16, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    table = {}
    for name, kind in PROBE_KINDS.items():
        # reads move the buffer; copies read half of it and write as much
        size = nbytes if kind in (0, 1, 4, 5) else nbytes // 2
        moved = nbytes
        for blocks in (1024, 4096, 8192):
            ms = ctypes.c_float()
            rc = f(kind, src.data_ptr(), dst.data_ptr(), size, blocks, reps, stream, ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"gmres_probe_bandwidth({name}, {blocks}) failed: {rc}")
            table[f"{name}_{blocks}"] = round(moved * reps / (ms.value * 1e-3) / 1e9, 1)
    del src, dst
    read = max(v for k, v in table.items() if k.startswith("read"))
    copy = max(v for k, v in table.items() if k.startswith("copy"))
    return {"read_GBps": read, "copy_GBps": copy, "buffer_MiB": mib, "probes": table,
            "how": f"own HIP probe kernels (gmres_probe.hip): reads of a {mib} MiB float64 buffer and "
                   f"copies of {mib // 2} MiB into a second buffer, 16-byte vectors, 256-thread "
                   "workgroups, grid-stride or tiled (each workgroup streaming one contiguous chunk), "
                   "best of 1024-8192 workgroups and of plain or non-temporal loads/stores, "
                   f"{reps} timed launches each after one untimed"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, m):
    """The oracle on the host cores: its OpenMP timing build (the same
    arithmetic per row; length-n loops on all threads the process may use,
    OMP_NUM_THREADS or else the affinity set) for restart cycles of the same
    system until about 4 s have passed, then one cycle on a single thread."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    oracle.omp_threads(threads)
    oracle.solve(p.row_ptr, p.col_idx, p.vals, p.b, p.x0, m, "mgs1r", 0.0, 2, acc="openmp")
    its, dt = 0, 0.0
    while dt < 4.0 and its < 20 * m:
        t0 = time.perf_counter()
        r = oracle.solve(p.row_ptr, p.col_idx, p.vals, p.b, p.x0, m, "mgs1r", 0.0, m, acc="openmp")
        dt += time.perf_counter() - t0
        its += r.iters
    oracle.omp_threads(1)
    t0 = time.perf_counter()
    r1 = oracle.solve(p.row_ptr, p.col_idx, p.vals, p.b, p.x0, m, "mgs1r", 0.0, m, acc="openmp")
    dt1 = time.perf_counter() - t0
    oracle.omp_threads(threads)
    return {"value": its / dt, "unit": "Arnoldi iters/s", "cores": threads, "kind": "oracle",
            "sample": f"{its // m} {m}-column restart cycles (one-reduce scheme, no early exit) of the "
                      f"same system from x0=0 on {threads} threads: {its} iterations in {dt:.2f} s; "
                      "the oracle's OpenMP timing build (its sequential build is the parity reference)",
            "one_thread_iters_per_s": r1.iters / dt1,
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(),
                     "affinity_cpus": len(os.sched_getaffinity(0)), "threads_used": threads}}


def kernel_table(kt, ms_per_solve):
    out = {}
    for name, st in kt.items():
        if st["launches"]:
            out[name] = {"launches": st["launches"], "avg_us": st["ms"] / st["launches"] * 1e3,
                         "avg_bytes": st["bytes"] / st["launches"],
                         "GBps": st["bytes"] / (st["ms"] * 1e-3) / 1e9,
                         "time_share": st["ms"] / ms_per_solve}
    return out


def ir32_result(args, p, rp, ci, va, b, x, x64, s64_per_solve, iters64, scheme="mgs1r_ir32"):
    """A reduced-precision-basis scheme (float32, or the bfloat16 experiment)
    on the same system and tolerance: speed, and its solution's error against
    the float64 one and against x_true."""
    import numpy as np
    import torch

    from paper_1809_05805_amd.native import GmresSolver

    s = GmresSolver(rp, ci, va, p.m, scheme)
    k = max(1, min(args.steps, 5))
    dt, iters, res, kt = time_solves(s, b, x, p.rtol, args.max_iters, k, 1, timing=True)
    xr = x.cpu().numpy()
    A = p.scipy()
    rel_res = float(np.linalg.norm(p.b - A @ xr) / np.linalg.norm(p.b))
    x64n = x64.cpu().numpy()
    err64 = float(np.linalg.norm(xr - x64n) / np.linalg.norm(x64n))
    errt = float(np.linalg.norm(xr - p.x_true) / np.linalg.norm(p.x_true))
    err64t = float(np.linalg.norm(x64n - p.x_true) / np.linalg.norm(p.x_true))
    log(f"{scheme}: {iters / k:.0f} iters/solve, {dt / k * 1e3:.2f} ms/solve, rel_res {rel_res:.2e}, "
        f"err vs fp64 {err64:.2e}")
    s.close()
    basis = "float32" if scheme == "mgs1r_ir32" else "bfloat16 (float32 arithmetic)"
    return {"scheme": f"one-reduce on a {basis} basis, float64 refinement at every restart",
            "m": p.m, "iters_per_s": round(iters / dt, 2), "ms_per_solve": round(dt / k * 1e3, 3),
            "iters_per_solve": iters // k, "fp64_iters_per_solve": iters64,
            "speedup_vs_fp64_solve": round(s64_per_solve / (dt / k), 3),
            "converged": bool(res.converged), "rel_res_true_fp64_recomputed": rel_res,
            "err_vs_fp64_solution": err64, "err_vs_x_true": errt, "fp64_err_vs_x_true": err64t,
            "kernels": kernel_table(kt, dt / k * 1e3)}


def precision_config(args):
    """The 256^3 precision workload: float64 one-reduce GMRES(40) vs the
    FP32-basis scheme at 1e-10, one solve each after a warm-up."""
    import numpy as np
    import torch

    from paper_1809_05805_amd import problems
    from paper_1809_05805_amd.native import GmresSolver

    t0 = time.perf_counter()
    p = problems.make_config("convdiff3d", N=args.precision_N)
    log(f"precision config n={p.n} nnz={p.nnz} built in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (p.row_ptr, p.col_idx, p.vals))
    b = torch.from_numpy(p.b).to(dev)
    x = torch.zeros(p.n, dtype=torch.float64, device=dev)
    out = {"workload": f"3D 7-point upwind convection-diffusion {args.precision_N}^3, GMRES(40) to 1e-10",
           "n": p.n, "nnz": p.nnz}
    sols = {}
    A = p.scipy()
    for scheme in ("mgs1r", "mgs1r_ir32", "mgs1r_ir16"):
        s = GmresSolver(rp, ci, va, 40, scheme)
        dt, iters, res, kt = time_solves(s, b, x, 1e-10, args.max_iters, 1, 1, timing=True,
                                         timed_runs=1)
        sols[scheme] = x.cpu().numpy()
        rel_res = float(np.linalg.norm(p.b - A @ sols[scheme]) / np.linalg.norm(p.b))
        out[scheme] = {"iters_per_s": round(iters / dt, 2), "ms_per_solve": round(dt * 1e3, 3),
                       "iters": iters, "converged": bool(res.converged),
                       "rel_res_true_fp64_recomputed": rel_res,
                       "err_vs_x_true": float(np.linalg.norm(sols[scheme] - p.x_true) /
                                              np.linalg.norm(p.x_true)),
                       "kernels": kernel_table(kt, dt * 1e3)}
        log(f"precision {scheme}: {iters} iters, {dt * 1e3:.1f} ms, rel_res {rel_res:.2e}")
        s.close()
    out["mgs1r_ir32"]["err_vs_fp64_solution"] = float(
        np.linalg.norm(sols["mgs1r_ir32"] - sols["mgs1r"]) / np.linalg.norm(sols["mgs1r"]))
    out["mgs1r_ir16"]["err_vs_fp64_solution"] = float(
        np.linalg.norm(sols["mgs1r_ir16"] - sols["mgs1r"]) / np.linalg.norm(sols["mgs1r"]))
    out["speedup_vs_fp64_solve"] = round(out["mgs1r"]["ms_per_solve"] / out["mgs1r_ir32"]["ms_per_solve"], 3)
    out["bf16_speedup_vs_fp64_solve"] = round(out["mgs1r"]["ms_per_solve"] / out["mgs1r_ir16"]["ms_per_solve"], 3)
    return out


def orth_study(args):
    """Stability study: loss of orthogonality per Arnoldi step for every
    Gram-Schmidt scheme on the row-scaled 27-point system (rows scaled
    log-uniformly over eight decades, kappa ~ 1e8): one 100-column cycle from
    x0 = 0 per scheme; ||I - V_k^T V_k||_2 of the GPU's own basis for the
    leading k columns (Gram matrix formed on the GPU, norms on the host), and
    Paige's ||S_k||_2 from the T or L the device built, where the scheme forms
    one. Each scheme's cycle is also timed (after a warm-up, without the
    host-side S history)."""
    import numpy as np
    import torch

    from paper_1809_05805_amd import problems
    from paper_1809_05805_amd.native import GmresSolver

    m = 100
    p = problems.make_config("stencil27", N=args.orth_study_N)
    dev = torch.device("cuda:0")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (p.row_ptr, p.col_idx, p.vals))
    b = torch.from_numpy(p.b).to(dev)
    out = {"workload": f"27-point stencil {args.orth_study_N}^3, off-diagonals N(0,1)/27, rows scaled "
                       "by 10^(8 U(0,1)); one GMRES(100) cycle from x0 = 0", "n": p.n, "m": m}
    marks = [10, 20, 40, 60, 80, 100]
    for scheme in ("mgs", "mgs1r", "cgs2", "cgs2_3r", "two_synch"):
        s = GmresSolver(rp, ci, va, m, scheme)
        x = torch.zeros(p.n, dtype=torch.float64, device=dev)
        s.solve(b, x, 0.0, m)  # warm-up, then one timed cycle without the host-side S history
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve(b, x, 0.0, m)
        dt = time.perf_counter() - t0
        # per-kernel rates from a separate cycle with HIP events on each dispatch
        x.zero_()
        s.set_timing(True)
        s.solve(b, x, 0.0, m)
        kt = s.timing()
        s.set_timing(False)
        kernels = {name: {"launches": st["launches"], "avg_us": round(st["ms"] / st["launches"] * 1e3, 2),
                          "GBps": round(st["bytes"] / (st["ms"] * 1e-3) / 1e9, 1)}
                   for name, st in kt.items() if st["launches"]}
        x.zero_()
        r = s.solve(b, x, 0.0, m, orth=True)
        _, _, _, j = s.last_cycle()
        V = s.basis()[:, :j]
        G = (V.t() @ V).cpu().numpy()
        loss = [float(np.linalg.norm(np.eye(k) - G[:k, :k], 2)) for k in range(1, j + 1)]
        rec = {"columns": j, "orth_loss_at": {str(k): loss[k - 1] for k in marks if k <= j},
               "relative_residual_after_cycle": r.rel_res_true,
               "iters_per_s": round(r.iters / dt, 1), "ms_per_cycle": round(dt * 1e3, 2),
               "reductions": r.reductions, "kernels": kernels}
        if r.orth is not None and np.all(np.isfinite(r.orth)):
            rec["paige_s_at"] = {str(k): float(r.orth[k - 1]) for k in marks if k <= len(r.orth)}
            rec["paige_s_per_iteration"] = [float(v) for v in r.orth]
        rec["orth_loss_per_iteration"] = loss
        out[scheme] = rec
        log(f"orth study {scheme}: {r.iters / dt:.0f} iters/s, ||I - V^T V|| at k=10..100: "
            + " ".join(f"{loss[k - 1]:.1e}" for k in marks if k <= j) + " | "
            + " ".join(f"{k}: {v['avg_us']:.1f} us {v['GBps']:.0f} GB/s" for k, v in kernels.items()))
        s.close()
        del V, x
    # the one-reduce cycle with the rotations batched two steps at a time
    s = GmresSolver(rp, ci, va, m, "mgs1r", pipeline_depth=2)
    x = torch.zeros(p.n, dtype=torch.float64, device=dev)
    s.solve(b, x, 0.0, m)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.solve(b, x, 0.0, m)
    dt = time.perf_counter() - t0
    out["mgs1r_pipeline_depth_2"] = {"iters_per_s": round(r.iters / dt, 1),
                                     "ms_per_cycle": round(dt * 1e3, 2), "reductions": r.reductions}
    s.close()
    return out


def small_config(args):
    """The 2D 5-point 64^2 system (n = 4,096, GMRES(30), rtol 1e-8): it sits in
    the caches, so every step is latency-bound. Per scheme: one-cycle solves
    with a fixed budget of 30 and of 10 columns (no early exit), timed over
    many repetitions; the difference over the 20 extra columns gives the
    marginal microseconds per step (columns 10..29, around k = m/2), the
    30-column solve divided by 30 the whole-cycle rate. Then the solve to
    1e-8."""
    import numpy as np
    import torch

    from paper_1809_05805_amd import problems
    from paper_1809_05805_amd.native import GmresSolver

    p = problems.make_config("convdiff2d")
    dev = torch.device("cuda:0")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (p.row_ptr, p.col_idx, p.vals))
    b = torch.from_numpy(p.b).to(dev)
    x = torch.zeros(p.n, dtype=torch.float64, device=dev)
    out = {"workload": "2D 5-point upwind convection-diffusion 64^2 (wind (1,1), Peclet 10), GMRES(30)",
           "n": p.n, "nnz": p.nnz, "m": p.m, "rtol": p.rtol}
    reps = 60

    def cycle_time(s, cols):
        x.zero_()
        s.solve(b, x, 0.0, cols)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            x.zero_()
            s.solve(b, x, 0.0, cols)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    for scheme in ("mgs1r", "mgs", "cgs2"):
        s = GmresSolver(rp, ci, va, p.m, scheme)
        t30, t10 = cycle_time(s, p.m), cycle_time(s, 10)
        dt, iters, res, _ = time_solves(s, b, x, p.rtol, args.max_iters, 20, 2)
        err = float(np.linalg.norm(x.cpu().numpy() - p.x_true) / np.linalg.norm(p.x_true))
        out[scheme] = {"us_per_step_marginal": round((t30 - t10) / (p.m - 10) * 1e6, 2),
                       "us_per_step_whole_cycle": round(t30 / p.m * 1e6, 2),
                       "solve_ms": round(dt / 20 * 1e3, 3), "iters_per_solve": iters // 20,
                       "converged": bool(res.converged), "rel_res_true": res.rel_res_true,
                       "err_vs_x_true": err, "reductions_per_solve": res.reductions}
        log(f"64^2 {scheme}: {out[scheme]['us_per_step_marginal']:.1f} us/step marginal, "
            f"solve {out[scheme]['solve_ms']:.2f} ms ({iters // 20} iters)")
        s.close()
    for base in ("mgs", "cgs2"):
        out[f"one_reduce_speedup_per_step_vs_{base}"] = round(
            out[base]["us_per_step_marginal"] / out["mgs1r"]["us_per_step_marginal"], 3)
    return out


# The paper's own GPU timings (Section V-B, the Parabolic FEM timing table),
# for context only: other hardware, another matrix, a preconditioner, and no
# one-reduce scheme among them. Orth is the Gram-Schmidt time of a solve.
PAPER_CONTEXT = {
    "note": "context on other hardware, not a target; the paper times no one-reduce step",
    "source": "Section V-B, Parabolic FEM timing table",
    "hardware": "NVIDIA P100 16 GB HBM2 (Summit-Dev), CUDA 9.0, FP64",
    "workload": "Parabolic FEM n=525,825 nnz=3,674,625, BoomerAMG-preconditioned GMRES(72) to 1e-13, "
                "78 iterations",
    "orth_s_per_solve": {"level1_mgs_hypre": 0.95, "level1_mgs_device": 0.25, "cgs2_alg1": 0.14,
                         "two_synch_alg3": 0.12},
    "orth_ms_per_iteration": {"level1_mgs_hypre": 12.18, "level1_mgs_device": 3.21, "cgs2_alg1": 1.79,
                              "two_synch_alg3": 1.54},
}

BATCH_WORKLOAD = ("512 independent 2D 5-point upwind convection-diffusion systems, grid side "
                  "U{32..256} (n 1,024-65,536), Peclet U(1,100), wind angle U(0,2pi), GMRES(30) to 1e-10")
BATCH3D_WORKLOAD = ("64 independent 3D 7-point upwind convection-diffusion systems, grid side "
                    "U{32..64} (n 32,768-262,144), Peclet U(1,50), wind (cos t, sin t, 1/2) with "
                    "t U(0,2pi), GMRES(50) to 1e-10: about 3.1 GB of float64 basis in use at once, "
                    "12x the 256 MB last-level cache")


def batch_bytes(info, sizes, nnz_sys, m, vb):
    """Algorithmic HBM bytes of a batched solve from each system's iteration and
    cycle counts (cycles taken full but the last). Per Arnoldi step k: A, the
    projection's read of V[:,0:k+1], w written; MAXPY's read of V[:,0:k+1] and w
    and its two column writes; per cycle the norm-only step, the x update and
    the restart residual. vb: bytes per basis entry (8 or 4)."""
    import numpy as np

    total = 0.0
    for it, cyc, n, nnz in zip(info["iters"], info["cycles"], sizes, nnz_sys):
        A = 12.0 * nnz + 4.0 * (n + 1)
        full = max(int(cyc) - 1, 0)
        js = [m] * full + [int(it) - m * full] if cyc else []
        for j in js:
            k = np.arange(j)
            total += j * A + vb * n * float(np.sum(2 * (k + 1) + 4))       # steps
            total += vb * n + 8.0 * n * j + 16.0 * n + A + 24.0 * n        # norm step, x update, restart
        total += A + 24.0 * n                                              # the final residual check
    return total


def batch_result(args, dim=2):
    """The batched form: one persistent launch per solve of the whole batch,
    float64 and float32 basis, each with the autotuned launch configuration,
    against single-system float64 solves of a stratified sample run one by one.
    dim 2: the 512-system batch; dim 3: the 64-system 3D batch whose bases far
    exceed the last-level cache."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    from paper_1809_05805_amd import problems
    from paper_1809_05805_amd.native import BatchSolver, GmresSolver

    t0 = time.perf_counter()
    bp = problems.make_batch(nsys=args.batch_systems) if dim == 2 else problems.make_batch3d()
    tag = "batch" if dim == 2 else "batch3d"
    log(f"{tag}: {bp.nsys} systems, n={bp.n} nnz={bp.nnz}, built in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (bp.row_ptr, bp.col_idx, bp.vals))
    b = torch.from_numpy(bp.b).to(dev)
    A = sp.csr_matrix((bp.vals, bp.col_idx, bp.row_ptr), shape=(bp.n, bp.n))
    sizes = np.diff(bp.row_off)
    nnz_sys = bp.row_ptr[bp.row_off[1:]].astype(np.int64) - bp.row_ptr[bp.row_off[:-1]]
    bnorm = np.sqrt(np.add.reduceat(bp.b ** 2, bp.row_off[:-1]))
    if dim == 3:
        workload = BATCH3D_WORKLOAD
    else:
        workload = BATCH_WORKLOAD if args.batch_systems == 512 else f"{bp.nsys} systems"
    out = {"workload": workload, "systems": bp.nsys, "rows": bp.n, "nnz": bp.nnz, "m": bp.m,
           "rtol": bp.rtol}
    for scheme, key, vb in (("mgs1r", "fp64", 8), ("mgs1r_ir32", "fp32_basis", 4)):
        s = BatchSolver(bp.row_off, rp, ci, va, bp.m, scheme)
        x = torch.zeros(bp.n, dtype=torch.float64, device=dev)
        trials = []
        if args.batch_config:
            s.set_config(*(int(v) for v in args.batch_config.split(",")))
        elif not args.no_batch_autotune:
            trials = s.autotune(b, x, bp.rtol, args.max_iters)
        cfg = s.config()
        times = []
        for rep in range(1 + args.batch_steps):
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, info = s.solve(b, x, bp.rtol, args.max_iters)
            times.append(time.perf_counter() - t)
        dt = float(np.mean(times[1:]))
        xs = x.cpu().numpy()
        res = np.sqrt(np.add.reduceat((bp.b - A @ xs) ** 2, bp.row_off[:-1])) / bnorm
        iters = int(info["iters"].sum())
        nbytes = batch_bytes(info, sizes, nnz_sys, bp.m, vb)
        out[key] = {"iters_per_s": round(iters / dt, 1), "ms_per_solve": round(dt * 1e3, 2),
                    "iters": iters, "max_iters_one_system": int(info["iters"].max()),
                    "all_converged": bool(np.all(info["converged"] == 1)) and rc == 0,
                    "worst_rel_res_true_fp64_recomputed": float(res.max()),
                    "algorithmic_GBps": round(nbytes / dt / 1e9, 1),
                    "config": cfg,
                    "spmv_format": s.format()[0],
                    "autotune_trials": [{"block_size": t[0], "grid": t[1],
                                         "order": "largest_first" if t[2] else "natural",
                                         "part_rows": t[4], "streamed": bool(t[5]),
                                         "ms": round(t[3], 2)} for t in trials]}
        log(f"{tag} {scheme}: {iters} iters in {dt * 1e3:.1f} ms ({iters / dt:.0f} it/s), cfg {cfg}, "
            f"worst rel res {res.max():.2e}")
        s.close()
        del x
    # single-system float64 solves, one after another, on systems spread over the sizes
    order = np.argsort(sizes, kind="stable")
    sample = order[np.linspace(0, bp.nsys - 1, min(16 if dim == 2 else 8, bp.nsys)).astype(int)]
    it_s, t_s = 0, 0.0
    for i in sample:
        p = bp.system(int(i))
        r2, c2, v2 = (torch.from_numpy(a).to(dev) for a in (p.row_ptr, p.col_idx, p.vals))
        g = GmresSolver(r2, c2, v2, bp.m, "mgs1r")
        bb = torch.from_numpy(p.b).to(dev)
        xx = torch.zeros(p.n, dtype=torch.float64, device=dev)
        g.solve(bb, xx, bp.rtol, args.max_iters)
        xx.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = g.solve(bb, xx, bp.rtol, args.max_iters)
        t_s += time.perf_counter() - t
        it_s += r.iters
        g.close()
    seq = it_s / t_s
    out["sequential_fp64"] = {"iters_per_s": round(seq, 1), "iters": it_s, "seconds": round(t_s, 3),
                              "sample": f"{len(sample)} systems evenly spread over the sorted sizes, "
                                        "each solved alone by the single-system float64 path"}
    out["fp64_speedup_vs_sequential"] = round(out["fp64"]["iters_per_s"] / seq, 2)
    out["fp32_basis_speedup_vs_sequential"] = round(out["fp32_basis"]["iters_per_s"] / seq, 2)
    log(f"{tag}: sequential sample {seq:.0f} it/s")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128, help="grid side (default: the 128^3 workload)")
    ap.add_argument("--max-iters", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-baselines", action="store_true", help="skip the MGS and CGS2 solves")
    ap.add_argument("--no-ir32", action="store_true", help="skip the FP32-basis solve")
    ap.add_argument("--precision-N", type=int, default=256,
                    help="the float64 vs float32- and bfloat16-basis comparison on an N^3 system "
                         "(default 256: the precision workload; 0 skips it)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a reference kernel "
                         "for hardware byte counters)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solver section")
    ap.add_argument("--no-batch3d", action="store_true",
                    help="skip the 3D batch whose bases exceed the last-level cache")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the device copy and sum rates reported beside the peak")
    ap.add_argument("--orth-study-N", type=int, default=100,
                    help="the loss-of-orthogonality study of every scheme on the row-scaled 27-point "
                         "N^3 system (default 100: its full size; 0 skips it)")
    ap.add_argument("--no-small", action="store_true", help="skip the latency-bound 64^2 system")
    ap.add_argument("--no-batch-autotune", action="store_true",
                    help="batched solves with the default launch configuration")
    ap.add_argument("--batch-systems", type=int, default=512)
    ap.add_argument("--batch-config", type=str, default="",
                    help="block_size,grid,order,part_rows for the batched solves instead of autotuning")
    ap.add_argument("--batch-steps", type=int, default=2, help="timed batched solves per scheme")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver is built and measured for a single "
              "MI355X; a multi-GPU (row-sharded) run is not part of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1809_05805_amd import problems
    from paper_1809_05805_amd.native import GmresSolver

    p = problems.make_config("convdiff3d", N=args.N)
    n, nnz, m, rtol = p.n, p.nnz, p.m, p.rtol
    log(f"workload n={n} nnz={nnz} m={m} rtol={rtol}")
    dev = torch.device("cuda:0")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (p.row_ptr, p.col_idx, p.vals))
    b = torch.from_numpy(p.b).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib * 2**20 // 8
        src = torch.ones(nb, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t0 = time.perf_counter()
    s1 = GmresSolver(rp, ci, va, m, "mgs1r")
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    fmt, stored = s1.format()
    dt, iters, res, kt = time_solves(s1, b, x, rtol, args.max_iters, args.steps, args.warmup,
                                     timing=True)
    err = float(torch.linalg.norm(x.cpu() - torch.from_numpy(p.x_true)) / np.linalg.norm(p.x_true))
    log(f"mgs1r: {iters / args.steps:.0f} iters/solve, {dt / args.steps * 1e3:.2f} ms/solve, "
        f"converged={res.converged} rel_res={res.rel_res_true:.3e} err={err:.2e}")
    kernels = {}
    for name, st in kt.items():
        if st["launches"]:
            avg_us = st["ms"] / st["launches"] * 1e3
            gbps = st["bytes"] / (st["ms"] * 1e-3) / 1e9
            kernels[name] = {"launches": st["launches"], "avg_us": avg_us,
                             "avg_bytes": st["bytes"] / st["launches"], "GBps": gbps,
                             "time_share": st["ms"] / (dt * 1e3 / args.steps)}
    dom = max(kernels, key=lambda k: kt[k]["ms"])
    d = kernels[dom]
    roofline = {"bound": "hbm", "achieved": round(d["GBps"], 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(d["GBps"] / HBM_PEAK_GBPS, 4),
                "traffic": counted_traffic(KERNEL_NAMES[dom]),
                "kernel": KERNEL_LABELS[dom],
                "bytes_per_launch": round(d["avg_bytes"]), "avg_us": round(d["avg_us"], 2),
                "bytes_model": "per step k with its SpMV: 12 nnz + 4 (n+1) (the CSR arrays) + 16 n (u "
                               "read, w written) + 8 n (k+1) (V[:,0:k+1] read); the cycle's norm-only "
                               "step: 8 n (u read)"}
    arnoldi_bytes = sum(kt[k]["bytes"] for k in kt)
    out = {
        "metric": "Arnoldi iters/s + achieved HBM GB/s, one-reduce vs plain GMRES at 1e-10 residual",
        "value": round(iters / dt, 2),
        "unit": "Arnoldi iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": n, "nnz": nnz, "m": m, "rtol": rtol,
                   "scheme": "one-reduce lagged compact-WY MGS", "iters_per_solve": iters // args.steps,
                   "converged": bool(res.converged), "rel_res_true": res.rel_res_true,
                   "reductions_per_solve": res.reductions, "spmv_format": fmt,
                   "stored_matrix_entries": stored, "setup_ms": round(setup_ms, 2)},
        # step-kernel bytes of the instrumented solve over the mean solve time
        "hbm_GBps_arnoldi": round(arnoldi_bytes / (dt / args.steps) / 1e9, 1),
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_ceilings and not args.copy_calibration_mib:
        # (a counter run keeps its one calibration copy the only large copy)
        ceil = measured_ceilings(dev)
        ceil["dominant_kernel_frac_of_read"] = round(d["GBps"] / ceil["read_GBps"], 4)
        if "maxpy" in kernels:
            ceil["maxpy_frac_of_copy"] = round(kernels["maxpy"]["GBps"] / ceil["copy_GBps"], 4)
        out["measured_ceilings"] = ceil
        log(f"ceilings: copy {ceil['copy_GBps']:.0f} GB/s, read {ceil['read_GBps']:.0f} GB/s")
    x64 = x.clone()
    # the same solve with the rotations and stopping test batched two steps at a time
    sd = GmresSolver(rp, ci, va, m, "mgs1r", pipeline_depth=2)
    kd = max(1, min(args.steps, 5))
    dtd, itd, rd, _ = time_solves(sd, b, x, rtol, args.max_iters, kd, 1)
    out["pipeline_depth_2"] = {"iters_per_s": round(itd / dtd, 2), "ms_per_solve": round(dtd / kd * 1e3, 3),
                               "iters_per_solve": itd // kd, "reductions_per_solve": rd.reductions,
                               "converged": bool(rd.converged)}
    log(f"mgs1r depth 2: {itd / kd:.0f} iters/solve, {dtd / kd * 1e3:.2f} ms/solve, {rd.reductions} reductions")
    sd.close()
    if not args.no_ir32:
        out["fp32_ir"] = ir32_result(args, p, rp, ci, va, b, x, x64, dt / args.steps, res.iters)
        out["bf16_ir"] = ir32_result(args, p, rp, ci, va, b, x, x64, dt / args.steps, res.iters,
                                     scheme="mgs1r_ir16")
    if args.precision_N:
        out["fp32_ir_precision_config"] = precision_config(args)
    if not args.no_baselines:
        for scheme in ("mgs", "cgs2", "cgs2_3r", "two_synch"):
            sv = GmresSolver(rp, ci, va, m, scheme)
            dt2, it2, r2, _ = time_solves(sv, b, x, rtol, args.max_iters, max(1, min(args.steps, 3)),
                                          1)
            k2 = max(1, min(args.steps, 3))
            out[f"{scheme}_baseline"] = {"iters_per_s": round(it2 / dt2, 2),
                                         "ms_per_solve": round(dt2 / k2 * 1e3, 3),
                                         "iters_per_solve": it2 // k2, "converged": bool(r2.converged),
                                         "reductions_per_solve": r2.reductions}
            log(f"{scheme}: {it2 / k2:.0f} iters/solve, {dt2 / k2 * 1e3:.2f} ms/solve")
            sv.close()
        out["speedup_vs_mgs"] = round(out["value"] / out["mgs_baseline"]["iters_per_s"], 3)
        # this GPU's whole Arnoldi iteration (SpMV included) per scheme, beside the paper's figures
        here = {s2: round(1e3 / out[f"{s2}_baseline"]["iters_per_s"], 4)
                for s2 in ("mgs", "cgs2", "cgs2_3r", "two_synch")}
        here["mgs1r"] = round(1e3 / out["value"], 4)
        out["paper_context"] = dict(PAPER_CONTEXT, this_gpu_ms_per_iteration=here,
                                    this_gpu_workload="the 128^3 system above (n=2,097,152, GMRES(50), "
                                                      "no preconditioner), whole iteration")
    if not args.no_small:
        out["small_64x64"] = small_config(args)
    if not args.no_batch:
        out["batch"] = batch_result(args)
    if not args.no_batch3d:
        out["batch_3d"] = batch_result(args, dim=3)
    if args.orth_study_N:
        out["orth_study"] = orth_study(args)
    if not args.no_cpu_baseline:
        log("cpu baseline: the oracle's OpenMP timing build on the host cores ...")
        out["cpu_baseline"] = cpu_baseline(p, m)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.1f} iters/s on "
            f"{out['cpu_baseline']['cores']} threads, {out['cpu_baseline']['one_thread_iters_per_s']:.1f} on one")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
