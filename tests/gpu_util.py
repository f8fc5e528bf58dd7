"""Helpers for the GPU tests: run the HIP library and the oracle on the same seeded inputs."""

from __future__ import annotations

import sys

import numpy as np

import oracle
from oracle import diagnostics as D


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(p):
    import torch

    return (torch.from_numpy(p.row_ptr).cuda(), torch.from_numpy(p.col_idx).cuda(),
            torch.from_numpy(p.vals).cuda())


def gpu_run(p, scheme, m=None, rtol=None, max_iters=None, b=None, x0=None, basis=False, fmt=None,
            orth=False, **options):
    """One solve through the C ABI; returns a dict with x, info, hist and the last cycle.
    fmt: None (the library's choice), "csr", "sell", "sell_d16" or "sell_diag";
    further keyword options (rows_per_lane, pipeline_depth, ...) go to
    gmres_create_ex."""
    import torch

    from paper_1809_05805_amd.native import GmresSolver

    m = p.m if m is None else m
    rtol = p.rtol if rtol is None else rtol
    max_iters = min(10 * p.n, 10**6) if max_iters is None else max_iters
    rp, ci, va = dev(p)
    if fmt is not None:
        options["format"] = fmt
    s = GmresSolver(rp, ci, va, m, scheme, **options)
    bt = torch.from_numpy(np.ascontiguousarray(p.b if b is None else b)).cuda()
    xt = torch.from_numpy(np.array(p.x0 if x0 is None else x0, dtype=np.float64)).cuda()
    r = s.solve(bt, xt, rtol, max_iters, hist=True, orth=orth)
    torch.cuda.synchronize()
    H, T, g, j = s.last_cycle()
    out = {"res": r, "x": xt.cpu().numpy(), "H": H, "T": T, "g": g, "j": j, "solver": s}
    if basis:
        out["V"] = s.basis()[:, : j + 1].cpu().numpy()
    return out


def oracle_run(p, scheme, m=None, rtol=None, max_iters=None, b=None, x0=None, dump=True):
    m = p.m if m is None else m
    rtol = p.rtol if rtol is None else rtol
    return oracle.solve(p.row_ptr, p.col_idx, p.vals, p.b if b is None else b,
                        p.x0 if x0 is None else x0, m, scheme, rtol, max_iters, dump)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


__all__ = ["log", "dev", "gpu_run", "oracle_run", "rel", "D"]
