"""Host-side logic of bench.py (CPU only): the batched solve's byte model."""

import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_batch_bytes_by_hand():
    bench = load_bench()
    n, nnz, m = 100, 460, 3
    A = 12.0 * nnz + 4.0 * (n + 1)
    # 5 iterations in 2 cycles: a full cycle of 3 steps, then 2 steps
    info = {"iters": np.array([5]), "cycles": np.array([2])}
    got = bench.batch_bytes(info, [n], [nnz], m, 8)
    want = 0.0
    for j in (3, 2):
        for k in range(j):
            want += A + 8 * n * (2 * (k + 1) + 4)       # SpMV, two sweeps of V[:,0:k+1], w, 2 columns
        want += 8 * n + 8.0 * n * j + 16.0 * n + A + 24.0 * n  # norm step, x update, restart
    want += A + 24.0 * n                                 # closing residual check
    assert got == want
    # a system that converged at its first restart check moves only that check
    info0 = {"iters": np.array([0]), "cycles": np.array([0])}
    assert bench.batch_bytes(info0, [n], [nnz], m, 8) == A + 24.0 * n
    # the float32 basis halves the vector bytes of the steps
    got4 = bench.batch_bytes({"iters": np.array([3]), "cycles": np.array([1])}, [n], [nnz], m, 4)
    steps4 = sum(A + 4 * n * (2 * (k + 1) + 4) for k in range(3))
    assert got4 == steps4 + 4 * n + 8.0 * n * 3 + 16.0 * n + A + 24.0 * n + A + 24.0 * n


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    for argv, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        e = dict(os.environ, **env)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, env=e,
                           capture_output=True, text=True, timeout=60)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""
