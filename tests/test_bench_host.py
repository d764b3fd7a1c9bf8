"""Host-side checks of bench.py (no GPU): the contract's refusal of more than
one GPU, the flop model, and that every name the measurement legs call exists
(a static check over the module's own syntax tree)."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_every_called_module_function_exists():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    defined = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    called = {n.func.id for n in ast.walk(tree) if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    local_names = set()
    for n in ast.walk(tree):
        if isinstance(n, (ast.Assign, ast.AugAssign)):
            for t in (n.targets if isinstance(n, ast.Assign) else [n.target]):
                for m in ast.walk(t):
                    if isinstance(m, ast.Name):
                        local_names.add(m.id)
        elif isinstance(n, ast.FunctionDef):
            local_names.update(a.arg for a in n.args.args)
            for m in ast.walk(n):
                if isinstance(m, ast.FunctionDef):
                    local_names.add(m.name)
    missing = {c for c in called if c not in defined and c not in local_names and not hasattr(bench, c)
               and c not in dir(__import__("builtins"))}
    assert not missing, missing
    for leg in ("bench_batch", "bench_diff", "bench_accel", "bench_cstr", "bench_rti", "bench_fp64_chain", "bench_table1",
                "cpu_baseline", "measured_traffic"):
        assert leg in defined, leg


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_stage_flop_model():
    # 2 F + 45 nb with F = nb^2 + nu nb + 2 nx^2 + 3 nx nu (the 12-mass chain: nx = 24, nu = 11):
    # F = 3554 and 8683 flops per stage-iteration
    nb = 35
    F = nb * nb + 11 * nb + 2 * 24 * 24 + 3 * 24 * 11
    assert F == 3554
    assert bench.stage_flops(24, 11) == 2 * F + 45 * nb == 8683


def test_peak_is_the_non_packed_fp32_rate():
    assert abs(bench.PEAK_FP32_VALU - 78.6e12) < 0.1e12
    assert bench.PEAK_FP32_PACKED == 157.3e12


def test_info_check_refuses_failed_solves():
    import numpy as np
    import pytest
    from paper_2601_14414_amd import pimpc as P
    rec = np.zeros(3, dtype=P.INFO_DTYPE)
    rec["iters"] = 300
    bench.check_info(P, rec, 300, "ok")
    rec["status"][1] = P.PIMPC_E_HIP
    with pytest.raises(RuntimeError):
        bench.check_info(P, rec, 300, "bad status")
    rec["status"][1] = 0
    rec["iters"][2] = 120
    with pytest.raises(RuntimeError):
        bench.check_info(P, rec, 300, "short run")


def test_oracle_pool_worker_counts_solves():
    """The all-core CPU baseline's worker runs whole oracle solves of the
    headline workload for a bounded time."""
    reps, t = bench._oracle_worker((0, 0.0))
    assert reps == 1 and t > 0
