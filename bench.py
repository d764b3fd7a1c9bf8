"""Benchmark: ADMM stage-iterations/s of the piMPC hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra] [--no-accel]
    python bench.py --only {batch,diff,accel,cstr}   (one extra workload, for profiling)

A step is one full solve (all iterations) of the long-horizon workload: the
12-mass chain (nx=24, nu=11), horizon N=1024, 500 plain ADMM iterations, FP32
iteration arithmetic with the FP64 stage factorisation done at setup.
Inputs are resident in HBM before timing starts; the timed region is the
graph-replayed solve on the current torch stream.  value = N * iterations *
steps / seconds.  Extra keys report the 4096-instance uneven batch, the
differentiable batch (forward + backward against the plain forward), restart
acceleration against plain ADMM to a tolerance on the batch, the reactor NMPC
at N=5000 (seconds per sample, as in the paper's Table 2), and the CPU oracle
timed on the host.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published FP32 vector peak (FLOP/s); it needs packed FP32
# instructions (two FMAs per lane and cycle), which this library does not use.
PEAK_FP32_PACKED = 157.3e12
# The rate this library can reach: 256 CUs x 4 SIMDs x 16 lanes x one FMA
# (2 flop) per cycle at 2.4 GHz, non-packed FP32.
PEAK_FP32_VALU = 256 * 4 * 16 * 2 * 2.4e9
PEAK_HBM = 8.0e12           # bytes/s

METRIC = "ADMM stage-iterations/s (N=1024; 4096-batch) + fwd+bwd time vs plain"


def measured_traffic():
    """HBM bytes per launch of the row kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE runs (scaled by the copy calibration), or None if
    the kernel source changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "row_kernel_long_horizon_traffic.json")))
        src = open(os.path.join(ROOT, "paper_2601_14414_amd", "csrc", "admm_row.hip"), "rb").read()
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    return rec["traffic_bytes_per_launch"]


def stage_flops(nx: int, nu: int) -> int:
    """Algorithmic flops of one stage-iteration of eqn. (8) and Algorithm 1
    steps 1-4: 2 F(nx, nu) for the mat-vecs of steps 1-2 (F = nb^2 + nu nb
    + 2 nx^2 + 3 nx nu FMAs, counted with the block structure of Abar, Bbar)
    plus 45 nb for the element-wise work of steps 2-4 (the argument of the
    projection, the projection, the three dual updates and the six squared
    differences of c)."""
    nb = nx + nu
    F = nb * nb + nu * nb + 2 * nx * nx + 3 * nx * nu
    return 2 * F + 45 * nb


def check_info(P, rec, iters=None, what=""):
    """Refuse to report a timing whose solves did not complete: every
    instance's status must be 0 (and its iteration count `iters` when given)."""
    import numpy as np
    rec = np.atleast_1d(rec)
    bad = np.nonzero(rec["status"] != 0)[0]
    if bad.size:
        raise RuntimeError(f"{what}: instance {int(bad[0])} ended with status {int(rec['status'][bad[0]])}")
    if iters is not None and np.any(rec["iters"] != iters):
        raise RuntimeError(f"{what}: an instance ran {int(rec['iters'].min())} iterations, expected {iters}")


def time_solves(torch, fn, steps, warmup):
    """Run fn() warmup + steps times; return (total_ms, per-step event ms list)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1), [a.elapsed_time(b) for a, b in evs]


def _oracle_worker(args):
    """One process of the all-core oracle timing: full solves of the
    long-horizon instance until `seconds` have passed."""
    seed, seconds = args
    import oracle
    from paper_2601_14414_amd import workloads as W
    p = W.long_horizon_problem(seed=seed)
    oracle.solve(p, K=2)  # load
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds or reps < 1:
        oracle.solve(p)
        reps += 1
    return reps, time.perf_counter() - t0


def host_threads():
    """Host cores this process may use, at most 16 (the GPU machine's CPU share
    for one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(single_seconds=8.0, pool_seconds=6.0):
    """The unchanged FP64 C oracle on the host: one process (one core), then
    one process per usable host core, each solving its own copy of the
    workload (independent instances, as a batch would be), for a bounded
    time; value = the all-core aggregate."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    from paper_2601_14414_amd import workloads as W
    p = W.long_horizon_problem(seed=0)
    reps1, t1 = _oracle_worker((0, single_seconds))
    v1 = p.N * p.K * reps1 / t1
    ncores = host_threads()
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(ncores) as pool:
        res = pool.map(_oracle_worker, [(s, pool_seconds) for s in range(ncores)])
    wall = time.perf_counter() - t0
    reps = sum(r for r, _ in res)
    vall = p.N * p.K * reps / wall
    return {"value": vall, "unit": "stage-iterations/s", "cores": ncores, "kind": "oracle",
            "single_core_value": v1, "host_cpus_visible": os.cpu_count(),
            "sample": f"unchanged single-threaded FP64 C oracle, full solves of the N=1024, 500-iteration "
                      f"long-horizon instance: {reps1} solves on one core in {t1:.1f} s; then {ncores} "
                      f"processes (one per usable host core, x0 seeds 0..{ncores - 1}) for {pool_seconds:.0f} s: "
                      f"{reps} solves in {wall:.1f} s wall"}


def headline_error(p, gpu_state, gpu_u0):
    """FP32 GPU result of the headline solve against the FP64 oracle run on
    the same instance and iteration count: largest error of every iterate
    (scaled by max(1, |oracle|_inf)) and of u0."""
    import numpy as np
    import oracle
    r = oracle.solve(p)
    it = max(float(np.max(np.abs(gpu_state[w] - r["state"][w])) / max(1.0, float(np.max(np.abs(r["state"][w])))))
             for w in range(5))
    return {"max_scaled_iterate_error": it, "u0_max_abs_error": float(np.max(np.abs(gpu_u0 - r["u0"]))),
            "oracle_r_prim": float(r["hist"][-1][1]), "oracle_r_dual": float(r["hist"][-1][2]),
            "tolerance": 1e-4}


def sync_floor(torch, P, W, K, nwg_target, steps=5):
    """Per-iteration time of the same row-family kernel over the same grid
    of workgroups (4 compute waves each), on the narrowest stage class (a
    2-state, 1-input system padded to 4 + 4, eight stages side by side in a
    wave, one 8-row dot product per halo): almost no arithmetic, so this is
    the period of the cross-workgroup cycle itself (publish, hop to the
    neighbour's receiver wave, forward through LDS, the two halo products and
    the update)."""
    import numpy as np
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    N = 8 * 4 * nwg_target  # 8 stages per wave, 4 compute waves per workgroup
    p = W.paper_random_system(2, 1, N, seed=0, K=K)
    s = P.Solver([p], max_iter=K, precision=P.PIMPC_FP32, stream=stream, family=P.PIMPC_FAMILY_ROW)
    x0 = torch.tensor(p.x0, dtype=torch.float32, device=dev)
    u0 = torch.empty(p.nu, dtype=torch.float32, device=dev)
    info = torch.zeros(40, dtype=torch.uint8, device=dev)
    ms, per = time_solves(torch, lambda: P.pimpc_solve_batch(s.ctx, x0, None, u0, info, stream), steps, 2)
    rec = np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE)
    check_info(P, rec, K, "sync_floor")
    s.close()
    return {"us_per_iteration": float(np.mean(per)) / K * 1e3, "workgroups": nwg_target, "N": N,
            "workload": "2-state, 1-input random system (row class 4+4, 8 stages per wave), same grid of "
                        "workgroups as the headline, same iteration count"}


def bench_batch(torch, P, W, steps, warmup):
    problems = W.random_batch(4096, base_seed=1000, K=300)
    stream = torch.cuda.current_stream().cuda_stream
    s = P.Solver(problems, max_iter=300, precision=P.PIMPC_FP32, stream=stream)
    dev = torch.device("cuda")
    import numpy as np
    x0 = torch.tensor(np.concatenate([p.x0 for p in problems]), dtype=torch.float32, device=dev)
    u0 = torch.empty(s.sum_nu, dtype=torch.float32, device=dev)
    info = torch.zeros(40 * len(problems), dtype=torch.uint8, device=dev)
    fn = lambda: P.pimpc_solve_batch(s.ctx, x0, None, u0, info, stream)
    ms, per = time_solves(torch, fn, steps, warmup)
    rec = np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE)
    check_info(P, rec, 300, "batch_4096")
    stage_its = sum(p.N for p in problems) * 300
    flops = sum(p.N * stage_flops(p.nx, p.nu) for p in problems) * 300
    # the device-pointer path does not write the step-1 outputs (du, xbar);
    # one host-path solve of the same context (same kernels, same inputs)
    # does, and must give the same u0 bit for bit
    u0_dev = u0.cpu().numpy().astype(np.float64)
    u0_host, _ = s.solve(x0=x0.cpu().numpy().astype(np.float64))
    if not np.array_equal(u0_host, u0_dev):
        raise RuntimeError("batch_4096: host-path and device-path solves differ")
    err = batch_error(P, s, problems, u0_dev)
    s.close()
    # the same instances one launch each (the single-instance path, graph
    # replays back to back on one stream): every 32nd instance, scaled to 4096
    sub = problems[::32]
    singles = [P.Solver([p], max_iter=300, precision=P.PIMPC_FP32, stream=stream) for p in sub]
    bufs = [(torch.tensor(p.x0, dtype=torch.float32, device=dev), torch.empty(p.nu, dtype=torch.float32, device=dev))
            for p in sub]

    def one_by_one():
        for sv, (xb, ub) in zip(singles, bufs):
            P.pimpc_solve_batch(sv.ctx, xb, None, ub, None, stream)

    ms1, _ = time_solves(torch, one_by_one, 2, 1)
    for sv in singles:
        sv.close()
    single_ms = ms1 / 2 * len(problems) / len(sub)
    return {"value": stage_its * steps / (ms / 1e3), "unit": "stage-iterations/s",
            "ms_per_step": ms / steps, "instances": 4096, "sum_N": int(sum(p.N for p in problems)),
            "iterations": 300, "achieved_tflops": flops / (min(per) / 1e3) / 1e12,
            "one_launch_per_instance_ms": single_ms, "batched_speedup": single_ms / (ms / steps),
            "one_launch_per_instance_note": "128 of the instances (every 32nd) solved one launch each, "
                                            "back to back on one stream, time scaled to 4096",
            "error_vs_oracle": err}


def batch_error(P, s, problems, u0_all):
    """Largest FP32-vs-oracle error of the batch over a stratified sample (the
    shortest and the longest instance of every (nx, nu) class present):
    every iterate, du, xbar and u0, scaled by max(1, |oracle|_inf)."""
    import numpy as np
    import oracle
    by_cls = {}
    for i, p in enumerate(problems):
        by_cls.setdefault((p.nx, p.nu), []).append(i)
    pick = sorted({j for ids in by_cls.values() for j in (min(ids, key=lambda i: problems[i].N),
                                                          max(ids, key=lambda i: problems[i].N))})
    its = {w: s.iterate(w) for w in range(7)}
    uoff = np.cumsum([0] + [p.nu for p in problems])
    worst = 0.0
    for i in pick:
        r = oracle.solve(problems[i])
        refs = [r["state"][w] for w in range(5)] + [r["du"], r["xs"]]
        for w in range(7):
            worst = max(worst, float(np.max(np.abs(its[w][i] - refs[w])) / max(1.0, np.max(np.abs(refs[w])))))
        worst = max(worst, float(np.max(np.abs(u0_all[uoff[i]:uoff[i + 1]] - r["u0"]))
                                 / max(1.0, np.max(np.abs(r["u0"])))))
    return {"max_scaled_error": worst, "instances_compared": len(pick),
            "sample": "shortest and longest instance of each (nx, nu) class; all five iterates, du, xbar, u0"}


def bench_accel(torch, P, W, steps, warmup):
    """Time to solution on the 4096-instance batch, plain ADMM against restart
    acceleration (Algorithm 1 steps 6-7): both stop each instance at c <= eps
    (checked every 10 iterations), at most 6000 iterations, eps = 1e-6; and
    the same on 1024 4-mass chains (N = 128) to eps = 1e-5, at most 20000.
    A batched solve ends with its slowest instance.  The levels keep the
    iterate differences that make up c well above FP32 resolution."""
    import numpy as np
    problems = W.random_batch(4096, base_seed=1000, K=6000)
    stream = torch.cuda.current_stream().cuda_stream
    dev = torch.device("cuda")
    x0 = torch.tensor(np.concatenate([p.x0 for p in problems]), dtype=torch.float32, device=dev)
    Ns = np.array([p.N for p in problems])
    out = {}
    for eps in (1e-6,):
        res = {}
        for name, accel in (("plain", False), ("accel", True)):
            s = P.Solver(problems, max_iter=6000, eps=eps, check_every=10, precision=P.PIMPC_FP32,
                         accel=accel, stream=stream)
            u0 = torch.empty(s.sum_nu, dtype=torch.float32, device=dev)
            info = torch.zeros(40 * len(problems), dtype=torch.uint8, device=dev)
            fn = lambda: P.pimpc_solve_batch(s.ctx, x0, None, u0, info, stream)
            ms, per = time_solves(torch, fn, steps, warmup)
            rec = np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE)
            its = rec["iters"].astype(np.int64)
            res[name] = {"ms_per_solve": ms / steps, "mean_iters": float(its.mean()),
                         "max_iters": int(its.max()), "converged": int((rec["c"] <= eps).sum()),
                         "stage_iterations_per_s": float((Ns * its).sum() / (min(per) / 1e3))}
            if accel:
                res[name]["mean_restarts"] = float(rec["restarts"].mean())
            s.close()
        res["speedup"] = res["plain"]["ms_per_solve"] / res["accel"]["ms_per_solve"]
        res["iteration_ratio"] = res["accel"]["mean_iters"] / res["plain"]["mean_iters"]
        out[f"eps_{eps:g}"] = res
    out["workload"] = ("4096 random instances (batch recipe), FP32, to c <= eps, check every 10, max 6000; "
                       "about a tenth of the instances never reach eps with either method (their box is "
                       "infeasible for the dynamics), so both batched solves run 6000 iterations on those")
    # a batch where every instance converges: 1024 perturbed 4-mass chains, N=128
    eps_c = 1e-5
    db = W.diff_batch(count=1024, seed=7, N=128, K=20000)
    chains = [db.instance(i) for i in range(1024)]
    x0c = torch.tensor(np.concatenate([p.x0 for p in chains]), dtype=torch.float32, device=dev)
    res = {}
    for name, accel in (("plain", False), ("accel", True)):
        s = P.Solver(chains, max_iter=20000, eps=eps_c, check_every=10, precision=P.PIMPC_FP32, accel=accel,
                     stream=stream)
        u0 = torch.empty(s.sum_nu, dtype=torch.float32, device=dev)
        info = torch.zeros(40 * len(chains), dtype=torch.uint8, device=dev)
        fn = lambda: P.pimpc_solve_batch(s.ctx, x0c, None, u0, info, stream)
        ms, per = time_solves(torch, fn, steps, warmup)
        rec = np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE)
        its = rec["iters"].astype(np.int64)
        res[name] = {"ms_per_solve": ms / steps, "mean_iters": float(its.mean()), "max_iters": int(its.max()),
                     "converged": int((rec["c"] <= eps_c).sum())}
        if accel:
            res[name]["mean_restarts"] = float(rec["restarts"].mean())
        s.close()
    res["speedup"] = res["plain"]["ms_per_solve"] / res["accel"]["ms_per_solve"]
    res["iteration_ratio"] = res["accel"]["mean_iters"] / res["plain"]["mean_iters"]
    res["workload"] = "1024 4-mass chains (nx=8, nu=3), N=128, FP32, to c <= 1e-5, check every 10, max 20000"
    out["chains_1024"] = res
    # single long horizons on the row family (a global reduction of c after
    # every accelerated step): the 12-mass chain and the reactor
    for key, prob, eps_r, kmax, rho in (
            ("long_horizon_1024", W.long_horizon_problem(seed=0), 1e-4, 200000, 1.0),
            ("cstr_5000", W.cstr_problem(N=5000, K=1000, rho=0.1), 1e-6, 200000, 0.1)):
        res = {}
        x0r = torch.tensor(prob.x0, dtype=torch.float32, device=dev)
        upr = torch.tensor(prob.u_prev, dtype=torch.float32, device=dev)
        for name, accel in (("plain", False), ("accel", True)):
            s = P.Solver([prob], rho=rho, max_iter=kmax, eps=eps_r, check_every=10 if not accel else 1,
                         precision=P.PIMPC_FP32, accel=accel, stream=stream)
            u0 = torch.empty(prob.nu, dtype=torch.float32, device=dev)
            info = torch.zeros(40, dtype=torch.uint8, device=dev)
            fn = lambda: P.pimpc_solve_batch(s.ctx, x0r, upr, u0, info, stream)
            ms, per = time_solves(torch, fn, 2, 1)
            rec = np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE)
            check_info(P, rec, None, f"restart_accel {key} {name}")
            it = int(rec["iters"][0])
            res[name] = {"ms_per_solve": ms / 2, "iters": it, "c": float(rec["c"][0]),
                         "us_per_iteration": ms / 2 / it * 1e3}
            if accel:
                res[name]["restarts"] = int(rec["restarts"][0])
            s.close()
        res["speedup"] = res["plain"]["ms_per_solve"] / res["accel"]["ms_per_solve"]
        res["iteration_ratio"] = res["accel"]["iters"] / res["plain"]["iters"]
        res["workload"] = (f"one instance on the row family, FP32, to c <= {eps_r:g} (plain: checked every 10 "
                           f"iterations; accelerated: every iteration, as steps 6-7 need), max {kmax}")
        out[key] = res
    return out


def bench_diff(torch, P, W, steps, warmup):
    """Differentiable batch: 1024 chains (nx=8, nu=3, N=128), 200 iterations,
    checkpoints every 20.  Returns the time of (taped forward + backward) over
    the time of the plain forward on the same batch; the same for the tape
    the forward records in full (ckpt_every = 1: no checkpoints, no re-run in
    the backward, 3.25 GB of records)."""
    import numpy as np
    from paper_2601_14414_amd.autograd import PiMPCFunction
    db = W.diff_batch(count=1024, seed=7, N=128, K=200)
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    problems = [db.instance(i) for i in range(1024)]
    plain = P.Solver(problems, max_iter=200, precision=P.PIMPC_FP32, stream=stream)
    f = lambda a, g=False: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev,
                                        requires_grad=g)
    x0 = f(db.x0)
    u0 = torch.empty(1024 * 3, dtype=torch.float32, device=dev)
    info = torch.zeros(40 * 1024, dtype=torch.uint8, device=dev)
    ms_plain, per_plain = time_solves(torch, lambda: P.pimpc_solve_batch(plain.ctx, x0, None, u0, info, stream),
                                      steps, warmup)
    check_info(P, np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE), 200, "differentiable plain")
    plain.close()
    xq, Qd, Rd, A, B = f(db.x0, True), f(db.Qdiag, True), f(db.Rdiag, True), f(db.A, True), f(db.Bm, True)
    target = f(db.u_target)
    # the oracle's reverse mode on a sample of instances
    import oracle
    sample = list(range(0, 1024, 256))
    ref = {}
    for i in sample:
        pi = db.instance(i)
        r = oracle.solve(pi)
        ref[i] = oracle.grad(8, 3, db.N, pi.A, pi.B, db.Qdiag[i], db.Rdiag[i], pi.lb(), pi.ub(), pi.x0, pi.rho,
                             db.K, 2 * (r["u0"] - db.u_target[i]))

    def run(ckpt):
        taped = P.Solver(problems, max_iter=200, precision=P.PIMPC_FP32, ckpt_every=ckpt, stream=stream)

        def fwd_bwd():
            u = PiMPCFunction.apply(xq, Qd, Rd, A, B, taped)
            ((u - target) ** 2).sum().backward()

        def fwd_only():
            with torch.no_grad():
                PiMPCFunction.apply(xq, Qd, Rd, A, B, taped)

        ms_fb, _ = time_solves(torch, fwd_bwd, steps, warmup)
        ms_f, _ = time_solves(torch, fwd_only, steps, warmup)
        for t in (xq, Qd, Rd, A, B):
            t.grad = None
        fwd_bwd()
        torch.cuda.synchronize()
        got = {k: t.grad.detach().cpu().numpy().astype(np.float64) for k, t in
               dict(dx0=xq, dQd=Qd, dRd=Rd, dA=A, dB=B).items()}
        taped.close()
        worst = 0.0
        for i in sample:
            for key in ("dx0", "dQd", "dRd", "dA", "dB"):
                g = ref[i][key]
                worst = max(worst, float(np.max(np.abs(got[key][i] - g)) / max(1e-6, np.max(np.abs(g)))))
        return ms_fb, ms_f, worst

    ms_fb, ms_f, worst = run(20)
    ms_fb1, ms_f1, worst1 = run(1)
    return {"fwd_bwd_over_plain": ms_fb / ms_plain, "plain_fwd_ms": ms_plain / steps,
            "taped_fwd_ms": ms_f / steps, "fwd_bwd_ms": ms_fb / steps,
            "workload": "1024 x 4-mass chain (nx=8, nu=3), N=128, 200 iterations, checkpoints every 20, "
                        "loss sum ||u0 - u_target||^2, gradients w.r.t. x0, diag Q, diag R, A, B",
            "gradient_error_vs_oracle": {"max_rel_error": worst, "instances": sample,
                                         "norm": "per parameter, max |gpu - oracle| / max |oracle|"},
            "full_tape": {"fwd_bwd_over_plain": ms_fb1 / ms_plain, "taped_fwd_ms": ms_f1 / steps,
                          "fwd_bwd_ms": ms_fb1 / steps, "max_rel_gradient_error": worst1,
                          "tape": "ckpt_every = 1: the forward records all 200 steps (31 floats a stage "
                                  "and step, 3.25 GB), the backward re-runs nothing"},
            "plain_stage_iterations_per_s": 1024 * 128 * 200 * steps / (ms_plain / 1e3)}


def bench_cstr(steps=21):
    """Reactor NMPC of Section V: N=5000, 1000 warm-started iterations per
    sample, re-linearised every sample.  Per-sample time = pimpc_linearize
    (FP64 refactorisation on the device) + pimpc_solve (host pointers,
    synchronous); the first sample is dropped."""
    import numpy as np
    from paper_2601_14414_amd import rti
    log = rti.run_cstr_nmpc(steps=steps, N=5000, iters=1000, rho=0.1)
    if any(int(st.info["iters"][0]) != 1000 for st in log):
        raise RuntimeError("cstr_nmpc_5000: a sample did not run 1000 iterations")
    t = np.array([st.solve_s for st in log[1:]])
    return {"median_s_per_sample": float(np.median(t)), "max_s_per_sample": float(np.max(t)),
            "stage_iterations_per_s": 5000 * 1000 / float(np.median(t)), "samples": len(t),
            "C_A_start": float(log[0].x[0]), "C_A_end": float(log[-1].x[0]),
            "paper_context": "0.526 s median / 0.610 s max per sample (RTX 3080, Table 2)",
            "workload": "CSTR, nx=2, nu=1, N=5000, 1000 iterations per sample, W_y=1, W_u=0, "
                        "W_du=0.1, rho=0.1, FP32, online linearisation at each sample"}


def bench_rti(steps=21):
    """Cart-pole swing-up with real-time iterations: N=256, time-varying
    A_k, B_k, e_k from the Jacobians along the shifted predicted trajectory,
    100 warm-started iterations per step, FP32 iteration with FP64
    refactorisation on the device.  Library time per step = pimpc_linearize
    + pimpc_solve (host pointers, synchronous); the whole step adds the host
    Jacobians and the read-back of the predicted trajectory.  The first step
    is dropped."""
    import numpy as np
    from paper_2601_14414_amd import rti
    log = rti.run_cartpole_rti(steps=steps, N=256, iters=100)
    if any(int(st.info["iters"][0]) != 100 for st in log):
        raise RuntimeError("rti_cartpole_256: a step did not run 100 iterations")
    lib = np.array([st.lib_s for st in log[1:]])
    step = np.array([st.step_s for st in log[1:]])
    jac = np.array([st.jac_s for st in log[1:]])
    return {"median_lib_s_per_step": float(np.median(lib)), "max_lib_s_per_step": float(np.max(lib)),
            "median_s_per_step": float(np.median(step)), "median_host_jacobian_s": float(np.median(jac)),
            "stage_iterations_per_s": 256 * 100 / float(np.median(lib)), "steps": len(lib),
            "theta_start": float(log[0].x[2]), "theta_end": float(log[-1].x[2]),
            "workload": "cart-pole swing-up RTI, nx=4, nu=1, N=256, 100 iterations per step, "
                        "Q=diag(10,1,10,1), R=0.01, |u|<=10, FP32 iteration, FP64 refactorisation"}


def bench_fp64_chain(torch, P, W, n):
    """Plain linear MPC in FP64: 4-mass chain (nx=8, nu=3), N=20, 200 fixed
    iterations, one instance; device-resident solves on the caller's stream."""
    p = W.plain_fp64_problem(seed=0)
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    s = P.Solver([p], max_iter=p.K, precision=P.PIMPC_FP64, stream=stream)
    x0 = torch.tensor(p.x0, dtype=torch.float64, device=dev)
    u0 = torch.empty(p.nu, dtype=torch.float64, device=dev)
    info = torch.zeros(40, dtype=torch.uint8, device=dev)
    fn = lambda: P.pimpc_solve_batch(s.ctx, x0, None, u0, info, stream)
    ms, per = time_solves(torch, fn, n, 2)
    import numpy as np
    check_info(P, np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE), p.K, "fp64_chain_20")
    s.close()
    sol_ms = ms / n
    return {"ms_per_solve": sol_ms, "stage_iterations_per_s": p.N * p.K / (sol_ms / 1e3),
            "kernel_ms": float(sum(per) / len(per)),
            "workload": "4-mass chain (nx=8, nu=3), N=20, 200 iterations, rho=1, FP64, one instance"}


# Table 1 of the paper (random systems of Section V-B, averages over 200 iterations): milliseconds per
# iteration of piMPC on its GPU (RTX 3080) and CPU (Ryzen 9 5900X), and of OSQP, for the stage sizes
# this build compiles.  Context only: other hardware, precision not stated.
PAPER_TABLE1_MS = {  # (n, m): {N: (piMPC GPU, piMPC CPU, OSQP)}
    (10, 3): {20: (0.53, 0.15, 0.02), 50: (0.55, 0.31, 0.06), 100: (0.54, 0.58, 0.11), 200: (0.55, 1.12, 0.23),
              500: (0.56, 2.75, 0.59)},
    (20, 6): {20: (0.56, 0.17, 0.07), 50: (0.56, 0.35, 0.18), 100: (0.55, 0.68, 0.35), 200: (0.55, 1.38, 0.72),
              500: (0.56, 3.52, 1.85)},
    (30, 10): {20: (0.54, 0.18, 0.15), 50: (0.54, 0.38, 0.37), 100: (0.58, 0.73, 0.74), 200: (0.56, 1.61, 1.56),
               500: (0.56, 3.90, 5.78)},
}


def bench_table1(torch, P, W, n_solves=10):
    """The random-system recipe of the paper's scalability study at the sizes
    of its Table 1 that this build compiles: one instance per solve, 200
    iterations, FP32, device pointers; milliseconds per iteration beside the
    paper's numbers."""
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for (n, m), row in PAPER_TABLE1_MS.items():
        for N, (gpu, cpu, osqp) in row.items():
            p = W.paper_random_system(n, m, N, seed=0, K=200)
            s = P.Solver([p], rho=p.rho, max_iter=200, precision=P.PIMPC_FP32, stream=stream)
            x0 = torch.tensor(p.x0, dtype=torch.float32, device=dev)
            u0 = torch.empty(m, dtype=torch.float32, device=dev)
            info = torch.zeros(40, dtype=torch.uint8, device=dev)
            ms, _ = time_solves(torch, lambda: P.pimpc_solve_batch(s.ctx, x0, None, u0, info, stream), n_solves, 2)
            import numpy as np
            check_info(P, np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE), 200, f"table1 {n},{m},{N}")
            s.close()
            out[f"n{n}_m{m}_N{N}"] = {"ms_per_iteration": ms / n_solves / 200, "paper_gpu_ms_per_iteration": gpu,
                                      "paper_cpu_ms_per_iteration": cpu, "paper_osqp_ms_per_iteration": osqp}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-accel", action="store_true", help="skip the restart-acceleration extra")
    ap.add_argument("--only", choices=["batch", "diff", "accel", "cstr", "rti", "fp64", "table1"],
                    help="run one extra workload alone and print its JSON (for profiling)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 256 MiB device copy (to scale FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calib:
        import torch
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")  # 256 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "launches": 3}))
        return
    if args.only:
        import torch
        from paper_2601_14414_amd import pimpc as P
        from paper_2601_14414_amd import workloads as W
        torch.cuda.set_device(0)
        n = max(3, args.steps // 4)
        res = {"batch": lambda: bench_batch(torch, P, W, n, 1), "diff": lambda: bench_diff(torch, P, W, n, 1),
               "accel": lambda: bench_accel(torch, P, W, 2, 1), "cstr": lambda: bench_cstr(),
               "rti": lambda: bench_rti(), "fp64": lambda: bench_fp64_chain(torch, P, W, 20),
               "table1": lambda: bench_table1(torch, P, W)}[args.only]()
        print(json.dumps({args.only: res}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for {args.gpus}); "
              "more GPUs would shard the batch by instance and a long horizon by stage blocks, "
              "which is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2601_14414_amd import pimpc as P
    from paper_2601_14414_amd import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda")
    side = torch.cuda.Stream()  # a created stream, so the solve is graph-captured
    torch.cuda.set_stream(side)
    stream = torch.cuda.current_stream().cuda_stream
    p = W.long_horizon_problem(seed=0)
    s = P.Solver([p], max_iter=p.K, precision=P.PIMPC_FP32, stream=stream)
    x0 = torch.tensor(p.x0, dtype=torch.float32, device=dev)
    u0 = torch.empty(p.nu, dtype=torch.float32, device=dev)
    info = torch.zeros(40, dtype=torch.uint8, device=dev)
    fn = lambda: P.pimpc_solve_batch(s.ctx, x0, None, u0, info, stream)
    ms, per = time_solves(torch, fn, args.steps, args.warmup)
    rec = np.frombuffer(info.cpu().numpy().tobytes(), dtype=P.INFO_DTYPE)[0]
    check_info(P, rec, p.K, "headline")
    stage_its = p.N * p.K
    value = stage_its * args.steps / (ms / 1e3)
    step_ms = float(np.mean(per))
    flops_per_launch = p.N * p.K * stage_flops(p.nx, p.nu)
    achieved = flops_per_launch / (step_ms / 1e3)
    gpu_state = s.state(0)
    gpu_u0 = u0.cpu().numpy().astype(np.float64)
    floor = sync_floor(torch, P, W, p.K, nwg_target=p.N // 4)
    out = {
        "metric": METRIC, "value": value, "unit": "stage-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "long horizon: 12-mass spring chain (nx=24, nu=11), N=1024, "
                               "500 plain ADMM iterations, rho=1, FP32 iteration, FP64 stage "
                               "factorisation at setup, x0 ~ U[-2,2] seed 0",
                   "N": p.N, "nx": p.nx, "nu": p.nu, "iterations": p.K, "instances": 1},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU, "traffic": measured_traffic(),
                     "kernel": "row_kernel<24,12,1,false,false,false> (one solve = one launch)",
                     "flops_per_launch": flops_per_launch,
                     "flops_per_stage_iteration": stage_flops(p.nx, p.nu), "avg_launch_ms": step_ms,
                     "peak_note": "non-packed FP32 FMA rate 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz; "
                                  "the published 157.3 TFLOP/s needs packed FP32, which this library does not "
                                  "use",
                     "frac_of_published_packed_peak": achieved / PEAK_FP32_PACKED,
                     "sync_floor": {**floor, "us_per_iteration_headline": step_ms / p.K * 1e3,
                                    "floor_over_headline": floor["us_per_iteration"] / (step_ms / p.K * 1e3)}},
        "residuals": {"c": float(rec["c"]), "r_prim": float(rec["r_prim"]), "r_dual": float(rec["r_dual"])},
    }
    s.close()
    out["error_vs_oracle"] = headline_error(p, gpu_state, gpu_u0)
    if not args.no_extra:
        out["batch_4096"] = bench_batch(torch, P, W, max(3, args.steps // 4), 1)
        out["differentiable_1024"] = bench_diff(torch, P, W, max(3, args.steps // 4), 1)
        if not args.no_accel:
            out["restart_accel_4096"] = bench_accel(torch, P, W, 2, 1)
        out["cstr_nmpc_5000"] = bench_cstr()
        out["rti_cartpole_256"] = bench_rti()
        out["fp64_chain_20"] = bench_fp64_chain(torch, P, W, 20)
        out["paper_table1_context"] = bench_table1(torch, P, W)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
