"""Benchmark: space-time FGMRES time-to-1e-8 and DOF-iterations/s on one MI355X.

A step is one FGMRES(30) solve to a true relative residual of 1e-8 of the whole
linearised space-time MHD system (every slab at once) with the block
preconditioner P_T applied in FP32 (Krylov, residual and least squares in
FP64).  Workload (default): 64 x 64 mesh, Q2-Q1 velocity/pressure and Q1
current/potential, Nt = 128 backward-Euler slabs, dt = 0.01, Re = S = 100,
seeded smooth synthetic state and N(0,1) right-hand side.  The same solve with
an FP64 preconditioner is timed beside it (speed-up of FP32 over FP64).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ST-FGMRES time-to-1e-8 residual + DOF-iters/s; FP32-precond vs FP64, % HBM"
HBM_PEAK_GBS = 8000.0
# HBM traffic of one J apply at the default workload from FETCH_SIZE / WRITE_SIZE
# counter runs calibrated with a 1 GiB copy (profiles/pmc_cfg3_jacobian_fetch_write.md),
# valid while the kernel source it measured is unchanged (digest of that source).
JAC_COUNTERS = {"config": "cfg3", "j_slabs": 8, "source_sha256_16": "9e73605d16ae5780", "traffic_bytes": 2.332e9}
# The same for one launch of the paired sweep-step kernel at the default workload
# (profiles/pmc_cfg3_sweep_step_fetch_write.md).
SWEEP_COUNTERS = {"config": "cfg3", "source_sha256_16": "17a2f7a3c39f8932", "traffic_bytes": 1.051e7}
# rocprofv3 average duration of that kernel at the default workload without event sampling
# (profiles/kstats_cfg3_fgmres_fp32_pipeline.md), valid for the same kernel source.
SWEEP_ROCPROF = {"config": "cfg3", "source_sha256_16": "17a2f7a3c39f8932", "avg_us": 4.13}


def jacobian_kernel_digest():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2309_00768_amd", "csrc", "kernels.h")).read()
    a = src.index("struct SpmvSlabsArgs {")
    b = src.index("// Fused Chebyshev-Jacobi step for A x = b")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def sweep_kernel_digest():
    """Digest of the stencil step kernel source (the paired sweep-step kernel's bodies)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2309_00768_amd", "csrc", "kernels.h")).read()
    a = src.index("// Operator on a structured node grid")
    b = src.index("// A Chebyshev-Jacobi sweep solve (or a run of its steps)")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


# Workloads whose residual plateau is longer than FGMRES(30)'s restart (the
# shear-layer state of cfg2; Re = S = 1000): a restart past the plateau.
CONFIG_DEFAULTS = {"cfg2": {"restart": 1000, "maxit": 3000},
                   "cfg3_re1000": {"restart": 2000, "maxit": 2500, "precision": "fp64"}}

GROUPING = {"all": "every member in one lockstep batch", "mesh": "one lockstep batch per mesh size",
            "split": "members with n < 64 in one lockstep batch, the others one at a time"}


def orth_name(orth, m, N):
    delayed = orth == "delayed" or (orth == "auto" and (m > 64 or N >= 1 << 20))
    return "CGS2 with delayed reorthogonalisation" if delayed else "CGS2"


def variant_name(v):
    return {"PT": "P_T", "Ptilde": "P-tilde", "P": "full P"}[v]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def jacobian_bytes(plan, nt, N):
    """Algorithmic bytes of one J apply: every per-slab value once (8 B), every shared value
    once (8 B), every index once (4 B, shared by all slabs), x read and y written (16 B/DOF)."""
    state = sum(plan.block_nnz(b) for b in ("Fu", "Zj", "ZA", "Y", "FA"))
    const = 2 * plan.block_nnz("B") + plan.block_nnz("Mj") + plan.block_nnz("KjA") + plan.block_nnz("Mu") \
        + plan.block_nnz("MA")
    return 8 * nt * state + 8 * const + 4 * (state + const) + 16 * N, state, const


def _oracle_worker(cfg_name, nt_sample, seed, rtol, keep_x, barrier, queue):
    """One oracle solve (exact inner solves, GMRES(30)) on the first nt_sample
    slabs of a workload, right-hand side seed `seed`; single-threaded.  The
    setup (assembly and factorisations) runs first; all workers then start
    their solves together."""
    import oracle
    from paper_2309_00768_amd import inputs
    cfg = inputs.CONFIGS[cfg_name]
    t0 = time.perf_counter()
    ub, ab = inputs.state(cfg)
    sysm = oracle.SpaceTimeSystem(cfg.n, nt_sample, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub[:nt_sample],
                                  ab[:nt_sample])
    b = inputs.rhs(inputs.Config("s", cfg.n, nt_sample, cfg.dt, cfg.re, cfg.s), seed)
    sysm.apply_PT_inv(b)            # factorisations (setup) outside the timed solve
    setup = time.perf_counter() - t0
    barrier.wait()
    t1 = time.perf_counter()
    x, its, _ = oracle.solve_fgmres(sysm, b, rtol=rtol)
    t2 = time.perf_counter()
    queue.put({"seed": seed, "N": sysm.N, "its": its, "setup_s": setup, "t_start": t1, "t_end": t2,
               "x": x if keep_x else None})


def _get_result(queue, procs, poll=10.0):
    """The next worker result; raises if a worker ended without delivering one."""
    import queue as q
    while True:
        try:
            return queue.get(timeout=poll)
        except q.Empty:
            dead = [p.exitcode for p in procs if p.exitcode not in (None, 0)]
            if dead:
                raise RuntimeError(f"an oracle worker process failed (exit codes {dead})")


def cpu_baseline(cfg, nt_sample, rtol, workers):
    """The oracle (exact inner solves, GMRES(30)) on the first `nt_sample` slabs of
    the same workload, in `workers` single-threaded processes at once, each with
    its own right-hand side seed (the first with the benchmark's); value = all
    their DOF-iterations over the wall time from the common start of the solves
    to the last one's end.  Runs before the GPU is touched (worker processes are
    started fresh).  Also returns worker 0's solution: J is block
    lower-bidiagonal in time, so the first nt_sample slabs of the full system's
    x* are the solution of the nt_sample-slab system."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    barrier, queue = ctx.Barrier(workers), ctx.Queue()
    env_threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_threads:
        os.environ[k] = "1"
    procs = [ctx.Process(target=_oracle_worker,
                         args=(cfg.name, nt_sample, cfg.rhs_seeds[0] + 100 * i, rtol, i == 0, barrier, queue))
             for i in range(workers)]
    try:
        for p in procs:
            p.start()
        res = [_get_result(queue, procs) for _ in procs]
        for p in procs:
            p.join()
    finally:
        for k, v in env_threads.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    t0 = min(r["t_start"] for r in res)
    t1 = max(r["t_end"] for r in res)
    dof_its = sum(r["N"] * r["its"] for r in res)
    r0 = next(r for r in res if r["x"] is not None)
    one = r0["N"] * r0["its"] / (r0["t_end"] - r0["t_start"])
    out = {"value": dof_its / (t1 - t0), "unit": "DOF-iter/s", "cores": workers, "kind": "oracle",
           "sample": f"oracle GMRES(30)+P_T with sparse-LU inner solves to {rtol:g} on the first {nt_sample} of "
                     f"{cfg.nt} slabs of the same workload (N={r0['N']}), {workers} single-threaded processes "
                     f"at once, one right-hand side each; {dof_its:.3g} DOF-iterations in {t1 - t0:.1f} s "
                     f"(host has {os.cpu_count()} logical CPUs)",
           "iterations": [r["its"] for r in res],
           "one_process_dof_iters_per_s": one,
           "setup_s_per_process": max(r["setup_s"] for r in res)}
    return out, r0["x"], r0["its"]


def _oracle_batch_worker(index, rtol, timed, queue):
    """The oracle on uneven-batch member `index`, single-threaded: x* by the
    direct forward substitution in time (sparse LU of every slab Jacobian), then
    (if timed) GMRES(30) + P_T with exact inner solves, timed after its setup."""
    import oracle
    from paper_2309_00768_amd import inputs
    c = inputs.batch_configs()[index]
    ub, ab = inputs.state(c)
    sysm = oracle.system_from_config(c, ub, ab)
    b = inputs.rhs(c, c.rhs_seeds[0])
    xs = sysm.direct_solve(b)
    its, t1, t2 = 0, None, None
    if timed:
        sysm.apply_PT_inv(b)            # factorisations (setup) outside the timed solve
        t1 = time.perf_counter()
        _, its, _ = oracle.solve_fgmres(sysm, b, rtol=rtol, maxit=2000)
        t2 = time.perf_counter()
    queue.put({"index": index, "N": sysm.N, "its": its, "t_start": t1, "t_end": t2, "x": xs})


def cpu_baseline_batch(members, timed, rtol):
    """The oracle on the given uneven-batch members, one single-threaded process
    each, started before the GPU is touched: every member's direct solution x*,
    and GMRES + P_T timed on the members in `timed`; value = their DOF-iterations
    over the wall time from the common start of their solves to the last one's end."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    queue = ctx.Queue()
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    procs = [ctx.Process(target=_oracle_batch_worker, args=(i, rtol, i in timed, queue)) for i in members]
    try:
        for p in procs:
            p.start()
        res = [_get_result(queue, procs) for _ in procs]
        for p in procs:
            p.join()
    finally:
        for k, v in env.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    tres = [r for r in res if r["t_start"] is not None]
    t0, t1 = min(r["t_start"] for r in tres), max(r["t_end"] for r in tres)
    dof_its = sum(r["N"] * r["its"] for r in tres)
    out = {"value": dof_its / (t1 - t0), "unit": "DOF-iter/s", "cores": len(tres), "kind": "oracle",
           "sample": f"oracle GMRES(30)+P_T with sparse-LU inner solves to {rtol:g} on uneven-batch member(s) "
                     f"{sorted(timed)}, one single-threaded process each; {dof_its:.3g} DOF-iterations in "
                     f"{t1 - t0:.1f} s",
           "iterations": {r["index"]: r["its"] for r in tres}}
    return out, {r["index"]: r["x"] for r in res}


def probe_jacobian(cfg, ub, ab, b, dev, launches=5, copy_bytes=1 << 30):
    """A few J applies and one device copy of `copy_bytes` (read + write), for
    FETCH_SIZE / WRITE_SIZE counter runs: the copy calibrates the counters."""
    import torch
    from paper_2309_00768_amd import binding
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision="fp32")
    N = plan.ns * cfg.nt
    jbytes, _, _ = jacobian_bytes(plan, cfg.nt, N)
    sysg = binding.System(plan, dev)
    plan.close()
    x = torch.from_numpy(b).to(dev)
    y = torch.empty_like(x)
    src = torch.ones(copy_bytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(launches):
        sysg.apply_jacobian(x, y)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "jacobian", "launches": launches, "algorithmic_bytes_per_launch": jbytes,
                      "copy_bytes_read": copy_bytes, "copy_bytes_written": copy_bytes}), flush=True)


def probe_sweeps(cfg, ub, ab, b, dev, applies=3, copy_bytes=1 << 30):
    """A few recorded P_T^{-1} applies (FP32) and one device copy of `copy_bytes`,
    for FETCH_SIZE / WRITE_SIZE counter runs of the paired sweep-step kernel."""
    import torch
    from paper_2309_00768_amd import binding
    plan = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision="fp32")
    nnz = {k: plan.block_nnz(k) for k in ("Fu", "C0")}
    sysg = binding.System(plan, dev)
    plan.close()
    nu, na = sysg.offsets[2] - sysg.offsets[0], sysg.offsets[5] - sysg.offsets[4]
    r = torch.from_numpy(b).to(dev)
    z = torch.empty_like(r)
    src = torch.ones(copy_bytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(applies):
        sysg.apply_precond(r, z)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "sweeps", "applies": applies,
                      "algorithmic_bytes_per_launch": 4 * (nnz["Fu"] + nnz["C0"]) + 28 * (nu + na),
                      "nnz_Fu": nnz["Fu"], "nnz_CA": nnz["C0"], "rows_u": nu, "rows_A": na,
                      "copy_bytes_read": copy_bytes, "copy_bytes_written": copy_bytes}), flush=True)


def bench_batch(args, dev, cpu=None):
    """Uneven batch: 16 systems (n in {16,...,96}, Nt in {16,...,256}, dt = 1/Nt,
    Re = S = 300), FP32 preconditioner, solved together in lockstep; a step is
    one batched solve of every member.  The same systems solved one at a time
    (each with its own recorded preconditioner pipeline) are timed beside it."""
    import torch
    from paper_2309_00768_amd import binding, inputs
    cfgs = inputs.batch_configs()
    systems, rhs, singles, ntot = [], [], [], 0
    t0 = time.perf_counter()
    for c in cfgs:
        ub, ab = inputs.state(c)
        plan = binding.Plan(c.n, c.nt, c.dt, c.mu, c.eta, c.mu0, ub, ab, precision="fp32",
                            autotune=not args.no_autotune)
        si = plan.solver_info()
        systems.append(binding.System(plan, dev))
        plan.close()
        rhs.append(torch.from_numpy(inputs.rhs(c, c.rhs_seeds[0])).to(dev))
        ntot += systems[-1].N
        log(f"setup {c.name}: n={c.n} Nt={c.nt} N={systems[-1].N}, inner degrees F_u {si[0]} C_A {si[1]} "
            f"(kappa {si[2]:.1f}, {si[3]:.1f}), launches {systems[-1].tuning()}")
    log(f"setup {time.perf_counter() - t0:.1f} s, {len(cfgs)} systems, N total {ntot}")
    # Lockstep groups: every member in one batch, or one batch per mesh size
    # (members of one size have launches of similar length, so a grouped
    # launch does not wait for a much larger member's op).
    if args.batch_groups == "mesh":
        sizes = sorted({c.n for c in cfgs})
        groups = [[i for i, c in enumerate(cfgs) if c.n == nn] for nn in sizes]
    elif args.batch_groups == "split":
        # members whose sweep steps fill the GPU alone (n >= 64: 32,258 F_u rows
        # per slab or more) solved one at a time, the latency-bound rest in lockstep
        groups = [[i for i, c in enumerate(cfgs) if c.n < 64]] + [[i] for i, c in enumerate(cfgs) if c.n >= 64]
    else:
        groups = [list(range(len(cfgs)))]
    batches = [binding.Batch([systems[i] for i in g], restart=30) if len(g) > 1 else None for g in groups]
    counts = [b.launch_counts() if b is not None else (0, 0) for b in batches]
    lock, sep = sum(c[0] for c in counts), sum(c[1] for c in counts)
    # Iteration budget per member, in calls of whole restart cycles (the next
    # call restarts from the iterate); members that stagnate use all of it.
    budget = args.batch_budget
    chunk = min(240, budget)
    # Second phase: a member still open after the lockstep budget (P_T is weak
    # at Re = S = 300 with long steps, and FGMRES(30) stalls there) continues
    # alone from its iterate with a long restart (delayed reorthogonalisation).
    # Its long-restart system (2 m + 1 Krylov vectors) is set up when needed
    # and released after the solve; that setup is not timed.
    long_m = args.long_restart
    longs = set()
    setup_in_timed = [0.0]

    def finish(i, x, total, status, res):
        """Phase two for member i from iterate x; updates the tallies."""
        if long_m <= 0 or status[i] == 0:
            return x
        t1 = time.perf_counter()
        c = cfgs[i]
        # restart within the memory given to the long-restart Krylov vectors (V and Z, FP64)
        m_i = max(30, min(long_m, int(args.long_mem_gb * 1e9 / (16 * systems[i].N))))
        ub, ab = inputs.state(c)
        plan = binding.Plan(c.n, c.nt, c.dt, c.mu, c.eta, c.mu0, ub, ab, precision="fp32",
                            autotune=not args.no_autotune, max_restart=m_i)
        sg = binding.System(plan, dev)
        plan.close()
        torch.cuda.synchronize()
        setup_in_timed[0] += time.perf_counter() - t1
        x, info, rc, _ = sg.solve(rhs[i], x, restart=m_i, rtol=args.rtol, maxit=args.long_maxit, x0=True)
        if rc < 0:
            raise RuntimeError(f"long-restart solve of member {i}: status {rc}")
        log(f"  member {i}: FGMRES({m_i}) {info.iterations} its, {info.seconds:.2f} s, "
            f"residual {info.true_rel_residual:.1e}")
        total[i] += info.iterations
        status[i], res[i] = rc, info.true_rel_residual
        longs.add(i)
        t1 = time.perf_counter()
        sg.close()
        del sg
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        setup_in_timed[0] += time.perf_counter() - t1
        return x

    final = {}

    def solve_all(label):
        total = [0] * len(rhs)
        status = [1] * len(rhs)
        res = [1.0] * len(rhs)
        for g, batch in zip(groups, batches):
            bs = [rhs[i] for i in g]
            xs = [torch.zeros_like(b) for b in bs]
            for call in range(max(1, budget // chunk)):
                if batch is None:   # one member: its own recorded pipeline
                    x1, info1, rc, _ = systems[g[0]].solve(bs[0], xs[0], rtol=args.rtol, maxit=chunk, x0=call > 0)
                    xs, infos, sts = [x1], [info1], [rc]
                else:
                    xs, infos, sts, rc, _ = batch.solve(bs, xs, rtol=args.rtol, maxit=chunk, x0=call > 0)
                if rc < 0:
                    raise RuntimeError(f"batched solve: status {rc}, member statuses {sts}")
                for i, inf, st in zip(g, infos, sts):
                    total[i] += inf.iterations
                    status[i], res[i] = st, inf.true_rel_residual
                if rc == 0:
                    break
            xs = [finish(i, x, total, status, res) for i, x in zip(g, xs)]
            final.update(zip(g, xs))
            log(f"  {label}: group {g}: {sum(total[i] for i in g)} member iterations, open: "
                f"{[(k, f'{res[k]:.1e}') for k in g if status[k] != 0]}")
        return total, status, res

    for i in range(args.warmup):
        solve_all(f"warmup {i}")
    torch.cuda.synchronize()
    setup_in_timed[0] = 0.0
    t0 = time.perf_counter()
    runs = [solve_all(f"step {i}") for i in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0 - setup_in_timed[0]
    dof_its = sum(s.N * k for its, _, _ in runs for s, k in zip(systems, its))
    its, status, res = runs[-1]
    converged = [st == 0 for st in status]
    log(f"batched: {elapsed / args.steps:.2f} s per batch, iterations {its}")
    out = {
        "metric": METRIC, "value": dof_its / elapsed, "unit": "DOF-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-precond/f64-krylov", "data": "synthetic",
        "config": {"workload": f"cfg4: {len(cfgs)} uneven systems (n, Nt) = "
                               f"{[(c.n, c.nt) for c in cfgs]}, dt = 1/Nt, Re=S=300; lockstep FGMRES(30) "
                               f"({GROUPING[args.batch_groups]}) to "
                               f"{args.rtol:g} within {budget} iterations per member"
                               + (f", then FGMRES(m <= {long_m}, Krylov vectors within {args.long_mem_gb:g} GB) alone "
                                  f"for the members still open (at most {args.long_maxit} iterations)"
                                  if long_m > 0 else "") + ", P_T in FP32",
                   "N_total": ntot},
        "time_to_1e8_s": elapsed / args.steps if all(converged) else None,
        "fgmres_iters": its, "converged": converged, "true_rel_residual": res,
        "launches_per_arnoldi_step": {"lockstep": lock, "one_at_a_time": sep},
        "lockstep_groups": groups,
        "long_restart_members": sorted(longs),
        "setup_excluded_s": setup_in_timed[0],
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu[0]
        out["error_vs_oracle"] = {
            str(i): float(np.linalg.norm(final[i].cpu().numpy() - xs) / np.linalg.norm(xs)) for i, xs in cpu[1].items()}
        out["error_vs_oracle"]["reference"] = "the oracle's direct forward substitution in time (sparse LU per slab)"
        log(f"error vs oracle x*: {out['error_vs_oracle']}")
    if not args.no_separate:
        # the same systems one at a time, same budget (each with its own recorded pipeline)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sep_its = []
        setup_in_timed[0] = 0.0
        for k, (sg, b) in enumerate(zip(systems, rhs)):
            x = torch.zeros_like(b)
            tally, st_k, res_k = [0] * len(rhs), [1] * len(rhs), [1.0] * len(rhs)
            for call in range(max(1, budget // chunk)):
                x, info, rc, _ = sg.solve(b, x, rtol=args.rtol, maxit=chunk, x0=call > 0)
                tally[k] += info.iterations
                st_k[k] = rc
                if rc < 0:
                    raise RuntimeError(f"separate solve: status {rc}")
                if rc == 0:
                    break
            x = finish(k, x, tally, st_k, res_k)
            sep_its.append(tally[k])
            log(f"  one at a time: member {k} ({tally[k]} its), {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        tsep = time.perf_counter() - t0 - setup_in_timed[0]
        sep_rate = sum(s.N * k for s, k in zip(systems, sep_its)) / tsep
        out["one_at_a_time_s"] = tsep
        out["one_at_a_time_dof_iters_per_s"] = sep_rate
        out["batch_speedup"] = out["value"] / sep_rate
        log(f"one at a time: {tsep:.2f} s")
    print(json.dumps(out), flush=True)


def bench_newton(args, dev):
    """Space-time Newton on the paper's model problems (island coalescence and
    the tearing mode's Harris sheet on the unit square), mu = eta = mu0 = 1,
    Newton to ||R|| <= 1e-10 with FGMRES(30) + P_T to a relative 1e-2 or an
    absolute 1e-14 per correction (the paper's tolerances), over a grid of
    mesh and time-step sizes with T = 1: the shape of the paper's Table 1."""
    import torch
    from paper_2309_00768_amd import binding, inputs
    rows = []
    sizes = [(16, 16), (32, 16), (32, 32), (32, 64), (64, 32)]
    # spatial solves of the sweeps: one SA-AMG V(1,1) cycle (these problems are
    # diffusion-dominated: mu dt / h^2 = 16 to 256), the automatic choice per
    # solve, or converged ones (EXACT mode: the paper's exact inner solves)
    inner = {"vcycle": {"fu_solver": -1, "ca_solver": -1}, "auto": {}, "exact": {"inner": "exact"}}
    t_all = time.perf_counter()
    for name, n, nt, how in [(nm, n, nt, h) for nm in ("island", "tearing") for (n, nt) in sizes
                             for h in ("vcycle", "auto", "exact") if h == "vcycle" or (n, nt) in ((16, 16), (32, 32))]:
            prob = inputs.ModelProblem(name, n, nt, 1.0 / nt)
            fl = inputs.model_newton_fields(prob)
            t0 = time.perf_counter()
            nw = binding.Newton(n, nt, prob.dt, prob.mu, prob.eta, prob.mu0, fl, device=dev, precision=args.precision,
                                **inner[how])
            setup = time.perf_counter() - t0
            torch.cuda.synchronize()
            x, info, rc = nw.solve(atol=1e-10, lin_rtol=1e-2, lin_atol=1e-14)
            its = list(info.linear_iterations[:info.newton_iterations])
            rows.append({"problem": name, "n": n, "nt": nt, "inner": how, "N": nw.N, "newton": info.newton_iterations,
                         "fgmres_per_newton": sum(its) / max(len(its), 1), "converged": bool(info.converged),
                         "final_residual": info.residual_norm[info.newton_iterations],
                         "seconds": info.seconds, "reassembly_seconds": info.setup_seconds, "setup_s": setup})
            log(f"{name} n={n} Nt={nt} ({how}): Newton {info.newton_iterations} ({rows[-1]['fgmres_per_newton']:.2f} "
                f"FGMRES its each), ||R|| {rows[-1]['final_residual']:.1e}, {info.seconds:.2f} s "
                f"({info.setup_seconds:.2f} s re-assembly)")
            del nw
    total = time.perf_counter() - t_all
    dofs = sum(r["N"] * sum([r["fgmres_per_newton"] * r["newton"]]) for r in rows)
    out = {"metric": METRIC, "value": dofs / sum(r["seconds"] for r in rows), "unit": "DOF-iter/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": 1e3 * sum(r["seconds"] for r in rows),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32-precond/f64-krylov" if args.precision == "fp32" else "f64", "data": "synthetic",
           "config": {"workload": "space-time Newton on island coalescence and the tearing mode (unit square, "
                                  "Dirichlet u and A, mu = eta = mu0 = 1, T = 1), Newton to 1e-10, FGMRES(30) + P_T "
                                  "to rel 1e-2 / abs 1e-14"},
           "newton": rows, "wall_s": total}
    print(json.dumps(out), flush=True)


def bench_adjoint(args, dev):
    """Adjoint workload: 128 x 128 mesh, Nt = 128, dt = 0.005, Re = S = 500, FP64.
    A step is one gradient of J = 1/2 |A(T) - A_target|^2 with respect to the
    initial potential A0 and the forcing f through the autograd Function: a
    forward solve and the transposed, backward-in-time adjoint solve, both to
    1e-12.  The gradient is checked against central differences in 8 seeded
    directions (J is exactly quadratic, so the differences are exact up to the
    solve tolerance)."""
    import torch
    from paper_2309_00768_amd import autograd as stg
    from paper_2309_00768_amd import inputs
    cfg = inputs.CONFIGS["cfg5"]
    ub, ab = inputs.state(cfg)
    t0 = time.perf_counter()
    prob = stg.SpaceTimeProblem(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision="fp64",
                                rtol=1e-12, checkpoint="auto", device=dev)
    log(f"setup {time.perf_counter() - t0:.1f} s, N={prob.N}")
    n, nt = cfg.n, cfg.nt
    na, nu = (n - 1) ** 2, 2 * (2 * n - 1) ** 2
    a0 = torch.from_numpy(inputs.free_a_field(cfg, 2)).to(dev).requires_grad_(True)
    f = torch.from_numpy(inputs.random_vector(nt * nu, 1)).to(dev).requires_grad_(True)
    target = torch.from_numpy(inputs.free_a_field(cfg, 3)).to(dev)

    def loss(a, ff):
        return 0.5 * ((stg.terminal_potential(prob, a, ff) - target) ** 2).sum()

    def gradient():
        a0.grad = None
        f.grad = None
        L = loss(a0, f)
        L.backward()
        return L

    for i in range(args.warmup):
        gradient()
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        L = gradient()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ga, gf = a0.grad.detach().clone(), f.grad.detach().clone()
    worst, checks = 0.0, []
    if not args.no_fd:
        for s in range(8):
            da = torch.from_numpy(inputs.random_vector(na, 10 + s)).to(dev)
            df = torch.from_numpy(inputs.random_vector(nt * nu, 20 + s) * 0.1).to(dev)
            eps = 1e-3
            with torch.no_grad():
                fd = (loss(a0 + eps * da, f + eps * df) - loss(a0 - eps * da, f - eps * df)).item() / (2 * eps)
            ad = (ga @ da + gf @ df).item()
            err = abs(fd - ad) / max(abs(fd), 1e-30)
            worst = max(worst, err)
            checks.append(err)
            log(f"  direction {s}: finite difference {fd:.10e}, adjoint {ad:.10e}, relative {err:.2e}")
    out = {
        "metric": METRIC, "value": prob.N * 2 / (elapsed / args.steps), "unit": "DOF-solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"cfg5: {n}x{n} Q2-Q1/Q1/Q1, Nt={nt}, dt={cfg.dt}, Re=S={cfg.re:g}; gradient of "
                               f"1/2|A(T) - A_target|^2 w.r.t. A0 and f: forward + adjoint FGMRES(30) to 1e-12, "
                               f"FP64", "N": prob.N},
        "gradient_s": elapsed / args.steps, "loss": float(L.item()), "rebuilds": prob.rebuilds,
        "fd_worst_relative": worst if checks else None, "fd_relative": checks,
    }
    print(json.dumps(out), flush=True)


def parse_args(argv=None):
    """The command line, with the per-workload defaults of the options left unset."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cfg3")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=None,
                    help="FGMRES iteration cap of a solve (default 1000; cfg2 3000, cfg3_re1000 2500)")
    ap.add_argument("--restart", type=int, default=None,
                    help="FGMRES restart length m (default 30; cfg2 1000, cfg3_re1000 2000: restarts longer than "
                         "the residual plateau of these workloads)")
    ap.add_argument("--orth", choices=["auto", "cgs2", "delayed"], default="auto",
                    help="Gram-Schmidt of the Arnoldi steps (auto: delayed reorthogonalisation above restart 64 "
                         "or from 2^20 unknowns)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-slabs", type=int, default=16)
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes at once (0: min(16, CPUs))")
    ap.add_argument("--cpu-rtol", type=float, default=1e-12,
                    help="oracle tolerance (its solution on the sampled slabs is the reference x*)")
    ap.add_argument("--sweep-lanes", type=int, default=0, choices=[0, 1, 2],
                    help="lanes per row of the F_u sweep steps when not autotuned (0: library default)")
    ap.add_argument("--time-parallel", type=int, default=0,
                    help="Parareal iterations for the two sweeps of P_T (0: forward substitution in time)")
    ap.add_argument("--time-coarse", type=int, default=1,
                    help="Chebyshev steps of the Parareal coarse propagator per slab")
    ap.add_argument("--sweep-chunk", type=int, default=0,
                    help="slabs per chunk of the recorded P_T pipeline (0: library default)")
    ap.add_argument("--single-stream", action="store_true",
                    help="P_T step by step in program order instead of the recorded two-program replay")
    ap.add_argument("--inner", choices=["auto", "vcycle"], default="auto",
                    help="spatial solves of the F_u and C_A sweeps: automatic (Chebyshev-Jacobi alone at the "
                         "default workload) or one SA-AMG V(1,1) cycle per sweep step")
    ap.add_argument("--inner-degrees", default="",
                    help="F,C: Chebyshev-Jacobi degrees of the F_u and C_A sweep solves (default: the plan's choice)")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default=None,
                    help="preconditioner precision of the timed solves (cfg1-cfg3; fp64 leaves out the second, "
                         "all-FP64 comparison; default fp32, for cfg3_re1000 fp64, the faster there, whose "
                         "2000-vector basis leaves no room for a second system) and of the Newton corrections")
    ap.add_argument("--variant", choices=["PT", "Ptilde", "P"], default="PT",
                    help="preconditioner: P_T (default), P-tilde or the full P (step by step)")
    ap.add_argument("--window", type=int, default=1,
                    help="with --timestep: slabs per step (1: sequential time stepping with P_{T,k}; W > 1: "
                         "windows of W slabs solved all at once in turn)")
    ap.add_argument("--window-restart", type=int, default=0,
                    help="with --timestep: FGMRES restart per step (0: 30 for single slabs, 200 for windows)")
    ap.add_argument("--timestep", action="store_true",
                    help="also solve the workload by sequential time stepping with P_{T,k} (one-slab systems)")
    ap.add_argument("--profile-every", type=int, default=32,
                    help="time every k-th launch of the paired sweep-step kernel with HIP events")
    ap.add_argument("--no-separate", action="store_true", help="cfg4: skip the one-at-a-time comparison")
    ap.add_argument("--batch-budget", type=int, default=480,
                    help="cfg4: lockstep FGMRES(30) iterations per member")
    ap.add_argument("--long-restart", type=int, default=1200,
                    help="cfg4: restart of the second phase for members still open after the lockstep budget "
                         "(0: none)")
    ap.add_argument("--long-maxit", type=int, default=2400, help="cfg4: iteration cap of the second phase")
    ap.add_argument("--long-mem-gb", type=float, default=150.0,
                    help="cfg4: device memory for the second phase's Krylov vectors (caps its restart per member)")
    ap.add_argument("--batch-groups", choices=sorted(GROUPING), default="all",
                    help="cfg4: " + "; ".join(f"{k}: {v}" for k, v in GROUPING.items()))
    ap.add_argument("--no-fd", action="store_true", help="cfg5: skip the finite-difference check")
    ap.add_argument("--no-autotune", action="store_true",
                    help="default launch choices instead of timing them at st_create")
    ap.add_argument("--probe", choices=["jacobian", "sweeps"], default=None,
                    help="run only a few J applies (or P_T applies) and a copy of known size (for hardware-counter runs)")
    args = ap.parse_args(argv)
    # per-workload defaults of the options left unset
    dflt = {"restart": 30, "maxit": 1000, "precision": "fp32"}
    dflt.update(CONFIG_DEFAULTS.get(args.config, {}))
    for k, v in dflt.items():
        if getattr(args, k) is None:
            setattr(args, k, v)
    return args


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the solve of one system "
              f"is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)

    from paper_2309_00768_amd import inputs

    cpu = None
    if args.config == "cfg4" and not args.no_cpu:
        # the oracle on the smallest members (n = 16), before anything touches the GPU
        # (x* of every n = 16 member; GMRES timed on the shortest of them)
        bc = inputs.batch_configs()
        members = [i for i, c in enumerate(bc) if c.n == 16]
        timed = [min(members, key=lambda i: bc[i].nt)]
        log(f"cpu baseline (oracle, members {members}, GMRES timed on {timed}) ...")
        t0 = time.perf_counter()
        cpu = cpu_baseline_batch(members, timed, args.rtol)
        log(f"cpu baseline done in {time.perf_counter() - t0:.1f} s: {cpu[0]['value']:.3g} DOF-iter/s")
    # (cfg2 and cfg3_re1000: the oracle's GMRES(30) stalls on their plateaus and
    # a restart past it is no bounded CPU sample; no oracle leg by default)
    if args.config in ("cfg2", "cfg3_re1000"):
        args.no_cpu = True
    if args.config not in ("cfg4", "cfg5", "newton") and not args.no_cpu and args.probe is None:
        # before anything touches the GPU: the oracle's worker processes start fresh
        cfg = inputs.CONFIGS[args.config]
        args.cpu_slabs = min(args.cpu_slabs, cfg.nt)
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        log(f"cpu baseline (oracle, {workers} processes, first {args.cpu_slabs} slabs) ...")
        t0 = time.perf_counter()
        cpu = cpu_baseline(cfg, args.cpu_slabs, args.cpu_rtol, workers)
        log(f"cpu baseline done in {time.perf_counter() - t0:.1f} s: {cpu[0]['value']:.3g} DOF-iter/s")

    import torch
    from paper_2309_00768_amd import binding

    dev = torch.device("cuda:0")
    if args.config == "cfg4":
        bench_batch(args, dev, cpu)
        return
    if args.config == "cfg5":
        bench_adjoint(args, dev)
        return
    if args.config == "newton":
        bench_newton(args, dev)
        return
    cfg = inputs.CONFIGS[args.config]
    ub, ab = inputs.state(cfg)
    b = inputs.rhs(cfg, cfg.rhs_seeds[0])
    if args.probe == "jacobian":
        probe_jacobian(cfg, ub, ab, b, dev)
        return
    if args.probe == "sweeps":
        probe_sweeps(cfg, ub, ab, b, dev)
        return
    t0 = time.perf_counter()
    tune = not args.no_autotune
    m = args.restart
    # spatial solves of the sweeps: the automatic choice (Chebyshev-Jacobi alone where it reaches the
    # target reduction), or one SA-AMG V(1,1) cycle per sweep step on F_u,k and C_A,k
    solver = {"fu_solver": -1, "ca_solver": -1} if args.inner == "vcycle" else {}
    if args.inner_degrees:
        fu_d, ca_d = (int(v) for v in args.inner_degrees.split(","))
        solver.update(fu_solver=fu_d, ca_solver=ca_d)
    if args.time_parallel > 0:
        solver.update(time_parallel=args.time_parallel, time_coarse_degree=args.time_coarse)
    if args.single_stream:
        solver.update(single_stream=True)
    if args.sweep_chunk > 0:
        solver.update(sweep_chunk=args.sweep_chunk)
    prec = args.precision
    fp32 = prec == "fp32"
    plan32 = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision=prec, autotune=tune,
                          max_restart=m, sweep_lanes=args.sweep_lanes, variant=args.variant, **solver)
    N = plan32.ns * cfg.nt
    jbytes, nnz_state, nnz_const = jacobian_bytes(plan32, cfg.nt, N)
    plan_nnz = {b: plan32.block_nnz(b) for b in ("Fu", "C0")}
    fu_deg, ca_deg, _, _ = plan32.solver_info()
    inner = (f"Chebyshev-Jacobi sweeps of degree {fu_deg} on F_u,k and {ca_deg} on C_A,k "
             f"(0 = SA-AMG V(1,1)), SA-AMG V(1,1) on K_p")
    if args.time_parallel > 0:
        inner += (f"; both sweeps by {args.time_parallel} Parareal iterations (coarse propagator: "
                  f"{args.time_coarse} Chebyshev step(s) per slab), step by step")
    sys32 = binding.System(plan32, dev)
    plan32.close()
    log(f"setup {prec} {time.perf_counter() - t0:.1f} s, N={N}, launches {sys32.tuning()}")
    sys64 = None
    if fp32 and not args.no_fp64:
        t0 = time.perf_counter()
        plan64 = binding.Plan(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, precision="fp64",
                              autotune=tune, max_restart=m, sweep_lanes=args.sweep_lanes, variant=args.variant,
                              **solver)
        sys64 = binding.System(plan64, dev)
        plan64.close()
        log(f"setup fp64 {time.perf_counter() - t0:.1f} s, launches {sys64.tuning()}")
    # a step solves every right-hand side of the workload in turn (cfg2: three)
    bts = [torch.from_numpy(b).to(dev)] + [torch.from_numpy(inputs.rhs(cfg, sd)).to(dev) for sd in cfg.rhs_seeds[1:]]
    xs = [torch.zeros_like(bt) for bt in bts]

    statuses = []

    def solve(sysg):
        step = []
        for bt, x in zip(bts, xs):
            _, info, rc, _ = sysg.solve(bt, x, rtol=args.rtol, restart=m, maxit=args.maxit, orth=args.orth)
            if rc < 0:
                raise RuntimeError(f"solve failed: status {rc}")
            statuses.append(rc)
            step.append(info)
        return step

    for i in range(args.warmup):
        info = solve(sys32)
        log(f"warmup {i}: {sum(k.iterations for k in info)} its, {sum(k.seconds for k in info):.3f} s")
    profiled = sys32.tuning()["precond_launches"] > 0 and args.profile_every > 0
    if profiled:
        sys32.profile_kernel(1, args.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [k for _ in range(args.steps) for k in solve(sys32)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    x32 = xs[0].clone()
    its = sum(i.iterations for i in infos)
    converged = all(rc == 0 for rc in statuses)
    value = N * its / elapsed
    jac_s = sum(i.jacobian_seconds for i in infos)
    jac_n = sum(i.jacobian_calls for i in infos)
    jac_avg = jac_s / max(jac_n, 1)
    res = max(i.true_rel_residual for i in infos)
    log(f"{prec} precond: {its / args.steps:.1f} its/step, {elapsed / args.steps:.3f} s/step ({len(bts)} right-hand "
        f"side(s) per step), residual {res:.2e}")

    out = {
        "metric": METRIC, "value": value, "unit": "DOF-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-precond/f64-krylov" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.n}x{cfg.n} Q2-Q1/Q1/Q1, Nt={cfg.nt}, dt={cfg.dt}, "
                               f"Re=S={cfg.re:g}; FGMRES({m}, {orth_name(args.orth, m, N)}) to {args.rtol:g}, {variant_name(args.variant)} in "
                               f"{prec.upper()}: {inner}",
                   "N": N, "nt": cfg.nt, "n": cfg.n, "rhs_per_step": len(bts)},
        "time_to_1e8_s": elapsed / args.steps if converged else None,
        "converged": converged,
        "fgmres_iters": its / args.steps,
        "true_rel_residual": res,
        "precond_share": sum(i.precond_seconds for i in infos) / elapsed,
        "launch_choices": {prec: sys32.tuning(), "autotuned": tune},
    }
    x64 = None
    if sys64 is not None:
        statuses.clear()
        solve(sys64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info64 = solve(sys64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        x64 = xs[0].clone()
        ok64 = all(rc == 0 for rc in statuses)
        its64 = sum(k.iterations for k in info64)
        out["fp64_time_to_1e8_s"] = t64 if ok64 else None
        out["fp64_fgmres_iters"] = its64
        out["fp32_vs_fp64_speedup"] = t64 / (elapsed / args.steps) if (ok64 and converged) else None
        out["launch_choices"]["fp64"] = sys64.tuning()
        log(f"fp64 precond: {its64} its, {t64:.3f} s")
    # Roofline of the dominant kernel: the paired sweep-step kernel (one
    # Chebyshev-Jacobi step of an F_u,k solve and one of a C_A,k solve per
    # launch).  Algorithmic bytes per launch: every true nonzero of the two
    # slab operators once (4 B in FP32, 8 in FP64) and 7 vector passes per row
    # (r, x read and written; d_old, D^{-1} read; d_new written).
    nnz_fu, nnz_ca = plan_nnz["Fu"], plan_nnz["C0"]
    nu, na = sys32.offsets[2] - sys32.offsets[0], sys32.offsets[5] - sys32.offsets[4]
    wb = 4 if fp32 else 8
    sweep_bytes = wb * (nnz_fu + nnz_ca) + 7 * wb * (nu + na)
    jac = {"kernel": (f"k_spmv_slabs<{sys32.tuning()['j_slabs']}, 4> (space-time Jacobian apply)"),
           "bytes_per_launch": jbytes, "avg_launch_ms": jac_avg * 1e3, "launches": jac_n,
           "achieved_GBs": jbytes / jac_avg / 1e9, "frac": jbytes / jac_avg / 1e9 / HBM_PEAK_GBS,
           "traffic": None, "nnz_state_per_slab": nnz_state, "nnz_shared": nnz_const}
    nv = sys32.tuning()["j_slabs"]
    if (args.config == JAC_COUNTERS["config"] and nv == JAC_COUNTERS["j_slabs"]
            and jacobian_kernel_digest() == JAC_COUNTERS["source_sha256_16"]):
        jac["traffic"] = JAC_COUNTERS["traffic_bytes"]
    psec, pn, pseen = sys32.profile_read() if profiled else (0.0, 0, 0)
    if pn > 0:
        # (no paired sweep step runs when the sweeps take V-cycles: then J is the kernel reported)
        p_avg = psec / pn
        achieved = sweep_bytes / p_avg / 1e9
        traffic = None
        if (fp32 and args.config == SWEEP_COUNTERS["config"]
                and sweep_kernel_digest() == SWEEP_COUNTERS["source_sha256_16"]):
            traffic = SWEEP_COUNTERS["traffic_bytes"]
        frac_rp = None
        if (fp32 and args.config == SWEEP_ROCPROF["config"]
                and sweep_kernel_digest() == SWEEP_ROCPROF["source_sha256_16"]):
            frac_rp = sweep_bytes / (SWEEP_ROCPROF["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
        out["roofline"] = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "frac_rocprof": frac_rp,
            "kernel": f"k_two<BodyStCheb<{'float' if fp32 else 'double'}>, BodyStCheb<{'float' if fp32 else 'double'}>> "
                      "(paired sweep step: one Chebyshev-Jacobi step of a C_A,k solve and one of an F_u,k solve)",
            "bytes_per_launch": sweep_bytes, "avg_launch_ms": p_avg * 1e3, "launches_timed": pn,
            "launches": pseen, "share_of_solve_time": pseen * p_avg / elapsed,
            "nnz_Fu_per_slab": nnz_fu, "nnz_CA_per_slab": nnz_ca, "rows_u": nu, "rows_A": na,
            "jacobian": jac}
    else:
        out["roofline"] = {"bound": "hbm", "achieved": jac["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": jac["frac"], "traffic": jac["traffic"], "kernel": jac["kernel"],
                           "bytes_per_launch": jbytes, "avg_launch_ms": jac_avg * 1e3, "launches": jac_n}
    if args.timestep:
        # the same workload by sequential time stepping with P_{T,k}: one one-slab
        # system per slab (or one per window of W slabs; the preconditioner in the
        # precision of the timed solves), each step to ||r_k|| <= rtol ||b|| sqrt(W / Nt)
        t0 = time.perf_counter()
        W = max(1, args.window)
        wm = args.window_restart or (30 if W == 1 else 200)
        ts = binding.TimeStepping(cfg.n, cfg.nt, cfg.dt, cfg.mu, cfg.eta, cfg.mu0, ub, ab, device=dev,
                                  precision=prec, window=W, restart=wm)
        log(f"time stepping setup {time.perf_counter() - t0:.1f} s ({len(ts.systems)} systems of {W} slab(s))")
        bt = bts[0]
        xts = torch.zeros_like(bt)
        ts.solve(bt, xts, rtol=args.rtol)        # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xts, tinfos, trc = ts.solve(bt, xts, rtol=args.rtol)
        torch.cuda.synchronize()
        tts = time.perf_counter() - t0
        step_its = [i.iterations for i in tinfos]
        avg = sum(step_its) / len(step_its)
        out["time_stepping"] = {
            "preconditioner": (f"P_{{T,k}} (single step), {prec.upper()}, FGMRES({wm}) per step, warm start"
                               if W == 1 else
                               f"P_T of each window of {W} slabs (windowed space-time), {prec.upper()}, "
                               f"FGMRES({wm}) per window, warm start"),
            "window": W,
            "time_s": tts, "converged": trc == 0, "iterations_total": sum(step_its),
            "iterations_per_step_avg": avg, "iterations_per_step_max": max(step_its),
            # against the first right-hand side's space-time solves
            "space_time_over_time_stepping_iterations":
                sum(infos[i].iterations for i in range(0, len(infos), len(bts))) / args.steps / avg,
            "time_stepping_over_space_time_time":
                tts / (sum(infos[i].seconds for i in range(0, len(infos), len(bts))) / args.steps)}
        log(f"time stepping: {tts:.3f} s, {sum(step_its)} iterations ({avg:.1f} per step)")
    if cpu is not None:
        base, xs, its_cpu = cpu
        k = args.cpu_slabs
        nk = k * sys32.ns
        ref = xs[:nk]

        def err(xg):
            return None if xg is None else float(np.linalg.norm(xg[:nk].cpu().numpy() - ref) / np.linalg.norm(ref))
        out["error_vs_oracle"] = {
            f"{prec}_precond": err(x32), **({"fp64_precond": err(x64)} if fp32 else {}),
            "reference": f"the oracle's solution of the first {k} slabs (GMRES to {args.cpu_rtol:g} with exact "
                         f"inner solves, {its_cpu} iterations); J is block lower-bidiagonal in time, so it is the "
                         f"full system's x* on those slabs"}
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
