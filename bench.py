#!/usr/bin/env python3
"""Exp-ParaDiag benchmark on one MI355X.

Headline workload (the metric's subject): 256 independent 2D Allen-Cahn
instances u_t = eps^2 Lap u + u - u^3 on periodic [0,2pi)^2, n in
{64, 128, 256}, Nt in {16, 32, 64, 128}, T = 2, eps ~ U[0.02, 0.1],
alpha in {1e-2, 1e-3}, ETD1, u0 ~ U[-0.9, 0.9] (instance i drawn from
default_rng([0, i])), solved together in one batched plan in mixed
precision (fp32 spatial FFTs and nonlinearity in the bulk phase, fp64
residual, time transform and iterate), synthetic.

One step = one batched solve from U = 0 in which every instance runs to the
first fixed-point iteration whose iterate lies within 1e-10 of sequential
stepping (the paper's stopping rule: L_inf(0,T; L2) error against the
sequential solution, normalised).  Those counts come from comparing the
GPU iterates with the oracle's sequential solutions, which the oracle leg
computes on the host cores before the GPU sections (without that leg the
run-time rule ||S||/||U|| <= 1e-11 decides instead, and the line says so).
Inputs are resident in HBM when the timed region starts.

value = space-time DOF-iterations per second of that batched mixed solve
(sum over instances of n^2 * Nt * iterations, over wall time).  Beside it:
  * time-to-1e-10 of the batch against the plain FP64 single-instance path
    (the same 256 instances solved one after another, each to its own
    first iteration within 1e-10), and the errors reached;
  * the roofline of the batch's dominant kernel class: fixed-count batched
    solves (every instance the same number of iterations, so every launch
    does full work) with HIP start/stop events attached to every launch
    (hipExtLaunchKernel, on the batch's stream), algorithmic bytes per
    launch over the average launch time; the per-iteration fraction of the
    HBM peak for the design's bytes and for the method's minimum (40 B per
    real space-time DOF);
  * cpu_baseline: the oracle (numpy fp64) on the host cores, one worker
    process per core up to 16: a bounded sample of its fixed point (one
    iteration of every 8th batched instance) as DOF-iters/s, and its
    sequential stepping of every instance (the CPU time-to-solution);
  * single_256: the 256^2 x 64 Allen-Cahn instance (eps = 0.05, alpha =
    1e-3) alone, fp64 and mixed, to the run-time tolerance and to 1e-10,
    with its kernel classes against the roofline;
  * heat1d: the 1D heat window (n = 64, Nt = 16, alpha = 1e-2, fp64):
    us per iteration and time-to-1e-10 (latency-bound);
  * mixed_error: the relative difference between one mixed (fp32 bulk)
    and one fp64 fixed-point update from the same iterate, per alpha;
  * rd2d / ac3d: the 512^2 x 128 reaction-diffusion window (Newton-GMRES
    and fixed point, fp64 and mixed) and a 3D 128^3 x 32 Allen-Cahn window
    (fp64 and mixed), both larger than the Infinity Cache;
  * ebdf2/4/6, krylov, advection, schroedinger, if1: the next rows of the
    scope (exponential BDFs, GMRES vs BiCGStab, complex symbols and states,
    the implicit IF1 scheme);
  * served: batch-shaped 2D requests mixed with 3D 128^3 x 32 requests into
    the continuous-batching server: a burst (its capacity), then Poisson
    arrivals at 0.25 .. 1.2 of that capacity; p50/p99 latency and solves/s.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F64_PEAK_TFLOPS = 78.6
TOL = 1e-11        # run-time rule ||S|| / ||U||
ERR_BAR = 1e-10    # error against sequential stepping that ends a solve
BATCH_SEED = 0


DEVICE_SOURCES = ("cx.hpp", "fft_core.hpp", "kernels_fft.hpp",
                  "kernels_passb.hpp", "kernels_krylov.hpp",
                  "kernels_dense.hpp", "kernels_bdf.hpp")


# the device sources a workload's kernels are built from: its counter
# record stays valid while these are unchanged
WORKLOAD_SOURCES = {
    "batch256_mixed": ("cx.hpp", "fft_core.hpp", "kernels_fft.hpp",
                       "kernels_passb.hpp", "kernels_dense.hpp"),
    "single256_fp64": ("cx.hpp", "fft_core.hpp", "kernels_fft.hpp",
                       "kernels_passb.hpp", "kernels_dense.hpp",
                       "kernels_bdf.hpp"),
}


def _src_hash(sources=DEVICE_SOURCES):
    """Hash of device-code sources (what the counters depend on)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2603_04350_amd", "csrc")
    for name in sources:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(workload, kernel, src_hash):
    """HBM bytes per launch of kernel class `kernel` in `workload` from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    w = rec.get("workloads", {}).get(workload)
    if w is None or w.get("src_hash") != src_hash:
        return None
    k = w.get("classes", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _copy_rate(nbytes, reps=50):
    """GB/s (bytes read + bytes written over time) of torch's device copy of
    `nbytes` bytes: the rate a plain streaming kernel reaches at that size.
    Copies whose two buffers fit the 256 MB Infinity Cache run faster than
    ones that stream from HBM."""
    import torch
    n = max(1, int(nbytes) // 8)
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (us * 1e-6) / 1e9


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# The oracle leg: host worker processes (numpy only, no GPU)
# --------------------------------------------------------------------------
_WORKER_BATCH = None


def _ref_instances():
    """Single instances whose sequential solution the GPU sections compare
    against, by name."""
    import dataclasses
    import workloads as W
    _, stream = W.served_stream(64, 1.0, seed=1)
    return {
        "heat1d": W.heat1d(),
        "ac256": W.allen_cahn2d(),
        "rd2d": W.rd2d(),
        "ac3d": next(i for i in stream if i.name.startswith("ac3d")),
        "advection": W.advection2d(),
        "schroedinger": W.schroedinger2d(),
        "if1": dataclasses.replace(W.allen_cahn2d(scheme=4), jac=0),
        "ebdf2_65": W.diffusion2d_ebdf(2, Nt=65, T=2.0),
    }


def _worker_init(count, seed):
    global _WORKER_BATCH
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import oracle  # noqa: F401  (imported once, outside the timed tasks)
    import workloads as W
    _WORKER_BATCH = W.batch(count, seed=seed, precision=1)


def _noop(_):
    time.sleep(0.2)
    return os.getpid()


def _o1_batch_task(i):
    import oracle as O
    inst = _WORKER_BATCH[i]
    t0 = time.perf_counter()
    ref = O.sequential(O.Setup.from_instance(inst), inst.u0)
    return i, ref, time.perf_counter() - t0


def _o1_named_task(name):
    import oracle as O
    inst = _ref_instances()[name]
    t0 = time.perf_counter()
    ref = O.sequential(O.Setup.from_instance(inst), inst.u0)
    return name, ref, time.perf_counter() - t0


def _o2_task(arg):
    import oracle as O
    i, iters = arg
    inst = _WORKER_BATCH[i]
    st = O.Setup.from_instance(inst)
    t0 = time.perf_counter()
    O.fixed_point(st, inst.u0, max_iter=iters, tol=0.0)
    return inst.dof * iters, time.perf_counter() - t0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _host_workers():
    """One worker per host core, at most 16 (the host share of one GPU)."""
    return max(1, min(16, os.cpu_count() or 1))


def oracle_leg(count, sample_iters, names):
    """The oracle on the host cores, in a pool of worker processes:
      * a bounded sample of its fixed point (`sample_iters` iterations of
        every 8th batched instance) as DOF-iters/s over the pool's wall
        time;
      * its sequential stepping of every batched instance (the CPU
        time-to-solution of the batch), whose results also decide the GPU's
        time-to-1e-10;
      * the sequential solutions of the single instances in `names`.
    Returns (cpu_baseline record, batch references, named references)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    workers = _host_workers()
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(workers, mp_context=ctx,
                             initializer=_worker_init,
                             initargs=(count, BATCH_SEED)) as pool:
        list(pool.map(_noop, range(2 * workers)))
        sample = list(range(0, count, 8))
        t0 = time.perf_counter()
        res = list(pool.map(_o2_task, [(i, sample_iters) for i in sample]))
        t_o2 = time.perf_counter() - t0
        # largest windows first, so the pool's tail is short
        order = sorted(range(count), key=lambda i: -_batch_dof(i, count))
        refs = [None] * count
        cpu_s = 0.0
        t0 = time.perf_counter()
        for i, ref, dt in pool.map(_o1_batch_task, order):
            refs[i] = ref
            cpu_s += dt
        t_o1 = time.perf_counter() - t0
        named = {}
        named_s = {}
        for name, ref, dt in pool.map(_o1_named_task, names):
            named[name] = ref
            named_s[name] = dt
    dof_iters = sum(r[0] for r in res)
    rec = {
        "value": dof_iters / t_o2,
        "unit": "DOF-iters/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{sample_iters} fixed-point iteration(s) of each of "
                  f"{len(sample)} of the {count} batched Allen-Cahn "
                  f"instances (every 8th; the oracle's numpy fp64 fixed "
                  f"point), {workers} worker processes, {t_o2:.1f} s wall, "
                  f"{sum(r[1] for r in res):.1f} s CPU",
        "cpu_model": _cpu_model(),
        "host_cpus": os.cpu_count(),
        "o1_batch_time_to_solution_s": t_o1,
        "o1_batch_cpu_seconds": cpu_s,
        "o1_single_cpu_seconds": named_s,
    }
    return rec, refs, named


_BATCH_DOF = None


def _batch_dof(i, count):
    global _BATCH_DOF
    if _BATCH_DOF is None or len(_BATCH_DOF) != count:
        import workloads as W
        _BATCH_DOF = [b.dof for b in W.batch(count, seed=BATCH_SEED)]
    return _BATCH_DOF[i]


# --------------------------------------------------------------------------
# GPU helpers
# --------------------------------------------------------------------------
def _rel_err_t(U, R):
    """max_n ||u_n - r_n||_2 / max_n ||r_n||_2 on the device: the paper's
    L_inf(0,T; L2) error against the reference R, normalised by R."""
    nt = U.shape[0]
    d = (U - R).reshape(nt, -1).norm(dim=1).max()
    r = R.reshape(nt, -1).norm(dim=1).max()
    return float(d / r)


def _first_within(run, errs_of, start, bar=ERR_BAR, max_rounds=40):
    """Per instance, the first iteration count whose iterate lies within
    `bar` of the reference.  run(caps) solves every instance from zero for
    exactly caps[i] iterations; errs_of() returns the errors of that run.
    The search starts at `start` (the run-time rule's counts) and moves down
    while the error stays within the bar, or up until it is."""
    n = len(start)
    caps = list(start)
    best = [None] * n
    up = [False] * n
    done = [False] * n
    for _ in range(max_rounds):
        run(caps)
        e = errs_of()
        for i in range(n):
            if done[i]:
                continue
            if e[i] <= bar:
                best[i] = caps[i]
                if up[i] or caps[i] == 1:
                    done[i] = True
                else:
                    caps[i] -= 1
            elif best[i] is not None:
                done[i] = True
                caps[i] = best[i]
            else:
                up[i] = True
                caps[i] += 1
        if all(done):
            break
    if any(b is None for b in best):
        raise RuntimeError("an instance did not reach the error bar")
    return best


def _classes(X, ms, cnt, by, tm, runs):
    """Per kernel class: launches per run, algorithmic bytes per launch,
    average event-timed launch, GB/s."""
    out = {}
    for i in range(len(ms)):
        if not cnt[i]:
            continue
        d = {"launches_per_run": cnt[i] / runs,
             "bytes_per_launch": by[i] / cnt[i],
             "avg_us": 1e3 * ms[i] / tm[i] if tm[i] else 0.0,
             "ms_per_run": ms[i] / runs,
             "timed_launches": tm[i]}
        if tm[i]:
            d["GBps"] = d["bytes_per_launch"] / (d["avg_us"] * 1e-6) / 1e9
        out[X.PROFILE_CLASSES[i]] = d
    return out


# --------------------------------------------------------------------------
# Headline: the batched mixed-precision solve
# --------------------------------------------------------------------------
def bench_batch(count, steps, warmup, refs, tune_file=None):
    """256 heterogeneous Allen-Cahn instances in one batched plan, mixed
    precision, against the same instances on the plain FP64 single-instance
    path.  With `refs` (the oracle's sequential solutions) every instance
    runs to its first iteration within 1e-10 of them; without, to the
    run-time rule."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    dev = "cuda:0"
    insts = W.batch(count, seed=BATCH_SEED, precision=1)
    n = len(insts)
    u0s = [torch.from_numpy(i.u0).to(dev) for i in insts]
    Us = [torch.zeros((i.Nt,) + i.shape, dtype=torch.float64, device=dev)
          for i in insts]
    R = None
    if refs is not None:
        R = [torch.from_numpy(r).to(dev) for r in refs]

    def zero(vs):
        for v in vs:
            v.zero_()

    def errs(vs):
        return [_rel_err_t(v, r) for v, r in zip(vs, R)]

    t0 = time.perf_counter()
    solvers = [X.Solver.from_instance(i, precision=1) for i in insts]
    b = X.Batch(solvers)
    setup_s = time.perf_counter() - t0
    # per-shape tuning (time transform, column width) and graph replay
    # against plain launches for this batch, measured by the library
    t0 = time.perf_counter()
    tune = b.autotune(u0s, Us, tune_file)
    tune["seconds"] = time.perf_counter() - t0
    per_shape = {}
    for inst, s in zip(insts, solvers):
        key = f"{inst.n}^2 x Nt{inst.Nt}"
        if key not in per_shape:
            tv, cw = X.expdiag_get_tuning(s.h)
            per_shape[key] = {"time_transform": "dense" if tv else "radix",
                              "column_width": "2C" if cw else "C"}
    tune["per_shape"] = per_shape
    # every solve starts from U = 0 (the library clears the instances'
    # iterates instead of transforming Us, which are output only)
    b.set_zero_guess(True)
    # the run-time rule ||S|| / ||U|| <= TOL (what a caller without a
    # reference uses)
    zero(Us)
    b.iterate(u0s, Us, max_iter=400, tol=TOL)
    zero(Us)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, its_rt, rels, sts = b.iterate(u0s, Us, max_iter=400, tol=TOL)
    torch.cuda.synchronize()
    t_rt = time.perf_counter() - t0
    out = {"instances": n, "total_dof": sum(i.dof for i in insts),
           "setup_s": setup_s, "autotune": tune,
           "run_time_rule": {
               "tol": TOL, "ms_per_solve": 1e3 * t_rt,
               "iters_min_max": [min(its_rt), max(its_rt)],
               "all_converged": all(s == 0 for s in sts)}}
    if R is not None:
        e_rt = errs(Us)
        out["run_time_rule"]["max_err_vs_oracle"] = max(e_rt)
        zeros = [0.0] * n

        def run(caps):
            zero(Us)
            b.iterate_each(u0s, Us, caps, zeros)

        caps = _first_within(run, lambda: errs(Us), its_rt)
        out["stop"] = "first iteration within 1e-10 of sequential stepping"
    else:
        caps = its_rt
        out["stop"] = "run-time rule ||S||/||U|| <= 1e-11 (no oracle leg)"
    tols0 = [0.0] * n

    def step():
        return b.iterate_each(u0s, Us, caps, tols0)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / steps
    dof_iters = sum(i.dof * k for i, k in zip(insts, caps))
    out.update({
        "ms_per_solve": ms,
        "dof_iters_per_s": dof_iters / (ms * 1e-3),
        "iters_min_max": [min(caps), max(caps)],
        "iters_mean": sum(caps) / n,
    })
    if R is not None:
        e = errs(Us)
        out["max_err_vs_oracle"] = max(e)
        out["instances_within_1e-10"] = sum(1 for v in e if v <= ERR_BAR)
    # kernel classes: fixed-count solves (every instance kfix iterations, so
    # every launch does full work), events on every launch; from a zeroed
    # U through the full entry, so that the first iteration's pass A runs
    # as every later one does (the zero-guess option skips it)
    b.set_zero_guess(False)
    kfix = min(caps)
    fixed = [kfix] * n
    X.expdiag_profile_enable(solvers[0].h, 0x1F)
    runs = 2
    for _ in range(runs):
        zero(Us)
        b.iterate_each(u0s, Us, fixed, tols0)
    pm, pc, pb, pt = X.expdiag_profile_read(solvers[0].h)
    X.expdiag_profile_enable(solvers[0].h, 0)
    kern = _classes(X, pm, pc, pb, pt, runs)
    dom = max(kern, key=lambda k: kern[k]["ms_per_run"])
    # marginal wall time of one batched iteration (plain launches, no
    # events): solves of kfix and 2 kfix iterations
    def timed(k, reps=3):
        ks = [k] * n
        zero(Us)
        b.iterate_each(u0s, Us, ks, tols0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            zero(Us)
            b.iterate_each(u0s, Us, ks, tols0)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps
    # algorithmic bytes of the same fixed-count solves (the library's
    # phase-exact accounting, no events): the bytes of iterations k+1..2k
    # are those of the 2k-iteration solve less those of the k-iteration one
    def prof_bytes(k):
        X.expdiag_profile_enable(solvers[0].h, 1 << 7)  # bytes, no events
        zero(Us)
        b.iterate_each(u0s, Us, [k] * n, tols0)
        _, _, pbytes, _ = X.expdiag_profile_read(solvers[0].h)
        X.expdiag_profile_enable(solvers[0].h, 0)
        return sum(v for c, v in zip(X.PROFILE_CLASSES, pbytes)
                   if c != "reduce")

    tot_dof = out["total_dof"]

    def marginal(k):
        t1, t2 = timed(k), timed(2 * k)
        us_iter = 1e6 * (t2 - t1) / k
        it_bytes = (prof_bytes(2 * k) - prof_bytes(k)) / k
        return {"iterations": [k + 1, 2 * k],
                "marginal_us_per_iter": us_iter,
                "algorithmic_bytes": it_bytes,
                "frac": round(it_bytes / (us_iter * 1e-6)
                              / (HBM_PEAK_GBS * 1e9), 4)}

    out["kernels"] = {k: {kk: round(vv, 4) for kk, vv in v.items()}
                      for k, v in kern.items()}
    out["dominant"] = dom
    # iterations kfix+1..2 kfix: every instance past its bulk phase (fp64:
    # the method's minimum is 40 B per real space-time DOF); iterations
    # 5..8: every instance in its fp32 bulk phase
    late = marginal(kfix)
    late.update({
        "fixed_count_iters": kfix,
        "method_min_bytes": 40 * tot_dof,
        "design_over_min": late["algorithmic_bytes"] / (40 * tot_dof),
        "min_bytes_frac": round(40 * tot_dof
                                / (late["marginal_us_per_iter"] * 1e-6)
                                / (HBM_PEAK_GBS * 1e9), 4),
        "note": "batched iteration of all instances past their bulk phase: "
                "the design's algorithmic bytes of those iterations (phase-"
                "exact) and the method's fp64 minimum (40 B per real "
                "space-time DOF) over the marginal wall time of one more "
                "iteration"})
    out["iteration_hbm"] = late
    out["iteration_hbm_bulk"] = marginal(4)
    out["iteration_hbm_bulk"]["note"] = (
        "iterations 5..8, every instance in its fp32 bulk phase (72 B per "
        "complex half-spectrum entry by the design)")
    b.close()
    for s in solvers:
        s.close()
    # the plain FP64 single-instance path on the same instances, one after
    # another (each to its own first iteration within 1e-10; the counts are
    # found with a batch of the same handles, whose results equal the solo
    # ones)
    solos = [X.Solver.from_instance(i, precision=0) for i in insts]
    V = [torch.zeros_like(u) for u in Us]
    b64 = X.Batch(solos)
    zero(V)
    rc, its64_rt, _, _ = b64.iterate(u0s, V, max_iter=400, tol=TOL)
    if R is not None:
        def run64(caps):
            zero(V)
            b64.iterate_each(u0s, V, caps, [0.0] * n)
        caps64 = _first_within(run64, lambda: errs(V), its64_rt)
    else:
        caps64 = its64_rt
    b64.close()

    for s in solos:
        s.set_zero_guess(True)

    def solo_pass():
        for s, u0, v, k in zip(solos, u0s, V, caps64):
            s.iterate(u0, v, max_iter=k, tol=0.0)

    solo_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solo_pass()
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    out["solo_fp64"] = {
        "ms_total": 1e3 * t_solo,
        "iters_min_max": [min(caps64), max(caps64)],
        "iters_mean": sum(caps64) / n,
        "dof_iters_per_s": sum(i.dof * k for i, k in zip(insts, caps64))
        / t_solo}
    if R is not None:
        out["solo_fp64"]["max_err_vs_oracle"] = max(errs(V))
    out["speedup_vs_solo_fp64"] = 1e3 * t_solo / ms
    for s in solos:
        s.close()
    del Us, V, R, u0s
    torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------------------
# Single instances
# --------------------------------------------------------------------------
def bench_time_variants(Nts=(8, 16, 32, 64, 128)):
    """Both time transforms of pass B on the 256^2 Allen-Cahn grid for each
    Nt, timed by the library's autotuner on one handle (20 preconditioner
    applies each after warm-up): the radix FFT, and the DFT products on
    FP64 MFMA with their executed flops (16 Nt^2 per kappa column: the
    2Nt x 2Nt real form of each of the two Nt-point DFTs, its entries read
    from a table of roots of unity) against the FP64 matrix peak; both
    against HBM (read R, write S: 32 B per complex entry)."""
    import dataclasses
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    out = {}
    for Nt in Nts:
        inst = dataclasses.replace(W.allen_cahn2d(), Nt=Nt)
        with X.Solver.from_instance(inst, precision=0) as s:
            v, us_fft, us_dense = X.expdiag_autotune(s.h)
        Nk = inst.n * (inst.n // 2 + 1)
        C = 64 if Nt <= 32 else 2048 // Nt
        flops = 16 * Nt * Nt * ((Nk + C - 1) // C) * C
        nbytes = 32 * Nt * Nk
        row = {"chosen": "dense" if v == 1 else "radix",
               "radix_us": us_fft, "dense_us": us_dense,
               "radix_hbm_frac": round(nbytes / (us_fft * 1e-6) / 1e9
                                       / HBM_PEAK_GBS, 4)}
        if us_dense > 0:
            tf = flops / (us_dense * 1e-6) / 1e12
            row.update({
                "dense_flops": flops,
                "dense_TFLOPs": round(tf, 2),
                "dense_mfma_frac": round(tf / MFMA_F64_PEAK_TFLOPS, 4),
                "dense_hbm_frac": round(nbytes / (us_dense * 1e-6) / 1e9
                                        / HBM_PEAK_GBS, 4)})
        out[f"Nt{Nt}"] = row
    return {"grid": "256x256 half spectrum (33024 columns), fp64",
            "per_Nt": out}


def bench_single(inst, prec, steps, warmup, ref=None):
    """One instance solved alone: to the run-time rule (timed, `steps`
    solves), then with events on every launch of fixed-count solves (kernel
    classes against the roofline); with `ref` (its sequential solution) also
    to its first iteration within 1e-10 of it (timed the same way)."""
    import torch
    from paper_2603_04350_amd import expdiag as X
    dev = "cuda:0"
    u0 = torch.from_numpy(inst.u0).to(dev)
    U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64, device=dev)
    s = X.Solver.from_instance(inst, precision=prec)

    def step():
        U.zero_()
        return s.iterate(u0, U, max_iter=400, tol=TOL)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(steps):
        rc, it, rel = step()
        iters += it
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {
        "ms_per_solve": 1e3 * wall / steps,
        "iters": it,
        "rel_update": rel,
        "dof_iters_per_s": inst.dof * iters / wall,
        "us_per_iter": 1e6 * wall / iters,
    }
    R = None
    if ref is not None:
        R = torch.from_numpy(ref).to(dev)
        out["err_vs_oracle"] = _rel_err_t(U, R)
    # Kernel timing runs every solve for exactly its iteration count with
    # tol = 0, so no launch is enqueued past convergence (such launches see
    # the instance done and return at once; averaged in, they would flatter
    # the per-launch time).
    def step_fixed(k=it):
        U.zero_()
        return s.iterate(u0, U, max_iter=k, tol=0.0)

    # events attached to every launch (hipExtLaunchKernel, on the library's
    # stream): each pair measures its own kernel and the averages agree
    # with rocprofv3's kernel times
    X.expdiag_profile_enable(s.h, 0x1F)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_fixed()
    torch.cuda.synchronize()
    wall2 = time.perf_counter() - t0
    ms, cnt, by, tm = X.expdiag_profile_read(s.h)
    X.expdiag_profile_enable(s.h, 0)
    kern = _classes(X, ms, cnt, by, tm, steps)
    dom = max(kern, key=lambda k: kern[k]["ms_per_run"])
    out["ms_per_solve_instrumented"] = 1e3 * wall2 / steps
    out["dominant"] = dom
    out["kernels"] = kern
    # algorithmic bytes of one iteration (launches of the iteration plan per
    # solve, over the solve's iterations) against the untimed wall clock
    it_bytes = sum(d["bytes_per_launch"] * d["launches_per_run"]
                   for d in kern.values()) / max(it, 1)
    out["iteration_bytes"] = it_bytes
    out["iteration_hbm_frac"] = it_bytes / (out["us_per_iter"] * 1e-6) / \
        (HBM_PEAK_GBS * 1e9)
    if R is not None:
        def run(caps):
            step_fixed(caps[0])
        k = _first_within(run, lambda: [_rel_err_t(U, R)], [it])[0]
        # time to 1e-10 from U = 0 with the zero-guess option (as the
        # batched headline and its solo comparison are timed): the library
        # clears its iterate instead of transforming U, which is output only
        s.set_zero_guess(True)
        for _ in range(warmup):
            s.iterate(u0, U, max_iter=k, tol=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.iterate(u0, U, max_iter=k, tol=0.0)
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        out["time_to_1e-10"] = {"iters": k, "ms": 1e3 * w / steps,
                                "err_vs_oracle": _rel_err_t(U, R),
                                "zero_guess": True}
    out["U"] = U.cpu().numpy().copy()
    s.close()
    return out


def bench_heat1d(steps, ref):
    """The 1D heat window (n = 64, Nt = 16, alpha = 1e-2, fp64): latency-
    bound, so us per iteration (a solve of 200 fixed iterations against one
    of 20) and the time to its first iteration within 1e-10 of the exact
    window (5 iterations by the per-mode closed form of the iteration)."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    inst = W.heat1d()
    dev = "cuda:0"
    u0 = torch.from_numpy(inst.u0).to(dev)
    U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64, device=dev)
    s = X.Solver.from_instance(inst)

    def solve(k, tol=0.0):
        U.zero_()
        return s.iterate(u0, U, max_iter=k, tol=tol)

    def timed(k, reps):
        solve(k)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            solve(k)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    t20, t200 = timed(20, steps), timed(200, steps)
    out = {"workload": "1D heat u_t = u_xx, periodic n=64, Nt=16, T=1, "
                       "ETD1 fixed point, alpha=1e-2, fp64",
           "us_per_iter_marginal": 1e6 * (t200 - t20) / 180,
           "ms_per_solve_200_iters": 1e3 * t200}
    rc, it, rel = solve(400, TOL)
    out["iters_to_tol"] = it
    if ref is not None:
        R = torch.from_numpy(ref).to(dev)
        k = _first_within(lambda c: solve(c[0]),
                          lambda: [_rel_err_t(U, R)], [it])[0]
        out["time_to_1e-10"] = {"iters": k, "ms": 1e3 * timed(k, steps),
                                "err_vs_oracle": _rel_err_t(U, R)}
    s.close()
    return out


def bench_mixed_error(alphas=(1e-2, 1e-3, 1e-4), k=3):
    """Per alpha, the relative difference between one mixed-precision
    fixed-point update (bulk phase: fp32 spatial FFTs and nonlinearity, fp64
    time transform and shifted solves) and the fp64 update from the same
    iterate (the fp64 iterate after k iterations of the 256^2 x 64
    Allen-Cahn instance): ||U_mixed - U_fp64|| / ||U_fp64 - U_k||."""
    import dataclasses
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    dev = "cuda:0"
    out = {}
    for a in alphas:
        inst = dataclasses.replace(W.allen_cahn2d(), alpha=a)
        u0 = torch.from_numpy(inst.u0).to(dev)
        Uk = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64,
                         device=dev)
        with X.Solver.from_instance(inst, precision=0) as s64, \
                X.Solver.from_instance(inst, precision=1) as smx:
            s64.iterate(u0, Uk, max_iter=k, tol=0.0)
            V64 = Uk.clone()
            s64.iterate(u0, V64, max_iter=1, tol=0.0)
            Vmx = Uk.clone()
            smx.iterate(u0, Vmx, max_iter=1, tol=0.0)
        upd = float((V64 - Uk).norm())
        out[f"{a:g}"] = float((Vmx - V64).norm()) / upd
    return {"per_alpha": out, "from_iterate": k,
            "note": "relative difference of one mixed (fp32 bulk) update "
                    "from the fp64 update, same iterate; 2D Allen-Cahn "
                    "256^2 x 64"}


def bench_rd2d(steps, ref):
    """The reaction-diffusion window (512^2 x 128, ETD2) solved as the paper
    uses Exp-ParaDiag there: as the preconditioner of Newton-GMRES(20), mixed
    precision (fp32 Jacobian products), to ||R_j|| <= 1e-11 ||R_0|| (which
    lands within 1e-10 of sequential stepping); beside it the fixed point in
    fp64 and mixed precision, to the run-time rule and to 1e-10.  The window
    (268 MB per array) streams from HBM."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    dev = "cuda:0"
    inst = W.rd2d()
    out = {"workload": "u_t = 0.1 Lap u + u - u^3, periodic 512x512, "
                       "Nt=128, T=1, ETD2, alpha=1e-3, u0 = 32 periodic "
                       "Gaussians (seed 0)",
           "dof": inst.dof}
    steps = max(1, min(steps, 3))
    u0 = torch.from_numpy(inst.u0).to(dev)
    U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64, device=dev)
    s = X.Solver.from_instance(inst, gmres_restart=20)

    def solve():
        U.zero_()
        return s.gmres(u0, U, restart=20, max_iter=400, tol=1e-11)

    solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, it, rel = solve()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    row = {"ms_per_solve": ms, "rel_resid": rel, "tol": 1e-11,
           "newton_steps": it // 1000, "gmres_iters": it % 1000}
    if ref is not None:
        row["err_vs_oracle"] = _rel_err_t(U, torch.from_numpy(ref).to(dev))
    # event time per kernel class over one more solve
    X.expdiag_profile_enable(s.h, 0x1F)
    solve()
    pm, pc, pb, pt = X.expdiag_profile_read(s.h)
    X.expdiag_profile_enable(s.h, 0)
    row["classes_ms"] = {X.PROFILE_CLASSES[i]: round(pm[i], 3)
                         for i in range(len(pm)) if pt[i]}
    row["classes_launches"] = {X.PROFILE_CLASSES[i]: int(pc[i])
                               for i in range(len(pm)) if pt[i]}
    row["classes_GBps"] = {X.PROFILE_CLASSES[i]:
                           round(pb[i] / (pm[i] * 1e-3) / 1e9, 1)
                           for i in range(len(pm)) if pt[i]}
    out["newton_gmres"] = row
    s.close()
    del U, u0
    torch.cuda.empty_cache()
    for prec, name in ((1, "fixed_point_mixed"), (0, "fixed_point_fp64")):
        fp = bench_single(inst, prec, steps, 1, ref)
        fp.pop("U")
        out[name] = _single_summary(fp)
        torch.cuda.empty_cache()
    out["mixed_speedup_time_to_tol"] = (
        out["fixed_point_fp64"]["ms_per_solve"]
        / out["fixed_point_mixed"]["ms_per_solve"])
    return out


def bench_ac3d(steps, ref):
    """The first 3D Allen-Cahn request of the served stream (128^3 x 32,
    eps ~ U[0.02, 0.1], alpha = 1e-3, T = 1) solved alone by the fixed
    point, fp64 and mixed (each array 545 MB: streams from HBM)."""
    import torch
    out = {}
    inst = _ref_instances()["ac3d"]
    out["workload"] = (f"3D Allen-Cahn eps^2={inst.a:.3g}, periodic 128^3, "
                       f"Nt=32, T=1, ETD1 fixed point, alpha=1e-3")
    for prec, name in ((1, "mixed"), (0, "fp64")):
        fp = bench_single(inst, prec, max(1, min(steps, 5)), 1, ref)
        fp.pop("U")
        out[name] = _single_summary(fp)
        torch.cuda.empty_cache()
    out["mixed_speedup_time_to_tol"] = (out["fp64"]["ms_per_solve"]
                                        / out["mixed"]["ms_per_solve"])
    return out


def _single_summary(fp):
    keep = ("ms_per_solve", "iters", "rel_update", "dof_iters_per_s",
            "us_per_iter", "err_vs_oracle", "time_to_1e-10", "dominant",
            "iteration_bytes")
    out = {k: fp[k] for k in keep if k in fp}
    out["iteration_hbm_frac"] = round(fp["iteration_hbm_frac"], 4)
    out["kernels"] = {k: {kk: round(vv, 3) for kk, vv in v.items()}
                      for k, v in fp["kernels"].items()}
    return out


def bench_ebdf2(steps, warmup, Nt, order=2):
    """Exponential BDF window of order 2 (Sec. 4) or 3..6 (Sec. bdfs) on the
    headline grid: solves from zero to ||S||/||U|| <= TOL, then the pass B
    launches timed with kernel-attached events.  Nt - order + 1 a power of
    two (64 unknown slices for Nt = 63 + order) takes the radix FFT pass B,
    HBM-bound: algorithmic bytes 32 per window entry plus the per-kappa
    tables.  Nt = 64 takes the dense pass B: per block of C kappa columns
    (C = 64 for Nt <= 32, else 2048 / Nt) two real products of the
    2Nt x 2Nt block matrix (entries from the table of roots of unity) with
    the 2Nt x C tile on FP64 MFMA: executed flops 2 * 2 * (2Nt)^2 * C per
    block."""
    import workloads as W
    inst = W.diffusion2d_ebdf(order, Nt=Nt, T=2.0)
    fp = bench_single(inst, 0, steps, warmup)
    kb = fp["kernels"]["passb"]
    us = kb["avg_us"] if "avg_us" in kb else kb["avg_us_all_classes_timed"]
    gbps = kb["bytes_per_launch"] / (us * 1e-6) / 1e9
    dense = (Nt & (Nt - 1)) == 0
    out = {
        "workload": f"2D diffusion u_t = eps^2 Lap u, eps=0.05, periodic "
                    f"256x256, Nt={Nt} ({Nt - order + 1} unknown slices), "
                    f"T=2, EBDF{order} Exp-ParaDiag fixed point, "
                    f"alpha=1e-3, u0~U[-0.9,0.9] seed 0",
        "time_transform": "dense MFMA" if dense else "radix FFT",
        "ms_per_solve": fp["ms_per_solve"],
        "iters_per_solve": fp["iters"],
        "us_per_iter": fp["us_per_iter"],
        "dof_iters_per_s": fp["dof_iters_per_s"],
        "dominant": fp["dominant"],
        "passb": {
            "avg_us": us,
            "bytes_per_launch": kb["bytes_per_launch"],
            "roofline_hbm": {"bound": "hbm", "achieved": round(gbps, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbps / HBM_PEAK_GBS, 4)},
        },
        "U": fp["U"],
    }
    if dense:
        Nk = inst.n * (inst.n // 2 + 1)
        C = 64 if Nt <= 32 else 2048 // Nt
        flops = 2 * 2 * (2 * Nt) ** 2 * C * ((Nk + C - 1) // C)
        tflops = flops / (us * 1e-6) / 1e12
        out["passb"]["flops_per_launch"] = flops
        out["passb"]["roofline_mfma"] = {
            "bound": "mfma", "achieved": round(tflops, 2),
            "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tflops / MFMA_F64_PEAK_TFLOPS, 4)}
    return out


def bench_krylov(steps, warmup):
    """GMRES(20) against BiCGStab on the left-preconditioned system, the
    comparison of Table cpu_time_combined: purely diffusive problem, a in
    {1e-1, 1e-5}, dt = 0.01, first-order (ETD1, Nt = 64) and EBDF2
    (Nt = 65) windows on the 256^2 grid, from zero to a relative
    preconditioned residual of 1e-10.  Each BiCGStab iteration applies the
    operator twice, each GMRES iteration once."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    dev = "cuda:0"
    out = {}
    for scheme, Nt, name in ((1, 64, "etd1"), (3, 65, "ebdf2")):
        for a in (1e-1, 1e-5):
            inst = W.heat2d_table(a, Nt=Nt, scheme=scheme)
            u0 = torch.from_numpy(inst.u0).to(dev)
            U = torch.zeros((Nt,) + inst.shape, dtype=torch.float64,
                            device=dev)
            s = X.Solver.from_instance(inst, gmres_restart=20)
            row = {}
            for meth in ("gmres", "bicgstab"):
                def solve():
                    U.zero_()
                    if meth == "gmres":
                        return s.gmres(u0, U, restart=20, max_iter=200,
                                       tol=1e-10)
                    return s.bicgstab(u0, U, max_iter=200, tol=1e-10)
                for _ in range(warmup):
                    solve()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    rc, it, rel = solve()
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / steps
                row[meth] = {"ms_per_solve": ms, "iters": it,
                             "operator_applications":
                                 it * (2 if meth == "bicgstab" else 1),
                             "rel_resid": rel}
                # kernel classes of the solve, events on every launch: the
                # dominant one against the HBM roofline
                X.expdiag_profile_enable(s.h, 0x1F)
                solve()
                pm, pc, pb, pt = X.expdiag_profile_read(s.h)
                X.expdiag_profile_enable(s.h, 0)
                dom = max(range(len(pm)), key=lambda i: pm[i])
                us = 1e3 * pm[dom] / pt[dom]
                gbps = pb[dom] / pc[dom] / (us * 1e-6) / 1e9
                row[meth]["classes_ms"] = {
                    X.PROFILE_CLASSES[i]: round(pm[i], 4)
                    for i in range(len(pm)) if pt[i]}
                row[meth]["roofline"] = {
                    "kernel": X.PROFILE_CLASSES[dom], "bound": "hbm",
                    "avg_launch_us": us,
                    "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4)}
            row["bicgstab_speedup"] = (row["gmres"]["ms_per_solve"]
                                       / row["bicgstab"]["ms_per_solve"])
            s.close()
            out[f"{name}_a{a:g}"] = row
    out["workload"] = ("u_t = a Lap u, periodic 256x256, dt=0.01, "
                       "alpha=1e-3, u0~U[-0.9,0.9] seed 0; ETD1 Nt=64 and "
                       "EBDF2 Nt=65; tol 1e-10 (preconditioned residual)")
    return out


def bench_advection(steps, warmup):
    """The headline instance with an advection term (complex symbol, real
    state): the same kernels with complex E and phi tables."""
    import workloads as W
    inst = W.advection2d()
    fp = bench_single(inst, 0, steps, warmup)
    dom = fp["dominant"]
    kb = fp["kernels"][dom]
    return {
        "workload": "2D Allen-Cahn eps=0.05 with advection b=(2,1), periodic "
                    "256x256, Nt=64, T=2, ETD1, alpha=1e-3, u0~U[-0.9,0.9] "
                    "seed 0",
        "ms_per_solve": fp["ms_per_solve"],
        "iters_per_solve": fp["iters"],
        "us_per_iter": fp["us_per_iter"],
        "dof_iters_per_s": fp["dof_iters_per_s"],
        "dominant": dom,
        "roofline": {"kernel": dom, "bound": "hbm",
                     "achieved": round(kb["GBps"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s",
                     "frac": round(kb["GBps"] / HBM_PEAK_GBS, 4),
                     "avg_launch_us": kb["avg_us"]},
        "U": fp["U"],
    }


def bench_schroedinger(steps, warmup):
    """Complex state: u_t = i Lap u - 2i u on 256^2 from a wave packet,
    full-spectrum pass B (complex symbols), C2C boundary transforms."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    inst = W.schroedinger2d()
    dev = "cuda:0"
    u0 = torch.from_numpy(inst.u0).to(dev)
    U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.complex128,
                    device=dev)
    s = X.Solver.from_instance(inst)

    def step():
        U.zero_()
        return s.iterate(u0, U, max_iter=400, tol=TOL)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(steps):
        rc, it, rel = step()
        iters += it
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # pass B launches, each solve run for its iteration count with tol = 0
    X.expdiag_profile_enable(s.h, 1 << X.PROFILE_CLASSES.index("passb"))
    for _ in range(steps):
        U.zero_()
        s.iterate(u0, U, max_iter=it, tol=0.0)
    ms, cnt, by, tm = X.expdiag_profile_read(s.h)
    X.expdiag_profile_enable(s.h, 0)
    pb = X.PROFILE_CLASSES.index("passb")
    us = 1e3 * ms[pb] / tm[pb]
    bpl = by[pb] / cnt[pb]
    out = {
        "workload": "2D Schroedinger u_t = i Lap u - 2i u (complex state), "
                    "periodic 256x256, Nt=64, T=1, ETD1, alpha=1e-3, "
                    "u0 = Gaussian wave packet (width 0.4, wavenumber 5)",
        "ms_per_solve": 1e3 * wall / steps,
        "iters_per_solve": it,
        "us_per_iter": 1e6 * wall / iters,
        "dof_iters_per_s": inst.dof * iters / wall,
        "passb": {"avg_us": us, "bytes_per_launch": bpl,
                  "roofline_hbm": {"bound": "hbm",
                                   "achieved": round(bpl / (us * 1e-6) / 1e9,
                                                     1),
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(bpl / (us * 1e-6) / 1e9 /
                                                 HBM_PEAK_GBS, 4)}},
        "U": U.cpu().numpy().copy(),
    }
    s.close()
    # the paper's use on this problem: GMRES(20) to 1e-10 on the
    # preconditioned system, complex arithmetic (complex state)
    with X.Solver.from_instance(inst, gmres_restart=20) as g:
        def gstep():
            U.zero_()
            return g.gmres(u0, U, restart=20, max_iter=200, tol=1e-10)
        for _ in range(warmup):
            gstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rc, git, grel = gstep()
        torch.cuda.synchronize()
        out["gmres"] = {"ms_per_solve": 1e3 * (time.perf_counter() - t0) /
                        steps, "iters": git, "rel_resid": grel,
                        "note": "complex GMRES(20) on the preconditioned "
                                "system, tol 1e-10"}
    return out


def bench_if1(steps, warmup):
    """The headline instance solved with the implicit IF1 scheme (Sec. 5),
    lagged iteration (jacobian = 0)."""
    import dataclasses
    import workloads as W
    inst = dataclasses.replace(W.allen_cahn2d(scheme=4), jac=0)
    fp = bench_single(inst, 0, steps, warmup)
    dom = fp["dominant"]
    kb = fp["kernels"][dom]
    return {
        "workload": "2D Allen-Cahn eps=0.05, periodic 256x256, Nt=64, T=2, "
                    "IF1 u_n = A u_{n-1} + dt N(u_n), lagged iteration, "
                    "alpha=1e-3, u0~U[-0.9,0.9] seed 0",
        "ms_per_solve": fp["ms_per_solve"],
        "iters_per_solve": fp["iters"],
        "us_per_iter": fp["us_per_iter"],
        "dof_iters_per_s": fp["dof_iters_per_s"],
        "dominant": dom,
        "roofline": {"kernel": dom, "bound": "hbm",
                     "achieved": round(kb["GBps"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s",
                     "frac": round(kb["GBps"] / HBM_PEAK_GBS, 4),
                     "avg_launch_us": kb["avg_us"]},
        "U": fp["U"],
    }


def _serve_run(times, insts, dev):
    """Submit instance k at time times[k] (seconds from the start) into a
    fresh server; returns (results, wall seconds)."""
    import torch
    from paper_2603_04350_amd import expdiag as X
    u0s = [torch.from_numpy(i.u0).to(dev) for i in insts]
    Us = [torch.zeros((i.Nt,) + i.shape, dtype=torch.float64, device=dev)
          for i in insts]
    torch.cuda.synchronize()
    srv = X.expdiag_server_create(64 << 30, 128)
    X.expdiag_server_autotune(srv)
    t0 = time.perf_counter()
    done = []
    for k, (ta, inst) in enumerate(zip(times, insts)):
        while time.perf_counter() - t0 < ta:
            res, _ = X.expdiag_server_poll(srv)
            done.extend(res)
            time.sleep(0.0005)
        prob = X.make_problem(inst.a, inst.c, inst.n1, inst.n2, inst.n3,
                              inst.precision)
        X.expdiag_server_submit(srv, inst.shape, inst.Nt, inst.dt,
                                inst.alpha, inst.scheme, prob, u0s[k], Us[k],
                                400, TOL)
    while len(done) < len(insts):
        res, _ = X.expdiag_server_poll(srv)
        done.extend(res)
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    X.expdiag_server_destroy(srv)
    del Us, u0s
    torch.cuda.empty_cache()
    return done, wall




def bench_served(rates_frac, n_req):
    """Continuous batching: first every request at once (the server's
    capacity in solves/s), then Poisson arrivals at fractions of that
    capacity; p50/p99 of submit-to-result latency per arrival rate."""
    import numpy as np
    import workloads as W
    dev = "cuda:0"

    def summary(done, wall, rate, frac, insts):
        lat = np.array([r["t_done"] - r["t_submit"] for r in done])
        return {
            "rate_solves_per_s": rate,
            "rate_frac_of_capacity": frac,
            "requests": len(insts),
            "requests_3d": sum(1 for i in insts if i.dim == 3),
            "converged": sum(1 for r in done if r["status"] == 0),
            "p50_latency_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_latency_ms": 1e3 * float(np.percentile(lat, 99)),
            "throughput_solves_per_s": len(insts) / wall,
        }

    _, insts = W.served_stream(n_req, 1.0, seed=1)
    done, wall = _serve_run([0.0] * n_req, insts, dev)
    cap = n_req / wall
    out = {"capacity_solves_per_s": cap, "tol": TOL,
           "burst": summary(done, wall, None, None, insts),
           "poisson": []}
    for frac in rates_frac:
        rate = frac * cap
        times, insts = W.served_stream(n_req, rate, seed=1)
        done, wall = _serve_run(times, insts, dev)
        out["poisson"].append(summary(done, wall, rate, frac, insts))
        _log(f"served at {frac:g} x capacity done")
    return out


# --------------------------------------------------------------------------
# Runs for profilers and counters
# --------------------------------------------------------------------------
def profile_run(steps):
    """Fixed-count solves only (tol = 0, so every launch does full work),
    for a profiler wrapped around this process: the Allen-Cahn instance in
    fp64 (22 iterations, its count to tolerance), the EBDF2 windows with
    Nt = 65 and 64 and the EBDF4 window with Nt = 67 (5 iterations).  Prints
    the event-timed average launch time of each kernel class for comparison
    with the profiler's."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    out = {}
    for name, inst, iters in (
            ("allen_cahn2d_fp64", W.allen_cahn2d(), 22),
            ("ebdf2_Nt65", W.diffusion2d_ebdf2(Nt=65, T=2.0), 5),
            ("ebdf2_Nt64", W.diffusion2d_ebdf2(Nt=64, T=2.0), 5),
            ("ebdf4_Nt67", W.diffusion2d_ebdf(4, Nt=67, T=2.0), 5)):
        u0 = torch.from_numpy(inst.u0).to("cuda:0")
        U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64,
                        device="cuda:0")
        s = X.Solver.from_instance(inst, precision=0)
        for _ in range(2):
            U.zero_()
            s.iterate(u0, U, max_iter=iters, tol=0.0)
        X.expdiag_profile_enable(s.h, 0x1F)
        for _ in range(steps):
            U.zero_()
            s.iterate(u0, U, max_iter=iters, tol=0.0)
        ms, cnt, by, tm = X.expdiag_profile_read(s.h)
        X.expdiag_profile_enable(s.h, 0)
        out[name] = {X.PROFILE_CLASSES[i]: round(1e3 * ms[i] / tm[i], 3)
                     for i in range(len(ms)) if tm[i]}
        s.close()
        _log(f"profile {name} done")
    print(json.dumps({"event_avg_us": out}), flush=True)


def profile_large(steps):
    """Fixed-count solves of the windows that stream from HBM, for a
    profiler wrapped around this process: the reaction-diffusion window
    (512^2 x 128, ETD2, mixed; the fixed point for 17 iterations, its count
    to tolerance, then one Newton-GMRES(20) solve to 1e-10) and the first 3D
    Allen-Cahn request of the served stream (128^3 x 32, mixed; 14
    iterations, its count to tolerance).  The counts are fixed here so that
    no solve to a tolerance (whose launches past convergence return at once)
    enters the profile.  Prints the event-timed average launch time of each
    kernel class."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    _, stream = W.served_stream(64, 1.0, seed=1)
    ac3d = next(i for i in stream if i.name.startswith("ac3d"))
    out = {}
    for name, inst, iters in (("rd2d_fixed_point", W.rd2d(), 17),
                              ("ac3d_128", ac3d, 14)):
        u0 = torch.from_numpy(inst.u0).to("cuda:0")
        U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64,
                        device="cuda:0")
        s = X.Solver.from_instance(inst)
        for _ in range(2):
            U.zero_()
            s.iterate(u0, U, max_iter=iters, tol=0.0)
        X.expdiag_profile_enable(s.h, 0x1F)
        for _ in range(steps):
            U.zero_()
            s.iterate(u0, U, max_iter=iters, tol=0.0)
        ms, cnt, by, tm = X.expdiag_profile_read(s.h)
        X.expdiag_profile_enable(s.h, 0)
        out[name] = {"iters": iters, "event_avg_us": {
            X.PROFILE_CLASSES[i]: round(1e3 * ms[i] / tm[i], 3)
            for i in range(len(ms)) if tm[i]}, "bytes_per_launch": {
            X.PROFILE_CLASSES[i]: by[i] / cnt[i]
            for i in range(len(ms)) if tm[i]}}
        s.close()
        del U, u0
        torch.cuda.empty_cache()
        _log(f"profile {name} done")
    inst = W.rd2d()
    u0 = torch.from_numpy(inst.u0).to("cuda:0")
    U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64,
                    device="cuda:0")
    s = X.Solver.from_instance(inst, gmres_restart=20)
    rc, it, rel = s.gmres(u0, U, restart=20, max_iter=400, tol=1e-10)
    out["rd2d_newton_gmres"] = {"newton_steps": it // 1000,
                                "gmres_iters": it % 1000}
    s.close()
    _log("profile rd2d_newton_gmres done")
    print(json.dumps({"event_avg_us_large": out}), flush=True)


def profile_batch(steps, count=256, kfix=17, tune_file=None):
    """Fixed-count batched solves only (every instance `kfix` iterations,
    tol = 0, so every launch does full work), for a profiler wrapped around
    this process: the headline batch.  Prints the event-timed average launch
    time of each kernel class for comparison with the profiler's."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    insts = W.batch(count, seed=BATCH_SEED, precision=1)
    n = len(insts)
    u0s = [torch.from_numpy(i.u0).to("cuda:0") for i in insts]
    Us = [torch.zeros((i.Nt,) + i.shape, dtype=torch.float64,
                      device="cuda:0") for i in insts]
    solvers = [X.Solver.from_instance(i, precision=1) for i in insts]
    b = X.Batch(solvers)
    b.autotune(u0s, Us, tune_file)
    caps, tols = [kfix] * n, [0.0] * n
    for _ in range(2):
        for u in Us:
            u.zero_()
        b.iterate_each(u0s, Us, caps, tols)
    X.expdiag_profile_enable(solvers[0].h, 0x1F)
    for _ in range(steps):
        for u in Us:
            u.zero_()
        b.iterate_each(u0s, Us, caps, tols)
    ms, cnt, by, tm = X.expdiag_profile_read(solvers[0].h)
    X.expdiag_profile_enable(solvers[0].h, 0)
    kern = _classes(X, ms, cnt, by, tm, steps)
    b.close()
    for s in solvers:
        s.close()
    _log("profile batch done")
    print(json.dumps({"batch_event_avg_us": {
        k: round(v["avg_us"], 3) for k, v in kern.items()},
        "batch_bytes_per_launch": {k: v["bytes_per_launch"]
                                   for k, v in kern.items()},
        "kfix": kfix, "steps": steps}), flush=True)


def profile_batch_solve(steps, count=256, tune_file=None):
    """Batched solves to the run-time rule (the headline batch, tuned, from
    U = 0 with the zero-guess option as the headline's solves), for a kernel
    trace of a whole solve: full-batch iterations, the tail where few
    instances remain, entry and exit transforms."""
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    insts = W.batch(count, seed=BATCH_SEED, precision=1)
    u0s = [torch.from_numpy(i.u0).to("cuda:0") for i in insts]
    Us = [torch.zeros((i.Nt,) + i.shape, dtype=torch.float64,
                      device="cuda:0") for i in insts]
    solvers = [X.Solver.from_instance(i, precision=1) for i in insts]
    b = X.Batch(solvers)
    tune = b.autotune(u0s, Us, tune_file)
    b.set_zero_guess(True)
    mark = torch.zeros(1, device="cuda:0")
    walls = []
    for _ in range(steps + 1):
        mark.add_(1.0)  # one small kernel ahead of each solve in the trace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, its, rels, sts = b.iterate(u0s, Us, max_iter=400, tol=TOL)
        torch.cuda.synchronize()
        walls.append(1e3 * (time.perf_counter() - t0))
    b.close()
    for s in solvers:
        s.close()
    _log("profile batch solve done")
    print(json.dumps({"batch_solve_ms": walls[1:], "graph": tune["graph_used"],
                      "iters_max": max(its)}), flush=True)


def profile_variants():
    """Both time transforms of pass B per Nt (bench_time_variants), for a
    profiler: kernel times and MFMA counters of the dense variant."""
    r = bench_time_variants()
    print(json.dumps(r), flush=True)


def calibrate(mib=512, reps=5):
    """A plain device-to-device copy of known size (`mib` MiB read and
    written, `reps` times, torch's copy kernel), run under rocprofv3 --pmc
    to find what FETCH_SIZE / WRITE_SIZE report per byte moved."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.rand(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_MiB": mib, "reps": reps}),
          flush=True)


KERNEL_CLASSES = (("col_kernel_host", "col_fft"), ("col_kernel_mp", "col_fft"),
                  ("row_kernel_mp", "row_fft"), ("passb", "passb"),
                  ("ctl_reduce", "reduce"))


def _pmc_rows(d, counter, last_run=False):
    """(kernel name, value) per dispatch of `counter` from a rocprofv3
    --pmc csv output directory, in dispatch order.  last_run: only the
    dispatches from the last run of consecutive output-zeroing fills on
    (a profiler mode zeroes its outputs before every solve, so these are
    the last solve's launches)."""
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"),
                          recursive=True):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") == counter:
                    rows.append((int(r.get("Dispatch_Id") or 0),
                                 r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort(key=lambda x: x[0])
    if last_run:
        fills = [i for i, (_, k, _) in enumerate(rows) if "FillFunctor" in k]
        start = 0
        for j in range(len(fills) - 1, -1, -1):
            start = fills[j]
            if j == 0 or fills[j - 1] != fills[j] - 1:
                break
        rows = rows[start:]
    return [(k, v) for _, k, v in rows]


def traffic(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, workload,
            mib=512, path=None, last_run=False):
    """HBM bytes per launch from two rocprofv3 counter runs (FETCH_SIZE,
    WRITE_SIZE, KiB per dispatch) of the `workload` profile run (last_run:
    its last solve only), each scaled by what the same counter reads for the
    calibration copy; merged into profiles/traffic.json under `workload`
    with the hash of the device sources its kernels are built from, and
    printed per kernel."""
    copy_kib = mib * 1024.0

    def factor(d, counter):
        v = [x for k, x in _pmc_rows(d, counter) if "copy" in k.lower()]
        big = [x for x in v if x > 0.25 * copy_kib]
        return copy_kib / (sum(big) / len(big))

    ff = factor(cal_fetch_dir, "FETCH_SIZE")
    fw = factor(cal_write_dir, "WRITE_SIZE")
    per = {}
    for counter, d, fac, key in (("FETCH_SIZE", fetch_dir, ff, "read"),
                                 ("WRITE_SIZE", write_dir, fw, "write")):
        for k, v in _pmc_rows(d, counter, last_run):
            e = per.setdefault(k, {"read": [], "write": []})
            e[key].append(v * 1024.0 * fac)
    kernels = {}
    for k, e in sorted(per.items()):
        if not e["read"] or not e["write"]:
            continue
        rd = sum(e["read"]) / len(e["read"])
        wr = sum(e["write"]) / len(e["write"])
        kernels[k] = {"dispatches": len(e["read"]), "read_bytes": rd,
                      "write_bytes": wr, "bytes_per_launch": rd + wr}
    classes = {}
    for k, v in kernels.items():
        for pat, cls in KERNEL_CLASSES:
            if pat in k:
                c = classes.setdefault(cls, {"kernels": [], "bytes": 0.0,
                                             "n": 0})
                c["kernels"].append(k)
                c["bytes"] += v["bytes_per_launch"] * v["dispatches"]
                c["n"] += v["dispatches"]
                break
    for c in classes.values():
        c["bytes_per_launch"] = c.pop("bytes") / c.pop("n")
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    rec.setdefault("workloads", {})[workload] = {
        "src_hash": _src_hash(WORKLOAD_SOURCES.get(workload,
                                                   DEVICE_SOURCES)),
        "fetch_factor": ff, "write_factor": fw,
        "classes": classes, "kernels": kernels}
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"fetch factor {ff:.4f}, write factor {fw:.4f}")
    print("| kernel | dispatches | read MB | write MB | total MB |")
    print("|---|---|---|---|---|")
    for k, v in kernels.items():
        print(f"| `{k}` | {v['dispatches']} | {v['read_bytes'] / 1e6:.2f} | "
              f"{v['write_bytes'] / 1e6:.2f} | "
              f"{v['bytes_per_launch'] / 1e6:.2f} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-iters", type=int, default=1,
                    help="oracle fixed-point iterations per batched "
                         "instance in the CPU baseline sample")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (then no time-to-1e-10: the "
                         "run-time rule ends every solve)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the sections beside the headline and the "
                         "single 256^2 instance")
    ap.add_argument("--quick", action="store_true",
                    help="headline without the oracle leg, nothing else")
    ap.add_argument("--profile", action="store_true",
                    help="fixed-count single-instance solves only, for "
                         "profiler runs")
    ap.add_argument("--profile-large", action="store_true",
                    help="fixed-count solves of the 512^2 x 128 and 3D "
                         "128^3 x 32 windows only, for profiler runs")
    ap.add_argument("--profile-batch", action="store_true",
                    help="fixed-count batched solves only, for profiler "
                         "runs")
    ap.add_argument("--profile-batch-solve", action="store_true",
                    help="batched solves to the run-time rule only, for "
                         "profiler runs")
    ap.add_argument("--profile-variants", action="store_true",
                    help="both time transforms per Nt only, for profiler "
                         "runs")
    ap.add_argument("--traffic-last-run", action="store_true",
                    help="with --traffic: count only the profiled run's last "
                         "solve (after its last zeroing of the outputs)")
    ap.add_argument("--tune-file", default=None,
                    help="the batch's tuning decisions: read from this JSON "
                         "file where it holds them, measured and written "
                         "to it otherwise (so that a profiled run can use "
                         "the decisions of an unprofiled one)")
    ap.add_argument("--calibrate", action="store_true",
                    help="a plain 512 MiB device copy, for the counter "
                         "calibration")
    ap.add_argument("--traffic", nargs=5,
                    metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR",
                             "CAL_WRITE_DIR", "WORKLOAD"),
                    help="merge rocprofv3 FETCH_SIZE / WRITE_SIZE outputs "
                         "into profiles/traffic.json (no GPU)")
    args = ap.parse_args()
    if args.traffic:
        traffic(*args.traffic, last_run=args.traffic_last_run)
        return
    if args.quick:
        args.no_serve = args.no_cpu_baseline = args.no_extra = True
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.calibrate:
        calibrate()
        return
    if args.profile:
        profile_run(args.steps)
        return
    if args.profile_large:
        profile_large(args.steps)
        return
    if args.profile_batch:
        profile_batch(args.steps, tune_file=args.tune_file)
        return
    if args.profile_batch_solve:
        profile_batch_solve(args.steps, tune_file=args.tune_file)
        return
    if args.profile_variants:
        import torch
        torch.zeros(1, device="cuda:0")
        profile_variants()
        return
    names = ["heat1d", "ac256"]
    if not args.no_extra:
        names += ["rd2d", "ac3d", "advection", "schroedinger", "if1",
                  "ebdf2_65"]
    cpu, brefs, refs = None, None, {}
    if not args.no_cpu_baseline and rank == 0:
        _log("oracle leg on the host cores (cpu baseline, references)")
        cpu, brefs, refs = oracle_leg(args.batch, args.cpu_iters, names)
    _log(f"batched: {args.batch} instances, mixed, against solo fp64")
    bt = bench_batch(args.batch, args.steps, args.warmup, brefs,
                     args.tune_file)
    del brefs
    src_hash = _src_hash()
    dom = bt["dominant"]
    kd = bt["kernels"][dom]
    achieved = kd["GBps"]
    roof = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": _traffic("batch256_mixed", dom,
                            _src_hash(WORKLOAD_SOURCES["batch256_mixed"])),
        "algorithmic_bytes_per_launch": kd["bytes_per_launch"],
        "avg_launch_us": kd["avg_us"],
        "measured_on": f"fixed-count batched solves "
                       f"({bt['iteration_hbm']['fixed_count_iters']} "
                       f"iterations of every instance), events on every "
                       f"launch",
    }
    roof["copy_GBps_1GiB"] = round(_copy_rate(1 << 30, reps=10), 1)
    roof["frac_of_copy_1GiB"] = round(achieved / roof["copy_GBps_1GiB"], 4)
    line = {
        "metric": "space-time DOF-iters/s + time-to-1e-10 "
                  "(mixed/batched vs plain FP64 GPU)",
        "value": bt["dof_iters_per_s"],
        "unit": "DOF-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bt["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": "256 batched 2D Allen-Cahn instances, periodic "
                        "n^2 with n in {64,128,256}, Nt in {16,32,64,128}, "
                        "T=2, eps~U[0.02,0.1], alpha in {1e-2,1e-3}, ETD1 "
                        "Exp-ParaDiag fixed point, mixed precision (fp32 "
                        "bulk FFTs and N, fp64 residual, time transform "
                        "and iterate), u0~U[-0.9,0.9], instance i from "
                        "default_rng([0, i]); step = one batched solve "
                        "from U=0, " + bt["stop"],
            "instances": bt["instances"],
            "total_space_time_dof": bt["total_dof"],
        },
        "time_to_1e-10": {
            "batched_mixed_ms": bt["ms_per_solve"],
            "solo_fp64_sequential_ms": bt["solo_fp64"]["ms_total"],
            "speedup_vs_solo_fp64": bt["speedup_vs_solo_fp64"],
            "stop": bt["stop"],
        },
        "roofline": roof,
        "batched": {k: v for k, v in bt.items() if k not in ("stop",)},
        "src_hash": src_hash,
    }
    if cpu is not None:
        line["time_to_1e-10"]["cpu_o1_sequential_s"] = \
            cpu["o1_batch_time_to_solution_s"]
        line["cpu_baseline"] = cpu
    _log("single 256^2 x 64 Allen-Cahn instance: fp64 and mixed")
    import workloads as W
    inst = W.allen_cahn2d()
    sg = {}
    for prec, name in ((0, "fp64"), (1, "mixed")):
        fp = bench_single(inst, prec, args.steps, args.warmup,
                          refs.get("ac256"))
        fp.pop("U")
        sg[name] = _single_summary(fp)
    sg["workload"] = ("2D Allen-Cahn eps=0.05, periodic 256x256, Nt=64, "
                      "T=2, ETD1 fixed point, alpha=1e-3, u0~U[-0.9,0.9] "
                      "seed 0 (arrays of 34 MB: Infinity Cache resident)")
    sg["mixed_speedup_time_to_tol"] = (sg["fp64"]["ms_per_solve"]
                                       / sg["mixed"]["ms_per_solve"])
    line["single_256"] = sg
    _log("time transform variants (radix FFT, DFT on FP64 MFMA)")
    line["time_transform"] = bench_time_variants()
    _log("1D heat window")
    line["heat1d"] = bench_heat1d(args.steps, refs.get("heat1d"))
    if not args.no_extra:
        _log("mixed-precision error per update, per alpha")
        line["mixed_error"] = bench_mixed_error()
        _log("reaction-diffusion 512^2 x 128: Newton-GMRES and fixed point")
        line["rd2d"] = bench_rd2d(args.steps, refs.get("rd2d"))
        _log("3D 128^3 x 32 Allen-Cahn: fp64 and mixed")
        line["ac3d"] = bench_ac3d(args.steps, refs.get("ac3d"))
        _log("ebdf2 (radix FFT, Nt = 65; dense, Nt = 64)")
        eb = bench_ebdf2(args.steps, args.warmup, 65)
        U_eb = eb.pop("U")
        ebd = bench_ebdf2(args.steps, args.warmup, 64)
        ebd.pop("U")
        eb["dense_variant_Nt64"] = ebd
        line["ebdf2"] = eb
        _log("ebdf4 (radix FFT, Nt = 67; dense, Nt = 64) and ebdf6 (Nt = 69)")
        e4 = bench_ebdf2(args.steps, args.warmup, 67, order=4)
        e4.pop("U")
        e4d = bench_ebdf2(args.steps, args.warmup, 64, order=4)
        e4d.pop("U")
        e4["dense_variant_Nt64"] = e4d
        e6 = bench_ebdf2(args.steps, args.warmup, 69, order=6)
        e6.pop("U")
        line["ebdf4"] = e4
        line["ebdf6"] = e6
        _log("krylov: GMRES vs BiCGStab")
        line["krylov"] = bench_krylov(args.steps, args.warmup)
        _log("advection (complex symbol)")
        adv = bench_advection(args.steps, args.warmup)
        U_adv = adv.pop("U")
        line["advection"] = adv
        _log("schroedinger (complex state)")
        se = bench_schroedinger(args.steps, args.warmup)
        U_se = se.pop("U")
        line["schroedinger"] = se
        _log("IF1 (implicit scheme)")
        if1 = bench_if1(args.steps, args.warmup)
        U_if1 = if1.pop("U")
        line["if1"] = if1
        if refs:
            import numpy as np
            import torch

            def err(Ug, name):
                return _rel_err_t(torch.from_numpy(np.ascontiguousarray(Ug)),
                                  torch.from_numpy(refs[name]))

            line["ebdf2"]["err_vs_oracle"] = err(U_eb, "ebdf2_65")
            line["advection"]["err_vs_oracle"] = err(U_adv, "advection")
            line["schroedinger"]["err_vs_oracle"] = err(U_se, "schroedinger")
            line["if1"]["err_vs_oracle"] = err(U_if1, "if1")
    if not args.no_serve:
        _log("served")
        line["served"] = bench_served((0.25, 0.5, 0.75, 0.9, 1.0, 1.2),
                                      args.serve_requests)
    if rank == 0:
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
