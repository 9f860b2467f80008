#!/usr/bin/env python3
"""Exp-ParaDiag benchmark on one MI355X.

Headline workload: 2D Allen-Cahn u_t = eps^2 Lap u + u - u^3, eps = 0.05,
periodic [0,2pi)^2 on 256^2 points, Nt = 64 steps over T = 2, ETD1,
alpha = 1e-3, u0 ~ U[-0.9, 0.9] i.i.d. (seed 0), synthetic.

One step = one complete Exp-ParaDiag solve from U = 0 to the run-time
tolerance ||S||/||U|| <= 1e-11 (which lands within 1e-10 of sequential
stepping), inputs already resident in HBM: boundary FFTs and every
fixed-point iteration (pass A: spatial FFTs + nonlinearity; pass B:
residual, alpha-scaled time transform, shifted solves, inverse transform,
update, norms), launched as the library chooses for this size (plain
launches; a captured hipGraph only for small iterates).

value = space-time DOF-iterations per second of the plain FP64 solve
(S = 256^2 * 64 DOF times iterations, over wall time).  Beside it:
  * the mixed-precision solve (fp32 bulk residual, fp64 refinement) timed
    the same way, with its time-to-tolerance against the FP64 path;
  * per-kernel durations from HIP events attached to the launches of the
    dominant kernel class (hipExtLaunchKernel start/stop events, on the
    library's stream) during a second timed region of the same solves, and
    the roofline of that class from its algorithmic bytes per launch;
  * batched: 256 heterogeneous Allen-Cahn instances (n in {64,128,256},
    Nt in {16..128}, eps ~ U[0.02,0.1], alpha in {1e-2,1e-3}) solved in one
    batched plan in mixed precision, against the same instances solved one
    after another by the plain FP64 single-instance path;
  * ebdf2: the same grid and window without the reaction term, solved by
    the second-order exponential BDF window: Nt = 65 (64 unknown slices,
    radix FFT time transform, pass B against HBM) and Nt = 64 (63, dense
    time transform on FP64 MFMA, pass B against both peaks);
  * advection: the headline instance with an advection term -b.grad u,
    b = (2, 1), whose symbol is complex (complex E and phi tables);
  * if1: the headline instance with the implicit IF1 scheme of the paper's
    nonlinear section (lagged iteration);
  * schroedinger: u_t = i Lap u - 2i u on the same grid, a complex state
    (full spectrum, C2C boundary transforms), from a wave packet;
  * served: batch-shaped 2D requests mixed with 3D 128^3 x 32 heat /
    Allen-Cahn requests into the continuous-batching server: all at once
    (its capacity), then Poisson arrivals at 0.5 and 0.9 of that capacity;
    p50/p99 latency and solves/s per arrival rate.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F64_PEAK_TFLOPS = 78.6
TOL = 1e-11


DEVICE_SOURCES = ("cx.hpp", "fft_core.hpp", "kernels_fft.hpp",
                  "kernels_passb.hpp", "kernels_krylov.hpp",
                  "kernels_dense.hpp", "kernels_bdf.hpp")


def _src_hash():
    """Hash of the device-code sources (what the counters depend on)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2603_04350_amd", "csrc")
    for name in DEVICE_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel, src_hash):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("src_hash") != src_hash:
        return None
    k = rec.get("kernels", {}).get(kernel)
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


def bench_single(inst, prec, steps, warmup):
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
    # timed region 1: graph replay, no instrumentation -> value
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
        "U": U.cpu().numpy().copy(),
    }
    # Kernel timing runs every solve for exactly its iteration count with
    # tol = 0, so no launch is enqueued past convergence (such launches see
    # the instance done and return at once; averaged in, they would flatter
    # the per-launch time).
    def step_fixed():
        U.zero_()
        return s.iterate(u0, U, max_iter=it, tol=0.0)

    # timed region 2: the same solves with HIP start/stop events attached to
    # every launch (hipExtLaunchKernel, on the library's stream).  With every
    # launch bracketed, each pair measures its own kernel and the averages
    # agree with rocprofv3's kernel times; events on one class alone also
    # count that launch's wait for the unbracketed kernel before it (1-2 us
    # more per launch), which is reported beside them.
    X.expdiag_profile_enable(s.h, 0x1F)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_fixed()
    torch.cuda.synchronize()
    wall2 = time.perf_counter() - t0
    ms, cnt, by, tm = X.expdiag_profile_read(s.h)
    dom = max(range(len(ms)), key=lambda i: ms[i])
    X.expdiag_profile_enable(s.h, 1 << dom)
    for _ in range(2):
        step_fixed()
    ms1, cnt1, by1, tm1 = X.expdiag_profile_read(s.h)
    X.expdiag_profile_enable(s.h, 0)
    out["ms_per_solve_instrumented"] = 1e3 * wall2 / steps
    out["dominant"] = X.PROFILE_CLASSES[dom]
    out["kernels"] = {}
    for i in range(len(ms)):
        d = {"launches_per_solve": cnt[i] / steps,
             "bytes_per_launch": by[i] / cnt[i] if cnt[i] else 0.0,
             "avg_us": 1e3 * ms[i] / tm[i] if tm[i] else 0.0,
             "timed_launches": tm[i]}
        if tm[i]:
            d["GBps"] = d["bytes_per_launch"] / (d["avg_us"] * 1e-6) / 1e9
        if i == dom:
            d["avg_us_events_on_this_class_only"] = 1e3 * ms1[i] / tm1[i]
        out["kernels"][X.PROFILE_CLASSES[i]] = d
    # algorithmic bytes of one iteration (launches of the iteration plan per
    # solve, over the solve's iterations) against the untimed wall clock
    it_bytes = sum(d["bytes_per_launch"] * d["launches_per_solve"]
                   for d in out["kernels"].values()) / max(it, 1)
    out["iteration_bytes"] = it_bytes
    out["iteration_hbm_frac"] = it_bytes / (out["us_per_iter"] * 1e-6) / \
        (HBM_PEAK_GBS * 1e9)
    s.close()
    return out


def bench_ebdf2(steps, warmup, Nt, order=2):
    """Exponential BDF window of order 2 (Sec. 4) or 3..6 (Sec. bdfs) on the
    headline grid: solves from zero to ||S||/||U|| <= TOL, then the pass B
    launches timed with kernel-attached events.  Nt - order + 1 a power of
    two (64 unknown slices for Nt = 63 + order) takes the radix FFT pass B,
    HBM-bound: algorithmic bytes 32 per window entry plus the per-kappa
    tables.  Nt = 64 takes the dense pass B, one 2Nt x 2Nt real GEMM pair
    per 16 kappa columns on FP64 MFMA: executed flops 2 * 2 * (2Nt)^2 * 16
    per block."""
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
        flops = 2 * 2 * (2 * Nt) ** 2 * 16 * ((Nk + 15) // 16)
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


def bench_rd2d(steps):
    """The reaction-diffusion window (512^2 x 128, ETD2, mixed precision)
    solved to 1e-10 as the paper uses Exp-ParaDiag there: as the
    preconditioner of Newton-GMRES(20); beside it the fixed point on the
    same window to ||S||/||U|| <= 1e-11, with its kernel classes against
    the HBM roofline (the window, 268 MB per array, streams from HBM).
    Time to tolerance per solve, Newton steps and GMRES iterations, and each
    result's error against sequential ETD2 stepping (the oracle, fp64)."""
    import torch
    import workloads as W
    import oracle as O
    from paper_2603_04350_amd import expdiag as X
    dev = "cuda:0"
    inst = W.rd2d()
    ref = O.sequential(O.Setup.from_instance(inst), inst.u0)
    out = {"workload": "u_t = 0.1 Lap u + u - u^3, periodic 512x512, "
                       "Nt=128, T=1, ETD2, alpha=1e-3, u0 = 32 periodic "
                       "Gaussians (seed 0), mixed precision",
           "dof": inst.dof}
    steps = max(1, min(steps, 3))
    u0 = torch.from_numpy(inst.u0).to(dev)
    U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64, device=dev)
    s = X.Solver.from_instance(inst, gmres_restart=20)

    def solve():
        U.zero_()
        return s.gmres(u0, U, restart=20, max_iter=400, tol=1e-10)

    solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, it, rel = solve()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    row = {"ms_per_solve": ms, "rel_resid": rel,
           "err_vs_oracle": float(O.rel_err(U.cpu().numpy(), ref)),
           "newton_steps": it // 1000, "gmres_iters": it % 1000}
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
    fp = bench_single(inst, 1, steps, 1)
    Ufp = fp.pop("U")
    out["fixed_point"] = {
        "ms_per_solve": fp["ms_per_solve"], "iters": fp["iters"],
        "rel_update": fp["rel_update"],
        "dof_iters_per_s": fp["dof_iters_per_s"],
        "us_per_iter": fp["us_per_iter"],
        "err_vs_oracle": float(O.rel_err(Ufp, ref)),
        "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()}
                    for k, v in fp["kernels"].items()},
        "iteration_bytes": fp["iteration_bytes"],
        "iteration_hbm_frac": round(fp["iteration_hbm_frac"], 4)}
    torch.cuda.empty_cache()
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


def bench_batched(count):
    import torch
    import workloads as W
    from paper_2603_04350_amd import expdiag as X
    dev = "cuda:0"
    insts = W.batch(count, seed=0, precision=1)
    u0s = [torch.from_numpy(i.u0).to(dev) for i in insts]
    Us = [torch.zeros((i.Nt,) + i.shape, dtype=torch.float64, device=dev)
          for i in insts]
    t0 = time.perf_counter()
    solvers = [X.Solver.from_instance(i, precision=1) for i in insts]
    b = X.Batch(solvers)
    setup_s = time.perf_counter() - t0
    b.iterate(u0s, Us, max_iter=400, tol=TOL)  # warmup
    for u in Us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, its, rels, sts = b.iterate(u0s, Us, max_iter=400, tol=TOL)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    dof_iters = sum(i.dof * k for i, k in zip(insts, its))
    b.close()
    for s in solvers:
        s.close()
    # the same instances one after another on the plain FP64 path
    solos = [X.Solver.from_instance(i, precision=0) for i in insts]
    V = [torch.zeros_like(u) for u in Us]
    for s, i, u0, v in zip(solos[:4], insts[:4], u0s[:4], V[:4]):
        s.iterate(u0, v, max_iter=400, tol=TOL)  # warmup
    for v in V:
        v.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its64 = []
    for s, u0, v in zip(solos, u0s, V):
        rc, it, rel = s.iterate(u0, v, max_iter=400, tol=TOL)
        its64.append(it)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    diff = max(float((a - c).abs().max() / c.abs().max())
               for a, c in zip(Us, V))
    for s in solos:
        s.close()
    return {
        "instances": count,
        "total_dof": sum(i.dof for i in insts),
        "setup_s": setup_s,
        "time_to_tol_s_batched_mixed": t_batch,
        "time_to_tol_s_solo_fp64_sequential": t_solo,
        "speedup_vs_solo_fp64": t_solo / t_batch,
        "dof_iters_per_s": dof_iters / t_batch,
        "iters_min_max": [min(its), max(its)],
        "iters_fp64_min_max": [min(its64), max(its64)],
        "all_converged": all(s == 0 for s in sts),
        "max_rel_diff_batched_mixed_vs_solo_fp64": diff,
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
    out = {"capacity_solves_per_s": cap,
           "burst": summary(done, wall, None, None, insts),
           "poisson": []}
    for frac in rates_frac:
        rate = frac * cap
        times, insts = W.served_stream(n_req, rate, seed=1)
        done, wall = _serve_run(times, insts, dev)
        out["poisson"].append(summary(done, wall, rate, frac, insts))
    return out


def cpu_baseline(inst, U_fp64, U_mixed, sample_iters):
    """The oracle timed on the host cores on a bounded sample: a few of its
    fixed-point iterations of the same instance, scaled to DOF-iters/s.  The
    oracle's sequential solution also checks the GPU answers."""
    import oracle as O
    st = O.Setup.from_instance(inst)
    t0 = time.perf_counter()
    O.fixed_point(st, inst.u0, max_iter=sample_iters, tol=0.0)
    t1 = time.perf_counter()
    ref = O.sequential(st, inst.u0)
    return {
        "value": inst.dof * sample_iters / (t1 - t0),
        "unit": "DOF-iters/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{sample_iters} fixed-point iterations of the 256^2 x 64 "
                  f"Allen-Cahn instance (numpy fp64, single-threaded FFTs), "
                  f"{t1 - t0:.1f} s",
        "err_fp64_vs_oracle": float(O.rel_err(U_fp64, ref)),
        "err_mixed_vs_oracle": float(O.rel_err(U_mixed, ref)),
    }


def cpu_baseline_ebdf2(U_gpu, sample_iters):
    """The oracle's EBDF2 fixed point on the Nt = 65 window (a bounded sample
    of iterations), and the GPU solution's error against sequential EBDF2."""
    import oracle as O
    import workloads as W
    inst = W.diffusion2d_ebdf2(Nt=65, T=2.0)
    st = O.Setup.from_instance(inst)
    t0 = time.perf_counter()
    O.fixed_point(st, inst.u0, max_iter=sample_iters, tol=0.0)
    t1 = time.perf_counter()
    ref = O.sequential(st, inst.u0)
    return {
        "value": inst.dof * sample_iters / (t1 - t0),
        "unit": "DOF-iters/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{sample_iters} EBDF2 fixed-point iterations of the "
                  f"256^2 x 65 diffusion window (numpy fp64), {t1 - t0:.1f} s",
        "err_vs_oracle": float(O.rel_err(U_gpu, ref)),
    }


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-ebdf2", action="store_true",
                    help="skip the EBDF, Krylov, advection, Schroedinger "
                         "and IF1 sections")
    ap.add_argument("--quick", action="store_true",
                    help="fp64 single-instance solves only")
    ap.add_argument("--profile-large", action="store_true",
                    help="fixed-count solves of the 512^2 x 128 and 3D "
                         "128^3 x 32 windows only, for profiler runs")
    ap.add_argument("--profile", action="store_true",
                    help="fixed-count solves only, for profiler runs")
    args = ap.parse_args()
    if args.quick:
        args.no_batch = args.no_serve = args.no_cpu_baseline = True
        args.no_ebdf2 = True
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.profile:
        profile_run(args.steps)
        return
    if args.profile_large:
        profile_large(args.steps)
        return
    import workloads as W
    inst = W.allen_cahn2d()
    _log("single-instance fp64")
    fp = bench_single(inst, 0, args.steps, args.warmup)
    _log("single-instance mixed")
    mx = fp if args.quick else bench_single(inst, 1, args.steps, args.warmup)
    kern = fp["kernels"]
    dom = fp["dominant"]
    src_hash = _src_hash()
    achieved = kern[dom]["GBps"]
    roof = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": _traffic(dom, src_hash),
        "algorithmic_bytes_per_launch": kern[dom]["bytes_per_launch"],
        "avg_launch_us": kern[dom]["avg_us"],
    }
    # what a plain device copy reaches at the dominant kernel's size (its
    # read and write arrays fit the Infinity Cache) and at 1 GiB (HBM)
    cp_same = _copy_rate(kern[dom]["bytes_per_launch"] / 2)
    cp_hbm = _copy_rate(1 << 30, reps=10)
    roof["copy_GBps_same_size"] = round(cp_same, 1)
    roof["copy_GBps_1GiB"] = round(cp_hbm, 1)
    roof["frac_of_copy_same_size"] = round(achieved / cp_same, 4)
    line = {
        "metric": "space-time DOF-iters/s + time-to-1e-10 "
                  "(mixed/batched vs plain FP64 GPU)",
        "value": fp["dof_iters_per_s"],
        "unit": "DOF-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "2D Allen-Cahn eps=0.05, periodic 256x256, Nt=64, "
                        "T=2, ETD1 Exp-ParaDiag fixed point, alpha=1e-3, "
                        "u0~U[-0.9,0.9] seed 0; step = one solve to "
                        "||S||/||U|| <= 1e-11",
            "global_batch": 1, "seq_len": 64, "parallelism": "none",
        },
        "iters_per_solve": fp["iters"],
        "time_to_tol_ms": {"fp64": fp["ms_per_solve"],
                           "mixed": mx["ms_per_solve"]},
        "mixed": {
            "dof_iters_per_s": mx["dof_iters_per_s"],
            "iters_per_solve": mx["iters"],
            "speedup_time_to_tol_vs_fp64":
                fp["ms_per_solve"] / mx["ms_per_solve"],
        },
        "us_per_iter": {"fp64": fp["us_per_iter"], "mixed": mx["us_per_iter"]},
        "ms_per_solve_instrumented": fp["ms_per_solve_instrumented"],
        "kernels_fp64": {k: {kk: round(vv, 3) for kk, vv in v.items()}
                         for k, v in kern.items()},
        "kernels_mixed": {k: {kk: round(vv, 3) for kk, vv in v.items()}
                          for k, v in mx["kernels"].items()},
        "roofline": roof,
        "iteration_hbm": {
            "algorithmic_bytes": fp["iteration_bytes"],
            "us_per_iter": fp["us_per_iter"],
            "achieved_GBps": fp["iteration_bytes"] / fp["us_per_iter"] / 1e3,
            "frac": round(fp["iteration_hbm_frac"], 4),
            "note": "all kernels of an iteration against the untimed wall "
                    "clock per iteration (launch gaps and the entry/exit "
                    "transforms included)",
            # the method's own minimum for a nonlinear fixed-point
            # iteration: pass A reads U^ and writes G^, pass B reads G^ and
            # U^ and writes U^, 8 B per real space-time DOF each (40 B/DOF);
            # the 2D FFT schedule adds the row pass and its intermediate
            "method_min_bytes": 40 * inst.dof,
            "design_over_min": fp["iteration_bytes"] / (40 * inst.dof),
            "min_bytes_frac": round(40 * inst.dof / (fp["us_per_iter"] * 1e-6)
                                    / (HBM_PEAK_GBS * 1e9), 4)},
        "src_hash": src_hash,
    }
    if not args.no_ebdf2:
        _log("ebdf2 single instance (radix FFT, Nt = 65; dense, Nt = 64)")
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
        _log("reaction-diffusion 512^2 x 128: Newton-GMRES and fixed point")
        line["rd2d"] = bench_rd2d(args.steps)
    if not args.no_ebdf2:
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
    if not args.no_batch:
        _log(f"batched: {args.batch} instances")
        line["batched"] = bench_batched(args.batch)
        if not args.no_serve:
            _log("served")
            line["served"] = bench_served((0.5, 0.9), args.serve_requests)
    if not args.no_cpu_baseline and rank == 0:
        _log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(inst, fp["U"], mx["U"],
                                            args.cpu_iters)
        if not args.no_ebdf2:
            line["ebdf2"]["cpu_baseline"] = cpu_baseline_ebdf2(
                U_eb, args.cpu_iters)
            import oracle as O
            import workloads as W
            ia = W.advection2d()
            line["advection"]["err_vs_oracle"] = float(O.rel_err(
                U_adv, O.sequential(O.Setup.from_instance(ia), ia.u0)))
            isc = W.schroedinger2d()
            line["schroedinger"]["err_vs_oracle"] = float(O.rel_err(
                U_se, O.sequential(O.Setup.from_instance(isc), isc.u0)))
            iif = W.allen_cahn2d(scheme=4)
            sif = O.Setup.from_instance(iif)
            line["if1"]["err_vs_oracle"] = float(O.rel_err(
                U_if1, O.sequential(sif, iif.u0)))
    if rank == 0:
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
