"""Batched solves and the continuous-batching server vs solo solves and the
oracle, through the C ABI.

Inside a batch an instance runs the same kernels on the same data with its
own reduction order, so its result must equal its solo result bit for bit;
against the oracle the usual bars apply (1e-12 fp64, 1e-10 mixed).
"""
import time

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(
        "cuda:0")


def _zeros(inst):
    import torch
    return torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64,
                       device="cuda:0")


def _mix(count, seed=3):
    insts = W.batch(count, seed=seed, ns=(16, 32, 64), nts=(8, 16, 32),
                    precision=1)
    # half fp64, a 1D heat and a 3D Allen-Cahn instance in the mix too
    for i, inst in enumerate(insts):
        inst.precision = i % 2
    rng = np.random.default_rng(seed)
    insts.append(W.Instance("heat1d", 1, 64, 16, 1.0, 1e-2, a=1.0,
                            u0=rng.uniform(-1, 1, 64)))
    insts.append(W.Instance("ac3d", 3, 16, 8, 1.0, 1e-3, a=0.0025, n1=1.0,
                            n3=-1.0, precision=1,
                            u0=rng.uniform(-0.9, 0.9, (16, 16, 16))))
    return insts


def test_graph_replay_equals_plain_launches():
    from paper_2603_04350_amd import Solver
    from paper_2603_04350_amd import expdiag as X
    inst = W.scaled(W.allen_cahn2d(precision=1), n=32, Nt=16)
    outs = []
    with Solver.from_instance(inst) as s:
        for graph in (True, False, True):
            X.expdiag_set_graph(s.h, graph)
            U = _zeros(inst)
            rc, it, rel = s.iterate(_dev(inst.u0), U, max_iter=200,
                                    tol=1e-12)
            outs.append((it, U.cpu().numpy()))
    for it, U in outs[1:]:
        assert it == outs[0][0]
        assert np.array_equal(U, outs[0][1])


def test_scheduled_batch_solves_equal_solo():
    """A batch solved a second time runs a schedule predicted from the first
    solve's counts (launches over just the instances predicted to run); a
    third solve from other initial values (so the predictions fall short
    for some instances and over-reach for others) pauses and completes
    them: every solve equals the solo solves bit for bit."""
    from paper_2603_04350_amd import Batch, Solver
    insts = _mix(16, seed=5)
    solvers = [Solver.from_instance(i) for i in insts]
    rng = np.random.default_rng(11)
    u0_sets = [[i.u0 for i in insts], [i.u0 for i in insts],
               [rng.uniform(-0.9, 0.9, i.u0.shape) * (0.3 + 0.7 * (k % 2))
                for k, i in enumerate(insts)]]
    b = Batch(solvers)
    for u0s_np in u0_sets:
        solo = []
        for s, inst, u0 in zip(solvers, insts, u0s_np):
            U = _zeros(inst)
            rc, it, rel = s.iterate(_dev(u0), U, max_iter=300, tol=1e-12)
            solo.append((it, U.cpu().numpy()))
        Us = [_zeros(i) for i in insts]
        rc, its, rels, sts = b.iterate([_dev(u) for u in u0s_np], Us,
                                       max_iter=300, tol=1e-12)
        for k in range(len(insts)):
            assert its[k] == solo[k][0], (k, its[k], solo[k][0])
            assert np.array_equal(Us[k].cpu().numpy(), solo[k][1]), k
    b.close()
    for s in solvers:
        s.close()


def test_batch_caps_schedule_equals_solo():
    """Per-instance caps with tolerance 0 fix every count ahead: the
    scheduled solve stops each instance at its cap, as solo solves do."""
    from paper_2603_04350_amd import Batch, Solver
    insts = _mix(10, seed=6)
    solvers = [Solver.from_instance(i) for i in insts]
    caps = [1 + (7 * k) % 23 for k in range(len(insts))]
    solo = []
    for s, inst, cap in zip(solvers, insts, caps):
        U = _zeros(inst)
        rc, it, rel = s.iterate(_dev(inst.u0), U, max_iter=cap, tol=0.0)
        assert it == cap
        solo.append(U.cpu().numpy())
    b = Batch(solvers)
    Us = [_zeros(i) for i in insts]
    rc, its, rels, sts = b.iterate_each([_dev(i.u0) for i in insts], Us,
                                        caps, [0.0] * len(insts))
    b.close()
    assert list(its) == caps
    for k in range(len(insts)):
        assert np.array_equal(Us[k].cpu().numpy(), solo[k]), k
    for s in solvers:
        s.close()


def test_batch_equals_solo_and_oracle():
    from paper_2603_04350_amd import Batch, Solver
    insts = _mix(12)
    solvers = [Solver.from_instance(i) for i in insts]
    solo = []
    for s, inst in zip(solvers, insts):
        U = _zeros(inst)
        rc, it, rel = s.iterate(_dev(inst.u0), U, max_iter=300, tol=1e-12)
        solo.append((it, U.cpu().numpy()))
    b = Batch(solvers)
    u0s = [_dev(i.u0) for i in insts]
    Us = [_zeros(i) for i in insts]
    rc, its, rels, sts = b.iterate(u0s, Us, max_iter=300, tol=1e-12)
    b.close()
    for k, inst in enumerate(insts):
        got = Us[k].cpu().numpy()
        assert its[k] == solo[k][0], (k, its[k], solo[k][0])
        assert np.array_equal(got, solo[k][1]), k
        st = O.Setup.from_instance(inst)
        ref = O.sequential(st, inst.u0)
        bar = 1e-10 if (inst.precision == 1 and inst.nonlinear) else 1e-12
        assert O.rel_err(got, ref) < bar, (k, inst.name)
    for s in solvers:
        s.close()


def test_batch_reused_twice():
    from paper_2603_04350_amd import Batch, Solver
    insts = _mix(4, seed=5)
    solvers = [Solver.from_instance(i) for i in insts]
    b = Batch(solvers)
    res = []
    for _ in range(2):
        Us = [_zeros(i) for i in insts]
        b.iterate([_dev(i.u0) for i in insts], Us, max_iter=300, tol=1e-12)
        res.append([u.cpu().numpy() for u in Us])
    b.close()
    for a, c in zip(res[0], res[1]):
        assert np.array_equal(a, c)


def test_server_continuous_batching():
    """Requests arrive while others run; every result equals its solo
    result, admission keeps the footprint within budget, timestamps are
    ordered."""
    import torch
    from paper_2603_04350_amd import Solver
    from paper_2603_04350_amd import expdiag as X
    insts = _mix(14, seed=11)
    solo = []
    for inst in insts:
        with Solver.from_instance(inst) as s:
            U = _zeros(inst)
            s.iterate(_dev(inst.u0), U, max_iter=300, tol=1e-12)
            solo.append(U.cpu().numpy())
    fps = [X.expdiag_footprint_bytes(i.shape, i.Nt, i.scheme, i.precision)
           for i in insts]
    budget = int(3.5 * max(fps))
    srv = X.expdiag_server_create(budget, 8)
    u0s = [_dev(i.u0) for i in insts]
    Us = [_zeros(i) for i in insts]
    torch.cuda.synchronize()
    ids = {}
    peak = 0
    rng = np.random.default_rng(0)
    for k, inst in enumerate(insts):
        prob = X.make_problem(inst.a, inst.c, inst.n1, inst.n2, inst.n3,
                              inst.precision)
        rid = X.expdiag_server_submit(srv, inst.shape, inst.Nt, inst.dt,
                                      inst.alpha, inst.scheme, prob, u0s[k],
                                      Us[k], 300, 1e-12)
        ids[rid] = k
        time.sleep(float(rng.exponential(0.002)))
        peak = max(peak, X.expdiag_server_stats(srv)["bytes_in_use"])
    done = []
    t_end = time.time() + 60
    while len(done) < len(insts) and time.time() < t_end:
        res, pending = X.expdiag_server_poll(srv)
        done.extend(res)
        peak = max(peak, X.expdiag_server_stats(srv)["bytes_in_use"])
        time.sleep(0.001)
    X.expdiag_server_destroy(srv)
    assert len(done) == len(insts)
    assert peak <= budget
    for r in done:
        k = ids[r["id"]]
        assert r["status"] == 0, r
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        assert np.array_equal(Us[k].cpu().numpy(), solo[k]), k


def _poll_all(X, srv, count, seconds):
    done = []
    t_end = time.time() + seconds
    while len(done) < count and time.time() < t_end:
        res, _ = X.expdiag_server_poll(srv)
        done.extend(res)
        time.sleep(0.001)
    return done


def test_server_failed_plan_build_reports_and_recovers(monkeypatch):
    """A launch plan that cannot be built (every plan upload forced to fail
    from the host, as a failed arena allocation under a full budget would)
    stops the server from launching for that set: every request comes back
    with EXPDIAG_EHIP, no slot or byte stays claimed, and once uploads work
    again the same server solves a new request to its solo result."""
    import torch
    from paper_2603_04350_amd import Solver
    from paper_2603_04350_amd import expdiag as X
    insts = W.batch(3, seed=5, ns=(16, 32), nts=(8, 16), precision=1)
    u0s = [_dev(i.u0) for i in insts]
    Us = [_zeros(i) for i in insts]
    torch.cuda.synchronize()
    srv = X.expdiag_server_create(1 << 30, 8)
    monkeypatch.setenv("EXPDIAG_FAIL_PLAN_UPLOAD", "1")
    for k, inst in enumerate(insts):
        prob = X.make_problem(inst.a, inst.c, inst.n1, inst.n2, inst.n3,
                              inst.precision)
        X.expdiag_server_submit(srv, inst.shape, inst.Nt, inst.dt,
                                inst.alpha, inst.scheme, prob, u0s[k],
                                Us[k], 200, 1e-12)
    done = _poll_all(X, srv, len(insts), 30)
    assert len(done) == len(insts)
    assert all(r["status"] == X.EXPDIAG_EHIP for r in done), done
    st = X.expdiag_server_stats(srv)
    assert st["active"] == 0 and st["pending"] == 0
    assert st["bytes_in_use"] == 0
    monkeypatch.delenv("EXPDIAG_FAIL_PLAN_UPLOAD")
    inst = insts[0]
    U = _zeros(inst)
    prob = X.make_problem(inst.a, inst.c, inst.n1, inst.n2, inst.n3,
                          inst.precision)
    X.expdiag_server_submit(srv, inst.shape, inst.Nt, inst.dt, inst.alpha,
                            inst.scheme, prob, u0s[0], U, 200, 1e-12)
    done = _poll_all(X, srv, 1, 30)
    X.expdiag_server_destroy(srv)
    assert len(done) == 1 and done[0]["status"] == 0, done
    with Solver.from_instance(inst) as s:
        V = _zeros(inst)
        s.iterate(u0s[0], V, max_iter=200, tol=1e-12)
    assert np.array_equal(U.cpu().numpy(), V.cpu().numpy())


TOL_BENCH = 1e-11  # the benchmark's tolerance on ||S|| / ||U||


def test_batched_configuration_full_size():
    """The batched configuration at full size, as the benchmark runs it: 256
    Allen-Cahn instances (n in {64, 128, 256}, Nt in {16 .. 128}, alpha in
    {1e-2, 1e-3}, eps ~ U[0.02, 0.1], mixed precision) in one batch.  Every
    instance converges and matches sequential stepping (the oracle) to the
    mixed bar 1e-10; the benchmark's timed form of the solve (per-instance
    caps at tolerance 0, zero-guess option) gives the same bits; the three
    largest and three smallest windows equal their solo solves bit for
    bit."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_2603_04350_amd import Batch, Solver
    insts = W.batch(256, seed=0, precision=1)
    solvers = [Solver.from_instance(i, precision=1) for i in insts]
    b = Batch(solvers)
    Us = [_zeros(i) for i in insts]
    u0s = [_dev(i.u0) for i in insts]
    rc, its, rels, sts = b.iterate(u0s, Us, max_iter=400, tol=TOL_BENCH)
    assert all(s == 0 for s in sts), [k for k, s in enumerate(sts) if s]
    # the benchmark's timed form of the same solves: per-instance caps at
    # tolerance 0 (a schedule known ahead), from zero with the zero-guess
    # option (the outputs' contents ignored: NaN here); same iterations,
    # same bits
    import torch
    b.set_zero_guess(True)
    V = [torch.full_like(u, float("nan")) for u in Us]
    rc2, its2, _, _ = b.iterate_each(u0s, V, its, [0.0] * len(insts))
    assert its2 == its
    for k in range(len(insts)):
        assert torch.equal(V[k], Us[k]), k
    del V
    b.close()
    order = sorted(range(len(insts)), key=lambda k: insts[k].dof)
    for k in order[:3] + order[-3:]:
        inst = insts[k]
        got = Us[k].cpu().numpy()
        U = _zeros(inst)
        rc1, it1, _ = solvers[k].iterate(_dev(inst.u0), U, max_iter=400,
                                         tol=TOL_BENCH)
        assert it1 == its[k] and np.array_equal(U.cpu().numpy(), got), k
    for s in solvers:
        s.close()

    def err_of(k):
        inst = insts[k]
        ref = O.sequential(O.Setup.from_instance(inst), inst.u0)
        return O.rel_err(Us[k].cpu().numpy(), ref)

    with ThreadPoolExecutor(8) as pool:
        errs = list(pool.map(err_of, range(len(insts))))
    worst = int(np.argmax(errs))
    print(f"256 batched instances against sequential stepping: max error "
          f"{errs[worst]:.2e} (instance {worst}: n {insts[worst].n}, "
          f"Nt {insts[worst].Nt}, alpha {insts[worst].alpha})")
    assert max(errs) < 1e-10, [(k, e) for k, e in enumerate(errs)
                               if e >= 1e-10]


def test_served_configuration_full_size_sampled():
    """The served configuration at full size, as the benchmark's burst:
    64 requests of the batch shapes with 3D 128^3 x 32 heat and Allen-Cahn
    requests among them, all submitted at once.  Every request converges,
    every 3D result equals its solo solve bit for bit, and one 3D request
    of each kind matches sequential stepping to the mixed bar."""
    import time
    import torch
    from paper_2603_04350_amd import Solver
    from paper_2603_04350_amd import expdiag as X
    _, insts = W.served_stream(64, 1.0, seed=1)
    assert any(i.dim == 3 for i in insts)
    u0s = [_dev(i.u0) for i in insts]
    Us = [_zeros(i) for i in insts]
    torch.cuda.synchronize()
    srv = X.expdiag_server_create(64 << 30, 128)
    ids = {}
    for k, inst in enumerate(insts):
        prob = X.make_problem(inst.a, inst.c, inst.n1, inst.n2, inst.n3,
                              inst.precision)
        rid = X.expdiag_server_submit(srv, inst.shape, inst.Nt, inst.dt,
                                      inst.alpha, inst.scheme, prob, u0s[k],
                                      Us[k], 400, TOL_BENCH)
        ids[rid] = k
    done = []
    t_end = time.time() + 90
    while len(done) < len(insts) and time.time() < t_end:
        res, _ = X.expdiag_server_poll(srv)
        done.extend(res)
        time.sleep(0.001)
    X.expdiag_server_destroy(srv)
    assert len(done) == len(insts)
    assert all(r["status"] == 0 for r in done)
    checked = set()
    for k, inst in enumerate(insts):
        if inst.dim != 3:
            continue
        got = Us[k].cpu().numpy()
        with Solver.from_instance(inst) as s:
            U = _zeros(inst)
            s.iterate(u0s[k], U, max_iter=400, tol=TOL_BENCH)
        assert np.array_equal(U.cpu().numpy(), got), k
        kind = inst.name.split("_")[0]
        if kind not in checked:
            checked.add(kind)
            ref = O.sequential(O.Setup.from_instance(inst), inst.u0)
            assert O.rel_err(got, ref) < 1e-10, (k, inst.name)
    assert checked, "no 3D request in the stream"


def test_server_autotune_results():
    """A server that tunes admitted handles by shape: every result equals
    the solo solve under the same (per-process) tuning and the oracle's
    sequential stepping at the mixed / fp64 bar."""
    import torch
    from paper_2603_04350_amd import Solver
    from paper_2603_04350_amd import expdiag as X
    insts = _mix(6, seed=21)
    u0s = [_dev(i.u0) for i in insts]
    Us = [_zeros(i) for i in insts]
    torch.cuda.synchronize()
    srv = X.expdiag_server_create(1 << 32, 8)
    X.expdiag_server_autotune(srv)
    ids = {}
    for k, inst in enumerate(insts):
        prob = X.make_problem(inst.a, inst.c, inst.n1, inst.n2, inst.n3,
                              inst.precision)
        rid = X.expdiag_server_submit(srv, inst.shape, inst.Nt, inst.dt,
                                      inst.alpha, inst.scheme, prob, u0s[k],
                                      Us[k], 300, 1e-12)
        ids[rid] = k
    done = _poll_all(X, srv, len(insts), 60)
    X.expdiag_server_destroy(srv)
    assert len(done) == len(insts)
    assert all(r["status"] == 0 for r in done), done
    for k, inst in enumerate(insts):
        with Solver.from_instance(inst) as s:
            X.expdiag_autotune(s.h)  # this shape's decision, from memory
            V = _zeros(inst)
            s.iterate(u0s[k], V, max_iter=300, tol=1e-12)
        got = Us[k].cpu().numpy()
        assert np.array_equal(V.cpu().numpy(), got), k
        ref = O.sequential(O.Setup.from_instance(inst), inst.u0)
        bar = 1e-10 if (inst.precision == 1 and inst.nonlinear) else 1e-12
        assert O.rel_err(got, ref) < bar, (k, inst.name)
