"""Benchmark of the AM-AMG-preconditioned FGMRES solve on one MI355X.

Workload (default): 256x256 lattice, quenched U(1) links from 200 Metropolis sweeps at
beta = 10, m0 = m_c + 0.01, three levels with 8x8 wirebaskets and overlap 2, 8 test vectors,
FGMRES(20) to relative residual 1e-10, Gaussian right-hand sides resident in HBM.

One step = the whole hot path on one batch: AM-AMG setup on the resident gauge field
(classification, test vectors, local Schur solves, normalisation, Galerkin operators,
smoother blocks, coarsest inverse) followed by the solve of --nrhs right-hand sides.
The headline value is right-hand sides solved per second in mixed precision (FP32 V-cycle
and Arnoldi matvec inside FP64 FGMRES); the same steps in pure FP64 are timed beside it.

Also reported: the fine-stencil bandwidth at a 4096^2 lattice, the roofline of the step's
dominant kernel (library kernel timer, HIP events on the solve stream), and the CPU oracle
timed on a bounded sample of the same workload.
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

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


FAMILIES = ["fine_matvec", "fine_gs", "restrict0", "prolong0", "coarse_gs", "dots", "update"]
KERNEL_NAMES = {"fine_matvec": "k_wilson_apply", "fine_gs": "k_wilson_gs",
                "restrict0": "k_restrict_partial (fine level)", "prolong0": "k_prolong (fine level)",
                "coarse_gs": "k_stencil_gs (level 1)", "dots": "k_gram<nv, s, w> (all basis sizes)",
                "update": "k_lag_update<nv, s> (all basis sizes)"}


def run_steps(lib, torch, ctx, h, b, x, nrhs, precision, steps, warmup, timer=None, groups=1):
    """warmup + timed steps; a step = in-place setup + solve of nrhs right-hand sides."""
    sp = lib.default_solve_params(precision=precision, groups=groups)
    infos = None
    for _ in range(warmup):
        h.update()
        infos, _ = h.solve_device(b.data_ptr(), x.data_ptr(), nrhs, sp)
    torch.cuda.synchronize()
    fams = [timer] if isinstance(timer, str) else list(timer or [])
    if fams:
        ctx.kernel_timer(fams)
    t_setup = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        h.update()                     # synchronous: returns when the setup has finished
        t_setup += time.perf_counter() - ts
        infos, st = h.solve_device(b.data_ptr(), x.data_ptr(), nrhs, sp)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timed = None
    if fams:
        timed = {f: ctx.kernel_timer_read(f) for f in fams}
        timed = timed[timer] if isinstance(timer, str) else timed
        ctx.kernel_timer([])
    return dt, t_setup, infos, timed


def copy_bandwidth(torch, gib=2.0, reps=10):
    """Device bandwidth of a plain elementwise kernel (y = -x, FP64, gib GiB each way), the
    practical ceiling the roofline fraction is read against beside the 8 TB/s data-sheet peak."""
    n = int(gib * 2 ** 30 / 8)
    a = torch.empty(n, dtype=torch.float64, device="cuda").normal_()
    y = torch.empty_like(a)
    torch.neg(a, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=y)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, y
    return gbs


def dominant_family(lib, torch, ctx, h, b, x, nrhs, precision, groups=1):
    """One instrumented step with every family timed; returns (family, {family: ms})."""
    ctx.kernel_timer(FAMILIES)
    h.update()
    h.solve_device(b.data_ptr(), x.data_ptr(), nrhs, lib.default_solve_params(precision=precision, groups=groups))
    torch.cuda.synchronize()
    tot = {f: ctx.kernel_timer_read(f)[1] for f in FAMILIES}
    ctx.kernel_timer([])
    return max(tot, key=tot.get), tot


def stencil_bandwidth(lib, torch, ctx, L=4096, reps=20):
    """Fine Wilson stencil on an L x L lattice (footprint far above the 256 MB last-level cache)."""
    U = np.exp(1j * np.random.default_rng(1).uniform(-np.pi, np.pi, (2, L, L)))
    g = lib.Gauge(ctx, synth.links_to_abi(U), 0.05)
    out = {}
    for prec, name, vb, lb in ((lib.FP64, "fp64", 16, 16), (lib.MIXED_FP32, "fp32", 8, 8),
                               (lib.MIXED_FP32_BF16LINKS, "fp32_bf16links", 8, 4)):
        dt = torch.float64 if prec == lib.FP64 else torch.float32
        xin = torch.randn(1, L, L, 2, 2, dtype=dt, device="cuda")
        y = torch.empty_like(xin)
        g.apply_dirac_device(xin.data_ptr(), y.data_ptr(), 1, prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g.apply_dirac_device(xin.data_ptr(), y.data_ptr(), 1, prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # algorithmic bytes per site: read 2 spinors-worth once (own + neighbours), 2 links, write
        bytes_site = 2 * vb + 2 * lb + 2 * vb
        out[name] = {"ms": ms, "GBps": bytes_site * L * L / ms / 1e6, "bytes_per_site": bytes_site}
        del xin, y
    g.close()
    return out


def cpu_baseline(w, m0, gpu_iterations, budget_s=25.0):
    """The oracle as it stands, timed on the host cores: setup once, then FGMRES steps until
    the time budget is spent; solves/s extrapolated to the GPU's FP64 iteration count."""
    import threadpoolctl  # noqa: F401  (BLAS threads left at their default: all cores)
    from oracle.amg import SetupParams, setup, vcycle
    U = w.links()
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed)[0].reshape(-1)
    prm = SetupParams(**w.oracle_kw())
    t0 = time.perf_counter()
    levs = setup(U, m0, prm)
    t_setup = time.perf_counter() - t0
    D = levs[0].A
    # Arnoldi steps of the oracle's FGMRES (same per-step work), timed until the budget is spent
    v = psi / np.linalg.norm(psi)
    V = [v]
    steps = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < max(2.0, budget_s - t_setup) and steps < 400:
        z = vcycle(levs, 0, V[-1], prm)
        wv = D @ z
        Vm = np.array(V)
        h = Vm.conj() @ wv
        wv = wv - Vm.T @ h
        h2 = Vm.conj() @ wv
        wv = wv - Vm.T @ h2
        wv /= np.linalg.norm(wv)
        V.append(wv)
        if len(V) > 20:
            V = [V[-1]]
        steps += 1
    t_step = (time.perf_counter() - t1) / steps
    solve_s = t_setup + t_step * gpu_iterations
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"oracle setup ({t_setup:.1f} s) + {steps} FGMRES steps ({t_step * 1e3:.0f} ms each) "
                      f"on the 256^2 workload, extrapolated to {gpu_iterations} steps per solve; "
                      "NumPy/SciPy FP64, sparse matvecs single-threaded"}


def generate_links(cfgs):
    """Gauge fields of `cfgs` (Metropolis on the host cores), generated by forked workers.
    Called before anything touches the GPU: a forked child of a process that has initialised
    HIP is not allowed, and a fork-context pool leaves no helper process behind."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(16, len(cfgs)), mp_context=mp.get_context("fork")) as ex:
        links = list(ex.map(synth.serving_links, cfgs))
    return links, time.perf_counter() - t0


def serve_leg(lib, n_requests, qps=None, n_configs=16, slots=16, instances=4, builders=4, load=0.7,
              capacity_requests=200, log_every=250, links=None):
    """Open-loop serving run on the continuous-batching server, mixed precision to 1e-10.

    16 resident gauge fields (L_j = 32..512 by j mod 5, beta_j from 2 to 10), each with a
    reference mass m_c + 0.0316 (the log-middle of the gap range) at which its hierarchy is set
    up before timing; each request draws a field, m0 = m_c + gap with the gap log-uniform in
    [0.01, 0.1] and 1..8 right-hand sides, and is solved with a hierarchy derived at its mass.
    Capacity is measured first: `capacity_requests` requests of the same distribution
    submitted at once, requests per second over their makespan.  Then n_requests Poisson
    arrivals at load x capacity (or at `qps` when given).  Latency = completion minus
    submission on the server clock (queueing, the derivation of the request's hierarchy and
    the solve)."""
    import threading
    cfgs = synth.serving_configs(n_configs)
    if links is None:
        t0 = time.perf_counter()                      # GPU already live: no fork, one process
        links = [synth.serving_links(c) for c in cfgs]
        t_gen = time.perf_counter() - t0
    else:
        links, t_gen = links
    m_c = synth.serving_critical()
    ref_gap = float(np.exp(0.5 * (np.log(synth.SERVING_GAPS[0]) + np.log(synth.SERVING_GAPS[1]))))
    srv = lib.Server(0, lib.default_server_params(slots=slots, max_instances=instances, builders=builders,
                                                  precision=lib.MIXED_FP32))
    gids = [srv.add_gauge(synth.links_to_abi(U)) for U in links]
    del links
    for k in range(len(cfgs)):
        srv.set_reference_mass(gids[k], m_c[k] + ref_gap)
    setups = [lib.default_setup_params(**synth.serving_setup(c["L"])) for c in cfgs]
    # right-hand-side pools (8 Gaussian fields per configuration); requests copy slices of them
    pools = [synth.field_to_abi(synth.gaussian_rhs(c["L"], c["L"], c["seed"] + 77, nrhs=8)) for c in cfgs]

    def submit(rq):
        rng = np.random.default_rng(rq["seed"])
        pick = rng.choice(8, rq["nrhs"], replace=False)
        return srv.submit(gids[rq["config"]], rq["m0"], pools[rq["config"]][pick], setups[rq["config"]])

    # warm cache: each field's hierarchy at its reference mass, built before timing
    t0 = time.perf_counter()
    for k in range(len(cfgs)):
        srv.submit(gids[k], m_c[k] + ref_gap, pools[k][:1], setups[k])
    srv.wait(1800)
    srv.poll(len(cfgs) + 1)
    warm = srv.stats()
    t_warm = time.perf_counter() - t0
    log(f"serving: {warm.setups} hierarchies built in {t_warm:.1f} s (setup {warm.setup_seconds:.1f} s, "
        f"longest {warm.setup_seconds_max:.2f} s)")
    # capacity: a burst of requests of the same distribution, all submitted at once
    burst = synth.near_critical_stream(capacity_requests, 1.0, m_c, seed=6007)
    t0 = time.perf_counter()
    for rq in burst:
        submit(rq)
    srv.wait(1800)
    cap_done = [i for i, _ in srv.poll(len(burst) + 1)]
    cap_span = max(i.t_done for i in cap_done) - min(i.t_submit for i in cap_done)
    capacity = len(burst) / cap_span
    rate = qps if qps else load * capacity
    log(f"serving: capacity {capacity:.1f} requests/s ({sum(i.nrhs for i in cap_done) / cap_span:.1f} solves/s); "
        f"stream at {rate:.1f} requests/s")
    before = srv.stats()
    stream = synth.near_critical_stream(n_requests, rate, m_c)
    lag = [0.0]

    def client():
        start = time.perf_counter()
        for k, rq in enumerate(stream):
            delay = rq["t"] - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            else:
                lag[0] = max(lag[0], -delay)
            submit(rq)
            if log_every and (k + 1) % log_every == 0:
                log(f"serving: submitted {k + 1}/{len(stream)}")
    th = threading.Thread(target=client)
    th.start()
    th.join()
    srv.wait(1800)
    done = srv.poll(len(stream) + 1)
    st = srv.stats()
    srv.close()
    infos = [i for i, _ in done]
    lat = np.array([i.t_done - i.t_submit for i in infos])
    queue = np.array([i.t_admit - i.t_submit for i in infos if i.instance >= 0] or [0.0])
    ok = sum(1 for i in infos if i.status == lib.OK and i.converged)
    rhs = sum(i.nrhs for i in infos)
    span = max(i.t_done for i in infos) - min(i.t_submit for i in infos)
    by_L = {}
    for i, rq in zip(sorted(infos, key=lambda i: i.id), stream):
        by_L.setdefault(cfgs[rq["config"]]["L"], []).append(i.t_done - i.t_submit)
    gaps = np.array([rq["m0"] - m_c[rq["config"]] for rq in stream])
    return {"requests": len(infos), "ok": ok, "rhs": rhs,
            "capacity_requests_per_s": capacity, "capacity_solves_per_s": sum(i.nrhs for i in cap_done) / cap_span,
            "load": rate / capacity, "qps": rate,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "queue_p50_ms": float(np.percentile(queue, 50) * 1e3),
            "queue_p99_ms": float(np.percentile(queue, 99) * 1e3),
            "solves_per_s": rhs / span, "span_s": span,
            "p50_ms_by_L": {str(L): float(np.percentile(v, 50) * 1e3) for L, v in sorted(by_L.items())},
            "p99_ms_by_L": {str(L): float(np.percentile(v, 99) * 1e3) for L, v in sorted(by_L.items())},
            "iterations_max": max(i.iterations for i in infos),
            "max_rel_residual": max(i.true_rel_residual for i in infos),
            "gap_min_max": [float(gaps.min()), float(gaps.max())], "reference_gap": ref_gap,
            "warmup_setups": warm.setups, "warmup_s": t_warm, "setup_s_max": st.setup_seconds_max,
            "setups_during_stream": st.setups - before.setups,
            "derivations_during_stream": st.derivations - before.derivations,
            "derive_s_mean": (st.derive_seconds - before.derive_seconds) / max(1, st.derivations - before.derivations),
            "derive_s_max": st.derive_seconds_max, "evictions": st.evictions,
            "peak_resident_GB": st.peak_resident_bytes / 1e9, "budget_GB": st.budget_bytes / 1e9,
            "client_max_lag_ms": lag[0] * 1e3,
            "slots": slots, "instances": instances, "builders": builders, "configs": len(cfgs),
            "lattices": sorted({c["L"] for c in cfgs}), "gauge_generation_s": t_gen}


def multi_lattice_leg(lib, torch, ctx, groups, instances=8, slots=8, nrhs_per=8, links=None):
    """(1) 64 right-hand sides on the 128^2 beta = 8 lattice at m0 = m_c + 0.01 as one batched
    solve (step = setup + solve, like the headline); (2) the 32 lattices of
    synth.multi_lattice_configs() (L in 32..256, beta in [2, 10], m0 = m_c + gap), nrhs_per
    right-hand sides each, submitted at once to the server in mixed precision: makespan cold
    (hierarchy builds included) and warm (hierarchies cached)."""
    out = {}
    w = synth.WORKLOADS["C4"]
    m0 = synth.critical_masses()["C4"] + w.gaps[0]
    g = lib.Gauge(ctx, synth.links_to_abi(w.links()), m0)
    h = lib.Hierarchy(g, lib.default_setup_params(**w.setup_kw()))
    b = torch.from_numpy(synth.field_to_abi(synth.gaussian_rhs(w.L, w.L, w.rhs_seed, nrhs=64))).to("cuda")
    x = torch.zeros_like(b)
    dt, ts, infos, _ = run_steps(lib, torch, ctx, h, b, x, 64, lib.MIXED_FP32, 2, 1, groups=groups)
    its = [i.iterations for i in infos]
    out["one_lattice_128_64rhs"] = {"solves_per_s": 128 / dt, "s_per_step": dt / 2, "setup_s": ts / 2,
                                    "iterations_min_max": [min(its), max(its)],
                                    "converged": all(i.converged for i in infos)}
    h.close()
    # the same with level 1 (16 x 16 nodes of 8 x 8 blocks) swept on matrix cores
    h = lib.Hierarchy(g, lib.default_setup_params(**w.setup_kw(block_smoother=1)))
    dt, ts, infos, _ = run_steps(lib, torch, ctx, h, b, x, 64, lib.MIXED_FP32, 2, 1, groups=groups)
    its = [i.iterations for i in infos]
    out["one_lattice_128_64rhs_matrix_core_smoother"] = {"solves_per_s": 128 / dt, "s_per_step": dt / 2,
                                                          "iterations_min_max": [min(its), max(its)],
                                                          "converged": all(i.converged for i in infos)}
    h.close()
    g.close()
    del b, x
    cfgs = synth.multi_lattice_configs()
    mcs = synth.multi_lattice_critical()
    links = [synth.serving_links(c) for c in cfgs] if links is None else links[0]
    srv = lib.Server(0, lib.default_server_params(slots=slots, max_instances=instances, precision=lib.MIXED_FP32))
    gids = [srv.add_gauge(synth.links_to_abi(U)) for U in links]
    setups = [lib.default_setup_params(**synth.serving_setup(c["L"])) for c in cfgs]
    rhs = [synth.field_to_abi(synth.gaussian_rhs(c["L"], c["L"], c["seed"] + 99, nrhs=nrhs_per)) for c in cfgs]
    for phase in ("cold", "warm"):
        t0 = time.perf_counter()
        for k, c in enumerate(cfgs):
            srv.submit(gids[k], mcs[k] + c["gap"], rhs[k], setups[k])
        srv.wait(1800)
        span = time.perf_counter() - t0
        done = [i for i, _ in srv.poll(len(cfgs) + 1)]
        out[f"lattices_32_{phase}"] = {
            "makespan_s": span, "solves_per_s": len(cfgs) * nrhs_per / span,
            "ok": sum(1 for i in done if i.status == lib.OK and i.converged),
            "iterations_max": max(i.iterations for i in done),
            "max_rel_residual": max(i.true_rel_residual for i in done)}
    st = srv.stats()
    srv.close()
    # the same 32 lattices as one lock-step solve: each Gram-Schmidt kernel launched once for all
    # lattices, and (graphs) one captured HIP graph per restart round
    ctx2 = lib.Context(0, torch.cuda.current_stream().cuda_stream)
    gs2 = [lib.Gauge(ctx2, synth.links_to_abi(U), mcs[k] + c["gap"]) for k, (U, c) in enumerate(zip(links, cfgs))]
    t0 = time.perf_counter()
    hs2 = [lib.Hierarchy(g2, st_) for g2, st_ in zip(gs2, setups)]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    bs = [torch.from_numpy(r).to("cuda") for r in rhs]
    for graphs in (0, 1):
        xs = [torch.zeros_like(b_) for b_ in bs]
        sp = lib.default_solve_params(precision=lib.MIXED_FP32, graphs=graphs)
        for rep in range(2):                       # the first call tunes and captures
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos, stt = lib.solve_multi_device(hs2, [nrhs_per] * len(cfgs), [b_.data_ptr() for b_ in bs],
                                                [x_.data_ptr() for x_ in xs], sp,
                                                torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            span = time.perf_counter() - t0
        flat = [i for li in infos for i in li]
        out[f"lattices_32_lockstep{'_graph' if graphs else ''}"] = {
            "makespan_s": span, "solves_per_s": len(cfgs) * nrhs_per / span, "setup_s_all": t_setup,
            "ok": sum(1 for i in flat if i.converged) // nrhs_per, "iterations_max": max(i.iterations for i in flat),
            "max_rel_residual": max(i.true_rel_residual for i in flat)}
    for h2 in hs2:
        h2.close()
    for g2 in gs2:
        g2.close()
    ctx2.close()
    out["lattices_32_setups"] = st.setups
    out["lattices"] = {str(L): sum(1 for c in cfgs if c["L"] == L) for L in synth.MULTI_SIZES}
    out["nrhs_per_lattice"] = nrhs_per
    out["instances"], out["slots"] = instances, slots
    return out


AGG_SWEEP = ((3, 4, 1), (3, 8, 1), (3, 8, 2), (2, 16, 2))      # (levels, a, o)


def agg_sweep_leg(lib, torch, ctx, groups, nrhs=64):
    """Sensitivity to the wirebasket size (the paper's parameter spread): the 256^2 workload's
    field and mass, 64 right-hand sides, mixed precision, setup + solve per (levels, a, o)."""
    w = synth.WORKLOADS["C3"]
    m0 = synth.critical_masses()["C3"] + w.gaps[0]
    g = lib.Gauge(ctx, synth.links_to_abi(w.links()), m0)
    b = torch.from_numpy(synth.field_to_abi(synth.gaussian_rhs(w.L, w.L, w.rhs_seed, nrhs=nrhs))).to("cuda")
    x = torch.zeros_like(b)
    out = []
    for levels, a, o in AGG_SWEEP:
        t0 = time.perf_counter()
        h = lib.Hierarchy(g, lib.default_setup_params(levels=levels, agg_size=a, overlap=o,
                                                       n_test_vectors=w.n_test_vectors,
                                                       test_vector_sweeps=w.test_vector_sweeps))
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        dt, ts, infos, _ = run_steps(lib, torch, ctx, h, b, x, nrhs, lib.MIXED_FP32, 1, 1, groups=groups)
        its = [i.iterations for i in infos]
        rec = {"levels": levels, "a": a, "o": o, "solves_per_s": nrhs / dt, "setup_s": ts,
               "first_setup_s": t_first, "iterations_min_max": [min(its), max(its)],
               "converged": all(i.converged for i in infos)}
        log("agg sweep", json.dumps(rec))
        out.append(rec)
        h.close()
    g.close()
    return out


TV_SWEEPS = (4, 16, 32, 64, 128)


def tv_sweep_leg(lib, torch, ctx, groups, nrhs=64):
    """The smoother sweeps that relax the test vectors (the paper leaves their number open): the
    256^2 workload's field and mass, 64 right-hand sides, mixed precision, setup + solve per
    value."""
    w = synth.WORKLOADS["C3"]
    m0 = synth.critical_masses()["C3"] + w.gaps[0]
    g = lib.Gauge(ctx, synth.links_to_abi(w.links()), m0)
    b = torch.from_numpy(synth.field_to_abi(synth.gaussian_rhs(w.L, w.L, w.rhs_seed, nrhs=nrhs))).to("cuda")
    x = torch.zeros_like(b)
    out = []
    for nu in TV_SWEEPS:
        h = lib.Hierarchy(g, lib.default_setup_params(**w.setup_kw(test_vector_sweeps=nu)))
        dt, ts, infos, _ = run_steps(lib, torch, ctx, h, b, x, nrhs, lib.MIXED_FP32, 1, 1, groups=groups)
        its = [i.iterations for i in infos]
        rec = {"test_vector_sweeps": nu, "solves_per_s": nrhs / dt, "setup_s": ts,
               "iterations_min_max": [min(its), max(its)], "converged": all(i.converged for i in infos)}
        log("test-vector sweeps", json.dumps(rec))
        out.append(rec)
        h.close()
    g.close()
    return out


BATCH_SWEEP = (1, 8, 32, 64, 128)


def batch_sweep_leg(lib, torch, ctx, h, w, groups):
    """Setup + solve of the 256^2 workload's first nrhs Gaussian right-hand sides per step, mixed
    precision (stream groups of at least 16 rhs), and the BF16-link mode at 64."""
    out = []
    for nrhs, prec in [(n, lib.MIXED_FP32) for n in BATCH_SWEEP] + [(64, lib.MIXED_FP32_BF16LINKS)]:
        psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed, nrhs=nrhs)
        b = torch.from_numpy(synth.field_to_abi(psi)).to("cuda")
        x = torch.zeros_like(b)
        gr = max(1, min(groups, nrhs // 16))
        dt, ts, infos, _ = run_steps(lib, torch, ctx, h, b, x, nrhs, prec, 1, 1, groups=gr)
        its = [i.iterations for i in infos]
        rec = {"nrhs": nrhs, "precision": {lib.MIXED_FP32: "mixed", lib.MIXED_FP32_BF16LINKS: "mixed_bf16links"}[prec],
               "groups": gr, "solves_per_s": nrhs / dt, "s_per_step": dt, "iterations_min_max": [min(its), max(its)],
               "converged": all(i.converged for i in infos)}
        log("batch sweep", json.dumps(rec))
        out.append(rec)
        del b, x
    return out


# the paper's own settings beside this library's defaults, on the headline workload
VARIANTS = (("coarsest GMRES to 0.1 (the paper's coarsest solver)", dict(coarsest_tol=0.1)),
            ("normalisation CONST (the paper's literal rule)", dict(norm=1)),
            ("normalisation NONE", dict(norm=2)))


def variants_leg(lib, torch, ctx, groups, nrhs=64):
    """The 256^2 workload's field and mass, 64 right-hand sides, mixed precision, setup + solve,
    with one setup parameter changed per record."""
    w = synth.WORKLOADS["C3"]
    m0 = synth.critical_masses()["C3"] + w.gaps[0]
    g = lib.Gauge(ctx, synth.links_to_abi(w.links()), m0)
    b = torch.from_numpy(synth.field_to_abi(synth.gaussian_rhs(w.L, w.L, w.rhs_seed, nrhs=nrhs))).to("cuda")
    x = torch.zeros_like(b)
    out = []
    for name, kw in VARIANTS:
        h = lib.Hierarchy(g, lib.default_setup_params(**w.setup_kw(**kw)))
        dt, ts, infos, _ = run_steps(lib, torch, ctx, h, b, x, nrhs, lib.MIXED_FP32, 1, 1, groups=groups)
        its = [i.iterations for i in infos]
        rec = {"variant": name, "setup": kw, "solves_per_s": nrhs / dt, "setup_s": ts,
               "iterations_min_max": [min(its), max(its)], "converged": all(i.converged for i in infos),
               "max_rel_residual": max(i.true_rel_residual for i in infos)}
        log("variant", json.dumps(rec))
        out.append(rec)
        h.close()
    g.close()
    return out


def flop_summary(w, iterations, s_per_step):
    """Operation count of one step (setup + the batch's solves) from the geometry model, the
    rate it implies, and the paper's AM-AMG counts at 256^2 for context (another coarsening,
    the real K-formulation, other ensembles: not a like-for-like target)."""
    from paper_2608_03515_amd import flops
    geo = flops.levels_of(w.L, w.L, w.levels, w.agg, w.overlap)
    st = flops.setup(geo, w.agg, w.overlap, w.n_test_vectors, w.test_vector_sweeps)
    sv = [flops.solve(geo, w.agg, w.overlap, it, restart=w.restart) for it in iterations]
    total = st["total"] + sum(v["total"] for v in sv)
    mean_solve = sum(v["total"] for v in sv) / len(sv)
    return {"model": "paper_2608_03515_amd.flops (real operations; algorithmic, setup included)",
            "setup_gflop": st["total"] / 1e9,
            "setup_parts_gflop": {k: v / 1e9 for k, v in st.items() if k != "total"},
            "solve_gflop_per_rhs_mean": mean_solve / 1e9,
            "gflop_per_solve_setup_per_rhs": st["total"] / 1e9 + mean_solve / 1e9,
            "gflop_per_solve_setup_shared": st["total"] / len(sv) / 1e9 + mean_solve / 1e9,
            "flop_per_site_per_iteration": sum(v["per_iteration_per_site"] for v in sv) / len(sv),
            "achieved_tflops": total / s_per_step / 1e12,
            "paper_am_amg_256": {"setup_gflop": 1.1, "kflop_per_site_per_iteration_range": [17.4, 17.6],
                                 "gflop_per_solve_range": [11.1, 1003.5],
                                 "note": "two-level algebraic AM-AMG, 9-point wirebaskets, beta 2-6, "
                                         "gaps 0.001-0.1; setup repeated per right-hand side"}}


# ------------------------------------------------------------------ profile summaries
# Kernel-name patterns of each timed family in the mixed step (the first pattern is the family's
# main kernel, one dispatch per timed launch; further patterns are kernels the same launch
# record covers), and the source file each is built from.
# kernel-name patterns of each family; "a&b" matches names holding both parts (the solve's FP32
# fused sweeps at any tuned tile width, not the setup's FP64 test-vector sweeps)
FAMILY_PATTERNS = {
    "fine_matvec": ("k_wilson_apply<64, 2, float",),
    "fine_gs": ("k_wilson_gs_fused<2, 16, &, float, ",),
    "restrict0": ("k_restrict_partial_tiled<32, 60, 32, float", "k_restrict_gather<float, HIP_vector_type<double"),
    "prolong0": ("k_prolong_tiled<32, 64, 32, float",),
    "coarse_gs": ("k_stencil_gs_quad_mfma<",),
    "dots": ("k_gram<",),
    "update": ("k_lag_update<",),
}


def pat_in(pat, name):
    return all(part in name for part in pat.split("&"))


_CSRC = os.path.join(ROOT, "paper_2608_03515_amd", "csrc")
FAMILY_SRC = {"fine_matvec": "fine.hip", "fine_gs": "fine.hip", "restrict0": "transfer.hip",
              "prolong0": "transfer.hip", "coarse_gs": "coarse.hip", "dots": "krylov.hip", "update": "krylov.hip"}
TRAFFIC_MD = os.path.join(ROOT, "profiles", "solve_families_256x256_64rhs_mixed_traffic.md")


def family_src_sha(fam):
    return _sha(os.path.join(_CSRC, FAMILY_SRC[fam]))


def _sha(path):
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def trace_summary(stats_csv, out_md, command, top=25):
    """Markdown summary of a rocprofv3 --kernel-trace --stats kernel_stats.csv."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# Kernel time, {os.path.basename(out_md)[:-3]}", "", "Command (from the repository root):", "",
             f"    {command}", "", f"Total kernel time {total / 1e6:.1f} ms over "
             f"{sum(int(r['Calls']) for r in rows)} dispatches.", "",
             "| total ms | calls | avg us | % | kernel |", "|---:|---:|---:|---:|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        name = r["Name"].split("(")[0].replace("|", "/")[:90]
        lines.append(f"| {float(r['TotalDurationNs']) / 1e6:.2f} | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} | `{name}` |")
    lines += ["", "Families (all instantiations):", "", "| family | calls | avg us | total ms |", "|---|---:|---:|---:|"]
    for fam, pats in FAMILY_PATTERNS.items():
        for pat in pats:
            sel = [r for r in rows if pat_in(pat, r["Name"])]
            n = sum(int(r["Calls"]) for r in sel)
            t = sum(float(r["TotalDurationNs"]) for r in sel)
            if n:
                lines.append(f"| {fam} (`{pat.replace('&', '…')}*`) | {n} | {t / n / 1e3:.2f} | {t / 1e6:.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def timer_families(t):
    """{family: {launches, avg_launch_us, algorithmic_bytes_per_launch}} from the JSON line of
    --profile-mixed (one family under "family", or several under "families")."""
    if "families" in t:
        return t["families"]
    return {t["family"]: t} if "family" in t else {}


def pmc_summary(fetch_csv, write_csv, out_md, command, timer_json, wait_csv=None):
    """HBM traffic per launch of the step's kernel families from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE), scaled by the same counters on a plain 1 GiB elementwise copy in
    the same run, beside the kernel timer's algorithmic bytes and launch times.  With wait_csv
    (a pass over SQ_WAIT_ANY, SQ_ACTIVE_INST_VALU, SQ_WAVES) also the cycles a wave waits per
    VALU-active cycle."""
    import csv
    from collections import defaultdict

    def load(path, counter=None):
        per = defaultdict(list)
        with open(path) as f:
            for row in csv.DictReader(f):
                if counter is None or row.get("Counter_Name") == counter:
                    per[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return per
    fe, wr = load(fetch_csv), load(write_csv)
    cal = [k for k in fe if "neg_kernel" in k]
    f_fac = fe[cal[0]][0] * 1024 / 2 ** 30          # counter bytes per byte read
    w_fac = wr[cal[0]][0] * 1024 / 2 ** 30          # counter bytes per byte written
    t = json.loads(timer_json)
    fams = timer_families(t)
    lines = [f"# HBM traffic, {os.path.basename(out_md)[:-3]}", "",
             "Counter passes (one counter each for the traffic), from the repository root:", ""]
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        lines.append(f"    {command.replace('COUNTER', c)}")
    if wait_csv:
        lines.append(f"    {command.replace('COUNTER', 'SQ_WAIT_ANY SQ_ACTIVE_INST_VALU SQ_WAVES')}")
    lines += ["", f"Calibration: a 1 GiB elementwise copy (`neg`) reads as {fe[cal[0]][0]:.0f} KiB of "
              f"FETCH_SIZE and writes as {wr[cal[0]][0]:.0f} KiB of WRITE_SIZE: scale factors "
              f"{f_fac:.4f} (fetch) and {w_fac:.4f} (write) counter bytes per byte.", "",
              "Per launch of each timed family (its kernels' traffic summed; algorithmic bytes and mean "
              "launch time from the library's kernel timer in the same command, one stream):", "",
              "| family | dispatches with traffic | read MB / launch | written MB / launch | "
              "algorithmic MB / launch (timer) | traffic / algorithmic | us / launch (timer) | "
              "algorithmic GB/s | % of 8 TB/s |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    rec = {}
    for fam, pats in FAMILY_PATTERNS.items():
        fv0 = [v for k, vs in fe.items() if pat_in(pats[0], k) for v in vs]
        nwork = sum(1 for v in fv0 if v * 1024 / f_fac > 1e6)
        if not nwork:
            continue
        fv = [v for k, vs in fe.items() if any(pat_in(p, k) for p in pats) for v in vs]
        wv = [v for k, vs in wr.items() if any(pat_in(p, k) for p in pats) for v in vs]
        rd = sum(fv) * 1024 / f_fac / nwork
        wt = sum(wv) * 1024 / w_fac / nwork
        ft = fams.get(fam, {})
        alg, us = ft.get("algorithmic_bytes_per_launch"), ft.get("avg_launch_us")
        rec[fam] = (rd, wt, nwork)
        gbs = alg / (us * 1e3) if alg and us else float("nan")
        lines.append(f"| {fam} | {nwork} | {rd / 1e6:.1f} | {wt / 1e6:.1f} | "
                     f"{alg / 1e6 if alg else float('nan'):.1f} | "
                     f"{(rd + wt) / alg if alg else float('nan'):.3f} | {us if us else float('nan'):.1f} | "
                     f"{gbs:.0f} | {100 * gbs / HBM_PEAK_GBS:.1f} |")
    if wait_csv:
        wa, va, wv_ = (load(wait_csv, c) for c in ("SQ_WAIT_ANY", "SQ_ACTIVE_INST_VALU", "SQ_WAVES"))
        lines += ["", "Latency: wave-cycles waiting on anything per VALU-active wave-cycle, summed over the "
                  "family's main kernel:", "", "| family | SQ_WAIT_ANY / SQ_ACTIVE_INST_VALU | waves / dispatch |",
                  "|---|---:|---:|"]
        for fam, pats in FAMILY_PATTERNS.items():
            w = sum(v for k, vs in wa.items() if pat_in(pats[0], k) for v in vs)
            a = sum(v for k, vs in va.items() if pat_in(pats[0], k) for v in vs)
            nw = [v for k, vs in wv_.items() if pat_in(pats[0], k) for v in vs]
            if a > 0:
                lines.append(f"| {fam} | {w / a:.2f} | {sum(nw) / max(1, len(nw)):.0f} |")
    lines.append("")
    for fam in fams:
        if fam in rec:
            lines.append(f"<!-- traffic family={fam} source_sha={family_src_sha(fam)} "
                         f"bytes_per_launch={rec[fam][0] + rec[fam][1]:.0f} -->")
    open(out_md, "w").write("\n".join(lines) + "\n")


STENCIL_L = 4096
STENCIL_BYTES_PER_SITE = {"fp64": 96, "fp32": 48, "fp32_bf16links": 40}


def stencil_traffic_summary(fetch_csv, write_csv, stats_csv, out_md, command, trace_command):
    """HBM bytes per launch of the fine stencil at 4096^2 (bench.py --stencil-only) from two
    rocprofv3 --pmc runs, scaled by the same counters on a 1 GiB elementwise copy, beside the
    algorithmic bytes (per site: 2 spinor reads, 2 links, 1 spinor write) and the rate over the
    kernel trace's mean duration."""
    import csv
    from collections import defaultdict

    def load(path):
        per = defaultdict(list)
        with open(path) as f:
            for row in csv.DictReader(f):
                per[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return per
    fe, wr = load(fetch_csv), load(write_csv)
    cal = [k for k in fe if "neg_kernel" in k]
    f_fac = fe[cal[0]][0] * 1024 / 2 ** 30
    w_fac = wr[cal[0]][0] * 1024 / 2 ** 30
    dur = {r["Name"].split("(")[0]: float(r["AverageNs"]) for r in csv.DictReader(open(stats_csv))}

    def mode(name):
        # template arguments: tile width, sites per thread, compute type, link storage, ...
        args = [a.strip() for a in name.split("k_wilson_apply<", 1)[1].split(",")]
        if "bf16" in args[3]:
            return "fp32_bf16links"
        return "fp64" if args[2] == "double" else "fp32"
    lines = [f"# HBM traffic, {os.path.basename(out_md)[:-3]}", "",
             "Two counter passes (one counter each) and a kernel trace, from the repository root:", ""]
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        lines.append(f"    {command.replace('COUNTER', c)}")
    lines += [f"    {trace_command}", "",
              f"Calibration: a 1 GiB elementwise copy (`neg`) reads as {fe[cal[0]][0]:.0f} KiB of "
              f"FETCH_SIZE and writes as {wr[cal[0]][0]:.0f} KiB of WRITE_SIZE: scale factors "
              f"{f_fac:.4f} (fetch) and {w_fac:.4f} (write) counter bytes per byte.", "",
              "| kernel | mode | dispatches | read MB | written MB | algorithmic MB | traffic / algorithmic "
              "| mean us (trace) | algorithmic GB/s | measured GB/s |",
              "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name in sorted(k for k in fe if "k_wilson_apply" in k):
        m = mode(name)
        n = len(fe[name])
        rd = sum(fe[name]) * 1024 / f_fac / n
        wt = sum(wr.get(name, [0.0])) * 1024 / w_fac / max(1, len(wr.get(name, [])))
        alg = STENCIL_BYTES_PER_SITE[m] * STENCIL_L * STENCIL_L
        us = dur.get(name.split("(")[0], float("nan")) / 1e3
        short = name.split("(")[0].replace("|", "/")[:70]
        lines.append(f"| `{short}` | {m} | {n} | {rd / 1e6:.1f} | {wt / 1e6:.1f} | {alg / 1e6:.1f} | "
                     f"{(rd + wt) / alg:.3f} | {us:.1f} | {alg / (us * 1e3):.0f} | {(rd + wt) / (us * 1e3):.0f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


MFMA_KERNELS = ("k_restrict_mfma", "k_prolong_mfma", "k_dense_apply_mfma", "k_stencil_gs_quad_mfma")
MFMA_PEAK_TFLOPS = {"F32": 157.3, "F64": 78.6}
SIMD_NUM = 1024


def mfma_summary(pmc_csv, stats_csv, out_md, command, trace_command):
    """Matrix-core use of the MFMA kernels: one rocprofv3 --pmc pass (SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_INSTS_VALU_MFMA_MOPS_F32/F64, GRBM_GUI_ACTIVE) and the kernel trace's mean durations.
    Utilisation = busy cycles / (active cycles x SIMDs), the vendor's MfmaUtil; flops = MOPS x 512."""
    import csv
    from collections import defaultdict
    per = defaultdict(lambda: defaultdict(list))
    with open(pmc_csv) as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            for k in MFMA_KERNELS:
                if k in name:
                    per[name][row["Counter_Name"]].append(float(row["Counter_Value"]))
    dur = {r["Name"]: float(r["AverageNs"]) for r in csv.DictReader(open(stats_csv))}
    lines = [f"# Matrix-core use, {os.path.basename(out_md)[:-3]}", "",
             "Counter pass and kernel trace, from the repository root:", "", f"    {command}",
             f"    {trace_command}", "",
             "| kernel | dispatches | MFMA util % (mean) | GFLOP / dispatch | mean us (trace) | TFLOP/s | peak | % of peak |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for name, c in sorted(per.items()):
        n = len(c.get("GRBM_GUI_ACTIVE", []))
        if not n:
            continue
        util = [100.0 * b / (a * SIMD_NUM) for b, a in zip(c["SQ_VALU_MFMA_BUSY_CYCLES"], c["GRBM_GUI_ACTIVE"]) if a > 0]
        f32 = sum(c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", [0])) * 512 / n
        f64 = sum(c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", [0])) * 512 / n
        kind = "F64" if f64 > f32 else "F32"
        flops = max(f32, f64)
        us = next((v / 1e3 for k, v in dur.items() if k.split("(")[0] == name.split("(")[0]), float("nan"))
        tf = flops / (us * 1e-6) / 1e12 if us == us and us > 0 else float("nan")
        short = name.split("(")[0].replace("|", "/")[:80]
        lines.append(f"| `{short}` | {n} | {sum(util) / max(1, len(util)):.1f} | {flops / 1e9:.3f} | {us:.2f} | "
                     f"{tf:.1f} | {MFMA_PEAK_TFLOPS[kind]} ({kind}) | {100 * tf / MFMA_PEAK_TFLOPS[kind]:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def committed_traffic(family):
    """Per-launch HBM bytes of `family` from the committed counter summary, or None when the
    summary is missing, covers another family, or the kernel source changed since."""
    import re
    try:
        text = open(TRAFFIC_MD).read()
    except OSError:
        return None
    for m in re.finditer(r"<!-- traffic family=(\w+) source_sha=(\w+) bytes_per_launch=([0-9.]+) -->", text):
        if m.group(1) == family and m.group(2) == family_src_sha(family):
            return float(m.group(3))
    return None


LEGS = ("multi", "agg", "batch", "tvs", "variants", "serving")
LEG_TIMEOUT_S = {"multi": 600, "serving": 900}


def leg_child(name, args, script=None):
    """One optional leg in a child process.  The full run starts these before it touches the GPU
    itself (a process that has initialised HIP may not start another program), one at a time,
    so that they never share the GPU with a timed pass; a failure or crash in a leg then costs
    that leg's record only, not the headline line.  The child's progress lines pass through."""
    import subprocess
    cmd = [sys.executable, script or os.path.abspath(__file__), "--leg", name, "--groups", str(args.groups),
           "--nrhs", str(args.nrhs), "--workload", args.workload, "--serve-requests", str(args.serve_requests)]
    if args.serve_qps is not None:
        cmd += ["--serve-qps", str(args.serve_qps)]
    if args.tv_sweeps is not None:
        cmd += ["--tv-sweeps", str(args.tv_sweeps)]
    if args.aug_vectors is not None:
        cmd += ["--aug-vectors", str(args.aug_vectors)]
    timeout = LEG_TIMEOUT_S.get(name, 300)
    log(f"leg {name}: child process")
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=None, text=True, timeout=timeout)
    except subprocess.TimeoutExpired:
        return {"error": f"child process timed out after {timeout} s"}
    for text in reversed(r.stdout.strip().splitlines()):
        try:
            d = json.loads(text)
        except ValueError:
            continue
        if isinstance(d, dict) and d.get("leg") == name:
            return d["result"]
    return {"error": f"child process ended with status {r.returncode} and no result"}


def run_leg(name, args):
    """Child side of leg_child: the leg's own gauge fields (host-generated before the GPU is
    touched), context and hierarchies."""
    serve_links = multi_links = None
    if name == "serving":
        serve_links = generate_links(synth.serving_configs(16))
    if name == "multi":
        if not os.path.exists(synth.MULTI_CRITICAL_PATH):
            return {"error": "critical masses not generated (python tests/golden/make_golden.py --multi-only)"}
        multi_links = generate_links(synth.multi_lattice_configs())
    import torch
    from paper_2608_03515_amd import amamg as lib
    if name == "serving":
        return serve_leg(lib, args.serve_requests, args.serve_qps, links=serve_links)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = lib.Context(0, stream.cuda_stream)
    if name == "multi":
        return multi_lattice_leg(lib, torch, ctx, args.groups, links=multi_links)
    if name == "agg":
        return agg_sweep_leg(lib, torch, ctx, args.groups)
    if name == "tvs":
        return tv_sweep_leg(lib, torch, ctx, args.groups)
    if name == "variants":
        return variants_leg(lib, torch, ctx, args.groups)
    w = synth.WORKLOADS[args.workload]
    m0 = synth.critical_masses()[w.name] + w.gaps[0] if w.m0 is None else w.m0
    g = lib.Gauge(ctx, synth.links_to_abi(w.links()), m0)
    h = lib.Hierarchy(g, lib.default_setup_params(**w.setup_kw()))
    out = batch_sweep_leg(lib, torch, ctx, h, w, args.groups)
    h.close()
    g.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--groups", type=int, default=2,
                    help="right-hand-side batches run concurrently on separate streams")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving leg (0: skip it)")
    ap.add_argument("--serve-qps", type=float, default=None,
                    help="arrival rate of the serving leg (default: 0.7 x its measured capacity)")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--multi", action="store_true",
                    help="also run the multi-lattice leg (off by default: one full run ended in a host "
                         "heap abort during it, cause not yet found)")
    ap.add_argument("--no-agg-sweep", action="store_true", help="skip the aggregate-size sweep")
    ap.add_argument("--no-batch-sweep", action="store_true",
                    help="skip the right-hand-side count sweep (1..128, mixed; BF16 links at 64)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the paper-setting variants (coarsest GMRES, CONST/NONE normalisation)")
    ap.add_argument("--stencil-only", action="store_true",
                    help="run only the 4096^2 fine-stencil bandwidth leg (for kernel traces)")
    ap.add_argument("--multi-only", action="store_true", help="run only the multi-lattice leg")
    ap.add_argument("--leg", default=None, choices=LEGS,
                    help="run one optional leg alone and print {\"leg\": name, \"result\": ...} (the full run "
                         "starts each optional leg this way in a child process)")
    ap.add_argument("--family", default=None, choices=FAMILIES,
                    help="kernel family of the roofline (default: the largest in an instrumented "
                         "one-stream step)")
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--aug-vectors", type=int, default=None,
                    help="test vectors augmenting the finest coarse space (default: the workload's)")
    ap.add_argument("--tv-sweeps", type=int, default=None,
                    help="smoother sweeps that relax the test vectors (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stencil", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="skip the single-rhs FP64 path")
    ap.add_argument("--trace-summary", nargs=3, metavar=("STATS_CSV", "OUT_MD", "COMMAND"))
    ap.add_argument("--mfma-summary", nargs=5, metavar=("PMC_CSV", "STATS_CSV", "OUT_MD", "COMMAND", "TRACE_COMMAND"))
    ap.add_argument("--stencil-traffic-summary", nargs=6,
                    metavar=("FETCH_CSV", "WRITE_CSV", "STATS_CSV", "OUT_MD", "COMMAND", "TRACE_COMMAND"))
    ap.add_argument("--pmc-summary", nargs="+",
                    metavar="ARG", help="FETCH_CSV WRITE_CSV OUT_MD COMMAND TIMER_JSON [WAIT_CSV]")
    ap.add_argument("--profile-mixed", action="store_true",
                    help="profiling run: only the one-stream timed mixed-precision steps of the "
                         "roofline pass (no FP64, single-rhs, stencil, serving or CPU legs), followed "
                         "by a device copy of known size")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(*args.trace_summary)
        return
    if args.mfma_summary:
        mfma_summary(*args.mfma_summary)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.stencil_traffic_summary:
        stencil_traffic_summary(*args.stencil_traffic_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent lattices and requests would run one per GPU).", file=sys.stderr)
        sys.exit(2)

    if args.serve_only or args.multi_only:
        args.leg = "serving" if args.serve_only else "multi"
    if args.leg:
        try:
            out = run_leg(args.leg, args)
        except Exception as e:              # reported in the leg's record
            out = {"error": f"{type(e).__name__}: {e}"}
        print(json.dumps({"leg": args.leg, "result": out}), flush=True)
        return
    # the optional legs, each in a child process, before this process touches the GPU
    full = not (args.stencil_only or args.profile_mixed)
    legs = {}
    if full:
        skip = {"multi": not args.multi, "agg": args.no_agg_sweep, "batch": args.no_batch_sweep,
                "tvs": args.no_variants, "variants": args.no_variants, "serving": args.serve_requests <= 0}
        for name in LEGS:
            if not skip[name]:
                legs[name] = leg_child(name, args)
                log(f"leg {name}", json.dumps(legs[name])[:400])

    import torch
    from paper_2608_03515_amd import amamg as lib

    if args.stencil_only:
        stream = torch.cuda.Stream()
        torch.cuda.set_stream(stream)
        ctx = lib.Context(0, stream.cuda_stream)
        st = stencil_bandwidth(lib, torch, ctx)
        # traffic-counter calibration: a plain elementwise copy of known size
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").normal_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)          # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        print(json.dumps({"stencil_4096": st}), flush=True)
        return

    stream = torch.cuda.Stream()          # default priority; the library runs on it
    torch.cuda.set_stream(stream)
    w = synth.WORKLOADS[args.workload]
    if args.tv_sweeps is not None or args.aug_vectors is not None:
        import dataclasses
        if args.tv_sweeps is not None:
            w = dataclasses.replace(w, test_vector_sweeps=args.tv_sweeps)
        if args.aug_vectors is not None:
            w = dataclasses.replace(w, aug_vectors=args.aug_vectors)
    m0 = synth.critical_masses()[w.name] + w.gaps[0] if w.m0 is None else w.m0
    log(f"workload {w.name}: L={w.L} beta={w.beta} m0={m0:.6f} levels={w.levels} a={w.agg} "
        f"o={w.overlap} nu={w.test_vector_sweeps} aug={w.aug_vectors} nrhs={args.nrhs}")
    U = w.links()
    ctx = lib.Context(0, stream.cuda_stream)
    g = lib.Gauge(ctx, synth.links_to_abi(U), m0)
    h = lib.Hierarchy(g, lib.default_setup_params(**w.setup_kw()))
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed, nrhs=args.nrhs)
    b = torch.from_numpy(synth.field_to_abi(psi)).to("cuda")
    x = torch.zeros_like(b)

    def summarize(dt, t_setup, infos, nrhs, steps):
        its = [i.iterations for i in infos]
        return {"s_per_step": dt / steps, "setup_s": t_setup / steps,
                "solves_per_s": nrhs * steps / dt,
                "solve_only_per_s": nrhs * steps / (dt - t_setup),
                "iterations_min_max": [min(its), max(its)],
                "true_rel_residual_max": max(i.true_rel_residual for i in infos),
                "converged": all(i.converged for i in infos)}

    res = {}
    if args.profile_mixed:
        # both Gram-Schmidt families are timed: they take nearly equal time, and the roofline
        # reports whichever the instrumented step finds dominant
        fams = list(FAMILY_PATTERNS)
        dt, ts, infos, timed = run_steps(lib, torch, ctx, h, b, x, args.nrhs, lib.MIXED_FP32, args.steps,
                                         args.warmup, timer=fams, groups=1)
        # traffic-counter calibration: a plain elementwise copy of known size
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").normal_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)          # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        print(json.dumps({"profile_mixed": summarize(dt, ts, infos, args.nrhs, args.steps),
                          "families": {f: {"launches": n, "avg_launch_us": ms * 1e3 / max(1, n),
                                           "algorithmic_bytes_per_launch": nb / max(1, n)}
                                       for f, (n, ms, nb) in timed.items()},
                          "copy_bytes_each_way": src.numel() * 8}), flush=True)
        return
    dt, ts, infos, _ = run_steps(lib, torch, ctx, h, b, x, args.nrhs, lib.FP64, args.steps, args.warmup,
                                 groups=args.groups)
    res["fp64"] = summarize(dt, ts, infos, args.nrhs, args.steps)
    rhs0_iterations = infos[0].iterations          # the right-hand side the CPU oracle samples
    x64 = x.clone()
    log("fp64", json.dumps(res["fp64"]))
    fam, fam_ms = dominant_family(lib, torch, ctx, h, b, x, args.nrhs, lib.MIXED_FP32)
    if args.family:
        fam = args.family
    log("dominant family (mixed):", fam, json.dumps({k: round(v, 2) for k, v in fam_ms.items()}))
    # headline: the stream-grouped step, no timer events
    dt, ts, infos, _ = run_steps(lib, torch, ctx, h, b, x, args.nrhs, lib.MIXED_FP32, args.steps,
                                 args.warmup, groups=args.groups)
    res["mixed"] = summarize(dt, ts, infos, args.nrhs, args.steps)
    res["mixed"]["rel_diff_vs_fp64"] = float((x - x64).norm() / x64.norm())
    log("mixed", json.dumps(res["mixed"]))
    op_count = flop_summary(w, [i.iterations for i in infos], res["mixed"]["s_per_step"])
    # roofline: the same step on one stream with the dominant family timed by the kernels' own
    # begin/end stamps (with two streams a kernel's duration includes sharing the GPU with the
    # other batch, which says nothing about the kernel)
    dt, ts, infos, timed = run_steps(lib, torch, ctx, h, b, x, args.nrhs, lib.MIXED_FP32, args.steps,
                                     args.warmup, timer=fam, groups=1)
    res["mixed_one_stream"] = summarize(dt, ts, infos, args.nrhs, args.steps)
    log("mixed one stream", json.dumps(res["mixed_one_stream"]))
    launches, ms, nbytes = timed
    traffic = committed_traffic(fam)
    roofline = {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": traffic,
                "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
                "kernel": KERNEL_NAMES[fam], "family": fam, "launches": launches,
                "avg_launch_us": ms * 1e3 / max(launches, 1),
                "algorithmic_bytes_per_launch": nbytes / max(launches, 1),
                "family_ms_instrumented_step": {k: round(v, 3) for k, v in fam_ms.items()}}
    roofline["frac"] = roofline["achieved"] / HBM_PEAK_GBS
    roofline["timed_pass"] = "mixed_one_stream (same workload and steps, one stream)"
    copy_gbs = copy_bandwidth(torch)
    roofline["measured_copy_GBs"] = copy_gbs
    roofline["frac_of_measured_copy"] = roofline["achieved"] / copy_gbs
    if not args.no_single:
        h1 = lib.Hierarchy(g, lib.default_setup_params(**w.setup_kw()))
        b1, x1 = b[:1].contiguous(), torch.zeros_like(b[:1])
        dt, ts, infos, _ = run_steps(lib, torch, ctx, h1, b1, x1, 1, lib.FP64, args.steps, args.warmup)
        res["fp64_single_rhs"] = summarize(dt, ts, infos, 1, args.steps)
        log("fp64 single rhs", json.dumps(res["fp64_single_rhs"]))
        h1.close()

    stencil = None if args.no_stencil else stencil_bandwidth(lib, torch, ctx)
    if stencil:
        log("stencil", json.dumps(stencil))
    multi, agg, batches = legs.get("multi"), legs.get("agg"), legs.get("batch")
    tvs, variants, serving = legs.get("tvs"), legs.get("variants"), legs.get("serving")
    head = res["mixed"]
    line = {
        "metric": "solves/s to rel. residual 1e-10 at L=256 (mixed vs FP64); stencil GB/s; p99",
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["s_per_step"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic quenched U(1) links (Metropolis), Gaussian right-hand sides",
        "config": {"workload": f"{w.L}x{w.L} beta={w.beta} m0=m_c+{w.gaps[0] if w.gaps else 0}, "
                               f"{w.levels} levels a={w.agg} o={w.overlap} Nv={w.n_test_vectors} nu={w.test_vector_sweeps}, "
                               f"FGMRES({w.restart}) to 1e-10; step = AM-AMG setup + solve of "
                               f"{args.nrhs} right-hand sides",
                   "nrhs": args.nrhs, "stream_groups": args.groups,
                   "precision": "FP32 V-cycle and Arnoldi matvec inside FP64 FGMRES"},
        "fp64": res["fp64"], "mixed": res["mixed"], "mixed_one_stream": res["mixed_one_stream"],
        "fp64_single_rhs": res.get("fp64_single_rhs"),
        "mixed_over_fp64": res["mixed"]["solves_per_s"] / res["fp64"]["solves_per_s"],
        "mixed_batched_over_fp64_single": (res["mixed"]["solves_per_s"] / res["fp64_single_rhs"]["solves_per_s"])
        if "fp64_single_rhs" in res else None,
        "roofline": roofline,
        "stencil_4096": stencil,
        "serving": serving,
        "multi_lattice": multi,
        "aggregate_sweep": agg,
        "operation_count": op_count,
        "paper_variants": variants,
        "test_vector_sweeps": tvs,
        "batch_sweep": batches,
        "autotuner": ctx.tuning_entries(),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(w, m0, rhs0_iterations)
    h.close()
    g.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
