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


def run_steps(lib, torch, g, h, b, x, nrhs, precision, steps, warmup):
    sp = lib.default_solve_params(precision=precision)
    infos = None
    for _ in range(warmup):
        h.update()
        infos, _ = h.solve_device(b.data_ptr(), x.data_ptr(), nrhs, sp)
    torch.cuda.synchronize()
    t_setup = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        h.update()                     # synchronous: returns when the setup has finished
        t_setup += time.perf_counter() - ts
        infos, st = h.solve_device(b.data_ptr(), x.data_ptr(), nrhs, sp)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, t_setup, infos


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
    prm = SetupParams(levels=w.levels, agg=w.agg, overlap=w.overlap, n_test_vectors=w.n_test_vectors)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stencil", action="store_true")
    ap.add_argument("--precisions", default="fp64,mixed")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent lattices and requests would run one per GPU).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_03515_amd import amamg as lib

    stream = torch.cuda.Stream()          # default priority; the library runs on it
    torch.cuda.set_stream(stream)
    w = synth.WORKLOADS[args.workload]
    m0 = synth.critical_masses()[w.name] + w.gaps[0] if w.m0 is None else w.m0
    log(f"workload {w.name}: L={w.L} beta={w.beta} m0={m0:.6f} levels={w.levels} a={w.agg} o={w.overlap}")
    U = w.links()
    ctx = lib.Context(0, torch.cuda.current_stream().cuda_stream)
    g = lib.Gauge(ctx, synth.links_to_abi(U), m0)
    h = lib.Hierarchy(g, lib.default_setup_params(levels=w.levels, agg_size=w.agg, overlap=w.overlap,
                                                   n_test_vectors=w.n_test_vectors))
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed, nrhs=args.nrhs)
    b = torch.from_numpy(synth.field_to_abi(psi)).to("cuda")
    x = torch.zeros_like(b)
    res = {}
    xs = {}
    for name in args.precisions.split(","):
        prec = {"fp64": lib.FP64, "mixed": lib.MIXED_FP32, "bf16": lib.MIXED_FP32_BF16LINKS}[name]
        dt, t_setup, infos = run_steps(lib, torch, g, h, b, x, args.nrhs, prec, args.steps, args.warmup)
        its = [i.iterations for i in infos]
        res[name] = {"s_per_step": dt / args.steps, "setup_s": t_setup / args.steps,
                     "solves_per_s": args.nrhs * args.steps / dt,
                     "solve_only_per_s": args.nrhs * args.steps / (dt - t_setup),
                     "iterations": its, "true_rel_residual": max(i.true_rel_residual for i in infos),
                     "converged": all(i.converged for i in infos)}
        xs[name] = x.clone()
        log(name, json.dumps(res[name]))
    if "fp64" in xs and "mixed" in xs:
        d = (xs["mixed"] - xs["fp64"]).norm() / xs["fp64"].norm()
        res["mixed"]["rel_diff_vs_fp64"] = float(d)

    stencil = None if args.no_stencil else stencil_bandwidth(lib, torch, ctx)
    if stencil:
        log("stencil", json.dumps(stencil))
    head = res.get("mixed") or res[next(iter(res))]
    line = {
        "metric": "solves/s to rel. residual 1e-10 at L=256 (mixed vs FP64); stencil GB/s; p99",
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["s_per_step"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32+fp64" if "mixed" in res else "f64",
        "data": "synthetic quenched U(1) links (Metropolis), Gaussian right-hand sides",
        "config": {"workload": f"{w.L}x{w.L} beta={w.beta} m0=m_c+{w.gaps[0] if w.gaps else 0}, "
                               f"{w.levels} levels a={w.agg} o={w.overlap}, Nv={w.n_test_vectors}, "
                               f"FGMRES({w.restart}) to 1e-10; step = setup + solve of {args.nrhs} rhs",
                   "nrhs": args.nrhs, "precision": "mixed FP32 V-cycle/matvec in FP64 FGMRES"},
        "fp64": res.get("fp64"), "mixed": res.get("mixed"),
        "mixed_over_fp64": (res["mixed"]["solves_per_s"] / res["fp64"]["solves_per_s"])
        if "mixed" in res and "fp64" in res else None,
        "stencil_4096": stencil,
    }
    if not args.no_cpu_baseline:
        its = (res.get("fp64") or head)["iterations"][0]
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(w, m0, its)
    h.close()
    g.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
