"""Writes the stored values under tests/golden/ using only the CPU oracle and the input generators.

critical_mass.json: m_c = -min Re lambda(D(m0 = 0)) of each workload's gauge field, from the
oracle's shift-invert Arnoldi (spectrum module).  The near-critical workloads use
m0 = m_c + gap.
multi_lattice_critical.json: the same for the 32 lattices of synth.multi_lattice_configs()
(computed in a process pool).
serving_critical.json: the same for the 16 gauge fields of synth.serving_configs() (the
serving workload draws each request's mass near its field's m_c).

c3_solve.json: the oracle's FP64 solve of the 256^2 workload's first right-hand side (the one
the benchmark's batch starts with): iteration and restart counts, the true relative residual,
||x||, 64 sampled solution entries and the first 40 residual-history values.

sweep_order_counts.json: the oracle's FGMRES iteration and restart counts with the coarse
Gauss-Seidel colours visited in the library's order (the 2 x 2 blocks of the 4 x 4 colour
pattern in a row) and in ascending colour order, for the 64^2 workload at its five masses and
the 256^2 workload's first right-hand side.  The paper fixes no colour order; the table is the
evidence that the order does not change the convergence.

Run from the repository root:
    python tests/golden/make_golden.py [--multi-only | --serving | --c3-solve | --sweep-order]
"""
import os
import sys

# one BLAS thread per process, set before numpy loads: the multi-lattice pool runs one process per
# core, and threads inherited by its forked workers would oversubscribe the cores many times over
# (the single-process 256^2 solve keeps the default)
if "--c3-solve" not in sys.argv and "--sweep-order" not in sys.argv:
    for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ.setdefault(_v, "1")

import json  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.spectrum import critical_mass  # noqa: E402


def _mc(cfg):
    return round(critical_mass(synth.serving_links(cfg)), 12)


def multi(workers=8):
    """One process per lattice (one BLAS thread each, see the top of this file)."""
    from concurrent.futures import ProcessPoolExecutor
    cfgs = synth.multi_lattice_configs()
    # largest lattices first, so that the pool's tail holds the short jobs
    order = sorted(range(len(cfgs)), key=lambda i: -cfgs[i]["L"])
    mcs = [None] * len(cfgs)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for i, mc in zip(order, ex.map(_mc, [cfgs[i] for i in order])):
            mcs[i] = mc
            print(i, cfgs[i]["L"], mc, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "multi_lattice_critical.json")
    with open(path, "w") as f:
        json.dump({"configs": cfgs, "m_c": mcs}, f, indent=1)
        f.write("\n")


def serving(workers=8):
    """Critical masses of the 16 serving configurations, one process per configuration."""
    from concurrent.futures import ProcessPoolExecutor
    cfgs = synth.serving_configs(16)
    order = sorted(range(len(cfgs)), key=lambda i: -cfgs[i]["L"])
    mcs = [None] * len(cfgs)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for i, mc in zip(order, ex.map(_mc, [cfgs[i] for i in order])):
            mcs[i] = mc
            print(i, cfgs[i]["L"], mc, flush=True)
    with open(synth.SERVING_CRITICAL_PATH, "w") as f:
        json.dump({"configs": cfgs, "m_c": mcs}, f, indent=1)
        f.write("\n")


def c3_solve():
    import numpy as np
    from oracle.amg import SetupParams
    from oracle.solve import solve
    w = synth.WORKLOADS["C3"]
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "critical_mass.json")) as f:
        m0 = json.load(f)["C3"] + w.gaps[0]
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed, nrhs=1)[0]
    prm = SetupParams(**w.oracle_kw())
    x, info, _ = solve(w.links(), m0, psi, prm, restart=w.restart, tol=1e-10)
    rng = np.random.default_rng(0)
    sites = sorted(int(s) for s in rng.choice(w.L * w.L, 64, replace=False))
    xf = x.reshape(-1, 2)
    out = {"workload": "C3", "m0": m0, "rhs_seed": w.rhs_seed, "test_vector_sweeps": w.test_vector_sweeps,
           "iterations": info.iterations,
           "restarts": info.restarts, "converged": bool(info.converged),
           "true_rel_residual": float(info.true_rel_residual), "x_norm": float(np.linalg.norm(x)),
           "samples": [[s, q, float(xf[s, q].real), float(xf[s, q].imag)] for s in sites for q in range(2)],
           "history": [[float(v), bool(t)] for v, t in info.history[:40]]}
    print("C3", info.iterations, info.restarts, info.true_rel_residual, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_solve.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def sweep_order():
    from oracle import amg
    from oracle.solve import solve
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "critical_mass.json")) as f:
        mc = json.load(f)
    orders = {"blocks": tuple(amg.COARSE_ORDER), "ascending": tuple(range(16))}
    cases = [("C2", g, synth.WORKLOADS["C2"].rhs_seed + i)
             for i, g in enumerate(synth.WORKLOADS["C2"].gaps)]
    cases.append(("C3", synth.WORKLOADS["C3"].gaps[0], synth.WORKLOADS["C3"].rhs_seed))
    rows = []
    links = {}
    for name, gap, seed in cases:
        w = synth.WORKLOADS[name]
        if name not in links:
            links[name] = w.links()
        psi = synth.gaussian_rhs(w.L, w.L, seed)[0]
        prm = amg.SetupParams(levels=w.levels, agg=w.agg, overlap=w.overlap,
                              n_test_vectors=w.n_test_vectors)
        row = {"workload": name, "gap": gap, "rhs_seed": seed}
        for key, order in orders.items():
            amg.COARSE_ORDER = order
            _, info, _ = solve(links[name], mc[name] + gap, psi, prm, restart=w.restart, tol=1e-10)
            row[key] = {"iterations": info.iterations, "restarts": info.restarts,
                        "true_rel_residual": float(info.true_rel_residual)}
        amg.COARSE_ORDER = orders["blocks"]
        print(row, flush=True)
        rows.append(row)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_order_counts.json")
    with open(path, "w") as f:
        json.dump({"orders": {k: list(v) for k, v in orders.items()}, "rows": rows}, f, indent=1)
        f.write("\n")


def main():
    if "--sweep-order" in sys.argv:
        sweep_order()
        return
    if "--multi-only" in sys.argv:
        multi()
        return
    if "--serving" in sys.argv:
        serving()
        return
    if "--c3-solve" in sys.argv:
        c3_solve()
        return
    out = {}
    for name in ("C2", "C3", "C4"):
        w = synth.WORKLOADS[name]
        out[name] = round(critical_mass(w.links()), 12)
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "critical_mass.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    multi()


if __name__ == "__main__":
    main()
