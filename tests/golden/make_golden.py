"""Writes the stored values under tests/golden/ using only the CPU oracle and the input generators.

critical_mass.json: m_c = -min Re lambda(D(m0 = 0)) of each workload's gauge field, from the
oracle's shift-invert Arnoldi (spectrum module).  The near-critical workloads use
m0 = m_c + gap.
multi_lattice_critical.json: the same for the 32 lattices of synth.multi_lattice_configs()
(computed in a process pool).

Run from the repository root:  python tests/golden/make_golden.py [--multi-only]
"""
import os

# one BLAS thread per process, set before numpy loads: the multi-lattice pool runs one process per
# core, and threads inherited by its forked workers would oversubscribe the cores many times over
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import json  # noqa: E402
import sys  # noqa: E402

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


def main():
    if "--multi-only" in sys.argv:
        multi()
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
