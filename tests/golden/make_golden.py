"""Writes the stored values under tests/golden/ using only the CPU oracle and the input generators.

critical_mass.json: m_c = -min Re lambda(D(m0 = 0)) of each workload's gauge field, from the
oracle's shift-invert Arnoldi (spectrum module).  The near-critical workloads use
m0 = m_c + gap.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.spectrum import critical_mass  # noqa: E402


def main():
    out = {}
    for name in ("C2", "C3", "C4"):
        w = synth.WORKLOADS[name]
        out[name] = round(critical_mass(w.links()), 12)
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "critical_mass.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
