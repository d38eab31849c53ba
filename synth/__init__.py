"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the solver: it only produces inputs.

* ``gen_theta`` / ``gen_links``: quenched U(1) gauge fields in two dimensions from
  Metropolis sweeps of the Wilson plaquette action S = beta * sum_P (1 - cos theta_P),
  beta = 1/g^2 in lattice units (paper, Numerical Results section).  The paper's
  configurations are dynamical two-flavour HMC ensembles that are not public; these
  quenched fields stand in for them with the same lattice shapes and coupling range.
* ``gaussian_rhs``: complex Gaussian right-hand sides (re, im ~ N(0, 1)).
* ``WORKLOADS``: the lattice sizes, couplings and hierarchy parameters of the
  benchmark and parity workloads.

Layouts: links are complex ``[2 mu][Nt][Nx]`` with mu = 0 the time direction; a
fermion field is complex ``[Nt][Nx][2 spin]`` (site index t*Nx + x, spin fastest).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = ["gen_theta", "gen_links", "gaussian_rhs", "plaquette_angles",
           "Workload", "WORKLOADS", "critical_masses", "links_to_abi", "field_to_abi",
           "field_from_abi", "SERVING_SIZES", "serving_setup", "serving_configs",
           "serving_links", "MULTI_SIZES", "MULTI_GAPS", "multi_lattice_configs",
           "multi_lattice_critical", "MULTI_CRITICAL_PATH", "SERVING_CRITICAL_PATH", "SERVING_GAPS",
           "serving_critical", "near_critical_stream"]


def plaquette_angles(theta: np.ndarray) -> np.ndarray:
    """theta_P(n) = theta_0(n) + theta_1(n + t^) - theta_0(n + x^) - theta_1(n), periodic links."""
    th0, th1 = theta[0], theta[1]
    return th0 + np.roll(th1, -1, axis=0) - np.roll(th0, -1, axis=1) - th1


def gen_theta(nt: int, nx: int, beta: float, sweeps: int, seed: int,
              step: float = 1.0) -> np.ndarray:
    """Link angles theta[mu, t, x] after ``sweeps`` checkerboard Metropolis sweeps from a cold start.

    One sweep: for mu in (0, 1), for parity in (0, 1), every mu-link whose x (mu = 0)
    or t (mu = 1) coordinate has that parity is updated at once.  Such links share no
    plaquette, so the simultaneous update is an exact Metropolis step.  A proposal
    theta -> theta + delta with delta ~ U(-step, step) is accepted with probability
    min(1, exp(-dS)).  Random numbers come from NumPy's PCG64(seed): per half-step a
    full-shape delta array, then a full-shape uniform array.
    """
    if nt % 2 or nx % 2:
        raise ValueError("checkerboard Metropolis needs even Nt and Nx")
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = np.zeros((2, nt, nx))
    tcoord = np.arange(nt)[:, None] * np.ones((1, nx), dtype=np.int64)
    xcoord = np.ones((nt, 1), dtype=np.int64) * np.arange(nx)[None, :]
    for _ in range(sweeps):
        for mu in (0, 1):
            for parity in (0, 1):
                delta = rng.uniform(-step, step, size=(nt, nx))
                u = rng.uniform(0.0, 1.0, size=(nt, nx))
                tp = plaquette_angles(theta)
                if mu == 0:
                    # theta_0(n) enters P(n) with + and P(n - x^) with -
                    p_plus = tp
                    p_minus = np.roll(tp, 1, axis=1)
                    sel = (xcoord % 2) == parity
                    ds = beta * ((np.cos(p_plus) - np.cos(p_plus + delta))
                                 + (np.cos(p_minus) - np.cos(p_minus - delta)))
                else:
                    # theta_1(n) enters P(n) with - and P(n - t^) with +
                    p_minus = tp
                    p_plus = np.roll(tp, 1, axis=0)
                    sel = (tcoord % 2) == parity
                    ds = beta * ((np.cos(p_plus) - np.cos(p_plus + delta))
                                 + (np.cos(p_minus) - np.cos(p_minus - delta)))
                accept = sel & (u < np.exp(-np.minimum(ds, 700.0)))
                theta[mu] = np.where(accept, theta[mu] + delta, theta[mu])
    return np.mod(theta + np.pi, 2.0 * np.pi) - np.pi


def gen_links(nt: int, nx: int, beta: float, sweeps: int, seed: int) -> np.ndarray:
    """Complex U(1) links U[mu, t, x] = exp(i theta) (host libm)."""
    return np.exp(1j * gen_theta(nt, nx, beta, sweeps, seed))


def gaussian_rhs(nt: int, nx: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """Complex Gaussian fields [nrhs][Nt][Nx][2 spin], re and im ~ N(0, 1) from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((nrhs, nt, nx, 2, 2))
    return z[..., 0] + 1j * z[..., 1]


def links_to_abi(U: np.ndarray) -> np.ndarray:
    """Complex [2][Nt][Nx] -> float64 [2][Nt][Nx][2 (re, im)], C-contiguous."""
    return np.ascontiguousarray(np.stack([U.real, U.imag], axis=-1), dtype=np.float64)


def field_to_abi(psi: np.ndarray) -> np.ndarray:
    """Complex [nrhs][Nt][Nx][2] -> float64 [nrhs][Nt][Nx][2][2 (re, im)], C-contiguous."""
    return np.ascontiguousarray(np.stack([psi.real, psi.imag], axis=-1), dtype=np.float64)


def field_from_abi(buf: np.ndarray) -> np.ndarray:
    return buf[..., 0] + 1j * buf[..., 1]


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: lattice, coupling, hierarchy parameters and seeds."""
    name: str
    L: int
    beta: float
    sweeps: int
    link_seed: int
    rhs_seed: int
    levels: int
    agg: int
    overlap: int
    n_test_vectors: int
    test_vector_sweeps: int = 4
    m0: float | None = None          # fixed bare mass, or None when given by critical mass + gap
    aug_vectors: int = 0             # test vectors augmenting the finest level's coarse space
    gaps: tuple = field(default_factory=tuple)
    restart: int = 20
    tol: float = 1e-10

    def links(self) -> np.ndarray:
        return gen_links(self.L, self.L, self.beta, self.sweeps, self.link_seed)

    def setup_kw(self, **extra) -> dict:
        """Hierarchy parameters as keyword arguments of the library's setup parameters."""
        kw = dict(levels=self.levels, agg_size=self.agg, overlap=self.overlap,
                  n_test_vectors=self.n_test_vectors, test_vector_sweeps=self.test_vector_sweeps,
                  aug_vectors=self.aug_vectors)
        kw.update(extra)
        return kw

    def oracle_kw(self, **extra) -> dict:
        """The same parameters as keyword arguments of the oracle's setup parameters."""
        kw = dict(levels=self.levels, agg=self.agg, overlap=self.overlap,
                  n_test_vectors=self.n_test_vectors, test_vector_sweeps=self.test_vector_sweeps,
                  aug_vectors=self.aug_vectors)
        kw.update(extra)
        return kw


WORKLOADS = {
    # two levels, FP64, 16x16
    "C1": Workload("C1", 16, 3.0, 200, 1001, 2001, 2, 4, 1, 4, m0=0.1),
    # three levels, FP64, 64x64, masses approaching the critical mass
    "C2": Workload("C2", 64, 6.0, 200, 1002, 2002, 3, 4, 1, 8,
                   gaps=(0.1, 0.05, 0.02, 0.01, 0.005)),
    # three levels, 256x256, mixed precision vs FP64
    "C3": Workload("C3", 256, 10.0, 200, 1003, 2003, 3, 8, 2, 8, test_vector_sweeps=64, gaps=(0.01,)),
    # one 128x128 lattice for many right-hand sides
    "C4": Workload("C4", 128, 8.0, 200, 1004, 2004, 3, 8, 2, 8, test_vector_sweeps=64, gaps=(0.01,)),
}

_GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "tests", "golden", "critical_mass.json")


def critical_masses() -> dict:
    """Critical masses m_c = -min Re lambda(D(m0 = 0)) of the workload lattices.

    The values are written by ``tests/golden/make_golden.py`` with the CPU oracle's
    shift-invert eigensolver and stored as plain numbers; this function only reads them.
    """
    with open(_GOLDEN) as f:
        return json.load(f)


# ------------------------------------------------------------------------- serving workload

SERVING_SIZES = (32, 64, 128, 256, 512)
def serving_setup(L: int) -> dict:
    """AM-AMG setup parameters used for an L x L serving lattice (the configurations above at
    their sizes; 512 keeps a = 8, o = 2 with a 2048-unknown coarsest level)."""
    if L <= 32:
        return dict(levels=2, agg_size=4, overlap=1, n_test_vectors=4, test_vector_sweeps=64)
    if L <= 64:
        return dict(levels=3, agg_size=4, overlap=1, n_test_vectors=8, test_vector_sweeps=64)
    return dict(levels=3, agg_size=8, overlap=2, n_test_vectors=8, test_vector_sweeps=64)


def serving_configs(n: int = 16, seed: int = 5005, sweeps: int = 50) -> list:
    """n gauge configurations: L_j = SERVING_SIZES[j mod 5], beta_j = 2 + 8 j / (n - 1) (from 2
    to 10); Metropolis from a cold start with its own seed."""
    out = []
    for i in range(n):
        out.append({"L": SERVING_SIZES[i % len(SERVING_SIZES)],
                    "beta": 2.0 + 8.0 * i / max(1, n - 1), "sweeps": sweeps, "seed": seed + 1 + i})
    return out


def serving_links(cfg: dict) -> np.ndarray:
    return gen_links(cfg["L"], cfg["L"], cfg["beta"], cfg["sweeps"], cfg["seed"])


# ------------------------------------------------------------------- multi-lattice workload

MULTI_SIZES = (32, 64, 128, 256)
MULTI_GAPS = (0.01, 0.02, 0.05)


def multi_lattice_configs(n: int = 32, seed: int = 4004, sweeps: int = 100) -> list:
    """n independent lattices: the first four cover every size once, the rest draw L uniformly;
    beta uniform in [2, 10]; a gap above the lattice's critical mass from MULTI_GAPS."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        L = MULTI_SIZES[i] if i < len(MULTI_SIZES) else int(rng.choice(MULTI_SIZES))
        out.append({"L": L, "beta": float(rng.uniform(2.0, 10.0)), "sweeps": sweeps,
                    "seed": seed + 1 + i, "gap": float(rng.choice(MULTI_GAPS))})
    return out


MULTI_CRITICAL_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests",
                                   "golden", "multi_lattice_critical.json")


def multi_lattice_critical() -> list:
    """Critical masses of multi_lattice_configs() (tests/golden/multi_lattice_critical.json)."""
    with open(MULTI_CRITICAL_PATH) as f:
        return json.load(f)["m_c"]


SERVING_CRITICAL_PATH = os.path.join(os.path.dirname(MULTI_CRITICAL_PATH), "serving_critical.json")
SERVING_GAPS = (0.01, 0.1)      # per-request gap above m_c: log-uniform in this range


def serving_critical() -> list:
    """Critical masses of serving_configs() (tests/golden/serving_critical.json)."""
    with open(SERVING_CRITICAL_PATH) as f:
        data = json.load(f)
    assert data["configs"] == serving_configs(len(data["configs"])), "serving configurations changed"
    return data["m_c"]


def near_critical_stream(n: int, qps: float, m_c: list, seed: int = 6006, max_rhs: int = 8) -> list:
    """Open-loop arrivals at rate qps (exponential gaps); per request a uniform configuration,
    m0 = m_c + gap with the gap log-uniform in SERVING_GAPS, and 1..max_rhs right-hand sides."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.log(SERVING_GAPS[0]), np.log(SERVING_GAPS[1])
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / qps))
        c = int(rng.integers(len(m_c)))
        out.append({"t": t, "config": c, "m0": float(m_c[c] + np.exp(rng.uniform(lo, hi))),
                    "nrhs": int(rng.integers(1, max_rhs + 1)), "seed": int(rng.integers(1 << 30))})
    return out
