"""Operation count of an AM-AMG setup and of an AM-AMG-preconditioned FGMRES solve.

The paper compares methods by their floating-point operation count, setup included
(Numerical Results: the GFLOP tables, and the statement that every right-hand side repeats
the setup there).  This module counts the operations of this library's algorithm from the
hierarchy's geometry alone. Counts are real operations. A complex multiply-add is 8, a complex
addition 2 and a complex times real 2. An LU factorisation of a complex n x n matrix is 8n^3/3,
and a pair of triangular solves with r right-hand sides is 8n^2 r. The counts are algorithmic:
redundant halo work, padding and repeated loads of the GPU kernels are not counted.

Per level k (grid Lt x Lx nodes, b unknowns per node, wirebasket spacing a, overlap o):

* a wirebasket's footprint has (a + o)^2 nodes, 4 o^2 of them vertices, so its local system
  A_FF has nF = ((a + o)^2 - 4 o^2) b rows and A_FV has 4 bc columns (bc = o^2 b);
* every non-vertex unknown of the level is an interpolation row over the 4 bc vertex unknowns
  of its wirebasket; a vertex couples to the wirebasket's other points only if it has a
  nearest neighbour there, which holds for 2o - 1 of the o^2 vertices of each corner (the
  others' columns of A_FV, hence of P, are zero), so a row has 4 (2o - 1) b nonzeros:
  nnz_F = (Lt Lx - nW o^2) b * 4 (2o - 1) b with nW = (Lt / a)(Lx / a).  (The GPU stores and
  multiplies the full 4 bc columns, 4/3 of this for o = 2.);
* the next level's operator has 21 nonzero b' x b' blocks per node (b' = bc), or is dense on
  the coarsest level.
"""
from __future__ import annotations

from dataclasses import dataclass

CMAC, CADD, CSCALE = 8, 2, 2
FINE_MATVEC_PER_SITE = 60      # spin-projected hops: 4 x (add 2 + multiply 6 + two adds 4) + mass 12
FINE_GS_PER_SITE = 72          # residual (matvec + subtract 4) + scale by 1/(m0 + 2) 4 + add 4
COARSE_BLOCKS = 21             # nonzero offsets of the coarse stencil


@dataclass
class LevelGeom:
    Lt: int
    Lx: int
    b: int

    @property
    def nodes(self) -> int:
        return self.Lt * self.Lx

    @property
    def ndof(self) -> int:
        return self.nodes * self.b


def levels_of(nt: int, nx: int, levels: int, a: int, o: int) -> list:
    out, Lt, Lx, b = [], nt, nx, 2
    for k in range(levels):
        out.append(LevelGeom(Lt, Lx, b))
        Lt, Lx, b = Lt // a, Lx // a, o * o * b
    return out


def wirebasket_counts(g: LevelGeom, a: int, o: int) -> dict:
    nW = (g.Lt // a) * (g.Lx // a)
    bc = o * o * g.b
    nF = ((a + o) ** 2 - 4 * o * o) * g.b
    nnzF = (g.nodes - nW * o * o) * g.b * 4 * (2 * o - 1) * g.b
    return {"nW": nW, "bc": bc, "nF": nF, "nnzF": nnzF}


def _period(L: int) -> int:
    for d in range(5, L + 1):
        if L % d == 0:
            return d
    return L


def smoother_sweep(g: LevelGeom, k: int) -> int:
    if k == 0:
        return FINE_GS_PER_SITE * g.nodes
    b = g.b
    return g.nodes * ((COARSE_BLOCKS + 1) * CMAC * b * b + 2 * CADD * b)


def operator_apply(g: LevelGeom, k: int, coarsest: bool) -> int:
    if coarsest:
        return CMAC * g.ndof * g.ndof
    if k == 0:
        return FINE_MATVEC_PER_SITE * g.nodes
    return g.nodes * COARSE_BLOCKS * CMAC * g.b * g.b


def vcycle(geo: list, a: int, o: int, pre: int = 0, post: int = 2) -> int:
    """One V-cycle for one right-hand side (coarsest level: the dense inverse applied)."""
    total = 0
    for k, g in enumerate(geo):
        if k == len(geo) - 1:
            total += CMAC * g.ndof * g.ndof
            break
        w = wirebasket_counts(g, a, o)
        transfers = 2 * CMAC * w["nnzF"]                     # restriction and interpolation
        total += transfers + (pre + post) * smoother_sweep(g, k)
        if pre > 0:                                          # residual after pre-smoothing
            total += operator_apply(g, k, False) + CADD * g.ndof
    return total


def gram_schmidt_step(n: int, j: int) -> int:
    """Step j (0-based) of the delayed CGS2 (DCGS2) Arnoldi process on vectors of n unknowns:
    pass A forms 2(j + 1) inner products, pass B applies j + (j + 1) projections and two
    scalings."""
    return CMAC * n * (2 * (j + 1) + j + (j + 1)) + 2 * CSCALE * n


def solve(geo: list, a: int, o: int, iterations: int, restart: int = 20, pre: int = 0, post: int = 2) -> dict:
    """Operations of one right-hand side's solve that took `iterations` Arnoldi steps."""
    n = geo[0].ndof
    per_vcycle = vcycle(geo, a, o, pre, post)
    matvec = operator_apply(geo[0], 0, False)
    steps, gs, ends = iterations, 0, 0
    while steps > 0:
        k = min(restart, steps)
        gs += sum(gram_schmidt_step(n, j) for j in range(k))
        gs += CMAC * n * (k + 1)                             # the cycle's last inner products
        # x += Z y, the true residual b - D x and its norm
        ends += CMAC * n * k + matvec + CADD * n + CMAC * n
        steps -= k
    start = matvec + CADD * n + CMAC * n + CSCALE * n        # r = b - D x0, ||r||, v_0 = r / ||r||
    total = iterations * (per_vcycle + matvec) + gs + ends + start
    return {"vcycle": per_vcycle, "matvec": matvec, "gram_schmidt": gs, "total": total,
            "per_iteration_per_site": (total / max(iterations, 1)) / geo[0].nodes}


def setup(geo: list, a: int, o: int, n_test_vectors: int, test_vector_sweeps: int = 4) -> dict:
    """Operations of one setup: test-vector relaxation, local solves, normalisation, Galerkin
    operator by probing, smoother block inverses and the coarsest inverse."""
    parts = {"test_vectors": 0, "local_solves": 0, "normalisation": 0, "galerkin": 0,
             "block_inverses": 0, "coarsest_inverse": 0}
    K = len(geo)
    for k in range(K - 1):
        g, gc = geo[k], geo[k + 1]
        w = wirebasket_counts(g, a, o)
        parts["test_vectors"] += n_test_vectors * test_vector_sweeps * smoother_sweep(g, k)
        nF, bc = w["nF"], w["bc"]
        nvc = 4 * (2 * o - 1) * g.b                            # nonzero columns of A_FV
        parts["local_solves"] += w["nW"] * (8 * nF ** 3 // 3 + CMAC * nF * nF * nvc)
        parts["normalisation"] += n_test_vectors * CMAC * w["nnzF"]
        probes = _period(gc.Lt) * _period(gc.Lx) * bc        # coloured unit vectors, bc per class
        parts["galerkin"] += probes * (2 * CMAC * w["nnzF"] + operator_apply(g, k, False))
        if k + 1 < K - 1:
            parts["block_inverses"] += gc.nodes * (8 * gc.b ** 3 // 3 + CMAC * gc.b ** 3)
    nc = geo[-1].ndof
    parts["coarsest_inverse"] = 8 * nc ** 3 // 3 + CMAC * nc ** 3
    parts["total"] = sum(v for v in parts.values())
    return parts
