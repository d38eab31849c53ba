"""Oracle: AM-AMG setup and V-cycle (test infrastructure).

Follows the paper's Multilevel approach section (setup = coarsening, interpolation,
Galerkin coarse operator; solution phase = two-level scheme algorithm) and the
SM-AMG for LQCD subsection (per-wirebasket block system, ideal presmoothing,
Schur-complement interpolation, normalisation, primary-wirebasket rule).

Readings where the paper is silent (all also used by the GPU library):
* interpolation: for each wirebasket W, A restricted to the points of W is split into
  F = E u I and V blocks; P_F^W = -A_FF^{-1} A_FV, which equals the paper's two Schur-
  complement formulas (pinned in the tests); a row of P comes from the row's primary
  wirebasket, vertex rows are the identity onto their coarse node;
* restriction is P^H (the complex form of the transpose used by the real K-formulation);
* normalisation N (the paper scales the interpolation rows so that constants are reproduced)
  has three modes: CONST (row sums of P equal 1, the literal rule), TESTVEC (the least-squares row
  scale that best reproduces smoothed random test vectors; equal to CONST for one test
  vector that is constant) and NONE;
* smoother (the paper smooths with its block solver, 0 pre and 2 post sweeps): multicolour point-block
  Gauss-Seidel; colours (t + x) mod 2 on the fine lattice, visited in increasing order, and
  (I mod 4) * 4 + (J mod 4) on coarse grids, visited in the order COARSE_ORDER, which takes the
  colours of each 2 x 2 block of the 4 x 4 colour pattern in a row (0, 1, 4, 5, then 2, 3, 6, 7,
  ...; any order is a valid multicolour sweep, the paper fixes none); a colour sets
  x_n <- x_n + A_nn^{-1} (f - A x)_n for all nodes n of the colour at once;
* test vectors: level 0 starts from the splitmix64 vectors of ``oracle.rng``; level k+1 starts
  from level k's smoothed vectors injected at the vertices; each level relaxes them with nu
  smoother sweeps on A w = 0;
* the coarsest level is solved exactly by LU with partial pivoting (coarsest_tol = 0), or, as
  in the paper's experiments, by unpreconditioned GMRES from x = 0 to the relative tolerance
  coarsest_tol (0.1 there) with at most coarsest_max_iters steps (``fgmres.gmres``);
* every level uses the same aggregate size a and overlap o.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import rng
from .dirac import dirac_matrix
from .fgmres import gmres
from .wirebasket import KIND_V, classify, coarse_dof_of_vertex, footprint

NORM_TESTVEC, NORM_CONST, NORM_NONE = 0, 1, 2


@dataclass
class SetupParams:
    levels: int = 2
    agg: int = 4
    overlap: int = 1
    n_test_vectors: int = 4
    test_vector_sweeps: int = 4
    pre_sweeps: int = 0
    post_sweeps: int = 2
    norm: int = NORM_TESTVEC
    seed: int = 0
    coarsest_tol: float = 0.0          # 0: exact solve; > 0: GMRES to this relative tolerance
    coarsest_max_iters: int = 32
    aug_vectors: int = 0               # test vectors augmenting the finest level's coarse space


@dataclass
class Level:
    A: sp.csr_matrix
    Lt: int
    Lx: int
    b: int
    index: int
    coarsest: bool = False
    colour_nodes: list = field(default_factory=list)
    Dinv: np.ndarray | None = None
    cls: dict | None = None
    P_tilde: sp.csr_matrix | None = None
    P: sp.csr_matrix | None = None
    test_vectors: np.ndarray | None = None
    lu: tuple | None = None

    @property
    def nnode(self) -> int:
        return self.Lt * self.Lx

    @property
    def ndof(self) -> int:
        return self.nnode * self.b


# ----------------------------------------------------------------------------- smoother

COARSE_ORDER = (0, 1, 4, 5, 2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15)


def colouring(Lt: int, Lx: int, fine: bool) -> list:
    """Node index arrays per colour in sweep order: colours 0, 1 on the fine lattice, the coarse
    colours in COARSE_ORDER."""
    T, X = np.meshgrid(np.arange(Lt), np.arange(Lx), indexing="ij")
    if fine:
        col = ((T + X) % 2).ravel()
    else:
        if Lt % 4 or Lx % 4:
            raise ValueError("coarse-level colouring needs grid sizes divisible by 4")
        col = ((T % 4) * 4 + (X % 4)).ravel()
    order = range(2) if fine else COARSE_ORDER
    return [np.nonzero(col == c)[0] for c in order]


def diagonal_block_inverses(A: sp.csr_matrix, nnode: int, b: int) -> np.ndarray:
    """A_nn^{-1} for every node n (b x b blocks on the diagonal)."""
    C = A.tocoo()
    blocks = np.zeros((nnode, b, b), dtype=complex)
    same = (C.row // b) == (C.col // b)
    np.add.at(blocks, (C.row[same] // b, C.row[same] % b, C.col[same] % b), C.data[same])
    return np.linalg.inv(blocks)


def gs_sweep(lev: Level, x: np.ndarray, f: np.ndarray) -> None:
    """One multicolour point-block Gauss-Seidel sweep on A x = f, in place."""
    xb = x.reshape(lev.nnode, lev.b)
    for nodes in lev.colour_nodes:
        r = (f - lev.A @ x).reshape(lev.nnode, lev.b)
        xb[nodes] += np.einsum("nij,nj->ni", lev.Dinv[nodes], r[nodes])


# ------------------------------------------------------------------------ interpolation

def local_interpolation(A: sp.csr_matrix, Lt: int, Lx: int, b: int, a: int, o: int,
                        cls: dict) -> sp.csr_matrix:
    """Unnormalised interpolation P~ (ndof x ndof_c): per-wirebasket block solves.

    For wirebasket W with F = E u I points and V points (paper's block system with
    rows in I, E, V order; the V rows are replaced by the identity under ideal
    presmoothing), the F rows of the local interpolator are -A_FF^{-1} A_FV.  Only the
    rows whose primary wirebasket is W are kept.  Vertex rows are the identity.
    """
    A = A.tocsr()
    nI, nJ = cls["nI"], cls["nJ"]
    kind, owner, node = cls["kind"], cls["owner"], cls["node"]
    bc = o * o * b
    ndof = Lt * Lx * b
    rows, cols, vals = [], [], []
    for I in range(nI):
        for J in range(nJ):
            w = I * nJ + J
            pts = [t * Lx + x for t, x, _, _ in footprint(I, J, Lt, Lx, a, o)]
            f_pts = [p for p in pts if kind[p] != KIND_V]
            v_pts = [p for p in pts if kind[p] == KIND_V]
            f_dofs = [p * b + q for p in f_pts for q in range(b)]
            v_dofs = [p * b + q for p in v_pts for q in range(b)]
            v_coarse = [coarse_dof_of_vertex(p, q, Lx, a, o, b, int(node[p]))
                        for p in v_pts for q in range(b)]
            A_ff = A[f_dofs][:, f_dofs].toarray()
            A_fv = A[f_dofs][:, v_dofs].toarray()
            Pw = -np.linalg.solve(A_ff, A_fv)
            for i, d in enumerate(f_dofs):
                if owner[d // b] == w:
                    rows.extend([d] * len(v_coarse))
                    cols.extend(v_coarse)
                    vals.extend(Pw[i])
    for p in np.nonzero(kind == KIND_V)[0]:
        for q in range(b):
            rows.append(int(p) * b + q)
            cols.append(coarse_dof_of_vertex(int(p), q, Lx, a, o, b, int(node[p])))
            vals.append(1.0)
    ncoarse = (Lt // a) * (Lx // a) * bc
    return sp.csr_matrix((np.asarray(vals, dtype=complex), (rows, cols)), shape=(ndof, ncoarse))


def inject(v: np.ndarray, Lt: int, Lx: int, b: int, a: int, o: int, cls: dict) -> np.ndarray:
    """Values of v at the vertices, as a coarse vector (rows of P~ that are the identity)."""
    nc = (Lt // a) * (Lx // a) * o * o * b
    out = np.zeros(v.shape[:-1] + (nc,), dtype=complex)
    for p in np.nonzero(cls["kind"] == KIND_V)[0]:
        for q in range(b):
            c = coarse_dof_of_vertex(int(p), q, Lx, a, o, b, int(cls["node"][p]))
            out[..., c] = v[..., int(p) * b + q]
    return out


def normalise(P_tilde: sp.csr_matrix, mode: int, b: int, cls: dict,
              tv: np.ndarray | None, tv_coarse: np.ndarray | None) -> sp.csr_matrix:
    """P = N P~ with N diagonal; vertex rows keep scale 1."""
    ndof = P_tilde.shape[0]
    f_row = np.repeat(cls["kind"] != KIND_V, b)
    c = np.ones(ndof, dtype=complex)
    if mode == NORM_CONST:
        rs = np.asarray(P_tilde.sum(axis=1)).ravel()
        c[f_row] = 1.0 / rs[f_row]
    elif mode == NORM_TESTVEC:
        q = np.stack([P_tilde @ tv_coarse[k] for k in range(tv.shape[0])])   # [Nv][ndof]
        num = np.sum(np.conj(q) * tv, axis=0)
        den = np.sum(np.abs(q) ** 2, axis=0)
        c[f_row] = num[f_row] / den[f_row]
    elif mode != NORM_NONE:
        raise ValueError("unknown normalisation")
    return (sp.diags(c) @ P_tilde).tocsr()


# ----------------------------------------------------------- augmented coarse space

def widen_columns(M: sp.csr_matrix, bc: int, bc_aug: int) -> sp.csr_matrix:
    """Renumber coarse columns node * bc + i as node * bc_aug + i (room for extra dofs per node)."""
    C = M.tocoo()
    cols = (C.col // bc) * bc_aug + C.col % bc
    nnode = M.shape[1] // bc
    return sp.csr_matrix((C.data, (C.row, cols)), shape=(M.shape[0], nnode * bc_aug))


def augment(P: sp.csr_matrix, tv: np.ndarray, tv_coarse: np.ndarray, b: int, bc: int, cls: dict,
            k: int):
    """Coarse space augmented with k test vectors (the paper's outlook: test vectors in the
    SM-AMG method to capture the near-kernel better).  For test vector w_j the wirebasket
    interpolation leaves the residual e_j = w_j - P (w_j at the vertices), which vanishes on
    vertex rows.  Each wirebasket W = (I, J) gets k coarse degrees of freedom on its node
    (I, J), numbered after the node's o^2 b vertex dofs: an orthonormal basis, by Gram-Schmidt
    in the order j = 0 .. k-1, of e_0 .. e_{k-1} restricted to the non-vertex rows W owns.

    Returns (P_aug, coarse test vectors): the coarse representation of w_j is its vertex values
    and its coefficients in W's basis, so that P_aug reproduces w_0 .. w_{k-1} exactly."""
    ndof = P.shape[0]
    bca = bc + k
    nW = cls["nI"] * cls["nJ"]
    owner = np.repeat(cls["owner"], b)
    frow = np.repeat(cls["kind"] != KIND_V, b)
    E = tv - (P @ tv_coarse.T).T                         # [Nv][ndof]: residuals of every test vector
    Pw = widen_columns(P, bc, bca)
    rows, cols, vals = [], [], []
    tvc = np.zeros((tv_coarse.shape[0], nW * bca), dtype=complex)
    for n in range(nW):
        idx = np.arange(bc)
        tvc[:, n * bca + idx] = tv_coarse[:, n * bc + idx]
    for w in range(nW):
        r = np.nonzero((owner == w) & frow)[0]
        Q = np.zeros((r.size, k), dtype=complex)
        for j in range(k):
            v = E[j, r].copy()
            for i in range(j):
                v -= Q[:, i] * np.vdot(Q[:, i], v)
            nrm = np.linalg.norm(v)
            if not nrm > 0:
                raise ValueError("test-vector residual has no component on a wirebasket")
            Q[:, j] = v / nrm
        for j in range(k):
            rows.extend(r.tolist())
            cols.extend([w * bca + bc + j] * r.size)
            vals.extend(Q[:, j].tolist())
        # coefficients of every test vector in W's basis (the next level's test vectors)
        tvc[:, w * bca + bc:(w + 1) * bca] = E[:, r] @ Q.conj()
    B = sp.csr_matrix((np.asarray(vals, dtype=complex), (rows, cols)), shape=(ndof, nW * bca))
    return (Pw + B).tocsr(), tvc


# ------------------------------------------------------------------------------- setup

def setup(U: np.ndarray, m0: float, prm: SetupParams) -> list:
    """Build the hierarchy; returns the list of Level objects (last one coarsest)."""
    nt, nx = U.shape[1], U.shape[2]
    A = dirac_matrix(U, m0)
    Lt, Lx, b = nt, nx, 2
    a, o = prm.agg, prm.overlap
    levels = []
    tv_in = None
    for k in range(prm.levels):
        lev = Level(A=A.tocsr(), Lt=Lt, Lx=Lx, b=b, index=k)
        levels.append(lev)
        if k == prm.levels - 1:
            lev.coarsest = True
            lev.lu = sla.lu_factor(lev.A.toarray())
            break
        lev.colour_nodes = colouring(Lt, Lx, fine=(k == 0))
        lev.Dinv = diagonal_block_inverses(lev.A, lev.nnode, b)
        cls = classify(Lt, Lx, a, o)
        lev.cls = cls
        tv = tv_coarse = None
        if prm.norm == NORM_TESTVEC:
            if k == 0:
                tv = rng.test_vectors(prm.seed, 0, prm.n_test_vectors, lev.ndof)
            else:
                tv = tv_in
            zero = np.zeros(lev.ndof, dtype=complex)
            for i in range(tv.shape[0]):
                for _ in range(prm.test_vector_sweeps):
                    gs_sweep(lev, tv[i], zero)
            lev.test_vectors = tv
            tv_coarse = inject(tv, Lt, Lx, b, a, o, cls)
            tv_in = tv_coarse.copy()
        lev.P_tilde = local_interpolation(lev.A, Lt, Lx, b, a, o, cls)
        lev.P = normalise(lev.P_tilde, prm.norm, b, cls, tv, tv_coarse)
        bc = o * o * b
        if k == 0 and prm.aug_vectors > 0:
            if tv is None or prm.aug_vectors > tv.shape[0]:
                raise ValueError("augmentation needs that many test vectors (TESTVEC normalisation)")
            lev.P, tv_in = augment(lev.P, tv, tv_coarse, b, bc, cls, prm.aug_vectors)
            bc += prm.aug_vectors
        A = (lev.P.conj().T @ lev.A @ lev.P).tocsr()
        Lt, Lx, b = Lt // a, Lx // a, bc
    return levels


def shift_mass(levels: list, U: np.ndarray, m0: float) -> list:
    """The hierarchy `levels` (built at another bare mass) with its operators at bare mass m0.

    Everything the setup derived from the old operator stays: the wirebaskets, the test vectors
    and the interpolation P of every level.  The operators follow their definitions at the new
    mass (Schwinger Model subsection for D; Multilevel approach section for the Galerkin
    products): A_0 = D(m0), A_{k+1} = P_k^H A_k P_k with the kept P_k; the smoother blocks and
    the coarsest factorisation are recomputed from them.
    """
    A = dirac_matrix(U, m0).tocsr()
    out = []
    for lev in levels:
        new = replace(lev, A=A)
        if lev.coarsest:
            new.lu = sla.lu_factor(A.toarray())
        else:
            new.Dinv = diagonal_block_inverses(A, lev.nnode, lev.b)
            A = (lev.P.conj().T @ A @ lev.P).tocsr()
        out.append(new)
    return out


def vcycle(levels: list, k: int, f: np.ndarray, prm: SetupParams) -> np.ndarray:
    """M_k f: the two-level scheme of the paper applied recursively, started at x = 0."""
    lev = levels[k]
    if lev.coarsest:
        if prm.coarsest_tol > 0:
            return gmres(lambda v: lev.A @ v, f, prm.coarsest_tol, prm.coarsest_max_iters)[0]
        return sla.lu_solve(lev.lu, f)
    x = np.zeros_like(f)
    for _ in range(prm.pre_sweeps):
        gs_sweep(lev, x, f)
    d = f - lev.A @ x
    e = vcycle(levels, k + 1, lev.P.conj().T @ d, prm)
    x = x + lev.P @ e
    for _ in range(prm.post_sweeps):
        gs_sweep(lev, x, f)
    return x
