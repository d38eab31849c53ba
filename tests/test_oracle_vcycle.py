"""Exact pin of the oracle's V-cycle (two-level scheme algorithm of the Multilevel approach
section, applied recursively; Numerical Results: V-cycle, 0 pre- and 2 post-smoothing steps of
a block smoother).

The V-cycle is rebuilt here from dense matrices only, without ``amg.gs_sweep`` or
``amg.vcycle``:

* P_k is the oracle's interpolation (pinned by the wirebasket and interpolation tests);
  A_{k+1} = P_k^H A_k P_k is formed as a dense product here;
* one multicolour point-block Gauss-Seidel sweep is the textbook splitting iteration
  x <- x + M^{-1} (f - A x) with M = D + L: D holds the couplings inside each node's block,
  L the couplings of a node to the nodes of colours visited earlier in the sweep (their new
  values are already in use when the node is updated); couplings to later colours and to
  other nodes of the same colour use the old values;
* the colour order is written out from its reading: (t + x) mod 2 ascending on the fine
  lattice; on coarse grids the colours (I mod 4) * 4 + (J mod 4) of each 2 x 2 block of the
  4 x 4 pattern in a row, blocks in row-major order;
* the coarsest level is solved with ``numpy.linalg.solve`` on the dense Galerkin matrix.

A plausible slip in the oracle -- post-sweeps run as pre-sweeps, one sweep instead of two, a
different colour order, a missing coarse correction, R = P^T instead of P^H -- changes the
result by far more than the 1e-12 bound; the last test checks that the comparison is sensitive
to exactly these changes.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import amg


def random_links(nt, nx, seed):
    return np.exp(1j * np.random.default_rng(seed).uniform(-np.pi, np.pi, (2, nt, nx)))


def sweep_rank(Lt, Lx, fine, order=None):
    """Rank of each node's colour in the sweep."""
    T, X = np.meshgrid(np.arange(Lt), np.arange(Lx), indexing="ij")
    if fine:
        return ((T + X) % 2).ravel()
    colour = ((T % 4) * 4 + (X % 4)).ravel()
    if order is None:
        order = [(2 * bi + di) * 4 + (2 * bj + dj)
                 for bi in range(2) for bj in range(2) for di in range(2) for dj in range(2)]
    rank = np.empty(16, dtype=int)
    rank[np.asarray(order)] = np.arange(16)
    return rank[colour]


def gs_splitting(A, Lt, Lx, b, fine, order=None):
    """M = D + L of the colour-ordered point-block Gauss-Seidel iteration (dense)."""
    node = np.arange(A.shape[0]) // b
    r = sweep_rank(Lt, Lx, fine, order)[node]
    same_node = node[:, None] == node[None, :]
    earlier = r[None, :] < r[:, None]
    return np.where(same_node | earlier, A, 0.0)


def dense_hierarchy(levels, order=None, restriction="PH"):
    """Per level: (A, P, LU of M) dense; A of level k+1 formed here as P^H A P (or P^T A P)."""
    out = []
    A = levels[0].A.toarray()
    for k, lev in enumerate(levels):
        if lev.coarsest:
            out.append((A, None, None))
            break
        P = lev.P.toarray()
        M = sla.lu_factor(gs_splitting(A, lev.Lt, lev.Lx, lev.b, fine=(k == 0), order=order))
        out.append((A, P, M))
        R = P.conj().T if restriction == "PH" else P.T
        A = R @ A @ P
    return out


def dense_vcycle(dense, k, f, pre, post, restriction="PH"):
    A, P, M = dense[k]
    if P is None:
        return np.linalg.solve(A, f)
    x = np.zeros_like(f)
    for _ in range(pre):
        x = x + sla.lu_solve(M, f - A @ x)
    R = P.conj().T if restriction == "PH" else P.T
    x = x + P @ dense_vcycle(dense, k + 1, R @ (f - A @ x), pre, post, restriction)
    for _ in range(post):
        x = x + sla.lu_solve(M, f - A @ x)
    return x


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    # (L, a, o, levels, m0)
    (8, 2, 1, 2, 0.1),
    (8, 2, 1, 3, 0.05),
    (16, 4, 1, 2, 0.1),     # the two-level 16^2 workload's hierarchy shape
    (16, 2, 1, 3, 0.1),
    (16, 4, 2, 2, 0.2),
    (32, 4, 2, 3, 0.1),     # coarse smoother on 8 x 8 nodes with 8 x 8 blocks
]


@pytest.mark.parametrize("L,a,o,levels,m0", CASES)
@pytest.mark.parametrize("norm", [amg.NORM_TESTVEC, amg.NORM_NONE])
def test_vcycle_equals_dense_two_level_recursion(L, a, o, levels, m0, norm):
    U = random_links(L, L, 100 + L + levels)
    prm = amg.SetupParams(levels=levels, agg=a, overlap=o, n_test_vectors=3, norm=norm)
    hier = amg.setup(U, m0, prm)
    dense = dense_hierarchy(hier)
    rng = np.random.default_rng(7 + L)
    for _ in range(2):
        f = rng.standard_normal(L * L * 2) + 1j * rng.standard_normal(L * L * 2)
        ref = dense_vcycle(dense, 0, f, pre=0, post=2)
        got = amg.vcycle(hier, 0, f, prm)
        assert _rel(got, ref) <= 1e-12, _rel(got, ref)


@pytest.mark.parametrize("L,a,o,levels", [(8, 2, 1, 2), (16, 4, 1, 2), (16, 4, 2, 2)])
def test_vcycle_without_smoothing_is_the_exact_coarse_correction(L, a, o, levels):
    """post_sweeps = 0 (and no pre-sweeps) gives x = P A_c^{-1} P^H f exactly."""
    U = random_links(L, L, 300 + L)
    prm = amg.SetupParams(levels=levels, agg=a, overlap=o, post_sweeps=0, n_test_vectors=2)
    hier = amg.setup(U, 0.1, prm)
    A = hier[0].A.toarray()
    P = hier[0].P.toarray()
    Ac = P.conj().T @ A @ P
    f = np.random.default_rng(11).standard_normal(L * L * 2) + 0j
    ref = P @ np.linalg.solve(Ac, P.conj().T @ f)
    got = amg.vcycle(hier, 0, f, prm)
    assert _rel(got, ref) <= 1e-12


@pytest.mark.parametrize("pre,post", [(1, 2), (1, 0), (2, 1)])
def test_vcycle_with_pre_sweeps_follows_the_two_level_scheme(pre, post):
    """Pre-smoothing from x = 0, residual, restricted correction, post-smoothing."""
    U = random_links(16, 16, 17)
    prm = amg.SetupParams(levels=3, agg=2, overlap=1, pre_sweeps=pre, post_sweeps=post,
                          n_test_vectors=3)
    hier = amg.setup(U, 0.1, prm)
    dense = dense_hierarchy(hier)
    f = np.random.default_rng(5).standard_normal(16 * 16 * 2) * (1 + 1j)
    ref = dense_vcycle(dense, 0, f, pre=pre, post=post)
    got = amg.vcycle(hier, 0, f, prm)
    assert _rel(got, ref) <= 1e-12


def test_vcycle_on_the_two_level_workload():
    """The 16^2, beta = 3 workload's own links, mass and hierarchy."""
    w = synth.WORKLOADS["C1"]
    U = w.links()
    prm = amg.SetupParams(levels=w.levels, agg=w.agg, overlap=w.overlap,
                          n_test_vectors=w.n_test_vectors)
    hier = amg.setup(U, w.m0, prm)
    dense = dense_hierarchy(hier)
    f = synth.gaussian_rhs(w.L, w.L, w.rhs_seed)[0].reshape(-1)
    assert _rel(amg.vcycle(hier, 0, f, prm), dense_vcycle(dense, 0, f, 0, 2)) <= 1e-12


def test_the_dense_pin_detects_plausible_slips():
    """Each variant below differs from the two-level scheme the oracle claims by far more than
    the comparison bound, so none of these mistakes could pass the tests above."""
    U = random_links(32, 32, 23)
    prm = amg.SetupParams(levels=3, agg=4, overlap=2, n_test_vectors=3)
    hier = amg.setup(U, 0.1, prm)
    f = np.random.default_rng(3).standard_normal(32 * 32 * 2) + 0j
    got = amg.vcycle(hier, 0, f, prm)
    dense = dense_hierarchy(hier)
    assert _rel(got, dense_vcycle(dense, 0, f, 0, 2)) <= 1e-12
    slips = {
        "pre instead of post": dense_vcycle(dense, 0, f, 2, 0),
        "one post-sweep": dense_vcycle(dense, 0, f, 0, 1),
        "three post-sweeps": dense_vcycle(dense, 0, f, 0, 3),
        "no coarse correction": (lambda A, M: sla.lu_solve(M, f) + sla.lu_solve(
            M, f - A @ sla.lu_solve(M, f)))(dense[0][0], dense[0][2]),
        "restriction P^T": dense_vcycle(dense_hierarchy(hier, restriction="PT"), 0, f, 0, 2,
                                        restriction="PT"),
        "ascending coarse colours": dense_vcycle(dense_hierarchy(hier, order=list(range(16))),
                                                 0, f, 0, 2),
    }
    for name, x in slips.items():
        assert _rel(x, got) > 1e-6, name
