"""Pins of the oracle's FGMRES and V-cycle against brute-force dense solves, and of the
critical-mass estimate against the free-field closed form."""
import numpy as np
import pytest

import synth
from oracle import amg
from oracle.dirac import dirac_matrix
from oracle.fgmres import fgmres, givens
from oracle.solve import solve
from oracle.spectrum import critical_mass


def test_givens_rotation_annihilates():
    for a, b in ((1 + 2j, 0.5), (-0.3j, 2.0), (0.0, 1.5), (2.0, 1e-20)):
        c, s = givens(a, b)
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-15
        assert abs(-np.conj(s) * a + c * b) < 1e-15


@pytest.mark.parametrize("L,a,levels", [(4, 2, 2), (8, 2, 2), (8, 4, 2), (16, 2, 3)])
def test_amg_fgmres_matches_dense_solve(L, a, levels):
    U = synth.gen_links(L, L, 2.0, 30, 100 + L)
    psi = synth.gaussian_rhs(L, L, 7)[0]
    m0 = 0.05
    D = dirac_matrix(U, m0).toarray()
    x_dense = np.linalg.solve(D, psi.reshape(-1))
    kappa = np.linalg.cond(D)
    prm = amg.SetupParams(levels=levels, agg=a, overlap=1, n_test_vectors=2)
    x, info, _ = solve(U, m0, psi, prm, tol=1e-13)
    assert info.converged
    err = np.linalg.norm(x.reshape(-1) - x_dense) / np.linalg.norm(x_dense)
    assert err <= 2 * kappa * 1e-13
    xp, infop, _ = solve(U, m0, psi, preconditioned=False, tol=1e-13)
    errp = np.linalg.norm(xp.reshape(-1) - x_dense) / np.linalg.norm(x_dense)
    assert errp <= 2 * kappa * 1e-13
    # the preconditioner pays off
    assert info.iterations < infop.iterations


def test_unpreconditioned_and_amg_solutions_agree():
    w = synth.WORKLOADS["C1"]
    U = w.links()
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed)[0]
    prm = amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=4)
    x1, i1, _ = solve(U, w.m0, psi, prm, tol=1e-12)
    x2, i2, _ = solve(U, w.m0, psi, preconditioned=False, tol=1e-12)
    assert i1.converged and i2.converged
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) < 1e-9
    assert i1.iterations < i2.iterations / 3


def test_exact_coarsest_is_direct_solve_when_fine_is_coarsest():
    """A one-level 'hierarchy' whose coarsest level is the fine lattice converges in one step."""
    L = 4
    U = synth.gen_links(L, L, 2.0, 10, 3)
    psi = synth.gaussian_rhs(L, L, 1)[0]
    prm = amg.SetupParams(levels=1)
    x, info, _ = solve(U, 0.1, psi, prm, tol=1e-12)
    assert info.iterations == 1 and info.converged


def test_residual_history_is_monotone_within_a_cycle():
    w = synth.WORKLOADS["C1"]
    U = w.links()
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed)[0]
    prm = amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=4)
    _, info, _ = solve(U, w.m0, psi, prm)
    est = []
    for v, is_true in info.history:
        if is_true:
            assert all(est[i + 1] <= est[i] * (1 + 1e-12) for i in range(len(est) - 1))
            est = []
        else:
            est.append(v)
    assert info.history[-1][1] and info.history[-1][0] <= 1e-10


@pytest.mark.parametrize("L", [16, 64])
def test_free_field_critical_mass(L):
    U = np.ones((2, L, L), dtype=complex)
    assert abs(critical_mass(U) - (-(1 - np.cos(np.pi / L)))) < 1e-10


def test_critical_mass_arnoldi_matches_dense():
    U = synth.gen_links(16, 16, 3.0, 100, 9)
    assert abs(critical_mass(U) - critical_mass(U, dense=True)) < 1e-9


def test_fgmres_iteration_cap_reports_not_converged():
    w = synth.WORKLOADS["C1"]
    U = w.links()
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed)[0]
    D = dirac_matrix(U, w.m0)
    x, info = fgmres(lambda v: D @ v, psi.reshape(-1), lambda v: v, m=10, max_iters=15)
    assert not info.converged and info.iterations == 15 and info.restarts == 1
