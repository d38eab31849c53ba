"""Pins of the oracle's FGMRES and V-cycle against brute-force dense solves, and of the
critical-mass estimate against the free-field closed form."""
import numpy as np
import pytest

import synth
from oracle import amg
from oracle.dirac import dirac_matrix
from oracle.fgmres import fgmres, givens, gmres
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


def _krylov_min_residual(A, b, k):
    """argmin over x in span{b, A b, ..., A^{k-1} b} of ||b - A x||, by least squares on an
    orthonormal basis of the explicit Krylov matrix (brute force, small k only)."""
    K = np.empty((b.shape[0], k), dtype=complex)
    K[:, 0] = b
    for i in range(1, k):
        K[:, i] = A @ K[:, i - 1]
    Q, _ = np.linalg.qr(K)
    y = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
    return Q @ y


def _coarsest_test_matrix(n=24, seed=5):
    rng = np.random.default_rng(seed)
    A = 2.5 * np.eye(n) + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_coarsest_gmres_is_the_krylov_minimum_residual_solution():
    """k steps of GMRES from x0 = 0 give the minimum-residual vector of the k-th Krylov space
    (the definition of GMRES), for every k, on a non-normal complex matrix."""
    A, b = _coarsest_test_matrix()
    for k in range(1, 9):
        x, steps = gmres(lambda v: A @ v, b, 0.0, k)
        xr = _krylov_min_residual(A, b, k)
        assert steps == k
        assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)


def test_coarsest_gmres_stops_at_the_first_step_below_the_tolerance():
    A, b = _coarsest_test_matrix(seed=9)
    nb = np.linalg.norm(b)
    for tol in (0.5, 0.1, 0.01):
        x, k = gmres(lambda v: A @ v, b, tol, 24)
        assert np.linalg.norm(b - A @ x) <= tol * nb * (1 + 1e-10)
        if k > 1:
            xp = _krylov_min_residual(A, b, k - 1)
            assert np.linalg.norm(b - A @ xp) > tol * nb
    # tolerance far below rounding: n steps reach the direct solution (or break down before)
    x, k = gmres(lambda v: A @ v, b, 1e-300, 24)
    xd = np.linalg.solve(A, b)
    assert k <= 24 and np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    x0, k0 = gmres(lambda v: A @ v, np.zeros_like(b), 0.1, 24)
    assert k0 == 0 and not np.any(x0)


def test_amg_with_coarsest_gmres_converges_to_the_dense_solution():
    """The paper's coarsest-level GMRES to 0.1 inside the V-cycle: FGMRES still reaches the
    direct solution; with a vanishing tolerance the V-cycle equals the exact-coarsest one."""
    w = synth.WORKLOADS["C1"]
    U = w.links()
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed)[0]
    D = dirac_matrix(U, w.m0).toarray()
    xd = np.linalg.solve(D, psi.reshape(-1))
    kappa = np.linalg.cond(D)
    prm = amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=4, coarsest_tol=0.1)
    x, info, levels = solve(U, w.m0, psi, prm, tol=1e-12)
    assert info.converged
    assert np.linalg.norm(x.reshape(-1) - xd) <= 2 * kappa * 1e-12 * np.linalg.norm(xd)
    f = synth.gaussian_rhs(w.L, w.L, 3)[0].reshape(-1)
    exact = amg.vcycle(levels, 0, f, amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=4))
    tight = amg.vcycle(levels, 0, f, amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=4,
                                                     coarsest_tol=1e-300, coarsest_max_iters=32))
    loose = amg.vcycle(levels, 0, f, prm)
    assert np.linalg.norm(tight - exact) <= 1e-9 * np.linalg.norm(exact)
    assert np.linalg.norm(loose - exact) > 1e-4 * np.linalg.norm(exact)

