"""Pins of the oracle's mass shift (a hierarchy built at one bare mass reused at another).

D depends on m0 only through its diagonal, D(m0') = D(m0) + (m0' - m0) I (Schwinger Model
subsection), so with the interpolation kept the Galerkin products of the Multilevel approach
section change by a closed form: A_{k+1}(m0') - A_{k+1}(m0) = (m0' - m0) G_{k+1} with
G_1 = P_0^H P_0 and G_{k+1} = P_k^H G_k P_k.  The tests compare the oracle's shifted operators
with that formula, check that a shift there and back returns the original hierarchy, and solve
with a shifted hierarchy against a dense solve at the new mass.
"""
import numpy as np
import pytest

import synth
from oracle import amg
from oracle.dirac import dirac_matrix
from oracle.solve import solve


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


@pytest.fixture(scope="module")
def c2_like():
    U = synth.gen_links(32, 32, 6.0, 40, 777)
    prm = amg.SetupParams(levels=3, agg=4, overlap=1, n_test_vectors=4, seed=5)
    return U, prm, amg.setup(U, 0.05, prm)


def test_shift_to_the_same_mass_reproduces_the_setup(c2_like):
    U, prm, levs = c2_like
    same = amg.shift_mass(levs, U, 0.05)
    for a, b in zip(levs, same):
        assert (a.A != b.A).nnz == 0
        if a.coarsest:
            assert np.array_equal(a.lu[0], b.lu[0])
        else:
            assert np.array_equal(a.Dinv, b.Dinv)
            assert a.P is b.P


@pytest.mark.parametrize("dm", [0.03, -0.02])
def test_shifted_operators_follow_the_mass_term_closed_form(c2_like, dm):
    U, prm, levs = c2_like
    new = amg.shift_mass(levs, U, 0.05 + dm)
    # fine level: only the diagonal moves
    d0 = (new[0].A - levs[0].A).toarray()
    assert np.abs(d0 - dm * np.eye(d0.shape[0])).max() < 1e-15
    G = None
    for k in range(1, len(levs)):
        P = levs[k - 1].P.toarray()
        G = P.conj().T @ P if G is None else P.conj().T @ G @ P
        diff = (new[k].A - levs[k].A).toarray()
        assert rel(diff, dm * G) < 1e-12, k
    # the interpolation is kept, the smoother blocks are those of the new operator
    assert new[1].P is levs[1].P
    ref = amg.diagonal_block_inverses(new[1].A, new[1].nnode, new[1].b)
    assert np.array_equal(new[1].Dinv, ref)


def test_shift_there_and_back_returns_the_operators(c2_like):
    U, prm, levs = c2_like
    back = amg.shift_mass(amg.shift_mass(levs, U, 0.11), U, 0.05)
    for a, b in zip(levs, back):
        assert rel(a.A.toarray(), b.A.toarray()) < 1e-14


def test_solve_with_a_shifted_hierarchy_matches_the_dense_solve():
    """An 8 x 8 hierarchy built at m0 = 0.2 and shifted to 0.05 preconditions FGMRES on
    D(0.05) to the dense solution (the preconditioner only changes the iteration count)."""
    L = 8
    U = synth.gen_links(L, L, 2.0, 30, 808)
    psi = synth.gaussian_rhs(L, L, 9)[0]
    prm = amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=2)
    levs = amg.shift_mass(amg.setup(U, 0.2, prm), U, 0.05)
    D = dirac_matrix(U, 0.05).toarray()
    x_dense = np.linalg.solve(D, psi.reshape(-1))
    x, info, _ = solve(U, 0.05, psi, prm, tol=1e-13, levels=levs)
    assert info.converged
    assert rel(x.reshape(-1), x_dense) <= 2 * np.linalg.cond(D) * 1e-13
    # the hierarchy really is the shifted one: its fine operator is D(0.05)
    assert np.abs((levs[0].A - dirac_matrix(U, 0.05)).toarray()).max() == 0
