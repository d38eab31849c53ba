"""Pins of the oracle's test-vector-augmented coarse space (the paper's outlook, Conclusion: test
vectors brought into the SM-AMG method to capture the near-kernel better).

The finest level's interpolation gets k extra columns per wirebasket: an orthonormal basis of the
part of the first k test vectors that the wirebasket interpolation does not reproduce, restricted
to the wirebasket's own non-vertex rows.  Consequences checked here, none of which the
construction states directly: the augmented interpolation reproduces those k test vectors
exactly (and no others); its vertex-row and wirebasket columns are the plain interpolation's;
each extra column lives on one wirebasket's own rows and the columns of a wirebasket are
orthonormal; k = 0 is the plain hierarchy; and the augmented preconditioner solves to the
dense solution.
"""
import numpy as np
import pytest

import synth
from oracle import amg
from oracle.dirac import dirac_matrix
from oracle.solve import solve
from oracle.wirebasket import KIND_V


@pytest.fixture(scope="module")
def setups():
    U = synth.gen_links(32, 32, 4.0, 40, 2024)
    base = dict(levels=3, agg=4, overlap=1, n_test_vectors=6, test_vector_sweeps=8, seed=4)
    plain = amg.setup(U, 0.05, amg.SetupParams(**base))
    aug = amg.setup(U, 0.05, amg.SetupParams(**base, aug_vectors=2))
    return U, plain, aug


def test_augmented_interpolation_reproduces_its_test_vectors(setups):
    U, plain, aug = setups
    lev = aug[0]
    k, b, bc = 2, lev.b, 2          # o = 1: o^2 b = 2 vertex dofs per node, then 2 extra
    tv = lev.test_vectors
    tvc = amg.inject(tv, lev.Lt, lev.Lx, b, 4, 1, lev.cls)
    # the coarse representation: vertex values, then each wirebasket's coefficients
    P = lev.P.toarray()
    nW = lev.cls["nI"] * lev.cls["nJ"]
    bca = bc + k
    assert P.shape[1] == nW * bca
    coarse = np.zeros((tv.shape[0], nW * bca), dtype=complex)
    for w in range(nW):
        coarse[:, w * bca:w * bca + bc] = tvc[:, w * bc:(w + 1) * bc]
        cols = P[:, w * bca + bc:(w + 1) * bca]
        coarse[:, w * bca + bc:(w + 1) * bca] = (tv - (plain[0].P @ tvc.T).T) @ cols.conj()
    for j in range(tv.shape[0]):
        err = np.linalg.norm(P @ coarse[j] - tv[j]) / np.linalg.norm(tv[j])
        if j < k:
            assert err < 1e-12, j
        else:
            assert err > 1e-3, j         # vectors beyond the first k are not in the space


def test_augmented_columns_are_local_orthonormal_and_keep_the_plain_interpolation(setups):
    U, plain, aug = setups
    lev, ref = aug[0], plain[0]
    k, b, bc = 2, lev.b, 2
    bca = bc + k
    P, P0 = lev.P.toarray(), ref.P.toarray()
    nW = lev.cls["nI"] * lev.cls["nJ"]
    owner = np.repeat(lev.cls["owner"], b)
    frow = np.repeat(lev.cls["kind"] != KIND_V, b)
    for w in range(nW):
        np.testing.assert_array_equal(P[:, w * bca:w * bca + bc], P0[:, w * bc:(w + 1) * bc])
        X = P[:, w * bca + bc:(w + 1) * bca]
        own = (owner == w) & frow
        assert np.all(X[~own] == 0)
        assert np.abs(X.conj().T @ X - np.eye(k)).max() < 1e-13
    # the coarse levels have the extra dofs per node
    assert aug[1].b == bc + k and aug[2].b == (bc + k)


def test_no_augmentation_is_the_plain_hierarchy(setups):
    U, plain, aug = setups
    again = amg.setup(U, 0.05, amg.SetupParams(levels=3, agg=4, overlap=1, n_test_vectors=6,
                                                test_vector_sweeps=8, seed=4, aug_vectors=0))
    for a, b in zip(plain, again):
        assert (a.A != b.A).nnz == 0


@pytest.mark.parametrize("L,a,levels", [(8, 4, 2), (16, 4, 2), (16, 2, 3)])
def test_augmented_fgmres_matches_the_dense_solve(L, a, levels):
    U = synth.gen_links(L, L, 2.0, 30, 300 + L)
    psi = synth.gaussian_rhs(L, L, 17)[0]
    m0 = 0.05
    D = dirac_matrix(U, m0).toarray()
    x_dense = np.linalg.solve(D, psi.reshape(-1))
    prm = amg.SetupParams(levels=levels, agg=a, overlap=1, n_test_vectors=4, aug_vectors=2)
    x, info, levs = solve(U, m0, psi, prm, tol=1e-13)
    assert info.converged and levs[1].b == 4
    err = np.linalg.norm(x.reshape(-1) - x_dense) / np.linalg.norm(x_dense)
    assert err <= 2 * np.linalg.cond(D) * 1e-13


def test_augmentation_needs_test_vectors():
    U = synth.gen_links(16, 16, 2.0, 10, 3)
    with pytest.raises(ValueError):
        amg.setup(U, 0.1, amg.SetupParams(levels=2, n_test_vectors=2, aug_vectors=3))
    with pytest.raises(ValueError):
        amg.setup(U, 0.1, amg.SetupParams(levels=2, norm=amg.NORM_NONE, aug_vectors=1))
