"""GPU parity of the test-vector-augmented coarse space (setup parameter aug_vectors) against the
oracle's (paper, Conclusion: test vectors brought into the SM-AMG method).

Bars as in the other parity tests: the augmented interpolation rows, the coarse operators and
the coarse levels' test vectors within 1e-10 relative of the oracle's (both orthonormalise per
wirebasket by Gram-Schmidt; the sums over a wirebasket's rows run in another order), FP64 solves
with the oracle's iteration and restart counts and a relative solution error <= 1e-9, mixed
precision within 1e-9.  Parameter errors are refused before any device work.
"""
import numpy as np
import pytest

import synth
from oracle import amg
from oracle.solve import solve as oracle_solve
from oracle.wirebasket import KIND_V
from test_gpu_parity import oracle_stencil

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def oracle_rows_aug(lev, a, o, k):
    """Oracle interpolation rows [p][i][4 bc] in the library's corner order, bc = o^2 b + k."""
    P = lev.P.tocsr()
    b, Lt, Lx = lev.b, lev.Lt, lev.Lx
    bc = o * o * b + k
    nI, nJ = Lt // a, Lx // a
    out = np.zeros((Lt * Lx, b, 4 * bc), dtype=complex)
    for p in range(Lt * Lx):
        if lev.cls["kind"][p] == KIND_V:
            continue
        I, J = divmod(int(lev.cls["owner"][p]), nJ)
        for c in range(4):
            node = ((I + (c >> 1)) % nI) * nJ + (J + (c & 1)) % nJ
            cols = node * bc + np.arange(bc)
            for i in range(b):
                out[p, i, c * bc:(c + 1) * bc] = P[p * b + i, cols].toarray().ravel()
    return out


CASES = [
    # L, beta, levels, a, o, nv, k, m0
    (32, 4.0, 3, 4, 1, 6, 2, 0.05),      # level 1: 8 x 8 nodes of 4 dofs, coarsest 2 x 2 x 4
    (32, 6.0, 2, 4, 1, 4, 3, 0.08),      # level 1 is the dense coarsest level (8 x 8 x 5)
    (128, 6.0, 3, 8, 2, 8, 8, 0.05),     # a = 8, o = 2: level 1 has 16 dofs per node
]


@pytest.mark.parametrize("case", CASES)
def test_augmented_setup_and_solves_match_the_oracle(lib, ctx, case):
    L, beta, levels, a, o, nv, k, m0 = case
    say("augmented", case)
    U = synth.gen_links(L, L, beta, 40, 1300 + L + k)
    prm = amg.SetupParams(levels=levels, agg=a, overlap=o, n_test_vectors=nv, test_vector_sweeps=16,
                          seed=9, aug_vectors=k)
    olev = amg.setup(U, m0, prm)
    g = lib.Gauge(ctx, synth.links_to_abi(U), m0)
    h = lib.Hierarchy(g, lib.default_setup_params(levels=levels, agg_size=a, overlap=o, n_test_vectors=nv,
                                                   test_vector_sweeps=16, seed=9, aug_vectors=k))
    assert h.level_info(1) == (olev[1].Lt, olev[1].Lx, olev[1].b) and olev[1].b == o * o * 2 + k
    assert rel(h.prolongator_rows(0, o, aug=k), oracle_rows_aug(olev[0], a, o, k)) < 1e-10
    for lvl in range(1, levels):
        lev = olev[lvl]
        if lev.coarsest:
            assert rel(h.coarse_operator(lvl, coarsest=True), lev.A.toarray()) < 1e-10
        else:
            assert rel(h.coarse_operator(lvl, coarsest=False), oracle_stencil(lev.A, lev.Lt, lev.Lx, lev.b)) < 1e-10
            assert rel(h.test_vectors(lvl, nv), lev.test_vectors) < 1e-10
    psi = synth.gaussian_rhs(L, L, 77, nrhs=2)
    x64, i64, st = h.solve(synth.field_to_abi(psi), lib.default_solve_params(precision=lib.FP64))
    x32, i32, st32 = h.solve(synth.field_to_abi(psi), lib.default_solve_params(precision=lib.MIXED_FP32))
    assert st == lib.OK and st32 == lib.OK
    plain = None
    for r in range(2):
        xo, io, _ = oracle_solve(U, m0, psi[r], prm, levels=olev)
        assert i64[r].iterations == io.iterations and i64[r].restarts == io.restarts
        assert rel(synth.field_from_abi(x64)[r], xo) <= 1e-9
        assert i32[r].converged and rel(synth.field_from_abi(x32)[r], xo) <= 1e-9
        if r == 0:
            _, plain, _ = oracle_solve(U, m0, psi[r], amg.SetupParams(
                levels=levels, agg=a, overlap=o, n_test_vectors=nv, test_vector_sweeps=16, seed=9))
    say("iterations augmented", i64[0].iterations, "plain", plain.iterations)
    h.close()
    g.close()


def test_augmented_parameters_are_checked(lib, ctx):
    U = synth.gen_links(32, 32, 4.0, 10, 5)
    g = lib.Gauge(ctx, synth.links_to_abi(U), 0.1)
    bad = [dict(levels=2, n_test_vectors=2, aug_vectors=3),                          # more than N_v
           dict(levels=2, norm=lib.NORM_NONE, aug_vectors=1),                        # no test vectors
           dict(levels=3, agg_size=4, overlap=1, n_test_vectors=4, aug_vectors=1)]   # level 1: 3 dofs
    codes = [lib.STATUS_CODES["INVALID_ARG"], lib.STATUS_CODES["INVALID_ARG"],
             lib.STATUS_CODES["UNSUPPORTED_SHAPE"]]
    for kw, code in zip(bad, codes):
        with pytest.raises(lib.AmamgError) as e:
            lib.Hierarchy(g, lib.default_setup_params(**kw))
        assert e.value.status == code, kw
    g.close()


def test_augmented_256_setup_sampled_parity(lib, ctx):
    """The 256^2 workload's field and mass (a = 8, o = 2, 3 levels, 64 test-vector sweeps) with
    k = 8: sampled augmented interpolation rows, sampled level-1 blocks (16 dofs per node) and
    the dense 1024-unknown coarsest operator against the oracle's setup."""
    w = synth.WORKLOADS["C3"]
    m0 = synth.critical_masses()["C3"] + w.gaps[0]
    U = w.links()
    say("C3 augmented setup parity")
    olev = amg.setup(U, m0, amg.SetupParams(**w.oracle_kw(aug_vectors=8)))
    g = lib.Gauge(ctx, synth.links_to_abi(U), m0)
    h = lib.Hierarchy(g, lib.default_setup_params(**w.setup_kw(aug_vectors=8)))
    bc = 16
    rows = h.prolongator_rows(0, 2, aug=8)
    P = olev[0].P.tocsr()
    rng = np.random.default_rng(1)
    for p in rng.choice(256 * 256, 200, replace=False):
        if olev[0].cls["kind"][p] == KIND_V:
            continue
        I, J = divmod(int(olev[0].cls["owner"][p]), 32)
        for c in range(4):
            nd = ((I + (c >> 1)) % 32) * 32 + (J + (c & 1)) % 32
            ref = P[2 * p:2 * p + 2, nd * bc:(nd + 1) * bc].toarray()
            assert np.abs(rows[p, :, c * bc:(c + 1) * bc] - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
    A1 = h.coarse_operator(1, coarsest=False)
    ref1 = olev[1].A.tocsr()
    for n in rng.choice(1024, 40, replace=False):
        t, x = divmod(int(n), 32)
        scale = max(1.0, np.abs(ref1[n * bc:(n + 1) * bc].toarray()).max())
        for off in (0, 1, 7, 12, 13, 17, 24):
            dt, dx = off // 5 - 2, off % 5 - 2
            m = ((t + dt) % 32) * 32 + (x + dx) % 32
            blk = ref1[n * bc:(n + 1) * bc, m * bc:(m + 1) * bc].toarray()
            assert np.abs(A1[n, off] - blk).max() <= 1e-10 * scale
    assert rel(h.test_vectors(1, 8), olev[1].test_vectors) < 1e-10
    assert rel(h.coarse_operator(2, coarsest=True), olev[2].A.toarray()) < 1e-10
    h.close()
    g.close()
