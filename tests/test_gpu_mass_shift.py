"""GPU parity of amamg_hierarchy_set_mass against the oracle's mass shift.

A hierarchy built at one bare mass is moved to another without a new setup: its wirebaskets,
test vectors and interpolation stay, its operators become those of the new mass (Schwinger
Model subsection: m0 enters D on the diagonal only; Multilevel approach: Galerkin operators
with the kept interpolation).  Bars as in the other parity tests: coarse operators within
1e-10 relative of the oracle's (its Galerkin products are recomputed at the new mass, the
library adds the mass term's Galerkin image), FP64 solves with the oracle's iteration and
restart counts and a relative solution error <= 1e-9, mixed precision within 1e-9.
"""
import numpy as np
import pytest

import synth
from oracle import amg
from oracle.solve import solve as oracle_solve
from test_gpu_parity import oracle_stencil

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def check_operators(h, olev):
    for k in range(1, len(olev)):
        lev = olev[k]
        if lev.coarsest:
            assert rel(h.coarse_operator(k, coarsest=True), lev.A.toarray()) < 1e-10, k
        else:
            assert rel(h.coarse_operator(k, coarsest=False), oracle_stencil(lev.A, lev.Lt, lev.Lx, lev.b)) < 1e-10, k


CASES = [
    # L, beta, levels, a, o, nv, built at, moved to, coarsest_tol
    (32, 6.0, 3, 4, 1, 4, 0.05, 0.11, 0.0),
    (32, 6.0, 2, 8, 2, 4, 0.2, 0.03, 0.1),
]


@pytest.mark.parametrize("case", CASES)
def test_set_mass_matches_the_oracle_shift(lib, ctx, case):
    L, beta, levels, a, o, nv, m_built, m_new, ctol = case
    say("set_mass", case)
    U = synth.gen_links(L, L, beta, 40, 900 + L + levels)
    prm = amg.SetupParams(levels=levels, agg=a, overlap=o, n_test_vectors=nv, seed=3, coarsest_tol=ctol)
    olev = amg.shift_mass(amg.setup(U, m_built, prm), U, m_new)
    g = lib.Gauge(ctx, synth.links_to_abi(U), m_built)
    h = lib.Hierarchy(g, lib.default_setup_params(levels=levels, agg_size=a, overlap=o, n_test_vectors=nv,
                                                   seed=3, coarsest_tol=ctol))
    h.set_mass(m_new)
    check_operators(h, olev)
    psi = synth.gaussian_rhs(L, L, 31, nrhs=2)
    x64, i64, st = h.solve(synth.field_to_abi(psi), lib.default_solve_params(precision=lib.FP64))
    assert st == lib.OK
    x32, i32, st32 = h.solve(synth.field_to_abi(psi), lib.default_solve_params(precision=lib.MIXED_FP32))
    assert st32 == lib.OK
    xg64, xg32 = synth.field_from_abi(x64), synth.field_from_abi(x32)
    for r in range(2):
        xo, io, _ = oracle_solve(U, m_new, psi[r], prm, levels=olev)
        assert i64[r].iterations == io.iterations and i64[r].restarts == io.restarts
        assert rel(xg64[r], xo) <= 1e-9
        assert i32[r].converged and rel(xg32[r], xo) <= 1e-9
    h.close()
    g.close()


def test_set_mass_on_the_128_workload_and_twice(lib, ctx):
    """128^2, a = 8, o = 2, 3 levels (8 x 8 blocks on level 1, 128 coarsest unknowns): built at
    m_c + 0.05, moved to m_c + 0.01 and on to m_c + 0.02; operators after each move and an FP64
    solve after the second against the oracle's shift of the same hierarchy."""
    w = synth.WORKLOADS["C4"]
    mc = synth.critical_masses()["C4"]
    U = w.links()
    prm = amg.SetupParams(levels=3, agg=8, overlap=2, n_test_vectors=8)
    base = amg.setup(U, mc + 0.05, prm)
    g = lib.Gauge(ctx, synth.links_to_abi(U), mc + 0.05)
    h = lib.Hierarchy(g, lib.default_setup_params(levels=3, agg_size=8, overlap=2, n_test_vectors=8))
    h.set_mass(mc + 0.01)
    check_operators(h, amg.shift_mass(base, U, mc + 0.01))
    h.set_mass(mc + 0.02)
    olev = amg.shift_mass(base, U, mc + 0.02)
    check_operators(h, olev)
    psi = synth.gaussian_rhs(w.L, w.L, 77, nrhs=1)
    x, infos, st = h.solve(synth.field_to_abi(psi), lib.default_solve_params(precision=lib.FP64))
    assert st == lib.OK
    xo, io, _ = oracle_solve(U, mc + 0.02, psi[0], prm, levels=olev)
    assert infos[0].iterations == io.iterations
    assert rel(synth.field_from_abi(x)[0], xo) <= 1e-9
    h.close()
    g.close()


def test_set_mass_refuses_a_non_finite_mass(lib, ctx):
    U = synth.gen_links(16, 16, 3.0, 10, 5)
    g = lib.Gauge(ctx, synth.links_to_abi(U), 0.1)
    h = lib.Hierarchy(g, lib.default_setup_params())
    with pytest.raises(lib.AmamgError) as e:
        h.set_mass(float("nan"))
    assert e.value.status == lib.STATUS_CODES["INVALID_ARG"]
    # the hierarchy is unchanged and still solves at its mass
    psi = synth.gaussian_rhs(16, 16, 2, nrhs=1)
    x, infos, st = h.solve(synth.field_to_abi(psi))
    xo, io, _ = oracle_solve(U, 0.1, psi[0], amg.SetupParams())
    assert st == lib.OK and infos[0].iterations == io.iterations
    h.close()
    g.close()


def test_derived_hierarchies_share_the_base_and_equal_a_moved_copy(lib, ctx):
    """Two hierarchies derived from one base at other masses: each matches the oracle's shift
    and is bitwise equal to a second setup of the base moved with set_mass; the base still solves
    bitwise as before; the base cannot be destroyed, updated or moved while they exist."""
    L, m_b = 32, 0.12
    U = synth.gen_links(L, L, 4.0, 40, 4242)
    prm = amg.SetupParams(levels=3, agg=4, overlap=1, n_test_vectors=4)
    sp = lib.default_setup_params(levels=3, agg_size=4, overlap=1, n_test_vectors=4)
    obase = amg.setup(U, m_b, prm)
    g = lib.Gauge(ctx, synth.links_to_abi(U), m_b)
    base = lib.Hierarchy(g, sp)
    psi = synth.field_to_abi(synth.gaussian_rhs(L, L, 5, nrhs=2))
    xb0, ib0, _ = base.solve(psi)
    derived = {m: base.derive_mass(m) for m in (0.04, 0.2)}
    for call in (base.update, lambda: base.set_mass(0.3), base.close):
        with pytest.raises(lib.AmamgError) as e:
            call()
        assert e.value.status == lib.STATUS_CODES["INVALID_ARG"]
    for m, h in derived.items():
        say("derived", m)
        olev = amg.shift_mass(obase, U, m)
        check_operators(h, olev)
        x, infos, st = h.solve(psi)
        assert st == lib.OK
        for r in range(2):
            xo, io, _ = oracle_solve(U, m, synth.field_from_abi(psi)[r], prm, levels=olev)
            assert infos[r].iterations == io.iterations
            assert rel(synth.field_from_abi(x)[r], xo) <= 1e-9
        moved = lib.Hierarchy(g, sp)
        moved.set_mass(m)
        xm, im, _ = moved.solve(psi)
        assert np.array_equal(xm, x) and [i.iterations for i in im] == [i.iterations for i in infos]
        moved.close()
    xb1, ib1, _ = base.solve(psi)
    assert np.array_equal(xb0, xb1)
    for h in derived.values():
        with pytest.raises(lib.AmamgError):
            h.update()
        h.close()
    base.close()
    g.close()
