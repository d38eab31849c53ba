"""GPU tests of the continuous-batching server (amamg_server_*), through the C ABI.

Bars: every request's solution matches the CPU oracle (FP64: relative error <= 1e-9 and the
oracle's iteration count); a request's solution is bitwise the same alone and in a mix of
requests on other lattices and masses that arrive while it runs; per-request failures stay
with their request; hierarchies are evicted under a small memory budget and rebuilt on demand
with unchanged results.
"""
import time

import numpy as np
import pytest

import synth
from oracle import amg
from oracle.solve import solve as oracle_solve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


SETUP = dict(levels=2, agg_size=4, overlap=1, n_test_vectors=4)


def lattices():
    """Two gauge fields: the 16^2 beta = 3 workload and a 32^2 beta = 4 field."""
    return [synth.WORKLOADS["C1"].links(), synth.gen_links(32, 32, 4.0, 60, 321)]


def requests():
    """(gauge index, m0, right-hand sides [nrhs][nt][nx][2]) in submission order."""
    out = []
    for k, (gi, m0, nrhs) in enumerate([(0, 0.1, 2), (1, 0.15, 1), (0, 0.2, 3), (1, 0.15, 2),
                                         (0, 0.1, 1), (1, 0.3, 1), (0, 0.2, 1)]):
        L = 16 if gi == 0 else 32
        out.append((gi, m0, synth.gaussian_rhs(L, L, 500 + k, nrhs=nrhs)))
    return out


def make_server(lib, precision=None, **kw):
    prm = lib.default_server_params(slots=4, max_instances=2,
                                    precision=lib.FP64 if precision is None else precision)
    for k, v in kw.items():
        setattr(prm, k, v)
    return lib.Server(0, prm)


def run(lib, srv, gids, reqs, stagger=0.0):
    sp = lib.default_setup_params(**SETUP)
    ids = []
    for i, (gi, m0, psi) in enumerate(reqs):
        ids.append(srv.submit(gids[gi], m0, synth.field_to_abi(psi), sp))
        if stagger and i % 2 == 1:
            time.sleep(stagger)          # later requests arrive while earlier ones run
    assert srv.wait(300)
    done = {info.id: (info, synth.field_from_abi(x)) for info, x in srv.poll()}
    return [done[i] for i in ids]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_server_matches_oracle_and_is_the_same_alone_and_in_a_mix(lib, prec):
    """FP64: the oracle's iteration counts and <= 1e-9; mixed precision (the serving default:
    FP32 V-cycle inside FP64 FGMRES): <= 1e-9 of the oracle.  Both: bitwise the same alone, in
    the mix and with captured cycles."""
    precision = lib.FP64 if prec == "fp64" else lib.MIXED_FP32
    Us = lattices()
    reqs = requests()
    # the mix: every request, staggered so that later ones join running instances
    srv = make_server(lib, precision)
    gids = [srv.add_gauge(synth.links_to_abi(U)) for U in Us]
    say("server mix")
    mix = run(lib, srv, gids, reqs, stagger=0.02)
    st = srv.stats()
    assert st.outstanding == 0 and st.setups == 4          # (16, 0.1) (32, 0.15) (16, 0.2) (32, 0.3)
    srv.close()
    prm = amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=4)
    for (gi, m0, psi), (info, x) in zip(reqs, mix):
        assert info.status == lib.OK and info.converged and 1e-14 < info.true_rel_residual <= 1e-10
        assert info.t_submit <= info.t_admit <= info.t_done
        its = []
        levels = None
        for r in range(psi.shape[0]):
            xo, io, levels = oracle_solve(Us[gi], m0, psi[r], prm, levels=levels)
            assert rel(x[r], xo) <= 1e-9
            its.append(io.iterations)
        if precision == lib.FP64:
            assert info.iterations == max(its)
    # each request alone on a fresh server: bitwise the same
    for k in (0, 3, 6):
        srv = make_server(lib, precision)
        gids = [srv.add_gauge(synth.links_to_abi(U)) for U in Us]
        say("server alone", k)
        (info, x), = run(lib, srv, gids, [reqs[k]])
        srv.close()
        assert info.iterations == mix[k][0].iterations
        assert np.array_equal(x, mix[k][1])
    # the mix again with every instance replaying its captured restart cycle: bitwise the same
    srv = make_server(lib, precision, graphs=1)
    gids = [srv.add_gauge(synth.links_to_abi(U)) for U in Us]
    say("server mix, graphs")
    mixg = run(lib, srv, gids, reqs, stagger=0.02)
    srv.close()
    for (info, x), (info0, x0) in zip(mixg, mix):
        assert info.status == lib.OK and info.iterations == info0.iterations
        assert np.array_equal(x, x0)


def test_server_request_errors_stay_with_their_request(lib):
    Us = lattices()
    srv = make_server(lib)
    gids = [srv.add_gauge(synth.links_to_abi(U)) for U in Us]
    sp = lib.default_setup_params(**SETUP)
    bad = synth.field_to_abi(synth.gaussian_rhs(16, 16, 9, nrhs=2))
    bad[1, 3, 4, 0, 1] = np.nan
    good = synth.field_to_abi(synth.gaussian_rhs(16, 16, 10, nrhs=1))
    zero = np.zeros_like(good)
    with pytest.raises(lib.AmamgError):
        srv.submit(7, 0.1, good, sp)                         # unknown gauge
    with pytest.raises(lib.AmamgError):
        srv.submit(gids[0], 0.1, np.zeros((5, 16, 16, 2, 2)), sp)   # more rhs than slots
    with pytest.raises(lib.AmamgError):
        srv.submit(gids[0], 0.1, good, lib.default_setup_params(levels=2, agg_size=5))  # 5 does not divide 16
    r_bad = srv.submit(gids[0], 0.1, bad, sp)
    r_good = srv.submit(gids[0], 0.1, good, sp)
    r_zero = srv.submit(gids[0], 0.1, zero, sp)
    assert srv.wait(120)
    out = {info.id: (info, x) for info, x in srv.poll()}
    srv.close()
    assert out[r_bad][0].status == lib.STATUS_CODES["NONFINITE"]
    assert out[r_good][0].status == lib.OK and out[r_good][0].converged
    assert out[r_zero][0].status == lib.OK and np.all(out[r_zero][1] == 0)


def test_server_evicts_under_a_small_budget_and_rebuilds(lib):
    Us = lattices()
    sp = lib.default_setup_params(**SETUP)
    psi = synth.field_to_abi(synth.gaussian_rhs(32, 32, 33, nrhs=1))
    masses = (0.15, 0.3, 0.15)
    # reference: ample budget, one request at a time; one builder, so that the setup scratch
    # held by the server is the same in both runs
    srv = make_server(lib, builders=1)
    g = srv.add_gauge(synth.links_to_abi(Us[1]))
    ref = []
    for m0 in masses:
        srv.submit(g, m0, psi, sp)
        assert srv.wait(120)
        (info, x), = srv.poll()
        ref.append((info, x))
    st = srv.stats()
    assert st.setups == 2 and st.evictions == 0
    work = st.resident_bytes - st.hierarchy_bytes            # the instance's workspace
    one = st.hierarchy_bytes // 2                             # one cached hierarchy
    srv.close()
    # room for one hierarchy only: a build needs workspace + estimate, which fits only after
    # the other hierarchy is evicted
    budget = work + st.last_estimate_bytes + one // 2
    srv = make_server(lib, hbm_budget=budget, builders=1)
    g = srv.add_gauge(synth.links_to_abi(Us[1]))
    for k, m0 in enumerate(masses):
        srv.submit(g, m0, psi, sp)
        assert srv.wait(120)
        (info, x), = srv.poll()
        assert info.status == lib.OK and info.hierarchy_built == 1
        assert info.iterations == ref[k][0].iterations and np.array_equal(x, ref[k][1])
    st = srv.stats()
    assert st.setups == 3 and st.evictions == 2 and st.peak_resident_bytes <= budget
    srv.close()
    # too small for any hierarchy: the request fails, the server stays usable
    srv = make_server(lib, hbm_budget=1 << 20)
    g = srv.add_gauge(synth.links_to_abi(Us[1]))
    srv.submit(g, 0.15, psi, sp)
    assert srv.wait(60)
    (info, _), = srv.poll()
    assert info.status == lib.STATUS_CODES["OUT_OF_MEMORY"]
    srv.close()


@pytest.mark.parametrize("graphs", [0, 1])
def test_one_instance_rebound_across_lattice_sizes(lib, graphs):
    """A single solver instance serves requests on lattices of different sizes in turn (same
    and different level counts): its workspace is resized for every hierarchy it is bound to,
    and with graphs on, the restart cycle is captured again for every binding."""
    cases = [(synth.WORKLOADS["C1"].links(), 0.1, dict(levels=2, agg_size=4, overlap=1, n_test_vectors=4)),
             (synth.gen_links(32, 32, 4.0, 60, 321), 0.15, dict(levels=2, agg_size=4, overlap=1, n_test_vectors=4)),
             (synth.gen_links(64, 64, 6.0, 60, 654), 0.1, dict(levels=3, agg_size=4, overlap=1, n_test_vectors=8))]
    srv = make_server(lib, max_instances=1, graphs=graphs)
    gids = [srv.add_gauge(synth.links_to_abi(U)) for U, _, _ in cases]
    for k in (0, 1, 2, 1, 0):
        U, m0, sp = cases[k]
        L = U.shape[1]
        psi = synth.gaussian_rhs(L, L, 40 + k, nrhs=2)
        say("rebind", L, "graphs", graphs)
        srv.submit(gids[k], m0, synth.field_to_abi(psi), lib.default_setup_params(**sp))
        assert srv.wait(120)
        (info, x), = srv.poll()
        assert info.status == lib.OK and info.instance == 0
        x = synth.field_from_abi(x)
        prm = amg.SetupParams(levels=sp["levels"], agg=sp["agg_size"], overlap=sp["overlap"],
                              n_test_vectors=sp["n_test_vectors"])
        levels = None
        for r in range(2):
            xo, io, levels = oracle_solve(U, m0, psi[r], prm, levels=levels)
            assert rel(x[r], xo) <= 1e-9
    srv.close()


def test_server_coarsest_gmres_requests(lib):
    """Requests whose setup asks for the paper's coarsest-level GMRES (to 0.1) get their own
    cached hierarchy beside the exact-coarsest one on the same gauge field and mass, and match
    the oracle's variant."""
    U = synth.WORKLOADS["C1"].links()
    srv = make_server(lib)
    gid = srv.add_gauge(synth.links_to_abi(U))
    psi = synth.gaussian_rhs(16, 16, 808, nrhs=2)
    ids = []
    for tol in (0.1, 0.0, 0.1):
        sp = lib.default_setup_params(**SETUP, coarsest_tol=tol)
        ids.append(srv.submit(gid, 0.1, synth.field_to_abi(psi), sp))
    assert srv.wait(120)
    done = {info.id: (info, synth.field_from_abi(x)) for info, x in srv.poll()}
    assert srv.stats().setups == 2
    srv.close()
    for k, tol in enumerate((0.1, 0.0, 0.1)):
        info, x = done[ids[k]]
        assert info.status == lib.OK and info.converged
        prm = amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=4, coarsest_tol=tol)
        its, levels = [], None
        for r in range(2):
            xo, io, levels = oracle_solve(U, 0.1, psi[r], prm, levels=levels)
            assert rel(x[r], xo) <= 1e-9
            its.append(io.iterations)
        assert info.iterations == max(its)
    assert np.array_equal(done[ids[0]][1], done[ids[2]][1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_reference_mass_requests_use_derived_hierarchies(lib, prec):
    """A gauge with a reference mass: one setup at that mass, and each other mass gets a
    hierarchy derived from it (interpolation from the reference mass, operators at the
    request's).  Every request matches the oracle's shift of the reference setup (FP64: its
    iteration counts); alone on a fresh server it is bitwise its result in the staggered mix."""
    precision = lib.FP64 if prec == "fp64" else lib.MIXED_FP32
    U = synth.gen_links(32, 32, 4.0, 60, 321)
    m_ref = 0.12
    masses = (0.05, 0.12, 0.3, 0.05, 0.08)
    reqs = [(0, m, synth.gaussian_rhs(32, 32, 700 + k, nrhs=1 + k % 2)) for k, m in enumerate(masses)]

    def serve(rs, stagger):
        srv = make_server(lib, precision)
        gid = srv.add_gauge(synth.links_to_abi(U))
        srv.set_reference_mass(gid, m_ref)
        out = run(lib, srv, [gid], rs, stagger=stagger)
        st = srv.stats()
        srv.close()
        return out, st

    mix, st = serve(reqs, 0.02)
    assert st.setups == 1 and st.derivations == 3             # 0.05, 0.3, 0.08 from 0.12
    prm = amg.SetupParams(levels=2, agg=4, overlap=1, n_test_vectors=4)
    base = amg.setup(U, m_ref, prm)
    for (gi, m0, psi), (info, x) in zip(reqs, mix):
        assert info.status == lib.OK and info.converged and 1e-14 < info.true_rel_residual <= 1e-10
        olev = amg.shift_mass(base, U, m0)
        its = []
        for r in range(psi.shape[0]):
            xo, io, _ = oracle_solve(U, m0, psi[r], prm, levels=olev)
            assert rel(x[r], xo) <= 1e-9
            its.append(io.iterations)
        if precision == lib.FP64:
            assert info.iterations == max(its)
    for k in (0, 2):
        (info, x), = serve([reqs[k]], 0.0)[0]
        assert info.iterations == mix[k][0].iterations and np.array_equal(x, mix[k][1])


def test_budget_holds_when_instances_are_rebound_across_lattice_sizes(lib):
    """Requests on a 16^2 and a 64^2 lattice, submitted together to a server with two instances
    whose budget is the peak of serving them one at a time with one instance: the server binds,
    creates and rebinds instances only when their workspace growth fits (releasing idle
    instances' memory and evicting when needed), so the peak stays within the budget and the
    results are bitwise those of the one-at-a-time run."""
    cases = [(synth.WORKLOADS["C1"].links(), 0.1, dict(levels=2, agg_size=4, overlap=1, n_test_vectors=4)),
             (synth.gen_links(64, 64, 6.0, 60, 654), 0.1, dict(levels=3, agg_size=4, overlap=1, n_test_vectors=8))]
    order = (0, 1, 0, 1)
    psis = [synth.field_to_abi(synth.gaussian_rhs(cases[k][0].shape[1], cases[k][0].shape[1], 60 + i, nrhs=2))
            for i, k in enumerate(order)]
    srv = make_server(lib, max_instances=1, builders=1)
    gids = [srv.add_gauge(synth.links_to_abi(U)) for U, _, _ in cases]
    ref = []
    for i, k in enumerate(order):
        srv.submit(gids[k], cases[k][1], psis[i], lib.default_setup_params(**cases[k][2]))
        assert srv.wait(120)
        (info, x), = srv.poll()
        assert info.status == lib.OK
        ref.append((info, x))
    budget = srv.stats().peak_resident_bytes
    srv.close()
    srv = make_server(lib, max_instances=2, builders=1, hbm_budget=budget)
    gids = [srv.add_gauge(synth.links_to_abi(U)) for U, _, _ in cases]
    ids = [srv.submit(gids[k], cases[k][1], psis[i], lib.default_setup_params(**cases[k][2]))
           for i, k in enumerate(order)]
    assert srv.wait(300)
    done = {info.id: (info, x) for info, x in srv.poll()}
    st = srv.stats()
    srv.close()
    assert st.peak_resident_bytes <= budget
    for i, rid in enumerate(ids):
        info, x = done[rid]
        assert info.status == lib.OK
        assert info.iterations == ref[i][0].iterations and np.array_equal(x, ref[i][1])
