"""GPU parity of the solver paths beyond the benchmark workloads, against the CPU oracle.

* pre-smoothing (the two-level scheme algorithm's optional pre-smoothing step; the paper runs 0),
  on the fine level alone and with a smoothed coarse level;
* a 2048-unknown coarsest level (128^2, a = 8, o = 2, two levels), solved exactly and by the
  paper's coarsest GMRES to 0.1 (Numerical Results), where the GMRES kernel splits the rows
  of the level over two halves of its workgroup;
* rectangular lattices (N_t != N_x), two and three levels, o = 1 and 2;
* the (3 levels, a = 8, o = 1) hierarchy of the aggregate-size sweep;
* the local-solve error path (a zero operator has only zero pivots).

Bars as in the other parity tests: classification bit-exact, setup products within 1e-10,
FP64 solves with the oracle's iteration and restart counts and a relative solution error
<= 1e-9, FP32 within 1e-9 with counts reported.
"""
import numpy as np
import pytest

import synth
from oracle import amg
from oracle.dirac import dirac_matrix
from oracle.solve import solve as oracle_solve
from test_gpu_parity import oracle_rows, oracle_stencil

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


GPU_NAMES = {"agg": "agg_size"}


def gpu_setup(lib, **kw):
    return lib.default_setup_params(**{GPU_NAMES.get(k, k): v for k, v in kw.items()})


def solve_both(lib, ctx, U, m0, psi, precision=0, olevels=None, **kw):
    """Oracle and GPU solves of the right-hand sides psi [nrhs][nt][nx][2] with the setup
    parameters kw (oracle names).  Returns (oracle results, GPU x, GPU infos, status, histories)."""
    prm = amg.SetupParams(**kw)
    outs = []
    for r in range(psi.shape[0]):
        xo, io, olevels = oracle_solve(U, m0, psi[r], prm, levels=olevels)
        outs.append((xo, io))
    g = lib.Gauge(ctx, synth.links_to_abi(U), m0)
    h = lib.Hierarchy(g, gpu_setup(lib, **kw))
    x, infos, st = h.solve(synth.field_to_abi(psi), lib.default_solve_params(precision=precision))
    hists = [h.residual_history(r) for r in range(psi.shape[0])]
    h.close()
    g.close()
    return outs, synth.field_from_abi(x), infos, st, hists, olevels


def check_fp64(outs, x, infos, st, hists):
    assert st == 0
    for r, (xo, io) in enumerate(outs):
        assert infos[r].converged and io.converged
        assert infos[r].iterations == io.iterations, (r, infos[r].iterations, io.iterations)
        assert infos[r].restarts == io.restarts
        assert rel(x[r], xo) <= 1e-9
        hist, flags = hists[r]
        assert np.array_equal(flags, np.array([f for _, f in io.history]))
        assert np.allclose(hist, np.array([v for v, _ in io.history]), rtol=1e-6, atol=1e-14)


# --------------------------------------------------------------------------- pre-smoothing

@pytest.mark.parametrize("wl,precision", [("C1", 0), ("C2", 0), ("C2", 1)])
def test_pre_sweeps_match_oracle(lib, ctx, wl, precision):
    """One pre-sweep and two post-sweeps: the V-cycle starts from x = 0, smooths, restricts the
    residual f - A x, adds the coarse correction and post-smooths, on every level (the 64^2
    hierarchy smooths its level-1 grid with the 16-colour sweep)."""
    w = synth.WORKLOADS[wl]
    U = w.links()
    m0 = w.m0 if wl == "C1" else synth.critical_masses()[wl] + 0.05
    psi = synth.gaussian_rhs(w.L, w.L, w.rhs_seed + 1, nrhs=2)
    say("pre-sweeps", wl, precision)
    kw = dict(levels=w.levels, agg=w.agg, overlap=w.overlap, n_test_vectors=w.n_test_vectors,
              pre_sweeps=1)
    outs, x, infos, st, hists, _ = solve_both(lib, ctx, U, m0, psi, precision, **kw)
    if precision == 0:
        check_fp64(outs, x, infos, st, hists)
    else:
        assert st == 0
        for r, (xo, io) in enumerate(outs):
            assert infos[r].converged and infos[r].true_rel_residual <= 1e-10
            assert abs(infos[r].iterations - io.iterations) <= max(5, io.iterations // 10)
            assert rel(x[r], xo) <= 1e-9
    # the pre-sweep changes the preconditioner: the counts differ from the default V-cycle's
    _, io0, _ = oracle_solve(U, m0, psi[0], amg.SetupParams(levels=w.levels, agg=w.agg, overlap=w.overlap,
                                                            n_test_vectors=w.n_test_vectors))
    assert [v for v, _ in io0.history] != [v for v, _ in outs[0][1].history]


# ------------------------------------------------------------------ 2048-unknown coarsest level

@pytest.fixture(scope="module")
def coarsest_2048():
    w = synth.WORKLOADS["C4"]
    U = w.links()
    m0 = synth.critical_masses()["C4"] + 0.05
    return U, m0


@pytest.mark.parametrize("coarsest_tol", [0.0, 0.1])
def test_2048_unknown_coarsest_level_matches_oracle(lib, ctx, coarsest_2048, coarsest_tol):
    """128^2 lattice, two levels of a = 8, o = 2: the coarsest level is 16 x 16 nodes with 8
    unknowns each.  The dense Galerkin operator matches the oracle's; FP64 solves with the exact
    coarsest solve and with GMRES to 0.1 take the oracle's iteration counts and agree to 1e-9;
    with GMRES each right-hand side of a batch is bitwise its single solve."""
    U, m0 = coarsest_2048
    psi = synth.gaussian_rhs(128, 128, 5151, nrhs=2)
    kw = dict(levels=2, agg=8, overlap=2, n_test_vectors=8, coarsest_tol=coarsest_tol)
    say("coarsest 2048", coarsest_tol)
    outs, x, infos, st, hists, olev = solve_both(lib, ctx, U, m0, psi, 0, **kw)
    assert olev[1].ndof == 2048
    check_fp64(outs, x, infos, st, hists)
    g = lib.Gauge(ctx, synth.links_to_abi(U), m0)
    h = lib.Hierarchy(g, gpu_setup(lib, **kw))
    assert h.level_info(1) == (16, 16, 8)
    assert rel(h.coarse_operator(1, coarsest=True), olev[1].A.toarray()) < 1e-10
    x1, i1, _ = h.solve(synth.field_to_abi(psi[1:2]))
    assert i1[0].iterations == infos[1].iterations
    assert np.array_equal(synth.field_from_abi(x1)[0], x[1])
    h.close()
    g.close()


# ------------------------------------------------------------------------ rectangular lattices

@pytest.fixture(scope="module")
def rect_links():
    return synth.gen_links(32, 64, 4.0, 100, 777)


@pytest.mark.parametrize("levels,a,o,nv", [(2, 4, 1, 4), (3, 4, 1, 8), (2, 4, 2, 4)])
def test_rectangular_lattice_matches_oracle(lib, ctx, rect_links, levels, a, o, nv):
    """32 x 64 lattice (N_t = 32 in time, N_x = 64 in space): classification, interpolation rows
    and coarse operators of every level, and FP64 solves of two right-hand sides."""
    U = rect_links
    m0 = 0.05
    psi = synth.gaussian_rhs(32, 64, 778, nrhs=2)
    kw = dict(levels=levels, agg=a, overlap=o, n_test_vectors=nv)
    say("rectangular", levels, a, o)
    outs, x, infos, st, hists, olev = solve_both(lib, ctx, U, m0, psi, 0, **kw)
    check_fp64(outs, x, infos, st, hists)
    g = lib.Gauge(ctx, synth.links_to_abi(U), m0)
    h = lib.Hierarchy(g, gpu_setup(lib, **kw))
    for k in range(levels - 1):
        lev = olev[k]
        assert h.level_info(k) == (lev.Lt, lev.Lx, lev.b)
        kind, owner, node = h.aggregates(k)
        assert np.array_equal(kind, lev.cls["kind"]) and np.array_equal(owner, lev.cls["owner"])
        assert np.array_equal(node, lev.cls["node"])
        assert rel(h.prolongator_rows(k, o), oracle_rows(lev, a, o)) < 1e-10
    for k in range(1, levels):
        lev = olev[k]
        if lev.coarsest:
            assert rel(h.coarse_operator(k, coarsest=True), lev.A.toarray()) < 1e-10
        else:
            assert rel(h.coarse_operator(k, coarsest=False), oracle_stencil(lev.A, lev.Lt, lev.Lx, lev.b)) < 1e-10
    # true residual with the oracle's operator (antiperiodic in time, periodic in space)
    D = dirac_matrix(U, m0)
    r = psi[0].reshape(-1) - D @ x[0].reshape(-1)
    assert np.linalg.norm(r) / np.linalg.norm(psi[0]) <= 1e-10
    h.close()
    g.close()


def test_rectangular_mixed_precision_within_bound(lib, ctx, rect_links):
    U = rect_links
    psi = synth.gaussian_rhs(32, 64, 779, nrhs=2)
    kw = dict(levels=3, agg=4, overlap=1, n_test_vectors=8)
    say("rectangular mixed")
    outs, x, infos, st, _, _ = solve_both(lib, ctx, U, 0.05, psi, 1, **kw)
    assert st == 0
    for r, (xo, io) in enumerate(outs):
        assert infos[r].converged and infos[r].true_rel_residual <= 1e-10
        assert rel(x[r], xo) <= 1e-9


# ----------------------------------------------------------------- (3 levels, a = 8, o = 1)

@pytest.mark.parametrize("precision", [0, 1])
def test_a8_o1_three_levels_matches_oracle(lib, ctx, coarsest_2048, precision):
    """The aggregate-sweep point (3, 8, 1) on the 128^2 lattice: level 1 is 16 x 16 nodes with
    2 unknowns (the two-spin block smoother), the coarsest 2 x 2 nodes."""
    U, m0 = coarsest_2048
    psi = synth.gaussian_rhs(128, 128, 5252, nrhs=2)
    kw = dict(levels=3, agg=8, overlap=1, n_test_vectors=8)
    say("a8 o1 three levels", precision)
    outs, x, infos, st, hists, olev = solve_both(lib, ctx, U, m0, psi, precision, **kw)
    assert (olev[1].Lt, olev[1].b, olev[2].ndof) == (16, 2, 8)
    if precision == 0:
        check_fp64(outs, x, infos, st, hists)
    else:
        assert st == 0
        for r, (xo, io) in enumerate(outs):
            assert infos[r].converged and infos[r].true_rel_residual <= 1e-10
            assert abs(infos[r].iterations - io.iterations) <= max(5, io.iterations // 10)
            assert rel(x[r], xo) <= 1e-9


# -------------------------------------------------------------------------------- errors

def test_zero_operator_reports_a_singular_local_system(lib, ctx):
    """Links U = 0 and m0 = -2 make D = 0, so every wirebasket's system A_FF is zero: the setup
    reports SINGULAR_LOCAL (nothing is written), and the context keeps working."""
    say("singular local")
    links = np.zeros((2, 16, 16, 2))
    g = lib.Gauge(ctx, links, -2.0)
    with pytest.raises(lib.AmamgError) as e:
        lib.Hierarchy(g, lib.default_setup_params(levels=2, agg_size=4, overlap=1, norm=2))
    assert e.value.status == lib.STATUS_CODES["SINGULAR_LOCAL"]
    g.close()
    w = synth.WORKLOADS["C1"]
    g = lib.Gauge(ctx, synth.links_to_abi(w.links()), w.m0)
    h = lib.Hierarchy(g, lib.default_setup_params(levels=2, agg_size=4, overlap=1))
    _, infos, st = h.solve(synth.field_to_abi(synth.gaussian_rhs(16, 16, w.rhs_seed)))
    assert st == lib.OK and infos[0].converged
    h.close()
    g.close()


# ------------------------------------------------------------------- caller's stream

def test_solve_device_follows_the_callers_stream(lib):
    """amamg_solve_device with a caller stream: the right-hand side is written on that stream
    behind a long queue of other work, and the solve (on the context's own stream) starts only
    after it, giving bitwise the host-buffer solve."""
    import torch
    w = synth.WORKLOADS["C1"]
    say("caller stream")
    ctx = lib.Context(0)                                   # the library's own stream
    g = lib.Gauge(ctx, synth.links_to_abi(w.links()), w.m0)
    h = lib.Hierarchy(g, lib.default_setup_params(levels=2, agg_size=4, overlap=1))
    psi = synth.field_to_abi(synth.gaussian_rhs(16, 16, w.rhs_seed, nrhs=2))
    x_ref, i_ref, _ = h.solve(psi)
    src = torch.from_numpy(psi).cuda()
    torch.cuda.synchronize()
    caller = torch.cuda.Stream()
    b = torch.zeros_like(src)
    x = torch.zeros_like(src)
    big = torch.ones(1 << 24, device="cuda")
    caller.wait_stream(torch.cuda.current_stream())       # b, x and big are initialised
    with torch.cuda.stream(caller):
        for _ in range(200):
            big.mul_(1.0000001)                           # ~0.1 s of queued work before b
        b.copy_(src)
    infos, st = h.solve_device(b.data_ptr(), x.data_ptr(), 2, stream=caller.cuda_stream)
    assert st == lib.OK
    torch.cuda.synchronize()
    assert [i.iterations for i in infos] == [i.iterations for i in i_ref]
    assert np.array_equal(x.cpu().numpy(), x_ref)
    h.close()
    g.close()
    ctx.close()
