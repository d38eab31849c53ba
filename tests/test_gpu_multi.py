"""GPU tests of amamg_solve_multi_device: several lattices of different sizes and hierarchies
solved in lock step, each Gram-Schmidt kernel launched once for all of them (and, with graphs,
one captured HIP graph per restart round for all lattices).

Bars: every right-hand side bitwise equal (solution, iteration count, residual history) to a
plain device solve of its lattice alone with the same number of right-hand sides, in FP64 and
mixed precision, with and without graphs; FP64 results also against the CPU oracle (the
oracle's iteration counts, relative error <= 1e-9).  Errors are refused before any device work.
"""
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


# (L, beta, setup keywords (library names), m0, nrhs)
LATTICES = [
    (16, 3.0, dict(levels=2, agg_size=4, overlap=1, n_test_vectors=4), 0.1, 2),
    (32, 4.0, dict(levels=2, agg_size=4, overlap=1, n_test_vectors=4), 0.08, 3),
    (64, 6.0, dict(levels=3, agg_size=4, overlap=1, n_test_vectors=8), 0.05, 2),
    (128, 8.0, dict(levels=3, agg_size=8, overlap=2, n_test_vectors=8), 0.05, 1),
]
ORACLE_NAMES = {"agg_size": "agg"}


@pytest.fixture(scope="module")
def lattices(lib):
    import torch
    stream = torch.cuda.Stream()
    ctx = lib.Context(0, stream.cuda_stream)
    out = []
    for k, (L, beta, sp, m0, nrhs) in enumerate(LATTICES):
        U = synth.gen_links(L, L, beta, 40, 7000 + L)
        g = lib.Gauge(ctx, synth.links_to_abi(U), m0)
        h = lib.Hierarchy(g, lib.default_setup_params(**sp))
        psi = synth.gaussian_rhs(L, L, 800 + k, nrhs=nrhs)
        b = torch.from_numpy(synth.field_to_abi(psi)).to("cuda")
        out.append(dict(U=U, g=g, h=h, psi=psi, b=b, m0=m0, sp=sp, nrhs=nrhs))
    yield ctx, stream, out
    for d in out:
        d["h"].close()
        d["g"].close()
    ctx.close()


def plain(lib, torch, stream, d, sp):
    x = torch.zeros_like(d["b"])
    with torch.cuda.stream(stream):
        infos, st = d["h"].solve_device(d["b"].data_ptr(), x.data_ptr(), d["nrhs"], sp, stream.cuda_stream)
    torch.cuda.synchronize()
    hist = [d["h"].residual_history(r) for r in range(d["nrhs"])]
    return x.cpu().numpy(), infos, st, hist


@pytest.mark.parametrize("precision,graphs", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_multi_lattice_solve_equals_each_lattice_alone(lib, lattices, precision, graphs):
    import torch
    ctx, stream, lats = lattices
    sp = lib.default_solve_params(precision=precision, graphs=graphs)
    say("multi lattice", precision, graphs)
    xs = [torch.zeros_like(d["b"]) for d in lats]
    with torch.cuda.stream(stream):
        infos, st = lib.solve_multi_device([d["h"] for d in lats], [d["nrhs"] for d in lats],
                                           [d["b"].data_ptr() for d in lats], [x.data_ptr() for x in xs],
                                           sp, stream.cuda_stream)
    torch.cuda.synchronize()
    assert st == lib.OK
    multi_hist = [[d["h"].residual_history(r) for r in range(d["nrhs"])] for d in lats]
    for k, d in enumerate(lats):
        x1, i1, st1, h1 = plain(lib, torch, stream, d, sp)
        assert st1 == lib.OK
        assert np.array_equal(xs[k].cpu().numpy(), x1), k
        assert [i.iterations for i in infos[k]] == [i.iterations for i in i1]
        assert [i.restarts for i in infos[k]] == [i.restarts for i in i1]
        for (va, fa), (vb, fb) in zip(multi_hist[k], h1):
            assert np.array_equal(va, vb) and np.array_equal(fa, fb)
        if precision == 0 and graphs == 0:
            prm = amg.SetupParams(**{ORACLE_NAMES.get(kk, kk): v for kk, v in d["sp"].items()})
            xo, io, _ = oracle_solve(d["U"], d["m0"], d["psi"][0], prm)
            assert infos[k][0].iterations == io.iterations
            assert rel(synth.field_from_abi(xs[k].cpu().numpy())[0], xo) <= 1e-9


def test_multi_lattice_errors(lib, lattices):
    import torch
    ctx, stream, lats = lattices
    d = lats[0]
    x = torch.zeros_like(d["b"])
    with pytest.raises(lib.AmamgError) as e:            # the same hierarchy twice
        lib.solve_multi_device([d["h"], d["h"]], [d["nrhs"]] * 2, [d["b"].data_ptr()] * 2, [x.data_ptr()] * 2)
    assert e.value.status == lib.STATUS_CODES["INVALID_ARG"]
    bad = d["b"].clone()
    bad[0, 1, 1, 0, 0] = float("nan")
    with pytest.raises(lib.AmamgError) as e:
        lib.solve_multi_device([d["h"], lats[1]["h"]], [d["nrhs"], lats[1]["nrhs"]],
                               [bad.data_ptr(), lats[1]["b"].data_ptr()],
                               [x.data_ptr(), torch.zeros_like(lats[1]["b"]).data_ptr()])
    assert e.value.status == lib.STATUS_CODES["NONFINITE"]
    torch.cuda.synchronize()
