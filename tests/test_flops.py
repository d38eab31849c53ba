"""The operation-count model (paper_2608_03515_amd.flops) against the oracle's structures.

The paper compares methods by operation counts with the setup included (Numerical Results).
The model counts this library's algorithm from the hierarchy geometry; its structural counts
(local system sizes, interpolation nonzeros, coarse stencil blocks, level sizes) are checked
here against the matrices the oracle actually builds.
"""
import numpy as np
import pytest

import synth
from oracle import amg
from oracle.wirebasket import KIND_V, footprint
from paper_2608_03515_amd import flops


@pytest.mark.parametrize("L,levels,a,o", [(32, 2, 4, 1), (64, 3, 4, 1), (32, 2, 8, 2), (48, 2, 8, 2)])
def test_structural_counts_match_the_oracle_hierarchy(L, levels, a, o):
    U = synth.gen_links(L, L, 4.0, 5, 40 + L)
    prm = amg.SetupParams(levels=levels, agg=a, overlap=o, n_test_vectors=2)
    olev = amg.setup(U, 0.1, prm)
    geo = flops.levels_of(L, L, levels, a, o)
    assert [(g.Lt, g.Lx, g.b) for g in geo] == [(lv.Lt, lv.Lx, lv.b) for lv in olev]
    for k in range(levels - 1):
        lev, g = olev[k], geo[k]
        w = flops.wirebasket_counts(g, a, o)
        # local system size of every wirebasket
        kind = lev.cls["kind"]
        for I in range(lev.Lt // a):
            for J in range(lev.Lx // a):
                pts = [t * lev.Lx + x for t, x, _, _ in footprint(I, J, lev.Lt, lev.Lx, a, o)]
                nf = sum(1 for p in pts if kind[p] != KIND_V) * lev.b
                nv = sum(1 for p in pts if kind[p] == KIND_V) * lev.b
                assert nf == w["nF"] and nv == 4 * w["bc"]
        # interpolation nonzeros in the non-vertex rows
        P = lev.P.tocsr()
        vrows = np.repeat(kind == KIND_V, lev.b)
        nnz_f = int(np.diff(P.indptr)[~vrows].sum())
        assert nnz_f == w["nnzF"]
        assert w["nW"] == (lev.Lt // a) * (lev.Lx // a)
        # the next level's operator: 21 nonzero blocks per node, or dense when coarsest
        nxt = olev[k + 1]
        A = nxt.A.toarray()
        if nxt.coarsest:
            assert A.shape == (geo[k + 1].ndof, geo[k + 1].ndof)
        else:
            b = nxt.b
            blocks = A.reshape(nxt.nnode, b, nxt.nnode, b).transpose(0, 2, 1, 3)
            per_node = (np.abs(blocks).sum(axis=(2, 3)) > 0).sum(axis=1)
            assert np.all(per_node == flops.COARSE_BLOCKS)


def test_operation_counts_scale_as_the_method_does():
    """Sanity relations of the model: the solve is linear in the iteration count at fixed
    cycle structure, the Gram-Schmidt share grows with the restart length, and a setup with
    larger wirebaskets costs more in local solves."""
    geo = flops.levels_of(256, 256, 3, 8, 2)
    s20 = flops.solve(geo, 8, 2, 200)
    s40 = flops.solve(geo, 8, 2, 400)
    assert s40["total"] == pytest.approx(2 * s20["total"], rel=1e-3)
    assert flops.solve(geo, 8, 2, 200, restart=10)["gram_schmidt"] < s20["gram_schmidt"]
    g4 = flops.levels_of(256, 256, 3, 4, 1)
    assert flops.setup(g4, 4, 1, 8)["local_solves"] < flops.setup(geo, 8, 2, 8)["local_solves"]
    # the fine level's share: matvec 60 and two smoother sweeps 144 flops per site
    assert flops.vcycle(geo, 8, 2) > 144 * 256 * 256
