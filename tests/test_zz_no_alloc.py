"""GPU test of amamg_apply_transfer_noalloc, the transfer entry point that allocates nothing.

It must give bitwise the results of amamg_apply_transfer (same kernels), on two calls in a row
with the second one smaller (the fixed scratch array keeps the first call's partial sums), and
refuse a restriction whose partial sums do not fit the array before doing any device work.
The 128^2 hierarchy (a = 8, o = 2, three levels) covers the register-tiled transfers of the
fine level (32 columns) and the matrix-core FP32 transfers of level 1 (128 columns).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c4_hierarchy(lib):
    ctx = lib.Context(0)
    w = synth.WORKLOADS["C4"]
    m0 = synth.critical_masses()["C4"] + w.gaps[0]
    g = lib.Gauge(ctx, synth.links_to_abi(w.links()), m0)
    h = lib.Hierarchy(g, lib.default_setup_params(levels=3, agg_size=8, overlap=2, n_test_vectors=8))
    yield h
    h.close()
    g.close()
    ctx.close()


def _device(arr, dtype):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(np.stack([arr.real, arr.imag], axis=-1))).to(dtype)
    return t.cuda()


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("direction", [0, 1])
def test_noalloc_transfer_equals_the_allocating_entry_point(lib, c4_hierarchy, level, precision, direction):
    import torch
    h = c4_hierarchy
    lt, lx, b = h.level_info(level)
    ltc, lxc, bc = h.level_info(level + 1)
    n, nc = lt * lx * b, ltc * lxc * bc
    nin, nout = (n, nc) if direction == 0 else (nc, n)
    rng = np.random.default_rng(100 * level + 10 * precision + direction)
    in_type = torch.float64 if (direction == 0 or precision == 0) else torch.float32
    out_type = torch.float64 if precision == 0 else torch.float32
    for nrhs in (5, 2):                       # the second call is smaller
        say("noalloc transfer", level, precision, direction, nrhs)
        vecs = rng.standard_normal((nrhs, nin)) + 1j * rng.standard_normal((nrhs, nin))
        if in_type == torch.float32:          # the values the FP32 kernels read
            vecs = (vecs.real.astype(np.float32).astype(np.float64)
                    + 1j * vecs.imag.astype(np.float32).astype(np.float64))
        ref = h.transfer(level, vecs, direction, precision)
        din = _device(vecs, in_type)
        dout = torch.full((nrhs, nout, 2), float("nan"), dtype=out_type, device="cuda")
        torch.cuda.synchronize()
        h.transfer_noalloc(level, din.data_ptr(), dout.data_ptr(), nrhs, direction, precision)
        torch.cuda.synchronize()
        got = dout.double().cpu().numpy()
        assert np.array_equal(got[..., 0] + 1j * got[..., 1], ref)


def test_noalloc_transfer_refuses_a_restriction_beyond_the_scratch_array(lib, c4_hierarchy):
    """600 right-hand sides on the fine level need at least 600 x 256 wirebaskets x 32 columns
    x 16 bytes = 78.6 MB of FP64 partial sums, more than the 64 MiB array: refused with
    INVALID_ARG (the buffers passed are large enough, so nothing could be out of bounds)."""
    import torch
    h = c4_hierarchy
    lt, lx, b = h.level_info(0)
    ltc, lxc, bc = h.level_info(1)
    nrhs = 600
    din = torch.zeros((nrhs, lt * lx * b, 2), dtype=torch.float64, device="cuda")
    dout = torch.zeros((nrhs, ltc * lxc * bc, 2), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(lib.AmamgError) as e:
        h.transfer_noalloc(0, din.data_ptr(), dout.data_ptr(), nrhs, 0, 0)
    assert e.value.status == lib.STATUS_CODES["INVALID_ARG"]
    assert "scratch" in str(e.value)
    # the prolongation needs no scratch: the same sizes are accepted
    h.transfer_noalloc(0, dout.data_ptr(), din.data_ptr(), nrhs, 1, 0)
    torch.cuda.synchronize()
