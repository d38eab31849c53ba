"""CPU checks of the C ABI: the library loads and exports every function include/amamg.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amamg.h")
LIB = os.path.join(ROOT, "paper_2608_03515_amd", "libamamg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amamg_[a-z_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_header():
    from paper_2608_03515_amd import amamg
    assert sorted(amamg.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_params_and_no_device_errors():
    from paper_2608_03515_amd import amamg
    p = amamg.default_setup_params()
    assert (p.levels, p.agg_size, p.overlap, p.n_test_vectors, p.post_sweeps) == (2, 4, 1, 4, 2)
    q = amamg.default_solve_params()
    assert (q.restart, q.max_iters, q.rel_tol, q.precision) == (20, 10000, 1e-10, 0)
    # without a GPU, creating a context fails cleanly with a negative status
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(amamg.AmamgError):
            amamg.Context(0)


def test_struct_layouts_match_header():
    from paper_2608_03515_amd import amamg
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    assert ctypes.sizeof(amamg.SetupParams) == 8 * 4 + 8
    assert ctypes.sizeof(amamg.SolveParams) == 4 + 4 + 8 + 4 + 4
    assert ctypes.sizeof(amamg.SolveInfo) == 16 + 8
