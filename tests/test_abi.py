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


def _c_layouts(structs):
    """sizeof and field offsets of header structs, from a C program compiled against it."""
    import subprocess
    import tempfile
    body = []
    for cname, fields in structs:
        body.append(f'printf("{cname} %zu", sizeof({cname}));')
        for f in fields:
            body.append(f'printf(" %zu", offsetof({cname}, {f}));')
        body.append('printf("\\n");')
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"amamg.h\"\nint main(void) {\n"
           + "\n".join(body) + "\nreturn 0;\n}\n")
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {ln.split()[0]: [int(v) for v in ln.split()[1:]] for ln in out.splitlines()}


def test_struct_layouts_match_header():
    """Every ctypes structure of the binding has the header's size and field offsets."""
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_2608_03515_amd import amamg
    pairs = [("amamg_setup_params", amamg.SetupParams), ("amamg_solve_params", amamg.SolveParams),
             ("amamg_solve_info", amamg.SolveInfo)]
    pairs += [("amamg_server_params", amamg.ServerParams), ("amamg_request_info", amamg.RequestInfo),
              ("amamg_server_counters", amamg.ServerCounters), ("amamg_tune_entry", amamg.TuneEntry)]
    c = _c_layouts([(cname, [f[0] for f in cls._fields_]) for cname, cls in pairs])
    for cname, cls in pairs:
        want = [ctypes.sizeof(cls)] + [getattr(cls, f[0]).offset for f in cls._fields_]
        assert c[cname] == want, (cname, c[cname], want)
