"""Thin ctypes binding of libamamg.so (the C ABI in include/amamg.h).

Argument marshalling only: every step of the solver runs in the HIP library.  The library
must have been built (``python -m paper_2608_03515_amd.build``); importing this module
raises ``ImportError`` when it is missing, there is no fallback.

Fields use the ABI layout: float64 arrays [nrhs][nt][nx][2 spin][2 (re, im)] (numpy), or
complex128 tensors [nrhs][nt][nx][2] on the GPU (torch) for the device entry points.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamamg.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2608_03515_amd.build")
_lib = C.CDLL(LIB_PATH)

OK, NOT_CONVERGED, PENDING = 0, 1, 2
FP64, MIXED_FP32, MIXED_FP32_BF16LINKS = 0, 1, 2
NORM_TESTVEC, NORM_CONST, NORM_NONE = 0, 1, 2
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "PENDING", -1: "INVALID_ARG", -2: "UNSUPPORTED_SHAPE",
                -3: "OUT_OF_MEMORY", -4: "DEVICE", -5: "SINGULAR_LOCAL",
                -6: "SINGULAR_COARSEST", -7: "NONFINITE"}
STATUS_CODES = {v: k for k, v in STATUS_NAMES.items()}

EXPORTED = ["amamg_default_setup_params", "amamg_default_solve_params", "amamg_context_create",
            "amamg_context_destroy", "amamg_last_error", "amamg_gauge_load",
            "amamg_gauge_set_mass", "amamg_gauge_update_links", "amamg_gauge_destroy",
            "amamg_setup", "amamg_hierarchy_update", "amamg_hierarchy_set_mass", "amamg_hierarchy_derive_mass", "amamg_hierarchy_destroy", "amamg_solve", "amamg_solve_device", "amamg_solve_multi_device",
            "amamg_residual_history", "amamg_apply_dirac", "amamg_apply_dirac_device", "amamg_dense_solve",
            "amamg_level_info",
            "amamg_get_aggregates", "amamg_get_prolongator", "amamg_get_coarse_operator",
            "amamg_get_test_vectors", "amamg_apply_transfer", "amamg_apply_transfer_noalloc", "amamg_apply_smoother", "amamg_context_set_tuning",
            "amamg_tuning_entries", "amamg_kernel_timer", "amamg_kernel_timer_read",
            "amamg_server_default_params", "amamg_server_create", "amamg_server_destroy",
            "amamg_server_add_gauge", "amamg_server_set_reference_mass", "amamg_server_submit", "amamg_server_poll", "amamg_server_wait",
            "amamg_server_stats", "amamg_server_last_error"]
KT = {"off": 0, "fine_matvec": 1, "fine_gs": 2, "restrict0": 3, "prolong0": 4, "coarse_gs": 5,
      "dots": 6, "update": 7}


class SetupParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("agg_size", C.c_int32), ("overlap", C.c_int32),
                ("n_test_vectors", C.c_int32), ("test_vector_sweeps", C.c_int32),
                ("pre_sweeps", C.c_int32), ("post_sweeps", C.c_int32), ("norm", C.c_int32),
                ("seed", C.c_uint64), ("coarsest_tol", C.c_double), ("coarsest_max_iters", C.c_int32),
                ("block_smoother", C.c_int32), ("aug_vectors", C.c_int32), ("reserved", C.c_int32)]


class SolveParams(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iters", C.c_int32), ("rel_tol", C.c_double),
                ("precision", C.c_int32), ("use_initial_guess", C.c_int32), ("groups", C.c_int32),
                ("graphs", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("reserved", C.c_int32), ("true_rel_residual", C.c_double)]


class ServerParams(C.Structure):
    _fields_ = [("slots", C.c_int32), ("max_instances", C.c_int32), ("precision", C.c_int32),
                ("restart", C.c_int32), ("max_iters", C.c_int32), ("builders", C.c_int32),
                ("graphs", C.c_int32), ("rel_tol", C.c_double), ("hbm_budget", C.c_uint64)]


class RequestInfo(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("nrhs", C.c_int32),
                ("iterations", C.c_int32), ("converged", C.c_int32), ("true_rel_residual", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("instance", C.c_int32), ("hierarchy_built", C.c_int32)]


class TuneEntry(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lt", C.c_int32), ("lx", C.c_int32), ("b", C.c_int32),
                ("precision", C.c_int32), ("nrhs", C.c_int32), ("choice", C.c_int32),
                ("ncand", C.c_int32), ("cand", C.c_int32 * 8), ("us", C.c_double * 8)]


TUNE_AUTO, TUNE_OFF, TUNE_FORCE = 0, 1, 2
TUNE_KINDS = {0: "fine_smoother_tile", 1: "block_smoother_launch"}


class ServerCounters(C.Structure):
    _fields_ = [("setups", C.c_int64), ("evictions", C.c_int64), ("resident_bytes", C.c_uint64),
                ("hierarchy_bytes", C.c_uint64),
                ("peak_resident_bytes", C.c_uint64), ("budget_bytes", C.c_uint64),
                ("outstanding", C.c_int64), ("clock", C.c_double), ("last_estimate_bytes", C.c_uint64),
                ("setup_seconds", C.c_double), ("setup_seconds_max", C.c_double),
                ("derivations", C.c_int64), ("derive_seconds", C.c_double), ("derive_seconds_max", C.c_double)]


_vp = C.c_void_p
_P = C.POINTER
_sig = {
    "amamg_default_setup_params": (None, [_P(SetupParams)]),
    "amamg_default_solve_params": (None, [_P(SolveParams)]),
    "amamg_context_create": (C.c_int, [C.c_int, _vp, _P(_vp)]),
    "amamg_context_destroy": (C.c_int, [_vp]),
    "amamg_last_error": (C.c_char_p, [_vp]),
    "amamg_gauge_load": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp, C.c_double, _P(_vp)]),
    "amamg_gauge_set_mass": (C.c_int, [_vp, C.c_double]),
    "amamg_gauge_update_links": (C.c_int, [_vp, _vp]),
    "amamg_gauge_destroy": (C.c_int, [_vp]),
    "amamg_setup": (C.c_int, [_vp, _P(SetupParams), _P(_vp)]),
    "amamg_hierarchy_update": (C.c_int, [_vp]),
    "amamg_hierarchy_set_mass": (C.c_int, [_vp, C.c_double]),
    "amamg_hierarchy_derive_mass": (C.c_int, [_vp, C.c_double, C.POINTER(_vp)]),
    "amamg_hierarchy_destroy": (C.c_int, [_vp]),
    "amamg_dense_solve": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _vp, _vp]),
    "amamg_solve": (C.c_int, [_vp, C.c_int32, _vp, _vp, _P(SolveParams), _P(SolveInfo)]),
    "amamg_solve_device": (C.c_int, [_vp, C.c_int32, _vp, _vp, _P(SolveParams), _P(SolveInfo), _vp]),
    "amamg_solve_multi_device": (C.c_int, [_P(_vp), C.c_int32, _P(C.c_int32), _P(_vp), _P(_vp), _P(SolveParams),
                                           _P(SolveInfo), _vp]),
    "amamg_residual_history": (C.c_int, [_vp, C.c_int32, _vp, C.c_int32, _P(C.c_int32), _vp]),
    "amamg_apply_dirac": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _vp]),
    "amamg_apply_dirac_device": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _vp]),
    "amamg_level_info": (C.c_int, [_vp, C.c_int32, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32)]),
    "amamg_get_aggregates": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp]),
    "amamg_get_prolongator": (C.c_int, [_vp, C.c_int32, _vp]),
    "amamg_get_coarse_operator": (C.c_int, [_vp, C.c_int32, _vp]),
    "amamg_get_test_vectors": (C.c_int, [_vp, C.c_int32, _vp]),
    "amamg_apply_transfer": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp, _vp]),
    "amamg_apply_transfer_noalloc": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp, _vp]),
    "amamg_apply_smoother": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp, _vp]),
    "amamg_context_set_tuning": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "amamg_tuning_entries": (C.c_int, [_vp, _vp, C.c_int32, _P(C.c_int32)]),
    "amamg_kernel_timer": (C.c_int, [_vp, C.c_uint32]),
    "amamg_kernel_timer_read": (C.c_int, [_vp, C.c_int32, _P(C.c_int64), _P(C.c_double), _P(C.c_double)]),
    "amamg_server_default_params": (None, [_P(ServerParams)]),
    "amamg_server_create": (C.c_int, [C.c_int32, _P(ServerParams), _P(_vp)]),
    "amamg_server_destroy": (C.c_int, [_vp]),
    "amamg_server_add_gauge": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _P(C.c_int32)]),
    "amamg_server_set_reference_mass": (C.c_int, [_vp, C.c_int32, C.c_double]),
    "amamg_server_submit": (C.c_int, [_vp, C.c_int32, C.c_double, _P(SetupParams), C.c_int32, _vp, _vp,
                                      _P(C.c_uint64)]),
    "amamg_server_poll": (C.c_int, [_vp, _P(RequestInfo), C.c_int32, _P(C.c_int32)]),
    "amamg_server_wait": (C.c_int, [_vp, C.c_double]),
    "amamg_server_stats": (C.c_int, [_vp, _P(ServerCounters)]),
    "amamg_server_last_error": (C.c_char_p, [_vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class AmamgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_vp)


def default_setup_params(**kw) -> SetupParams:
    p = SetupParams()
    _lib.amamg_default_setup_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def default_solve_params(**kw) -> SolveParams:
    p = SolveParams()
    _lib.amamg_default_solve_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Context:
    """amamg_context on a HIP device; stream: a raw hipStream_t handle (int) or None."""

    def __init__(self, device: int = 0, stream: int | None = None):
        h = _vp()
        st = _lib.amamg_context_create(device, _vp(stream) if stream else None, C.byref(h))
        if st != OK:
            raise AmamgError(st, "context creation failed")
        self.h = h

    def check(self, st: int, ok=(OK,)) -> int:
        if st not in ok:
            raise AmamgError(st, _lib.amamg_last_error(self.h).decode())
        return st

    def kernel_timer(self, families):
        """Time the named kernel families (list of KT keys; empty list stops)."""
        mask = 0
        for f in families:
            mask |= 1 << KT[f]
        self.check(_lib.amamg_kernel_timer(self.h, mask))

    def kernel_timer_read(self, family: str):
        """(launches, total ms, algorithmic bytes) of one family."""
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        self.check(_lib.amamg_kernel_timer_read(self.h, KT[family], C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def set_tuning(self, mode: int, force: int = 0):
        """TUNE_AUTO (default), TUNE_OFF or TUNE_FORCE with candidate number `force`."""
        self.check(_lib.amamg_context_set_tuning(self.h, mode, force))

    def dense_solve(self, aug: np.ndarray):
        """The setup's batched dense solve on complex [nsys][n][n + nrhs] augmented matrices
        (amamg_dense_solve): returns (the overwritten matrices, info per system)."""
        a = np.ascontiguousarray(aug, dtype=np.complex128).copy()
        nsys, n, ld = a.shape
        info = np.zeros(nsys, dtype=np.int32)
        self.check(_lib.amamg_dense_solve(self.h, n, ld - n, nsys, _ptr(a), _ptr(info)))
        return a, info

    def tuning_entries(self) -> list:
        """The launch shapes tuned so far: dicts with kind, grid, b, precision, nrhs, choice and
        the candidates' times (microseconds)."""
        n = C.c_int32()
        self.check(_lib.amamg_tuning_entries(self.h, None, 0, C.byref(n)))
        arr = (TuneEntry * max(1, n.value))()
        self.check(_lib.amamg_tuning_entries(self.h, arr, n.value, C.byref(n)))
        out = []
        for e in arr[:n.value]:
            out.append({"kind": TUNE_KINDS.get(e.kind, e.kind), "lt": e.lt, "lx": e.lx, "b": e.b,
                        "precision": e.precision, "nrhs": e.nrhs, "choice": e.choice,
                        "candidates_us": {int(e.cand[q]): round(e.us[q], 2) for q in range(e.ncand)}})
        return out

    def close(self):
        if self.h:
            _lib.amamg_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Gauge:
    """amamg_gauge: links float64 [2][nt][nx][2] (host), bare mass m0."""

    def __init__(self, ctx: Context, links: np.ndarray, m0: float):
        links = np.ascontiguousarray(links, dtype=np.float64)
        _, nt, nx, _ = links.shape
        h = _vp()
        ctx.check(_lib.amamg_gauge_load(ctx.h, nt, nx, _ptr(links), float(m0), C.byref(h)))
        self.ctx, self.h, self.nt, self.nx = ctx, h, nt, nx

    def set_mass(self, m0: float):
        self.ctx.check(_lib.amamg_gauge_set_mass(self.h, float(m0)))

    def update_links(self, links: np.ndarray):
        links = np.ascontiguousarray(links, dtype=np.float64)
        assert links.shape == (2, self.nt, self.nx, 2)
        self.ctx.check(_lib.amamg_gauge_update_links(self.h, _ptr(links)))

    def apply_dirac(self, fields: np.ndarray, precision: int = FP64) -> np.ndarray:
        fields = np.ascontiguousarray(fields, dtype=np.float64)
        out = np.empty_like(fields)
        nrhs = fields.shape[0]
        self.ctx.check(_lib.amamg_apply_dirac(self.h, precision, nrhs, _ptr(fields), _ptr(out)))
        return out

    def apply_dirac_device(self, in_ptr: int, out_ptr: int, nrhs: int, precision: int = FP64):
        """Asynchronous D on device buffers (FP64 fields for FP64, FP32 fields otherwise)."""
        self.ctx.check(_lib.amamg_apply_dirac_device(self.h, precision, nrhs, _vp(in_ptr), _vp(out_ptr)))

    def close(self):
        if self.h:
            self.ctx.check(_lib.amamg_gauge_destroy(self.h))
            self.h = None


def solve_multi_device(hierarchies, nrhs, psi_ptrs, x_ptrs, params: SolveParams | None = None,
                       stream: int | None = None):
    """Several lattices in lock step (amamg_solve_multi_device): hierarchies of one context,
    per lattice its right-hand-side count and raw device pointers.  Returns (infos per lattice,
    status)."""
    L = len(hierarchies)
    hs = (_vp * L)(*[h.h for h in hierarchies])
    nr = (C.c_int32 * L)(*nrhs)
    ps = (_vp * L)(*[_vp(p) for p in psi_ptrs])
    xs = (_vp * L)(*[_vp(p) for p in x_ptrs])
    infos = (SolveInfo * sum(nrhs))()
    st = _lib.amamg_solve_multi_device(hs, L, nr, ps, xs, C.byref(params) if params else None, infos,
                                       _vp(stream) if stream else None)
    hierarchies[0].ctx.check(st, ok=(OK, NOT_CONVERGED))
    out, k = [], 0
    for n in nrhs:
        out.append(list(infos[k:k + n]))
        k += n
    return out, st


class Hierarchy:
    """amamg_hierarchy built by amamg_setup on the GPU."""

    def __init__(self, gauge: Gauge, params: SetupParams | None = None):
        h = _vp()
        gauge.ctx.check(_lib.amamg_setup(gauge.h, C.byref(params) if params else None, C.byref(h)))
        self.gauge, self.ctx, self.h = gauge, gauge.ctx, h

    def update(self):
        """Re-run the setup in place from the gauge's current links and mass."""
        self.ctx.check(_lib.amamg_hierarchy_update(self.h))

    def set_mass(self, m0: float):
        """Move the hierarchy to bare mass m0, keeping its interpolation (no new setup)."""
        self.ctx.check(_lib.amamg_hierarchy_set_mass(self.h, C.c_double(m0)))

    def derive_mass(self, m0: float) -> "Hierarchy":
        """A hierarchy at bare mass m0 sharing this one's interpolation (close it first)."""
        h = _vp()
        self.ctx.check(_lib.amamg_hierarchy_derive_mass(self.h, C.c_double(m0), C.byref(h)))
        out = Hierarchy.__new__(Hierarchy)
        out.gauge, out.ctx, out.h = self.gauge, self.ctx, h
        return out

    def close(self):
        if self.h:
            self.ctx.check(_lib.amamg_hierarchy_destroy(self.h))
            self.h = None

    def solve(self, psi: np.ndarray, params: SolveParams | None = None, x0: np.ndarray | None = None):
        """Host solve; psi float64 [nrhs][nt][nx][2][2].  Returns (x, [SolveInfo], status)."""
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        nrhs = psi.shape[0]
        x = np.zeros_like(psi) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).copy()
        infos = (SolveInfo * nrhs)()
        p = params or default_solve_params()
        if x0 is not None:
            p.use_initial_guess = 1
        st = _lib.amamg_solve(self.h, nrhs, _ptr(psi), _ptr(x), C.byref(p), infos)
        self.ctx.check(st, ok=(OK, NOT_CONVERGED))
        return x, list(infos), st

    def solve_device(self, psi_ptr: int, x_ptr: int, nrhs: int, params: SolveParams | None = None,
                     stream: int | None = None):
        """Device solve on raw device pointers (e.g. torch ``data_ptr()``), after the work queued
        on `stream` (a raw hipStream_t handle, or None)."""
        infos = (SolveInfo * nrhs)()
        st = _lib.amamg_solve_device(self.h, nrhs, _vp(psi_ptr), _vp(x_ptr),
                                     C.byref(params) if params else None, infos,
                                     _vp(stream) if stream else None)
        self.ctx.check(st, ok=(OK, NOT_CONVERGED))
        return list(infos), st

    def residual_history(self, rhs: int = 0):
        n = C.c_int32()
        self.ctx.check(_lib.amamg_residual_history(self.h, rhs, None, 0, C.byref(n), None))
        vals = np.zeros(n.value)
        flags = np.zeros(n.value, dtype=np.int32)
        self.ctx.check(_lib.amamg_residual_history(self.h, rhs, _ptr(vals), n.value, C.byref(n),
                                                   _ptr(flags)))
        return vals, flags.astype(bool)

    def level_info(self, level: int):
        lt, lx, b = C.c_int32(), C.c_int32(), C.c_int32()
        self.ctx.check(_lib.amamg_level_info(self.h, level, C.byref(lt), C.byref(lx), C.byref(b)))
        return lt.value, lx.value, b.value

    def aggregates(self, level: int):
        lt, lx, _ = self.level_info(level)
        kind = np.zeros(lt * lx, dtype=np.int8)
        owner = np.zeros(lt * lx, dtype=np.int32)
        node = np.zeros(lt * lx, dtype=np.int32)
        self.ctx.check(_lib.amamg_get_aggregates(self.h, level, _ptr(kind), _ptr(owner), _ptr(node)))
        return kind, owner, node

    def prolongator_rows(self, level: int, overlap: int, aug: int = 0) -> np.ndarray:
        """complex [lt*lx][b][4*bc] interpolation rows (vertex rows zero); bc = o^2 b, plus the
        augmented dofs on level 0."""
        lt, lx, b = self.level_info(level)
        bc = overlap * overlap * b + (aug if level == 0 else 0)
        out = np.zeros((lt * lx, b, 4 * bc, 2))
        self.ctx.check(_lib.amamg_get_prolongator(self.h, level, _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def coarse_operator(self, level: int, coarsest: bool) -> np.ndarray:
        lt, lx, b = self.level_info(level)
        if coarsest:
            n = lt * lx * b
            out = np.zeros((n, n, 2))
        else:
            out = np.zeros((lt * lx, 25, b, b, 2))
        self.ctx.check(_lib.amamg_get_coarse_operator(self.h, level, _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def smooth(self, level: int, f: np.ndarray, x: np.ndarray, sweeps: int = 1, precision: int = 0) -> np.ndarray:
        """`sweeps` post-smoothing sweeps of level `level` on complex [nrhs][n_level] vectors with
        the kernels of the given precision's V-cycle; returns the new x."""
        lt, lx, b = self.level_info(level)
        n = lt * lx * b
        f = np.asarray(f, dtype=complex)
        x = np.asarray(x, dtype=complex)
        nrhs = f.shape[0]
        if f.shape != (nrhs, n) or x.shape != (nrhs, n):
            raise ValueError("vector shape does not match the level")
        fs = np.ascontiguousarray(np.stack([f.real, f.imag], axis=-1))
        xs = np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1))
        self.ctx.check(_lib.amamg_apply_smoother(self.h, level, precision, nrhs, sweeps, _ptr(fs), _ptr(xs)))
        return xs[..., 0] + 1j * xs[..., 1]

    def transfer(self, level: int, vecs: np.ndarray, direction: int, precision: int = 0) -> np.ndarray:
        """direction 0: P^H vecs (vecs complex [nrhs][n_level]); 1: P vecs (vecs complex
        [nrhs][n_coarse]); the kernels of the given precision's V-cycle."""
        lt, lx, b = self.level_info(level)
        ltc, lxc, bcn = self.level_info(level + 1)
        n, nc = lt * lx * b, ltc * lxc * bcn
        vecs = np.asarray(vecs, dtype=complex)
        nrhs = vecs.shape[0]
        if vecs.shape != (nrhs, n if direction == 0 else nc):
            raise ValueError("vector shape does not match the level")
        src = np.ascontiguousarray(np.stack([vecs.real, vecs.imag], axis=-1))
        out = np.zeros((nrhs, nc if direction == 0 else n, 2))
        self.ctx.check(_lib.amamg_apply_transfer(self.h, level, precision, direction, nrhs, _ptr(src),
                                                 _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def transfer_noalloc(self, level: int, in_ptr: int, out_ptr: int, nrhs: int, direction: int,
                         precision: int = 0):
        """amamg_apply_transfer_noalloc on raw device pointers (asynchronous, allocates nothing)."""
        self.ctx.check(_lib.amamg_apply_transfer_noalloc(self.h, level, precision, direction, nrhs,
                                                         _vp(in_ptr), _vp(out_ptr)))

    def test_vectors(self, level: int, nv: int) -> np.ndarray:
        lt, lx, b = self.level_info(level)
        out = np.zeros((nv, lt * lx * b, 2))
        self.ctx.check(_lib.amamg_get_test_vectors(self.h, level, _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]


def default_server_params(**kw) -> ServerParams:
    p = ServerParams()
    _lib.amamg_server_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Server:
    """amamg_server: continuous-batching solve server with its own device objects and worker
    thread.  Output arrays handed to submit() are kept alive here until poll() returns them."""

    def __init__(self, device: int = 0, params: ServerParams | None = None):
        s = _vp()
        st = _lib.amamg_server_create(device, C.byref(params) if params else None, C.byref(s))
        if st != OK:
            raise AmamgError(st, "amamg_server_create failed")
        self.s = s
        self._out = {}          # request id -> (x array, psi copy is made by the library)

    def _check(self, st, ok=(OK,)):
        if st not in ok:
            raise AmamgError(st, (_lib.amamg_server_last_error(self.s) or b"").decode())
        return st

    def add_gauge(self, links: np.ndarray) -> int:
        """links: float64 [2][nt][nx][2] (ABI layout); returns the gauge id."""
        a = np.ascontiguousarray(links, dtype=np.float64)
        gid = C.c_int32()
        self._check(_lib.amamg_server_add_gauge(self.s, a.shape[1], a.shape[2], _ptr(a), C.byref(gid)))
        return gid.value

    def set_reference_mass(self, gauge_id: int, m_ref: float):
        """Later requests on the gauge use hierarchies derived from one set up at m_ref (NaN:
        a setup per mass)."""
        self._check(_lib.amamg_server_set_reference_mass(self.s, gauge_id, C.c_double(m_ref)))

    def submit(self, gauge_id: int, m0: float, psi: np.ndarray, setup: SetupParams | None = None) -> int:
        """psi: float64 [nrhs][nt][nx][2][2]; returns the request id.  The solution is returned
        by poll()."""
        a = np.ascontiguousarray(psi, dtype=np.float64)
        x = np.zeros_like(a)
        rid = C.c_uint64()
        self._check(_lib.amamg_server_submit(self.s, gauge_id, m0, C.byref(setup) if setup else None,
                                             a.shape[0], _ptr(a), _ptr(x), C.byref(rid)))
        self._out[rid.value] = x
        return rid.value

    def poll(self, capacity: int = 256):
        """Finished requests: list of (RequestInfo, x)."""
        buf = (RequestInfo * capacity)()
        n = C.c_int32()
        self._check(_lib.amamg_server_poll(self.s, buf, capacity, C.byref(n)))
        return [(buf[i], self._out.pop(buf[i].id)) for i in range(n.value)]

    def wait(self, timeout_s: float = 600.0) -> bool:
        """True when nothing is outstanding, False on timeout."""
        return self._check(_lib.amamg_server_wait(self.s, timeout_s), ok=(OK, PENDING)) == OK

    def stats(self) -> ServerCounters:
        c = ServerCounters()
        self._check(_lib.amamg_server_stats(self.s, C.byref(c)))
        return c

    def close(self):
        if self.s:
            _lib.amamg_server_destroy(self.s)
            self.s = None
