"""ctypes binding of libedf.so (argument marshalling only; every numerical step
runs in the library's HIP kernels).  Names follow the C-ABI in include/edf.h."""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libedf.so")

EDF_OK = 0
STATUS_NAMES = {1: "EDF_ERR_ARG", 2: "EDF_ERR_OOM", 3: "EDF_ERR_HIP", 4: "EDF_ERR_STATE",
                5: "EDF_ERR_NO_CONVERGENCE", 6: "EDF_ERR_NONFINITE"}
PREC_F64, PREC_MIXED, PREC_MIXED_F16 = 0, 1, 2
SMOOTHER_POINT, SMOOTHER_LINE = 0, 1
SAMPLE_OK, SAMPLE_NEWTON_FAIL, SAMPLE_LINEAR_FAIL, SAMPLE_NONFINITE = 0, 1, 2, 3
SAMPLE_INADMISSIBLE = 4
N_XI = {0: 0, 1: 1, 2: 4, 3: 3}


class EDFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class GroupDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("n_levels", C.c_int32), ("n_samples", C.c_int32)]


class PhysicsC(C.Structure):
    _fields_ = [("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("rho0", C.c_double), ("rho1", C.c_double), ("mu", C.c_double),
                ("g", C.c_double), ("Dm", C.c_double), ("phi_mean", C.c_double),
                ("K_mean", C.c_double), ("patch", C.c_double * 4),
                ("field_model", C.c_int32), ("n_xi", C.c_int32)]


class SolverOpts(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("newton_atol", C.c_double),
                ("lin_rtol", C.c_double), ("newton_max_it", C.c_int32),
                ("ls_max_halvings", C.c_int32), ("lin_max_it", C.c_int32),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("precision", C.c_int32),
                ("check_every", C.c_int32), ("dt_max_halvings", C.c_int32),
                ("forcing", C.c_int32), ("concurrent_groups", C.c_int32),
                ("graph_vcycle", C.c_int32), ("substep_memory", C.c_int32),
                ("smoother", C.c_int32), ("matrix_free", C.c_int32), ("predictor", C.c_int32),
                ("lag_preconditioner", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_its", C.c_int32), ("lin_its", C.c_int32),
                ("ls_halvings", C.c_int32), ("substeps", C.c_int32), ("retries", C.c_int32),
                ("steps_total", C.c_int32), ("split_total", C.c_int32),
                ("substeps_total", C.c_int32), ("retries_total", C.c_int32),
                ("failed_step", C.c_int32), ("predicted", C.c_int32),
                ("defect0", C.c_double), ("defect", C.c_double),
                ("salt_balance_err", C.c_double), ("liquid_balance_err", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class QoiC(C.Structure):
    _fields_ = [("box", C.c_double * 6), ("rtol", C.c_double), ("kind", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGS = {
    "edf_create_problem": [C.POINTER(PhysicsC), C.POINTER(GroupDesc), C.c_int32,
                           C.POINTER(SolverOpts), C.c_void_p, C.POINTER(C.c_void_p)],
    "edf_set_parameters": [_P, _D],
    "edf_set_state": [_P, C.c_int32, C.c_void_p, C.c_int32],
    "edf_get_state": [_P, C.c_int32, C.c_void_p, C.c_int32],
    "edf_step": [_P, C.c_double, C.POINTER(StepStats)],
    "edf_solve": [_P, C.c_double, C.c_int32, C.c_int32, C.POINTER(StepStats)],
    "edf_moments": [_P, C.c_int32, C.c_int32, C.c_int32, C.c_double, _D, _D, _D, _D],
    "edf_moments_noalloc": [_P, C.c_int32, C.c_int32, C.c_int32, C.c_double, _D, _D, _D, _D],
    "edf_group_moments": [_P, C.c_int32, C.c_double, _D, _D, _D, _D],
    "edf_residual": [_P, C.c_int32, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_int32],
    "edf_get_jacobian": [_P, C.c_int32, _D, C.c_double, C.c_int32, _D],
    "edf_apply_vcycle": [_P, C.c_int32, C.c_double, _D, _D],
    "edf_apply_jacobian": [_P, C.c_int32, _D, _D],
    "edf_adjoint": [_P, C.POINTER(QoiC), _D, _D],
    "edf_gpc_project": [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _D,
                        C.POINTER(C.c_int32), _D, _D, _D, _D],
    "edf_gpc_exceed": [_P, C.c_int32, _D, C.c_double, _D, _D],
    "edf_autotune": [_P, C.c_double],
    "edf_get_tuning": [_P, C.c_int32, C.POINTER(C.c_int32), _D],
    "edf_set_tuning": [_P, C.c_int32, C.c_int32],
    "edf_get_line_tiles": [_P, C.c_int32, C.POINTER(C.c_int32)],
    "edf_set_line_tiles": [_P, C.c_int32, C.POINTER(C.c_int32)],
    "edf_profile": [_P, C.c_int32, _D],
    "edf_last_error": [_P],
    "edf_destroy": [_P],
}
EXPORTS = tuple(_SIGS)


def load_library(path: str = LIB_PATH):
    """Loads libedf.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1906_01632_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    lib = C.CDLL(path)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    lib.edf_last_error.restype = C.c_char_p
    lib.edf_destroy.restype = None
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _physics_c(phys: dict) -> PhysicsC:
    p = PhysicsC()
    for k in ("lx", "ly", "lz", "rho0", "rho1", "mu", "g", "Dm", "phi_mean", "K_mean"):
        setattr(p, k, float(phys[k]))
    for i, v in enumerate(phys["patch"]):
        p.patch[i] = float(v)
    p.field_model = int(phys.get("field_model", 0))
    p.n_xi = int(phys.get("n_xi", N_XI[p.field_model]))
    return p


def default_options(**over) -> dict:
    o = dict(newton_rtol=1e-10, newton_atol=0.0, lin_rtol=1e-6, newton_max_it=20,
             ls_max_halvings=5, lin_max_it=200, nu_pre=1, nu_post=1, precision=PREC_F64,
             check_every=4, dt_max_halvings=4, forcing=0, concurrent_groups=0, graph_vcycle=0,
             substep_memory=0, smoother=1, matrix_free=1, predictor=0,
             lag_preconditioner=0)
    o.update(over)
    return o


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # torch missing: the library uses the default stream
        pass
    return C.c_void_p(None)


def _is_device(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


class Problem:
    """A batch of Elder-box samples in resolution groups (edf_create_problem)."""

    def __init__(self, phys: dict, groups, opts: dict | None = None, stream=None):
        lib = load_library()
        self._lib = lib
        self.phys = dict(phys)
        self.groups = [tuple(int(v) for v in g) for g in groups]  # (nx, ny, nz, levels, S)
        o = default_options(**(opts or {}))
        self.opts = o
        gd = (GroupDesc * len(self.groups))(*[GroupDesc(*g) for g in self.groups])
        so = SolverOpts()
        for k, v in o.items():
            setattr(so, k, v)
        self._pc = _physics_c(phys)
        h = C.c_void_p()
        st = _current_stream() if stream is None else C.c_void_p(stream)
        rc = lib.edf_create_problem(C.byref(self._pc), gd, len(self.groups), C.byref(so), st,
                                    C.byref(h))
        if rc != EDF_OK:
            raise EDFError(rc, "edf_create_problem failed (see stderr)")
        self._h = h
        self.n_xi = self._pc.n_xi
        self.S = sum(g[4] for g in self.groups)
        self.offsets = np.cumsum([0] + [g[4] for g in self.groups])

    # -- helpers ----------------------------------------------------------
    def _check(self, rc):
        if rc != EDF_OK:
            raise EDFError(rc, self._lib.edf_last_error(self._h).decode())

    def group_of(self, sample: int) -> int:
        return int(np.searchsorted(self.offsets, sample, side="right") - 1)

    def n_vertices(self, sample: int) -> int:
        nx, ny, nz = self.groups[self.group_of(sample)][:3]
        return nx * ny * nz

    # -- C-ABI ------------------------------------------------------------
    def set_parameters(self, xi):
        xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(self.S, max(self.n_xi, 0)))
        self._check(self._lib.edf_set_parameters(self._h, _dptr(xi) if xi.size else None))

    def set_state(self, sample: int, pc):
        if _is_device(pc):
            self._check(self._lib.edf_set_state(self._h, sample, C.c_void_p(pc.data_ptr()), 1))
        else:
            a = np.ascontiguousarray(np.asarray(pc, dtype=np.float64).reshape(-1))
            assert a.size == 2 * self.n_vertices(sample)
            self._check(self._lib.edf_set_state(self._h, sample, a.ctypes.data_as(C.c_void_p), 0))

    def get_state(self, sample: int, out=None):
        if out is not None and _is_device(out):
            self._check(self._lib.edf_get_state(self._h, sample, C.c_void_p(out.data_ptr()), 1))
            return out
        a = np.empty(2 * self.n_vertices(sample))
        self._check(self._lib.edf_get_state(self._h, sample, a.ctypes.data_as(C.c_void_p), 0))
        nx, ny, nz = self.groups[self.group_of(sample)][:3]
        return a.reshape(nz, ny, nx, 2)

    def step(self, dt: float):
        st = (StepStats * self.S)()
        self._check(self._lib.edf_step(self._h, float(dt), st))
        return [s.as_dict() for s in st]

    def solve(self, dt: float, n_steps: int, checkpoint_every: int = 0, stats: bool = True):
        """n_steps steps (edf_solve); checkpoint_every > 0 records the trajectory for
        adjoint().  Returns the last step's statistics."""
        st = (StepStats * self.S)() if stats else None
        self._check(self._lib.edf_solve(self._h, float(dt), int(n_steps), int(checkpoint_every),
                                        st))
        return [s.as_dict() for s in st] if stats else None

    def moments(self, common, threshold=0.5, weights=None, noalloc=False):
        """Mean, variance and P(c > threshold) on the common grid (edf_moments, or
        edf_moments_noalloc, which allocates no device memory)."""
        cx, cy, cz = common
        n = cx * cy * cz
        mean, var, exc = np.empty(n), np.empty(n), np.empty(n)
        w = None
        if weights is not None:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
            assert w.size == self.S
        fn = self._lib.edf_moments_noalloc if noalloc else self._lib.edf_moments
        self._check(fn(self._h, cx, cy, cz, float(threshold), _dptr(w) if w is not None else None,
                       _dptr(mean), _dptr(var), _dptr(exc)))
        shape = (cz, cy, cx)
        return mean.reshape(shape), var.reshape(shape), exc.reshape(shape)

    def group_moments(self, group: int, threshold=0.5, weights=None):
        """Mean, variance and P(c > threshold) of one group's samples on the group's own
        grid (edf_group_moments); weights in the group's sample order."""
        nx, ny, nz = self.groups[group][:3]
        n = nx * ny * nz
        mean, var, exc = np.empty(n), np.empty(n), np.empty(n)
        w = None
        if weights is not None:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
            assert w.size == self.groups[group][4]
        self._check(self._lib.edf_group_moments(self._h, int(group), float(threshold),
                                                _dptr(w) if w is not None else None,
                                                _dptr(mean), _dptr(var), _dptr(exc)))
        shape = (nz, ny, nx)
        return mean.reshape(shape), var.reshape(shape), exc.reshape(shape)

    def gpc_project(self, group: int, common, degree: int, weights, truncation: int = 0,
                    coefficients: bool = True):
        """Polynomial chaos surrogate of the group's samples (edf_gpc_project): returns a
        dict with n_coef, coef [n_coef, cz, cy, cx] (if asked), mean, var [cz, cy, cx] and
        kernel_ms (the projection kernel's duration)."""
        cx, cy, cz = common
        n = cx * cy * cz
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        assert w.size == self.groups[group][4]
        nc = C.c_int32()
        ms = C.c_double()
        coef = np.empty(128 * n) if coefficients else None
        mean, var = np.empty(n), np.empty(n)
        self._check(self._lib.edf_gpc_project(
            self._h, group, cx, cy, cz, int(degree), int(truncation), _dptr(w), C.byref(nc),
            _dptr(coef) if coef is not None else None, _dptr(mean), _dptr(var),
            C.cast(C.pointer(ms), _D)))
        shape = (cz, cy, cx)
        out = {"n_coef": nc.value, "mean": mean.reshape(shape), "var": var.reshape(shape),
               "kernel_ms": ms.value}
        if coef is not None:
            out["coef"] = coef[:nc.value * n].reshape((nc.value,) + shape)
        return out

    def gpc_exceed(self, theta, threshold: float, common):
        """P(c > threshold) of the last surrogate sampled at points theta [N_s, M]
        (edf_gpc_exceed); returns (prob [cz, cy, cx], kernel_ms)."""
        t = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        cx, cy, cz = common
        prob = np.empty(cx * cy * cz)
        ms = C.c_double()
        self._check(self._lib.edf_gpc_exceed(self._h, t.shape[0], _dptr(t), float(threshold),
                                             _dptr(prob), C.cast(C.pointer(ms), _D)))
        return prob.reshape(cz, cy, cx), ms.value

    def adjoint(self, box, rtol: float = 0.0):
        """Salt mass J in `box` (x0, x1, y0, y1, z0, z1) at the end of the trajectory
        recorded by the last solve(..., checkpoint_every > 0), and dJ/dxi by the discrete
        adjoint (edf_adjoint) with its solves to rtol (0: the library's default 1e-12).
        Returns (J [S], dJ [S, n_xi])."""
        q = QoiC()
        for i, v in enumerate(box):
            q.box[i] = float(v)
        q.rtol = float(rtol)
        J = np.empty(self.S)
        g = np.empty((self.S, self.n_xi))
        self._check(self._lib.edf_adjoint(self._h, C.byref(q), _dptr(J), _dptr(g)))
        return J, g

    def gradient(self, box, dt: float, n_steps: int, checkpoint_every: int = 10,
                 rtol: float = 0.0):
        """solve() with checkpoints, then adjoint(): (J, dJ/dxi) after n_steps steps."""
        self.solve(dt, n_steps, checkpoint_every=min(max(1, checkpoint_every), max(n_steps, 1)),
                   stats=False)
        return self.adjoint(box, rtol)

    def residual(self, sample: int, u, u_old, dt: float):
        a = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1))
        b = np.ascontiguousarray(np.asarray(u_old, dtype=np.float64).reshape(-1))
        F = np.empty_like(a)
        self._check(self._lib.edf_residual(self._h, sample, a.ctypes.data_as(C.c_void_p),
                                           b.ctypes.data_as(C.c_void_p), float(dt),
                                           F.ctypes.data_as(C.c_void_p), 0))
        return F.reshape(np.shape(u))

    def get_jacobian(self, sample: int, u, dt: float, level: int = 0):
        """Scaled Jacobian as out[27][2][2][N_level] (see include/edf.h)."""
        a = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(-1))
        nx, ny, nz = self.groups[self.group_of(sample)][:3]
        for _ in range(level):
            nx, ny, nz = (nx - 1) // 2 + 1, (ny - 1) // 2 + 1, (nz - 1) // 2 + 1
        out = np.empty(108 * nx * ny * nz)
        self._check(self._lib.edf_get_jacobian(self._h, sample, _dptr(a), float(dt), level,
                                               _dptr(out)))
        return out.reshape(27, 2, 2, nz, ny, nx)

    def apply_vcycle(self, group: int, dt: float, x):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        y = np.empty_like(a)
        self._check(self._lib.edf_apply_vcycle(self._h, group, float(dt), _dptr(a), _dptr(y)))
        return y

    def apply_jacobian(self, group: int, x):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        y = np.empty_like(a)
        self._check(self._lib.edf_apply_jacobian(self._h, group, _dptr(a), _dptr(y)))
        return y

    def profile(self, enable: bool):
        """Starts (True) or stops (False) event timing of the smoother launches and of
        whole V-cycles; returns the totals since the last start."""
        out = np.zeros(16)
        self._check(self._lib.edf_profile(self._h, int(bool(enable)), _dptr(out)))
        return {"launches": int(out[0]), "ms": float(out[1]), "bytes": float(out[2]),
                "vcycles": int(out[3]), "vcycle_ms": float(out[4]), "vcycle_bytes": float(out[5]),
                "all_launches": int(out[6]), "all_bytes": float(out[7]),
                "large_launches": int(out[8]), "large_ms": float(out[9]),
                "large_bytes": float(out[10]), "large_all_launches": int(out[11]),
                "large_all_bytes": float(out[12]), "large_vcycles": int(out[13]),
                "large_vcycle_ms": float(out[14]), "large_vcycle_bytes": float(out[15])}

    def tuning_key(self) -> str:
        """What a V-cycle tuning depends on: the groups, the V-cycle's precision, smoother
        and sweep counts, and the device."""
        try:
            import torch
            dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
        except Exception:
            dev = "unknown"
        o = self.opts
        return json.dumps({"groups": [list(g) for g in self.groups], "precision": o["precision"],
                           "smoother": o["smoother"], "nu": [o["nu_pre"], o["nu_post"]],
                           "device": dev}, sort_keys=True)

    def autotune(self, dt: float, cache: str | None = None):
        """edf_autotune; with `cache` (a JSON file), a tuning stored there under this
        problem's tuning_key() is applied instead, and a new one is stored."""
        key = self.tuning_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                for g, rec in enumerate(table[key]):
                    self.set_tuning(g, rec["fuse_from"])
                    self.set_line_tiles(g, rec["line_tiles"])
                return False
        self._check(self._lib.edf_autotune(self._h, float(dt)))
        if cache:
            table[key] = [{"fuse_from": self.tuning(g)[0], "line_tiles": self.line_tiles(g),
                           "vcycle_ms": [float(v) for v in self.tuning(g)[1]]}
                          for g in range(len(self.groups))]
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return True

    def line_tiles(self, group: int):
        """Columns per workgroup of each level's line sweep (0: no line smoothing)."""
        L = self.groups[group][3]
        out = (C.c_int32 * L)()
        self._check(self._lib.edf_get_line_tiles(self._h, group, out))
        return [int(v) for v in out]

    def set_line_tiles(self, group: int, cols):
        L = self.groups[group][3]
        arr = (C.c_int32 * L)(*[int(v) for v in cols])
        self._check(self._lib.edf_set_line_tiles(self._h, group, arr))

    def tuning(self, group: int):
        """(first fused level, V-cycle ms per candidate level or -1) of a group."""
        f = C.c_int32()
        L = self.groups[group][3]
        ms = np.empty(L)
        self._check(self._lib.edf_get_tuning(self._h, group, C.byref(f), _dptr(ms)))
        return int(f.value), ms

    def set_tuning(self, group: int, fuse_from: int):
        self._check(self._lib.edf_set_tuning(self._h, group, fuse_from))

    def destroy(self):
        if getattr(self, "_h", None):
            self._lib.edf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()


def create_problem(phys: dict, groups, opts: dict | None = None, stream=None) -> Problem:
    return Problem(phys, groups, opts, stream)
