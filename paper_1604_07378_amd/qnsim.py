"""Python binding of libqnsim (argument marshalling only).

Every computation of the time step runs in the HIP library; this module only
converts NumPy arrays / torch tensors into the plain pointers and sizes of
the C ABI declared in include/qnsim.h. There is no fallback: if the compiled
library is missing the import of the binding fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqnsim.so")

KERNEL_ELEMENT, KERNEL_GATHER, KERNEL_SOLVE = 0, 1, 2
QNSIM_FP64 = 0
QNSIM_MIXED = 1
DIR_LBFGS, DIR_CHEBYSHEV = 0, 1
NEOHOOKEAN, STVK, SPLINE, COROTATED, POLYNOMIAL, MOONEY_RIVLIN = 0, 1, 2, 3, 4, 5

ERRORS = {
    -1: "QNSIM_E_INVALID", -2: "QNSIM_E_NONFINITE", -3: "QNSIM_E_DEGENERATE",
    -4: "QNSIM_E_INVERTED", -5: "QNSIM_E_STIFFNESS", -6: "QNSIM_E_NOT_SPD",
    -7: "QNSIM_E_H_MISMATCH", -8: "QNSIM_E_STATE", -9: "QNSIM_E_NOMEM",
    -10: "QNSIM_E_DEVICE", -11: "QNSIM_E_BUDGET",
}


class QnsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("history", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("dense_top", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("backtrack", ctypes.c_double),
                ("fit_lo", ctypes.c_double), ("fit_hi", ctypes.c_double),
                ("gravity", ctypes.c_double * 3),
                ("subtree_cap", ctypes.c_int32), ("level_merge", ctypes.c_int32),
                ("step_graph", ctypes.c_int32), ("trials_per_cycle", ctypes.c_int32),
                ("direction", ctypes.c_int32), ("cheb_delay", ctypes.c_int32),
                ("cheb_rho", ctypes.c_double), ("device_factor", ctypes.c_int32),
                ("elem_tile", ctypes.c_int32)]


class MaterialC(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mu", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("density", ctypes.c_double), ("spline_d2", ctypes.c_double * 8),
                ("fiber_kappa", ctypes.c_double), ("fiber_dir", ctypes.c_double * 3),
                ("mu2", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations_run", ctypes.c_int32), ("ls_trials", ctypes.c_int32),
                ("ls_exhausted", ctypes.c_int32), ("lbfgs_skipped", ctypes.c_int32),
                ("fallbacks", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("g_first", ctypes.c_double), ("g_last", ctypes.c_double),
                ("grad_norm_first", ctypes.c_double), ("grad_norm_last", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class TuneInfo(ctypes.Structure):
    _fields_ = [("dense_top", ctypes.c_int32), ("subtree_cap", ctypes.c_int32),
                ("level_merge", ctypes.c_int32), ("elem_tile", ctypes.c_int32),
                ("trials_per_cycle", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("schedule_ms", ctypes.c_double * 4), ("tile_ms", ctypes.c_double * 3),
                ("trials_ms", ctypes.c_double * 3)]

    def as_dict(self):
        return dict(dense_top=self.dense_top, subtree_cap=self.subtree_cap,
                    level_merge=self.level_merge, elem_tile=self.elem_tile,
                    trials_per_cycle=self.trials_per_cycle,
                    schedule_ms=list(self.schedule_ms), tile_ms=list(self.tile_ms),
                    trials_ms=list(self.trials_ms))


class FactorInfo(ctypes.Structure):
    _fields_ = [("n_free", ctypes.c_int32), ("n_supernodes", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("max_front", ctypes.c_int32),
                ("dense_top_cols", ctypes.c_int32), ("subtree_levels", ctypes.c_int32),
                ("nnz_L", ctypes.c_int64), ("nnz_L_exact", ctypes.c_int64),
                ("factor_bytes", ctypes.c_int64), ("factor_flops", ctypes.c_double),
                ("prepare_seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_verts", ctypes.c_int32), ("rest_xyz", ctypes.c_void_p),
                ("n_tets", ctypes.c_int32), ("tets", ctypes.c_void_p),
                ("n_pinned", ctypes.c_int32), ("pinned", ctypes.c_void_p),
                ("n_mat", ctypes.c_int32), ("mats", ctypes.c_void_p),
                ("tet_mat", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("v0", ctypes.c_void_p)]


class PoolInfo(ctypes.Structure):
    _fields_ = [("sims_staged", ctypes.c_int32), ("sims_resident", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("serving", ctypes.c_int32),
                ("budget_bytes", ctypes.c_int64), ("used_bytes", ctypes.c_int64),
                ("steps_done", ctypes.c_int64), ("batches_done", ctypes.c_int64),
                ("nnz_L", ctypes.c_int64), ("n_free", ctypes.c_int64), ("n_tets", ctypes.c_int64),
                ("groups_made", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int32

# name -> (restype, argtypes); every entry point of include/qnsim.h
SIGNATURES = {
    "qnsim_options_default": (ctypes.c_int, [ctypes.POINTER(Options)]),
    "qnsim_create": (ctypes.c_int, [ctypes.POINTER(Options), ctypes.POINTER(_P)]),
    "qnsim_destroy": (None, [_P]),
    "qnsim_set_mesh": (ctypes.c_int, [_P, _I, _P, _I, _P]),
    "qnsim_set_pinned": (ctypes.c_int, [_P, _I, _P]),
    "qnsim_set_materials": (ctypes.c_int, [_P, _I, ctypes.POINTER(MaterialC), _P]),
    "qnsim_prepare": (ctypes.c_int, [_P, _D]),
    "qnsim_analyze": (ctypes.c_int, [_P, _D]),
    "qnsim_step": (ctypes.c_int, [_P, _P, _P, _D, _P, _P, _P, ctypes.POINTER(Stats)]),
    "qnsim_step_device": (ctypes.c_int, [_P, _P, _P, _D, _P, _P, _P, _P, ctypes.POINTER(Stats)]),
    "qnsim_run_device": (ctypes.c_int, [_P, _P, _P, _D, _P, _I, _P, ctypes.POINTER(Stats)]),
    "qnsim_set_diagnostics": (ctypes.c_int, [_P, _I]),
    "qnsim_set_colliders": (ctypes.c_int, [_P, _I, _P, _D]),
    "qnsim_get_stiffness": (ctypes.c_int, [_P, _P]),
    "qnsim_get_masses": (ctypes.c_int, [_P, _P]),
    "qnsim_get_factor_info": (ctypes.c_int, [_P, ctypes.POINTER(FactorInfo)]),
    "qnsim_export_factor": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "qnsim_eval_device": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_D), _P, _P]),
    "qnsim_element_stress_device": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "qnsim_solve_device": (ctypes.c_int, [_P, _P, _P, _P]),
    "qnsim_solve_device_noalloc": (ctypes.c_int, [_P, _P, _P, _P]),
    "qnsim_refactor": (ctypes.c_int, [_P, _D, ctypes.POINTER(_D)]),
    "qnsim_time_kernel": (ctypes.c_int, [_P, _I, _I, ctypes.POINTER(_D)]),
    "qnsim_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "qnsim_last_error": (ctypes.c_char_p, [_P]),
    "qnsim_pool_create": (ctypes.c_int, [ctypes.POINTER(Options), _D, ctypes.c_int64,
                                         ctypes.POINTER(_P)]),
    "qnsim_pool_destroy": (None, [_P]),
    "qnsim_pool_add": (ctypes.c_int, [_P, _I, ctypes.POINTER(MeshDesc), _P]),
    "qnsim_pool_commit": (ctypes.c_int, [_P, _I, ctypes.POINTER(_I)]),
    "qnsim_pool_remove": (ctypes.c_int, [_P, _I]),
    "qnsim_pool_step": (ctypes.c_int, [_P, _I, _P, ctypes.POINTER(Stats)]),
    "qnsim_pool_get_state": (ctypes.c_int, [_P, _I, _P, _P]),
    "qnsim_pool_set_state": (ctypes.c_int, [_P, _I, _P, _P]),
    "qnsim_pool_serve_start": (ctypes.c_int, [_P, _I]),
    "qnsim_pool_submit": (ctypes.c_int, [_P, _I, ctypes.POINTER(ctypes.c_int64)]),
    "qnsim_pool_wait": (ctypes.c_int, [_P, ctypes.c_int64, _D, ctypes.POINTER(Stats),
                                       ctypes.POINTER(_D)]),
    "qnsim_pool_serve_stop": (ctypes.c_int, [_P]),
    "qnsim_pool_status": (ctypes.c_int, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "qnsim_pool_get_info": (ctypes.c_int, [_P, ctypes.POINTER(PoolInfo)]),
    "qnsim_pool_last_error": (ctypes.c_char_p, [_P]),
    "qnsim_pool_time_kernel": (ctypes.c_int, [_P, _I, _I, _I, ctypes.POINTER(_D)]),
    "qnsim_pool_set_h": (ctypes.c_int, [_P, _D, ctypes.POINTER(_D)]),
    "qnsim_pool_set_force": (ctypes.c_int, [_P, _I, _P]),
    "qnsim_pool_submit_force": (ctypes.c_int, [_P, _I, _P, ctypes.POINTER(ctypes.c_int64)]),
    "qnsim_tune": (ctypes.c_int, [_P, _D, _P, _P, _I, _I, ctypes.POINTER(TuneInfo)]),
    "qnsim_pool_tune": (ctypes.c_int, [_P, _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_D),
                                       ctypes.POINTER(_I), ctypes.POINTER(_D)]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libqnsim.so (built in-tree by build_lib.build()); no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "paper_1604_07378_amd.build_lib.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_options() -> Options:
    o = Options()
    load_library().qnsim_options_default(ctypes.byref(o))
    return o


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or t.dtype.__str__() != "torch.float64" or not t.is_contiguous():
        raise ValueError("device arrays must be contiguous float64 CUDA (HIP) tensors")
    return t.data_ptr()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _material_array(materials: Sequence):
    arr = (MaterialC * len(materials))()
    for i, m in enumerate(materials):
        get = (lambda k: m[k]) if isinstance(m, dict) else (lambda k: getattr(m, k))
        arr[i].type = int(get("type"))
        arr[i].mu = float(get("mu"))
        arr[i].lambda_ = float(get("lam"))
        arr[i].density = float(get("density"))
        d2 = get("spline_d2") if not isinstance(m, dict) else m.get("spline_d2")
        if d2 is not None:
            for j, val in enumerate(np.asarray(d2, dtype=np.float64)):
                arr[i].spline_d2[j] = float(val)
        opt = (lambda k: m.get(k)) if isinstance(m, dict) else (lambda k: getattr(m, k, None))
        if opt("fiber_kappa"):
            arr[i].fiber_kappa = float(opt("fiber_kappa"))
            for j, val in enumerate(np.asarray(opt("fiber_dir"), dtype=np.float64)):
                arr[i].fiber_dir[j] = float(val)
        if opt("mu2"):
            arr[i].mu2 = float(opt("mu2"))
    return arr


def _options_with(options: Optional[Options], overrides: dict) -> Options:
    o = options if options is not None else default_options()
    known = {f for f, _ in Options._fields_}
    for k, v in overrides.items():
        if k not in known:
            raise TypeError(f"unknown solver option {k!r}")
        if k == "gravity":
            o.gravity = (ctypes.c_double * 3)(*v)
        else:
            setattr(o, k, v)
    return o


class Sim:
    """One simulated mesh (a qnsim_t context)."""

    def __init__(self, options: Optional[Options] = None, **overrides):
        self._lib = load_library()
        o = _options_with(options, overrides)
        self.options = o
        h = ctypes.c_void_p()
        self._check(self._lib.qnsim_create(ctypes.byref(o), ctypes.byref(h)), None)
        self._h = h
        self.n = self.T = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.qnsim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, ctx="self"):
        if rc != 0:
            msg = ""
            if ctx is not None and getattr(self, "_h", None):
                msg = self._lib.qnsim_last_error(self._h).decode()
            raise QnsimError(rc, msg or self._lib.qnsim_strerror(rc).decode())

    # ---- setup ------------------------------------------------------------
    def set_mesh(self, rest, tets):
        rest = _f64(rest)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.n, self.T = rest.shape[0], tets.shape[0]
        self._check(self._lib.qnsim_set_mesh(self._h, self.n, _ptr(rest), self.T, _ptr(tets)))

    def set_pinned(self, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        self._check(self._lib.qnsim_set_pinned(self._h, idx.size, _ptr(idx) if idx.size else None))

    def set_materials(self, materials: Sequence, tet_mat=None):
        arr = _material_array(materials)
        tm = None
        if tet_mat is not None:
            tm = np.ascontiguousarray(tet_mat, dtype=np.int32)
        self._check(self._lib.qnsim_set_materials(self._h, len(materials), arr,
                                                  _ptr(tm) if tm is not None else None))

    def analyze(self, h: float):
        self._check(self._lib.qnsim_analyze(self._h, float(h)))

    def prepare(self, h: float):
        self._check(self._lib.qnsim_prepare(self._h, float(h)))

    def set_colliders(self, planes, stiffness: float):
        """planes: (p, 4) rows (nx, ny, nz, c) of half-spaces n . x >= c."""
        planes = _f64(planes).reshape(-1, 4)
        self._check(self._lib.qnsim_set_colliders(self._h, planes.shape[0],
                                                  _ptr(planes) if planes.size else None,
                                                  float(stiffness)))

    def set_diagnostics(self, final_gradient: bool):
        self._check(self._lib.qnsim_set_diagnostics(self._h, 1 if final_gradient else 0))

    # ---- queries ----------------------------------------------------------
    def stiffness(self) -> np.ndarray:
        k = np.empty(self.T)
        self._check(self._lib.qnsim_get_stiffness(self._h, _ptr(k)))
        return k

    def masses(self) -> np.ndarray:
        m = np.empty(self.n)
        self._check(self._lib.qnsim_get_masses(self._h, _ptr(m)))
        return m

    def factor_info(self) -> dict:
        fi = FactorInfo()
        self._check(self._lib.qnsim_get_factor_info(self._h, ctypes.byref(fi)))
        return fi.as_dict()

    def export_factor(self):
        info = self.factor_info()
        nf, nnz = info["n_free"], info["nnz_L"]
        perm = np.empty(nf, dtype=np.int32)
        cp = np.empty(nf + 1, dtype=np.int64)
        ri = np.empty(nnz, dtype=np.int32)
        va = np.empty(nnz)
        self._check(self._lib.qnsim_export_factor(self._h, _ptr(perm), _ptr(cp), _ptr(ri), _ptr(va)))
        return perm, cp, ri, va

    # ---- steps --------------------------------------------------------------
    def step(self, x, v, h: float, f_ext=None):
        """One step from host arrays; returns (x', v', stats dict)."""
        x = _f64(x, (self.n, 3))
        v = _f64(v, (self.n, 3))
        f = _f64(f_ext, (self.n, 3)) if f_ext is not None else None
        xo = np.empty_like(x)
        vo = np.empty_like(v)
        st = Stats()
        self._check(self._lib.qnsim_step(self._h, _ptr(x), _ptr(v), float(h),
                                         _ptr(f) if f is not None else None,
                                         _ptr(xo), _ptr(vo), ctypes.byref(st)))
        return xo, vo, st.as_dict()

    def step_device(self, x, v, h: float, f_ext=None, x_out=None, v_out=None,
                    stream=None, stats: bool = True):
        """One step on torch device tensors (n x 3 float64); in place by default."""
        x_out = x if x_out is None else x_out
        v_out = v if v_out is None else v_out
        st = Stats()
        self._check(self._lib.qnsim_step_device(
            self._h, _tptr(x), _tptr(v), float(h), _tptr(f_ext), _tptr(x_out), _tptr(v_out),
            _stream_ptr(stream), ctypes.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def run_device(self, x, v, h: float, steps: int, f_ext=None, stream=None):
        st = Stats()
        self._check(self._lib.qnsim_run_device(self._h, _tptr(x), _tptr(v), float(h),
                                               _tptr(f_ext), int(steps), _stream_ptr(stream),
                                               ctypes.byref(st)))
        return st.as_dict()

    def tune(self, x, v, h: float, reps: int = 3, schedule: bool = True, tile: bool = True,
             trials: bool = True) -> dict:
        """Keep the fastest solve schedule, element tile and line-search trials
        per cycle for steps from the device state (x, v) (torch n x 3 float64
        tensors, not modified)."""
        info = TuneInfo()
        what = (1 if schedule else 0) | (2 if tile else 0) | (4 if trials else 0)
        if what == 0:
            raise ValueError("nothing to tune")
        self._check(self._lib.qnsim_tune(self._h, float(h), _tptr(x), _tptr(v), int(reps), what,
                                         ctypes.byref(info)))
        return info.as_dict()

    def time_kernel(self, kernel: int, reps: int) -> float:
        """Mean milliseconds per launch of one step kernel (HIP events)."""
        ms = ctypes.c_double()
        self._check(self._lib.qnsim_time_kernel(self._h, int(kernel), int(reps), ctypes.byref(ms)))
        return ms.value

    # ---- kernel-level probes ------------------------------------------------
    def eval_device(self, x, y, grad_out, stream=None) -> float:
        g = ctypes.c_double()
        self._check(self._lib.qnsim_eval_device(self._h, _tptr(x), _tptr(y), ctypes.byref(g),
                                                _tptr(grad_out), _stream_ptr(stream)))
        return g.value

    def element_stress_device(self, x, psi_out, P_out, stream=None):
        self._check(self._lib.qnsim_element_stress_device(self._h, _tptr(x), _tptr(psi_out),
                                                          _tptr(P_out), _stream_ptr(stream)))

    def solve_device(self, q, r_out, stream=None):
        self._check(self._lib.qnsim_solve_device(self._h, _tptr(q), _tptr(r_out),
                                                 _stream_ptr(stream)))

    def solve_device_noalloc(self, q, r_out, stream=None):
        """As solve_device, with the working memory in the library's fixed
        device array (no allocation); stream-ordered."""
        self._check(self._lib.qnsim_solve_device_noalloc(self._h, _tptr(q), _tptr(r_out),
                                                         _stream_ptr(stream)))

    def refactor(self, h: float) -> float:
        """Refactor A for step size h on the device; returns the device time in ms."""
        ms = _D(0.0)
        self._check(self._lib.qnsim_refactor(self._h, float(h), ctypes.byref(ms)))
        return ms.value


def sim_from_workload(w, options: Optional[Options] = None, prepare: bool = True, **overrides):
    """Build a Sim from a workload description (rest, tets, pinned, materials...)."""
    if "gravity" not in overrides:
        overrides["gravity"] = tuple(w.gravity)
    s = Sim(options, **overrides)
    s.set_mesh(w.rest, w.tets)
    s.set_pinned(w.pinned)
    s.set_materials(_materials_of(w), w.tet_mat)
    if prepare:
        s.prepare(w.h)
    else:
        s.analyze(w.h)
    return s


def _materials_of(w):
    return [dict(type=m.type, mu=m.mu, lam=m.lam, density=m.density,
                 spline_d2=m.d2() if hasattr(m, "d2") else None,
                 fiber_kappa=getattr(m, "fiber_kappa", 0.0),
                 fiber_dir=getattr(m, "fiber_dir", None),
                 mu2=getattr(m, "mu2", 0.0)) for m in w.materials]


class Pool:
    """Resident simulations on one GPU (a qnsim_pool_t): batched steps of any
    subset, and the request loop that serves step requests."""

    def __init__(self, h: float, budget_bytes: int, options: Optional[Options] = None,
                 **overrides):
        self._lib = load_library()
        o = _options_with(options, overrides)
        self.options = o
        self.h = float(h)
        p = ctypes.c_void_p()
        self._p = None
        rc = self._lib.qnsim_pool_create(ctypes.byref(o), self.h, int(budget_bytes), ctypes.byref(p))
        if rc != 0:
            raise QnsimError(rc, self._lib.qnsim_strerror(rc).decode())
        self._p = p
        self.nverts = {}

    def close(self):
        if getattr(self, "_p", None):
            self._lib.qnsim_pool_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            msg = self._lib.qnsim_pool_last_error(self._p).decode() if self._p else ""
            raise QnsimError(rc, msg or self._lib.qnsim_strerror(rc).decode())

    def add(self, meshes: Sequence[dict]) -> list:
        """meshes: dicts with rest, tets, pinned, materials, tet_mat and
        optional x0, v0. Returns the new ids (staged)."""
        n = len(meshes)
        descs = (MeshDesc * n)()
        keep = []
        for i, m in enumerate(meshes):
            rest = _f64(m["rest"])
            tets = np.ascontiguousarray(m["tets"], dtype=np.int32)
            pinned = np.ascontiguousarray(m.get("pinned", np.zeros(0)), dtype=np.int32)
            mats = _material_array(m["materials"])
            tm = m.get("tet_mat")
            tm = np.ascontiguousarray(tm, dtype=np.int32) if tm is not None else None
            x0 = _f64(m["x0"], rest.shape) if m.get("x0") is not None else None
            v0 = _f64(m["v0"], rest.shape) if m.get("v0") is not None else None
            keep += [rest, tets, pinned, mats, tm, x0, v0]
            d = descs[i]
            d.n_verts, d.rest_xyz = rest.shape[0], rest.ctypes.data
            d.n_tets, d.tets = tets.shape[0], tets.ctypes.data
            d.n_pinned, d.pinned = pinned.size, (pinned.ctypes.data if pinned.size else None)
            d.n_mat, d.mats = len(m["materials"]), ctypes.addressof(mats)
            d.tet_mat = tm.ctypes.data if tm is not None else None
            d.x0 = x0.ctypes.data if x0 is not None else None
            d.v0 = v0.ctypes.data if v0 is not None else None
        ids = np.zeros(n, dtype=np.int32)
        self._check(self._lib.qnsim_pool_add(self._p, n, descs, _ptr(ids)))
        for i, m in enumerate(meshes):
            self.nverts[int(ids[i])] = int(np.asarray(m["rest"]).shape[0])
        return [int(i) for i in ids]

    def add_workloads(self, ws: Sequence) -> list:
        return self.add([dict(rest=w.rest, tets=w.tets, pinned=w.pinned,
                              materials=_materials_of(w), tet_mat=w.tet_mat,
                              x0=w.x0, v0=w.v0) for w in ws])

    def commit(self, max_group_sims: int = 0) -> int:
        n = ctypes.c_int32()
        self._check(self._lib.qnsim_pool_commit(self._p, int(max_group_sims), ctypes.byref(n)))
        return n.value

    def remove(self, sim_id: int):
        self._check(self._lib.qnsim_pool_remove(self._p, int(sim_id)))

    def step(self, ids: Sequence[int]) -> list:
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        st = (Stats * max(1, ids.size))()
        self._check(self._lib.qnsim_pool_step(self._p, ids.size, _ptr(ids), st))
        return [st[i].as_dict() for i in range(ids.size)]

    def set_force(self, sim_id: int, f_ext=None):
        """External force (n x 3, N) of a resident simulation for its later
        steps; None removes it."""
        n = self.nverts[int(sim_id)]
        f = _f64(f_ext, (n, 3)) if f_ext is not None else None
        self._check(self._lib.qnsim_pool_set_force(self._p, int(sim_id),
                                                   _ptr(f) if f is not None else None))

    def get_state(self, sim_id: int):
        n = self.nverts[int(sim_id)]
        x = np.zeros((n, 3)); v = np.zeros((n, 3))
        self._check(self._lib.qnsim_pool_get_state(self._p, int(sim_id), _ptr(x), _ptr(v)))
        return x, v

    def set_state(self, sim_id: int, x, v):
        n = self.nverts[int(sim_id)]
        x = _f64(x, (n, 3)); v = _f64(v, (n, 3))
        self._check(self._lib.qnsim_pool_set_state(self._p, int(sim_id), _ptr(x), _ptr(v)))

    def serve_start(self, lanes: int = 2):
        self._check(self._lib.qnsim_pool_serve_start(self._p, int(lanes)))

    def submit(self, sim_id: int) -> int:
        t = ctypes.c_int64()
        self._check(self._lib.qnsim_pool_submit(self._p, int(sim_id), ctypes.byref(t)))
        return t.value

    def submit_force(self, sim_id: int, f_ext) -> int:
        """Step request whose step uses f_ext (n x 3, N) in place of the
        simulation's own force."""
        n = self.nverts[int(sim_id)]
        f = _f64(f_ext, (n, 3))
        t = ctypes.c_int64()
        self._check(self._lib.qnsim_pool_submit_force(self._p, int(sim_id), _ptr(f), ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_s: float = -1.0):
        st = Stats()
        lat = ctypes.c_double()
        self._check(self._lib.qnsim_pool_wait(self._p, int(ticket), float(timeout_s),
                                              ctypes.byref(st), ctypes.byref(lat)))
        return st.as_dict(), lat.value

    def serve_stop(self):
        self._check(self._lib.qnsim_pool_serve_stop(self._p))

    def time_kernel(self, group: int, kernel: int, reps: int) -> float:
        ms = ctypes.c_double()
        self._check(self._lib.qnsim_pool_time_kernel(self._p, int(group), int(kernel), int(reps),
                                                     ctypes.byref(ms)))
        return ms.value

    def set_h(self, h: float) -> float:
        """New time step for every simulation (A refactored on the device);
        returns the device milliseconds."""
        ms = ctypes.c_double()
        self._check(self._lib.qnsim_pool_set_h(self._p, float(h), ctypes.byref(ms)))
        return ms.value

    def tune(self, reps: int = 3, candidates=(128, 256, 512), trials: bool = False):
        """Element-tile autotuning of every resident group among the candidate
        tiles: returns the chosen tile per group (admission order, 0 for a
        group with no resident member) and the measured milliseconds per
        batched step for the tiles 128, 256, 512 (groups x 3, NaN where not
        measured). With trials, also the kept line-search trials per cycle per
        group and their milliseconds per step (for 1, 2, 3), as two more lists."""
        mask = sum({128: 1, 256: 2, 512: 4}[int(t)] for t in set(candidates))
        n = self.info()["groups_made"]
        tiles = (_I * max(n, 1))()
        ms = (_D * (3 * max(n, 1)))()
        tr = (_I * max(n, 1))()
        tms = (_D * (3 * max(n, 1)))()
        self._check(self._lib.qnsim_pool_tune(self._p, mask, int(reps), n, tiles, ms,
                                              tr if trials else None, tms if trials else None))
        out = ([int(tiles[i]) for i in range(n)], [[float(ms[3 * i + k]) for k in range(3)] for i in range(n)])
        if trials:
            out += ([int(tr[i]) for i in range(n)], [[float(tms[3 * i + k]) for k in range(3)] for i in range(n)])
        return out

    def status(self, sim_id: int):
        """('staged' | 'resident' | 'removed', group index or -1)."""
        st, g = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.qnsim_pool_status(self._p, int(sim_id), ctypes.byref(st),
                                                ctypes.byref(g)))
        return ("staged", "resident", "removed")[st.value], g.value

    def info(self) -> dict:
        i = PoolInfo()
        self._check(self._lib.qnsim_pool_get_info(self._p, ctypes.byref(i)))
        return i.as_dict()
