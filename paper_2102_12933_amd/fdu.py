"""ctypes binding of libfdu (include/fdu.h): argument marshalling only.

Every step of the residual runs in the HIP library; this module checks tensor
shapes, dtypes and devices, passes raw pointers and the current HIP stream, and
raises FduError with the library's message on a non-zero status.  Importing it
fails loudly when libfdu.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdu.so")

F64, F32 = 0, 1
_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "HIP", 3: "OOM", 4: "STATE", 5: "UNSUPPORTED", 6: "NUMERIC"}


class FduError(RuntimeError):
    def __init__(self, func, code, msg):
        super().__init__(f"{func}: FDU_ERR_{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("weno_eps", C.c_double), ("entropy_frac", C.c_double),
                ("weno_power", C.c_int), ("riemann", C.c_int), ("positivity", C.c_int),
                ("interpolation", C.c_int), ("uniform_weno", C.c_int)]


class PrepView(C.Structure):
    _fields_ = [("nv_total", C.c_int64), ("nv_real", C.c_int64), ("ne_flux", C.c_int64),
                ("nnz_v", C.c_int64), ("nnz_e", C.c_int64),
                ("perm", C.c_void_p), ("iperm", C.c_void_p), ("flux_edge", C.c_void_p),
                ("sten6", C.c_void_p), ("geo", C.c_void_p), ("vptr", C.c_void_p), ("vcol", C.c_void_p),
                ("wfg", C.c_void_p), ("eptr", C.c_void_p), ("ecol", C.c_void_p), ("we", C.c_void_p),
                ("hmin", C.c_void_p), ("ghost_src", C.c_void_p), ("ghost_refl", C.c_void_p),
                ("n_artificial", C.c_int64), ("artificial", C.c_void_p)]


P, I64, I32, D, VP = C.POINTER, C.c_int64, C.c_int, C.c_double, C.c_void_p
_SIGS = {
    "fdu_last_error": (C.c_char_p, []),
    "fdu_default_params": (None, [P(Params)]),
    "fdu_prep_build": (I32, [P(VP), I64, I64, VP, I64, VP, I64, VP, VP, VP, I32, D, D, I32, I32, I32, I32, I32]),
    "fdu_prep_view_get": (I32, [VP, P(PrepView)]),
    "fdu_prep_destroy": (None, [VP]),
    "fdu_create": (I32, [P(VP), I32, I32, P(Params)]),
    "fdu_destroy": (None, [VP]),
    "fdu_upload_edge_stencils": (I32, [VP, I64, I64, I64, VP, VP]),
    "fdu_upload_vertex_stencils": (I32, [VP, VP, VP, VP, VP, VP, VP, VP]),
    "fdu_upload_ghosts": (I32, [VP, I64, VP, VP]),
    "fdu_upload_prep": (I32, [VP, VP]),
    "fdu_upload_ghost_states": (I32, [VP, I64, VP]),
    "fdu_finalize": (I32, [VP]),
    "fdu_sizes": (I32, [VP, P(I64), P(I64), P(I64), P(I64), P(I64)]),
    "fdu_fill_ghosts": (I32, [VP, VP, VP]),
    "fdu_edge_fluxes": (I32, [VP, VP, VP, VP]),
    "fdu_residual": (I32, [VP, VP, VP, VP]),
    "fdu_cfl_dt": (I32, [VP, VP, D, VP, VP]),
    "fdu_rk_stage": (I32, [VP, I32, VP, VP, VP, VP, VP]),
    "fdu_rk_step": (I32, [VP, VP, VP, D, VP, VP]),
    "fdu_kernel_times": (I32, [VP, VP, VP, I32, VP, VP]),
    "fdu_kernel_timer_start": (I32, [VP, I32, I32]),
    "fdu_vertex_block_info": (I32, [VP, P(I32), P(I64), P(I32)]),
    "fdu_check_state": (I32, [VP, VP, P(I64), P(I64), VP]),
    "fdu_kernel_timer_stop": (I32, [VP, VP, VP]),
    "fdu_enable_adjoint": (I32, [VP]),
    "fdu_set_variants": (I32, [VP, I32, I32]),
    "fdu_get_variants": (I32, [VP, P(I32), P(I32), P(I32), P(I32)]),
    "fdu_autotune": (I32, [VP, VP, VP, I32, VP, VP]),
    "fdu_batch_create": (I32, [P(VP), VP, I32]),
    "fdu_batch_destroy": (None, [VP]),
    "fdu_batch_set_states": (I32, [VP, VP, VP]),
    "fdu_batch_set_schedule": (I32, [VP, I32, I32, I32, I32]),
    "fdu_batch_step": (I32, [VP, D, VP]),
    "fdu_batch_capture": (I32, [VP, D, I32, VP]),
    "fdu_batch_launch": (I32, [VP, VP]),
    "fdu_batch_status": (I32, [VP, P(I32), VP]),
    "fdu_batch_info": (I32, [VP, P(I32), P(I32), P(I32), P(I32), P(I32), P(I32)]),
    "fdu_residual_vjp": (I32, [VP, VP, VP, VP, VP]),
    "fdu_rk_stage_vjp": (I32, [VP, I32, VP, VP, VP, VP, D, VP]),
    "fdu_rk_step_vjp": (I32, [VP, VP, VP, VP, VP, D, VP]),
    "fdu_rk_step_vjp_stages": (I32, [VP, VP, VP, VP, VP, VP, VP, D, VP]),
    "fdu_rk_step_static": (I32, [VP, VP, D, VP, VP]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(or python paper_2102_12933_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        raise FduError(name, st, lib().fdu_last_error().decode())


def _ptr(a: np.ndarray, dtype):
    assert a.dtype == dtype and a.flags["C_CONTIGUOUS"], (a.dtype, dtype)
    return a.ctypes.data_as(C.c_void_p)


def default_params(**kw) -> Params:
    p = Params()
    lib().fdu_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Prep:
    """Host preprocessing of a mesh (C++ inside libfdu)."""

    def __init__(self, mesh, deg: int = 5, level: int = 0, reorder: int = 1, nthreads: int = 0,
                 artificial: bool = False):
        self.mesh = mesh
        self.deg, self.level, self.reorder, self.artificial = deg, level, reorder, artificial
        xy = np.ascontiguousarray(mesh.xy, np.float64)
        edges = np.ascontiguousarray(mesh.edges, np.int32)
        tris = np.ascontiguousarray(mesh.tri, np.int32)
        gs = np.ascontiguousarray(mesh.ghost_src, np.int32)
        gr = np.ascontiguousarray(mesh.ghost_refl, np.int8)
        h = C.c_void_p()
        _call("fdu_prep_build", C.byref(h), mesh.nv, mesh.nv_real, _ptr(xy, np.float64), mesh.ne,
              _ptr(edges, np.int32), tris.shape[0], _ptr(tris, np.int32),
              gs.ctypes.data_as(C.c_void_p) if gs.size else None,
              gr.ctypes.data_as(C.c_void_p) if gr.size else None,
              {True: 1, "y": 2}.get(mesh.periodic, 0), float(mesh.box[0]), float(mesh.box[1]), deg, level,
              reorder, nthreads,
              int(bool(artificial)))
        self.handle = h
        v = PrepView()
        _call("fdu_prep_view_get", h, C.byref(v))
        self._view = v

    def arrays(self) -> dict:
        """Copies of the prep's arrays as numpy (library numbering)."""
        v = self._view
        nvt, nvr, nef, nzv, nze = v.nv_total, v.nv_real, v.ne_flux, v.nnz_v, v.nnz_e
        ng = nvt - nvr

        def arr(ptr, n, ctype, dt):
            if n == 0:
                return np.zeros(0, dt)
            return np.ctypeslib.as_array(C.cast(ptr, P(ctype)), shape=(n,)).astype(dt, copy=True)

        return dict(
            nv_total=nvt, nv_real=nvr, ne_flux=nef, nnz_v=nzv, nnz_e=nze,
            perm=arr(v.perm, nvt, C.c_int32, np.int64), iperm=arr(v.iperm, nvt, C.c_int32, np.int64),
            flux_edge=arr(v.flux_edge, nef, C.c_int32, np.int64),
            sten6=arr(v.sten6, 6 * nef, C.c_int32, np.int64).reshape(nef, 6),
            geo=arr(v.geo, 6 * nef, C.c_double, np.float64).reshape(nef, 6),
            vptr=arr(v.vptr, nvr + 1, C.c_int32, np.int64), vcol=arr(v.vcol, nzv, C.c_int32, np.int64),
            wfg=arr(v.wfg, 2 * nzv, C.c_double, np.float64).reshape(nzv, 2),
            eptr=arr(v.eptr, nvr + 1, C.c_int32, np.int64), ecol=arr(v.ecol, nze, C.c_int32, np.int64),
            we=arr(v.we, nze, C.c_double, np.float64), hmin=arr(v.hmin, nvr, C.c_double, np.float64),
            ghost_src=arr(v.ghost_src, ng, C.c_int32, np.int64), ghost_refl=arr(v.ghost_refl, ng, C.c_int8, np.int8),
            artificial=arr(v.artificial, 2 * v.n_artificial, C.c_int32, np.int64).reshape(-1, 2))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fdu_prep_destroy(self.handle)
            self.handle = None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """Device-resident stencils and weights of one mesh; compute calls take
    torch tensors on the solver's device and run on torch's current stream."""

    def __init__(self, prep: Prep | None = None, device: int = 0, precision: str = "f64", ghost_states=None,
                 **params):
        """ghost_states: [ng, 4] Dirichlet ghost states in the mesh's ghost order
        (needed when the mesh has Dirichlet ghosts)."""
        self.device = device
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.prec = F64 if precision == "f64" else F32
        p = default_params(**params)
        self.params = {name: getattr(p, name) for name, _ in Params._fields_}
        h = C.c_void_p()
        _call("fdu_create", C.byref(h), device, self.prec, C.byref(p))
        self.handle = h
        self.prep = prep
        if prep is not None:
            _call("fdu_upload_prep", h, prep.handle)
            if ghost_states is not None:
                self.set_ghost_states(ghost_states)
            _call("fdu_finalize", h)
            self._sizes()

    def set_ghost_states(self, states):
        """Dirichlet ghost states [ng, 4] (ghost order of the mesh = of the library)."""
        g = np.ascontiguousarray(states, np.float64)
        _call("fdu_upload_ghost_states", self.handle, g.shape[0], _ptr(g, np.float64))

    # -- uploads (library numbering)
    def upload(self, nv_total, nv_real, sten6, geo, vptr, vcol, wfg, eptr, ecol, we, hmin,
               ghost_src=None, ghost_refl=None):
        i32 = lambda a: np.ascontiguousarray(a, np.int32)
        f64 = lambda a: np.ascontiguousarray(a, np.float64)
        sten6, geo = i32(sten6), f64(geo)
        _call("fdu_upload_edge_stencils", self.handle, nv_total, nv_real, sten6.shape[0], _ptr(sten6, np.int32),
              _ptr(geo, np.float64))
        vptr, vcol, wfg, eptr, ecol, we, hmin = i32(vptr), i32(vcol), f64(wfg), i32(eptr), i32(ecol), f64(we), f64(hmin)
        _call("fdu_upload_vertex_stencils", self.handle, _ptr(vptr, np.int32), _ptr(vcol, np.int32),
              _ptr(wfg, np.float64), _ptr(eptr, np.int32), _ptr(ecol, np.int32), _ptr(we, np.float64),
              _ptr(hmin, np.float64))
        ng = nv_total - nv_real
        if ng:
            gs, gr = i32(ghost_src), np.ascontiguousarray(ghost_refl, np.int8)
            _call("fdu_upload_ghosts", self.handle, ng, _ptr(gs, np.int32), _ptr(gr, np.int8))
        else:
            _call("fdu_upload_ghosts", self.handle, 0, None, None)
        _call("fdu_finalize", self.handle)
        self._sizes()

    def _sizes(self):
        vals = [C.c_int64() for _ in range(5)]
        _call("fdu_sizes", self.handle, *[C.byref(v) for v in vals])
        self.nv_total, self.nv_real, self.ne_flux, self.nnz_v, self.nnz_e = (v.value for v in vals)

    def _state(self, w, rows=None):
        rows = self.nv_total if rows is None else rows
        if not (isinstance(w, torch.Tensor) and w.is_cuda and w.dtype == self.dtype and w.is_contiguous()
                and tuple(w.shape) == (rows, 4) and w.device.index == self.device):
            raise ValueError(f"expected a contiguous {self.dtype} cuda:{self.device} tensor of shape ({rows}, 4)")
        return C.c_void_p(w.data_ptr())

    def _dt(self, dt):
        if not (isinstance(dt, torch.Tensor) and dt.is_cuda and dt.dtype == torch.float64 and dt.numel() >= 1):
            raise ValueError("dt must be a float64 cuda tensor")
        return C.c_void_p(dt.data_ptr())

    # -- compute
    def fill_ghosts(self, w):
        _call("fdu_fill_ghosts", self.handle, self._state(w), _stream())

    def edge_fluxes(self, w, out=None):
        if out is None:
            out = torch.empty(self.ne_flux, 4, dtype=torch.float64, device=w.device)
        if tuple(out.shape) != (self.ne_flux, 4) or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("flux output must be a contiguous float64 (ne_flux, 4) tensor")
        _call("fdu_edge_fluxes", self.handle, self._state(w), C.c_void_p(out.data_ptr()), _stream())
        return out

    def residual(self, w, out=None):
        if out is None:
            out = torch.empty(self.nv_real, 4, dtype=self.dtype, device=w.device)
        _call("fdu_residual", self.handle, self._state(w), self._state(out, self.nv_real), _stream())
        return out

    def cfl_dt(self, w, cfl, dt=None):
        if dt is None:
            dt = torch.empty(1, dtype=torch.float64, device=w.device)
        _call("fdu_cfl_dt", self.handle, self._state(w), float(cfl), self._dt(dt), _stream())
        return dt

    def rk_stage(self, k, w_n, w_prev, w_out, dt):
        wn = self._state(w_n) if w_n is not None else None
        _call("fdu_rk_stage", self.handle, int(k), wn, self._state(w_prev), self._state(w_out), self._dt(dt), _stream())

    def rk_step(self, w, scratch, dt, cfl=0.0):
        if not (scratch.is_cuda and scratch.dtype == self.dtype and scratch.is_contiguous()
                and scratch.numel() >= 8 * self.nv_total):
            raise ValueError("scratch must hold two states")
        _call("fdu_rk_step", self.handle, self._state(w), C.c_void_p(scratch.data_ptr()), float(cfl),
              self._dt(dt), _stream())

    def rk_step_static(self, w, dt, cfl=0.0):
        """fdu_rk_step without a workspace: the stage states live in the library's
        static device array (no allocation; calls overlapping on one GPU race)."""
        _call("fdu_rk_step_static", self.handle, self._state(w), float(cfl), self._dt(dt), _stream())

    # -- adjoint
    def enable_adjoint(self):
        _call("fdu_enable_adjoint", self.handle)

    def residual_vjp(self, w, Rbar, out=None):
        if out is None:
            out = torch.empty(self.nv_total, 4, dtype=self.dtype, device=w.device)
        _call("fdu_residual_vjp", self.handle, self._state(w), self._state(Rbar, self.nv_real), self._state(out),
              _stream())
        return out

    def rk_stage_vjp(self, k, w_prev, obar, wbar_n, wbar_prev, dt: float):
        wn = self._state(wbar_n) if wbar_n is not None else None
        _call("fdu_rk_stage_vjp", self.handle, int(k), self._state(w_prev), self._state(obar), wn,
              self._state(wbar_prev), float(dt), _stream())

    def rk_step_vjp(self, w_n, wbar_np1, wbar_n, scratch, dt: float):
        if not (scratch.is_cuda and scratch.dtype == self.dtype and scratch.is_contiguous()
                and scratch.numel() >= 16 * self.nv_total):
            raise ValueError("scratch must hold four states")
        _call("fdu_rk_step_vjp", self.handle, self._state(w_n), self._state(wbar_np1), self._state(wbar_n),
              C.c_void_p(scratch.data_ptr()), float(dt), _stream())

    def rk_step_vjp_stages(self, w_n, w_1, w_2, wbar_np1, wbar_n, scratch, dt: float):
        """fdu_rk_step_vjp with the step's stage states given (not recomputed)."""
        if not (scratch.is_cuda and scratch.dtype == self.dtype and scratch.is_contiguous()
                and scratch.numel() >= 8 * self.nv_total):
            raise ValueError("scratch must hold two states")
        _call("fdu_rk_step_vjp_stages", self.handle, self._state(w_n), self._state(w_1), self._state(w_2),
              self._state(wbar_np1), self._state(wbar_n), C.c_void_p(scratch.data_ptr()), float(dt), _stream())

    # -- kernel variants
    def set_variants(self, edge: int, vertex: int):
        _call("fdu_set_variants", self.handle, int(edge), int(vertex))

    def variants(self):
        e, v, ne, nv = (C.c_int() for _ in range(4))
        _call("fdu_get_variants", self.handle, C.byref(e), C.byref(v), C.byref(ne), C.byref(nv))
        return dict(edge=e.value, vertex=v.value, n_edge=ne.value, n_vertex=nv.value)

    def autotune(self, w, reps: int = 10):
        """Time every kernel variant on state w; keep the fastest.  Returns the times (ms)."""
        info = self.variants()
        n = info["n_edge"] + info["n_vertex"]
        scratch = torch.empty(self.nv_total + 2, 4, dtype=self.dtype, device=w.device)
        out = (C.c_double * n)()
        _call("fdu_autotune", self.handle, self._state(w), C.c_void_p(scratch.data_ptr()), int(reps), out, _stream())
        ch = self.variants()
        return dict(edge_ms=list(out[:info["n_edge"]]), vertex_ms=list(out[info["n_edge"]:]),
                    edge=ch["edge"], vertex=ch["vertex"])

    def kernel_times(self, w, reps: int = 20):
        """Mean kernel durations in ms: ghost fill, edge flux, vertex step, CFL."""
        scratch = torch.empty(self.nv_total + 2, 4, dtype=self.dtype, device=w.device)
        out = (C.c_double * 4)()
        _call("fdu_kernel_times", self.handle, self._state(w), C.c_void_p(scratch.data_ptr()), int(reps), out,
              _stream())
        return dict(ghost=out[0], edge=out[1], vertex=out[2], cfl=out[3])

    def check_state(self, w):
        """(number of non-finite or non-physical real rows, first such row or -1)."""
        n, first = C.c_int64(), C.c_int64()
        _call("fdu_check_state", self.handle, self._state(w), C.byref(n), C.byref(first), _stream())
        return n.value, first.value

    def vertex_block_info(self):
        """Vertex blocks of the LDS-staged variants: count, total and largest row list."""
        n, rows, mx = C.c_int(), C.c_int64(), C.c_int()
        _call("fdu_vertex_block_info", self.handle, C.byref(n), C.byref(rows), C.byref(mx))
        return dict(n_blocks=n.value, halo_rows=rows.value, rows_max=mx.value)

    PHASES = ("ghost", "edge", "vertex", "cfl")

    def kernel_timer_start(self, capacity: int = 4096, phases=PHASES):
        """Bracket every later kernel launch of the given kinds by this solver
        with HIP events (first `capacity` launches of each kind) on the
        launching stream."""
        mask = sum(1 << self.PHASES.index(p) for p in phases)
        _call("fdu_kernel_timer_start", self.handle, int(capacity), int(mask))

    def kernel_timer_stop(self):
        """Stop the live timer; returns ({kind: mean ms}, {kind: launches})."""
        avg, cnt = (C.c_double * 4)(), (C.c_int * 4)()
        _call("fdu_kernel_timer_stop", self.handle, avg, cnt)
        keys = ("ghost", "edge", "vertex", "cfl")
        return dict(zip(keys, list(avg))), dict(zip(keys, list(cnt)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fdu_destroy(self.handle)
            self.handle = None


class Batch:
    """Several FP64 solvers advanced together (one persistent launch per stage,
    or per phase, or per instance), optionally captured in a HIP graph."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.handle.value for s in self.solvers])
        h = C.c_void_p()
        _call("fdu_batch_create", C.byref(h), arr, len(self.solvers))
        self.handle = h
        self._keep = None

    def set_states(self, states, scratches):
        for s, w, sc in zip(self.solvers, states, scratches):
            s._state(w)
            if not (sc.is_cuda and sc.dtype == torch.float64 and sc.is_contiguous() and sc.numel() >= 8 * s.nv_total):
                raise ValueError("each scratch must hold two states")
        n = len(self.solvers)
        ws = (C.c_void_p * n)(*[w.data_ptr() for w in states])
        ss = (C.c_void_p * n)(*[sc.data_ptr() for sc in scratches])
        _call("fdu_batch_set_states", self.handle, ws, ss)
        self._keep = (list(states), list(scratches))

    def set_schedule(self, schedule: int, edges_per_thread: int = 4, vertex_passes: int = 8, vertex_mode: int = 0):
        _call("fdu_batch_set_schedule", self.handle, int(schedule), int(edges_per_thread), int(vertex_passes),
              int(vertex_mode))

    def step(self, cfl: float):
        _call("fdu_batch_step", self.handle, float(cfl), _stream())

    def capture(self, cfl: float, nsteps: int):
        st = torch.cuda.current_stream().cuda_stream
        if not st:
            raise ValueError("capture needs a non-default stream (use torch.cuda.stream(...))")
        _call("fdu_batch_capture", self.handle, float(cfl), int(nsteps), C.c_void_p(st))

    def launch(self):
        _call("fdu_batch_launch", self.handle, _stream())

    def status(self):
        e = C.c_int()
        dt = np.zeros(len(self.solvers))
        _call("fdu_batch_status", self.handle, C.byref(e), dt.ctypes.data_as(C.c_void_p))
        return e.value, dt

    def info(self):
        vals = [C.c_int() for _ in range(6)]
        _call("fdu_batch_info", self.handle, *[C.byref(v) for v in vals])
        keys = ["schedule", "total_tiles", "grid", "edges_per_thread", "vertex_passes", "vertex_mode"]
        return {k: v.value for k, v in zip(keys, vals)}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fdu_batch_destroy(self.handle)
            self.handle = None


def exported_symbols():
    """Names declared in _SIGS (the binding's view of include/fdu.h)."""
    return list(_SIGS)
