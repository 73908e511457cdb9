"""MI355X moving-mesh finite-volume step (Chang, Wadsley & Quinn 2017).

Thin Python binding over the C ABI of ``libmm_mi355x.so`` (include/mm.h).
It only marshals arguments: every step of the path runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  Importing the
package does not need a GPU; creating a context does, and fails loudly if the
HIP library has not been built (``python -m paper_1707_05333_amd.build``).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

from .build import LIB_PATH

MM_FP64, MM_MIXED = 0, 1
MM_HLLC, MM_HLL = 0, 1
_STATUS = {0: "MM_OK", -1: "MM_EINVAL", -2: "MM_ENOMEM", -3: "MM_ECAPACITY", -4: "MM_EDEGENERATE",
           -5: "MM_ENONFINITE", -6: "MM_EHIP", -7: "MM_ESTATE", -8: "MM_EFULL"}
N_STAGES = 9
STAGE_NAMES = ("sort", "cells", "mesh", "cell_state", "gradient_predict", "gradient_half", "flux", "update", "remesh")


class MMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = _STATUS.get(code, str(code))


class Params(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("chi", ctypes.c_double),
        ("zeta", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("rho_floor", ctypes.c_double),
        ("p_floor", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("riemann", ctypes.c_int32),
        ("limit_mask", ctypes.c_int32),
        ("predictor_frame", ctypes.c_int32),
        ("half_step_mesh", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("mach_threshold", ctypes.c_double),
    ]


class StepInfo(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double),
        ("dt_cfl", ctypes.c_double),
        ("n_faces", ctypes.c_int64),
        ("max_faces_cell", ctypes.c_int32),
        ("deferred_cells", ctypes.c_int32),
        ("floor_hits", ctypes.c_int64 * 4),
        ("flags", ctypes.c_int32),
        ("rebuilt_cells", ctypes.c_int32),
    ]

    def as_dict(self):
        return dict(dt=self.dt, dt_cfl=self.dt_cfl, n_faces=self.n_faces, max_faces_cell=self.max_faces_cell,
                    deferred_cells=self.deferred_cells, rebuilt_cells=self.rebuilt_cells,
                    floor_hits=list(self.floor_hits), flags=self.flags)


class MeshView(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("n_faces", ctypes.c_int64),
        ("perm", ctypes.c_void_p),
        ("pos", ctypes.c_void_p),
        ("geo", ctypes.c_void_p),
        ("faces", ctypes.c_void_p),
    ]


class SimInfo(ctypes.Structure):
    _fields_ = [
        ("sim", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("steps", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("dt", ctypes.c_double),
        ("t", ctypes.c_double),
        ("floor_hits", ctypes.c_int64 * 4),
        ("flags", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return dict(sim=self.sim, status=self.status, steps=self.steps, n=self.n, dt=self.dt, t=self.t,
                    floor_hits=list(self.floor_hits), flags=self.flags)


class Request(ctypes.Structure):
    _fields_ = [
        ("arrival", ctypes.c_double),
        ("n", ctypes.c_int64),
        ("pos", ctypes.c_void_p),
        ("prim", ctypes.c_void_p),
        ("params", Params),
        ("dt_max", ctypes.c_double),
        ("steps", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("pos_out", ctypes.c_void_p),
        ("Q_out", ctypes.c_void_p),
    ]


class RequestResult(ctypes.Structure):
    _fields_ = [
        ("admitted", ctypes.c_double),
        ("finished", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("t", ctypes.c_double),
    ]


class ServeStats(ctypes.Structure):
    _fields_ = [
        ("wall", ctypes.c_double),
        ("batch_steps", ctypes.c_int64),
        ("sim_steps", ctypes.c_int64),
        ("cell_updates", ctypes.c_int64),
        ("cell_updates_per_s", ctypes.c_double),
        ("step_p50", ctypes.c_double),
        ("step_p99", ctypes.c_double),
        ("step_mean", ctypes.c_double),
        ("turnaround_p50", ctypes.c_double),
        ("turnaround_p99", ctypes.c_double),
        ("max_resident", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


# Functions declared in include/mm.h, with their ctypes signatures.
_vp, _i64, _i32, _d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
SIGNATURES = {
    "mm_default_params": (None, [ctypes.POINTER(Params)]),
    "mm_create": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(Params), _i64, _i64, _vp]),
    "mm_destroy": (_i32, [_vp]),
    "mm_set_params": (_i32, [_vp, ctypes.POINTER(Params)]),
    "mm_tessellate": (_i32, [_vp, _i64, _vp, ctypes.POINTER(StepInfo)]),
    "mm_get_mesh_view": (_i32, [_vp, ctypes.POINTER(MeshView)]),
    "mm_mesh_export": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_i64)]),
    "mm_init_charges": (_i32, [_vp, _vp, _vp]),
    "mm_init_entropy": (_i32, [_vp, _vp, _vp]),
    "mm_step_entropy": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _d, ctypes.POINTER(StepInfo)]),
    "mm_cell_state": (_i32, [_vp, _vp, _vp, _vp, ctypes.POINTER(_d), ctypes.POINTER(_i64)]),
    "mm_gradients": (_i32, [_vp, _vp, _vp, _i32]),
    "mm_predict": (_i32, [_vp, _vp, _vp, _vp, _d, _vp]),
    "mm_fluxes": (_i32, [_vp, _vp, _vp, _vp, _d, _vp]),
    "mm_step": (_i32, [_vp, _i64, _vp, _vp, _vp, _d, ctypes.POINTER(StepInfo)]),
    "mm_step_static": (_i32, [ctypes.POINTER(Params), _i64, _vp, _vp, _vp, _d, ctypes.POINTER(StepInfo), _vp]),
    "mm_last_error": (ctypes.c_char_p, [_vp]),
    "mm_version": (ctypes.c_char_p, []),
    "mm_set_stage_timing": (_i32, [_vp, _i32]),
    "mm_get_stage_ms": (_i32, [_vp, ctypes.POINTER(_d), _i32]),
    "mm_batch_footprint": (_i64, [_i32, _i64]),
    "mm_batch_create": (_i32, [ctypes.POINTER(_vp), _i32, _i64, _i32, _vp]),
    "mm_batch_destroy": (_i32, [_vp]),
    "mm_batch_admit": (_i32, [_vp, ctypes.POINTER(Params), _i64, _vp, _vp, _d, ctypes.POINTER(_i32)]),
    "mm_batch_step": (_i32, [_vp, ctypes.POINTER(SimInfo), _i32, ctypes.POINTER(_i32)]),
    "mm_batch_read": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "mm_batch_evict": (_i32, [_vp, _i32]),
    "mm_batch_usage": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "mm_batch_last_error": (ctypes.c_char_p, [_vp]),
    "mm_serve": (_i32, [_vp, ctypes.POINTER(Request), _i32, ctypes.POINTER(RequestResult),
                        ctypes.POINTER(ServeStats)]),
}

_lib = None


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Loads libmm_mi355x.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch first: it ships its own HIP runtime under the same soname, and
        # the process must use one runtime for torch's memory and our kernels.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing; build it with "
                               "`python -m paper_1707_05333_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def default_params() -> Params:
    p = Params()
    load_library().mm_default_params(ctypes.byref(p))
    return p


def make_params(box=(1.0, 1.0, 1.0), gamma=5.0 / 3.0, precision="fp64", **kw) -> Params:
    p = default_params()
    p.box[:] = [float(b) for b in box]
    p.gamma = float(gamma)
    p.precision = MM_MIXED if precision in ("mixed", MM_MIXED) else MM_FP64
    for k, v in kw.items():
        if k in ("cfl", "eta", "chi", "zeta", "theta", "rho_floor", "p_floor", "mach_threshold"):
            setattr(p, k, float(v))
        elif k in ("limit_mask", "predictor_frame", "half_step_mesh"):
            setattr(p, k, int(v))
        elif k == "riemann":
            p.riemann = {"hllc": MM_HLLC, "hll": MM_HLL}.get(v, v) if isinstance(v, str) else int(v)
        else:
            raise TypeError(f"unknown parameter {k}")
    return p


def _ptr(t, dtype=None, shape=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class MeshExport:
    V: object
    centroid: object
    face_i: object
    face_j: object
    face_code: object
    face_A: object
    face_f: object


class MovingMesh:
    """One simulation context on the current CUDA (HIP) device and stream."""

    def __init__(self, n_capacity: int, params: Params | None = None, face_capacity: int = 0, stream=None,
                 **param_kw):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.params = params if params is not None else make_params(**param_kw)
        self.mixed = self.params.precision == MM_MIXED
        self.rdtype = torch.float32 if self.mixed else torch.float64
        self.device = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        self.ctx = ctypes.c_void_p()
        rc = self.lib.mm_create(ctypes.byref(self.ctx), ctypes.byref(self.params), int(n_capacity),
                                int(face_capacity), ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            raise MMError(rc, "mm_create failed: " + self.lib.mm_last_error(None).decode())
        self.n_capacity = int(n_capacity)
        self.n = 0

    # -- helpers --------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise MMError(rc, self.lib.mm_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.lib.mm_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        self._check(self.lib.mm_set_params(self.ctx, ctypes.byref(params)))
        self.params = params

    # -- the C ABI calls ----------------------------------------------------
    def tessellate(self, pos) -> dict:
        n = int(pos.shape[0])
        info = StepInfo()
        self._check(self.lib.mm_tessellate(self.ctx, n, _ptr(pos, self._torch.float64, (n, 3), "pos"),
                                           ctypes.byref(info)))
        self.n = n
        return info.as_dict()

    def mesh_view(self) -> MeshView:
        v = MeshView()
        self._check(self.lib.mm_get_mesh_view(self.ctx, ctypes.byref(v)))
        return v

    def mesh_export(self) -> MeshExport:
        torch = self._torch
        nf = ctypes.c_int64()
        self._check(self.lib.mm_mesh_export(self.ctx, None, None, 0, None, None, None, None, None, ctypes.byref(nf)))
        n, F = self.n, int(nf.value)
        kw = dict(device=self.device)
        out = MeshExport(torch.empty(n, dtype=torch.float64, **kw), torch.empty(n, 3, dtype=torch.float64, **kw),
                         torch.empty(F, dtype=torch.int32, **kw), torch.empty(F, dtype=torch.int32, **kw),
                         torch.empty(F, dtype=torch.int32, **kw), torch.empty(F, dtype=torch.float64, **kw),
                         torch.empty(F, 3, dtype=torch.float64, **kw))
        self._check(self.lib.mm_mesh_export(self.ctx, _ptr(out.V), _ptr(out.centroid), F, _ptr(out.face_i),
                                            _ptr(out.face_j), _ptr(out.face_code), _ptr(out.face_A),
                                            _ptr(out.face_f), ctypes.byref(nf)))
        return out

    def init_charges(self, prim):
        torch = self._torch
        Q = torch.empty(self.n, 5, dtype=torch.float64, device=self.device)
        self._check(self.lib.mm_init_charges(self.ctx, _ptr(prim, torch.float64, (self.n, 5), "prim"), _ptr(Q)))
        return Q

    def cell_state(self, Q):
        torch = self._torch
        U = torch.empty(self.n, 5, dtype=self.rdtype, device=self.device)
        w = torch.empty(self.n, 3, dtype=torch.float64, device=self.device)
        dt = ctypes.c_double()
        hits = ctypes.c_int64()
        self._check(self.lib.mm_cell_state(self.ctx, _ptr(Q, torch.float64, (self.n, 5), "Q"), _ptr(U), _ptr(w),
                                           ctypes.byref(dt), ctypes.byref(hits)))
        return U, w, dt.value, hits.value

    def gradients(self, U, limit=True):
        G = self._torch.empty(self.n, 5, 3, dtype=self.rdtype, device=self.device)
        self._check(self.lib.mm_gradients(self.ctx, _ptr(U, self.rdtype, (self.n, 5), "U"), _ptr(G),
                                          1 if limit else 0))
        return G

    def predict(self, U, G, w, dt):
        Uh = self._torch.empty(self.n, 5, dtype=self.rdtype, device=self.device)
        self._check(self.lib.mm_predict(self.ctx, _ptr(U, self.rdtype, (self.n, 5), "U"),
                                        _ptr(G, self.rdtype, (self.n, 5, 3), "G"),
                                        _ptr(w, self._torch.float64, (self.n, 3), "w"), float(dt), _ptr(Uh)))
        return Uh

    def fluxes(self, Uh, Gh, w, dt):
        dQ = self._torch.empty(self.n, 5, dtype=self._torch.float64, device=self.device)
        self._check(self.lib.mm_fluxes(self.ctx, _ptr(Uh, self.rdtype, (self.n, 5), "U_half"),
                                       _ptr(Gh, self.rdtype, (self.n, 5, 3), "grad_half"),
                                       _ptr(w, self._torch.float64, (self.n, 3), "w"), float(dt), _ptr(dQ)))
        return dQ

    def step(self, pos, w, Q, dt_max=math.inf) -> dict:
        """One whole step in place on pos, w (output) and Q."""
        torch = self._torch
        n = int(pos.shape[0])
        info = StepInfo()
        self._check(self.lib.mm_step(self.ctx, n, _ptr(pos, torch.float64, (n, 3), "pos"),
                                     _ptr(w, torch.float64, (n, 3), "w"), _ptr(Q, torch.float64, (n, 5), "Q"),
                                     float(dt_max), ctypes.byref(info)))
        self.n = n
        return info.as_dict()

    def init_entropy(self, prim):
        """Entropy charges S = m P rho^-gamma (Sec. 4.3) on the last tessellation."""
        torch = self._torch
        S = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._check(self.lib.mm_init_entropy(self.ctx, _ptr(prim, torch.float64, (self.n, 5), "prim"), _ptr(S)))
        return S

    def step_entropy(self, pos, w, Q, S, mach=None, dt_max=math.inf) -> dict:
        """One whole step with the entropy column, in place on pos, w, Q and S;
        mach (float32 [n], optional) receives each cell's largest face Mach number."""
        torch = self._torch
        n = int(pos.shape[0])
        info = StepInfo()
        self._check(self.lib.mm_step_entropy(self.ctx, n, _ptr(pos, torch.float64, (n, 3), "pos"),
                                             _ptr(w, torch.float64, (n, 3), "w"),
                                             _ptr(Q, torch.float64, (n, 5), "Q"),
                                             _ptr(S, torch.float64, (n,), "S"),
                                             _ptr(mach, torch.float32, (n,), "mach") if mach is not None else None,
                                             float(dt_max), ctypes.byref(info)))
        self.n = n
        return info.as_dict()

    def set_stage_timing(self, enable: bool):
        self._check(self.lib.mm_set_stage_timing(self.ctx, 1 if enable else 0))

    def stage_ms(self) -> dict:
        arr = (ctypes.c_double * N_STAGES)()
        self._check(self.lib.mm_get_stage_ms(self.ctx, arr, N_STAGES))
        return dict(zip(STAGE_NAMES, list(arr)))


def batch_footprint(n: int, precision="mixed") -> int:
    """Device bytes one simulation of n points takes in a batch."""
    prec = MM_MIXED if precision in ("mixed", MM_MIXED) else MM_FP64
    return int(load_library().mm_batch_footprint(prec, int(n)))


class Batch:
    """Many simulations resident together, stepped in shared launches."""

    def __init__(self, hbm_budget: int, max_sims: int = 1024, precision="mixed", stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.precision = MM_MIXED if precision in ("mixed", MM_MIXED) else MM_FP64
        self.device = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        self.max_sims = int(max_sims)
        self.b = ctypes.c_void_p()
        rc = self.lib.mm_batch_create(ctypes.byref(self.b), self.precision, int(hbm_budget), self.max_sims,
                                      ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            raise MMError(rc, "mm_batch_create failed: " + self.lib.mm_batch_last_error(None).decode())
        self.n_of = {}

    def _check(self, rc):
        if rc != 0:
            raise MMError(rc, self.lib.mm_batch_last_error(self.b).decode())

    def close(self):
        if getattr(self, "b", None) and self.b.value:
            self.lib.mm_batch_destroy(self.b)
            self.b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, params: Params, pos, prim, dt_max=math.inf) -> int:
        """Admits a simulation (pos [n][3], prim [n][5] float64 CUDA tensors); returns its id."""
        torch = self._torch
        n = int(pos.shape[0])
        sim = ctypes.c_int32()
        self._check(self.lib.mm_batch_admit(self.b, ctypes.byref(params), n,
                                            _ptr(pos, torch.float64, (n, 3), "pos"),
                                            _ptr(prim, torch.float64, (n, 5), "prim"), float(dt_max),
                                            ctypes.byref(sim)))
        self.n_of[sim.value] = n
        return sim.value

    def try_admit(self, params: Params, pos, prim, dt_max=math.inf):
        """As admit, but returns None when the batch is full now."""
        try:
            return self.admit(params, pos, prim, dt_max)
        except MMError as e:
            if e.name == "MM_EFULL":
                return None
            raise

    def step(self) -> list:
        """One step of every resident simulation; a report per simulation."""
        info = (SimInfo * self.max_sims)()
        k = ctypes.c_int32()
        self._check(self.lib.mm_batch_step(self.b, info, self.max_sims, ctypes.byref(k)))
        return [info[i].as_dict() for i in range(k.value)]

    def read(self, sim: int):
        """(pos, Q, w) of a resident simulation, as new CUDA tensors."""
        torch = self._torch
        if sim not in self.n_of:
            self._check(self.lib.mm_batch_read(self.b, int(sim), None, None, None))
            raise MMError(-1, f"simulation {sim} was not admitted through this object")
        n = self.n_of[sim]
        kw = dict(dtype=torch.float64, device=self.device)
        pos, Q, w = torch.empty(n, 3, **kw), torch.empty(n, 5, **kw), torch.empty(n, 3, **kw)
        self._check(self.lib.mm_batch_read(self.b, int(sim), _ptr(pos), _ptr(Q), _ptr(w)))
        return pos, Q, w

    def evict(self, sim: int):
        self._check(self.lib.mm_batch_evict(self.b, int(sim)))
        self.n_of.pop(sim, None)

    def usage(self) -> dict:
        cells, cap, sims = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        self._check(self.lib.mm_batch_usage(self.b, ctypes.byref(cells), ctypes.byref(cap), ctypes.byref(sims)))
        return dict(cells=cells.value, cell_capacity=cap.value, sims=sims.value)

    def serve(self, requests: list):
        """Runs the serving loop over requests, each a dict with arrival (s),
        params, pos and prim (CUDA float64), steps, and optional dt_max,
        pos_out and Q_out tensors.  Returns (results, stats) as dicts."""
        torch = self._torch
        n_req = len(requests)
        arr = (Request * max(n_req, 1))()
        for k, r in enumerate(requests):
            n = int(r["pos"].shape[0])
            q = arr[k]
            q.arrival = float(r["arrival"])
            q.n = n
            q.pos = _ptr(r["pos"], torch.float64, (n, 3), "pos")
            q.prim = _ptr(r["prim"], torch.float64, (n, 5), "prim")
            q.params = r["params"]
            q.dt_max = float(r.get("dt_max", math.inf))
            q.steps = int(r["steps"])
            q.pos_out = _ptr(r.get("pos_out"), torch.float64, (n, 3), "pos_out")
            q.Q_out = _ptr(r.get("Q_out"), torch.float64, (n, 5), "Q_out")
        res = (RequestResult * max(n_req, 1))()
        stats = ServeStats()
        self._check(self.lib.mm_serve(self.b, arr, n_req, res, ctypes.byref(stats)))
        results = [dict(admitted=res[k].admitted, finished=res[k].finished, status=res[k].status,
                        steps=res[k].steps, t=res[k].t) for k in range(n_req)]
        return results, stats.as_dict()


STATIC_MAX_POINTS = 8192   # MM_STATIC_MAX_POINTS of include/mm.h


def step_static(params: Params, pos, w, Q, dt_max=math.inf, stream=None) -> dict:
    """mm_step_static: one whole step in place on pos, w (output) and Q with
    no context, for callers that cannot allocate device memory (n at most
    STATIC_MAX_POINTS; calls on one device must not overlap)."""
    import torch
    L = load_library()
    n = int(pos.shape[0])
    s = stream if stream is not None else torch.cuda.current_stream()
    info = StepInfo()
    rc = L.mm_step_static(ctypes.byref(params), n, _ptr(pos, torch.float64, (n, 3), "pos"),
                          _ptr(w, torch.float64, (n, 3), "w"), _ptr(Q, torch.float64, (n, 5), "Q"),
                          float(dt_max), ctypes.byref(info), ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise MMError(rc, L.mm_last_error(None).decode())
    return info.as_dict()


def version() -> str:
    return load_library().mm_version().decode()
