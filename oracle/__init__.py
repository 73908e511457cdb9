"""TEST INFRASTRUCTURE -- the plain FP64 CPU oracle (never the product path).

ctypes wrapper around ``liboracle.so`` built from ``mm_oracle.cpp`` (see
``build.py``).  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with ``paper_1707_05333_amd``: neither imports the other.

No function here reproduces a worked example printed in the paper (it
prints none, and its figures are absent); each is pinned instead by closed
forms, invariants and brute force in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


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
        ("limiter_disp", ctypes.c_int32),
        ("predictor_frame", ctypes.c_int32),
        ("limit_mask", ctypes.c_int32),
        ("riemann", ctypes.c_int32),
        ("half_step_mesh", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("mach_threshold", ctypes.c_double),
    ]


def make_params(box, gamma, cfl=0.3, eta=1.0, chi=1.0, zeta=0.25, theta=0.49,
                rho_floor=1e-12, p_floor=1e-14, limiter_disp=0, predictor_frame=0,
                limit_mask=3, riemann=0, half_step_mesh=0, mach_threshold=0.0, **_ignored) -> Params:
    p = Params()
    p.box[:] = [float(b) for b in box]
    p.gamma, p.cfl, p.eta, p.chi, p.zeta, p.theta = gamma, cfl, eta, chi, zeta, theta
    p.rho_floor, p.p_floor = rho_floor, p_floor
    p.limiter_disp, p.predictor_frame, p.limit_mask = limiter_disp, predictor_frame, limit_mask
    p.riemann = riemann
    p.half_step_mesh = half_step_mesh
    p.mach_threshold = mach_threshold
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.orc_mesh_build.restype = vp
        L.orc_mesh_build.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.orc_mesh_build_subset.restype = vp
        L.orc_mesh_build_subset.argtypes = [ctypes.c_int64, _dp, _dp, _i64p, ctypes.c_int64]
        L.orc_mesh_free.argtypes = [vp]
        L.orc_mesh_status.argtypes = [vp]
        L.orc_mesh_status.restype = ctypes.c_int32
        L.orc_mesh_delta_min.argtypes = [vp]
        L.orc_mesh_delta_min.restype = ctypes.c_double
        L.orc_mesh_nfaces.argtypes = [vp]
        L.orc_mesh_nfaces.restype = ctypes.c_int64
        L.orc_mesh_cells.argtypes = [vp, _dp, _dp, _dp, _dp, _i32p, _dp]
        L.orc_mesh_faces.argtypes = [vp, _i64p, _i32p, _i32p, _dp, _dp]
        P = ctypes.POINTER(Params)
        L.orc_init_charges.argtypes = [vp, P, _dp, _dp]
        L.orc_cell_state.argtypes = [vp, P, _dp, _dp, _dp, _dp, _i64p]
        L.orc_cell_state.restype = ctypes.c_double
        L.orc_gradient.argtypes = [vp, P, _dp, _dp, ctypes.c_int32]
        L.orc_predict.argtypes = [vp, P, _dp, _dp, _dp, ctypes.c_double, _dp, ctypes.c_int32, _i64p]
        L.orc_fluxes.argtypes = [vp, P, _dp, _dp, _dp, ctypes.c_double, _dp, _i64p]
        L.orc_face_states.argtypes = [vp, P, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_fluxes.restype = ctypes.c_int32
        L.orc_step.argtypes = [ctypes.c_int64, _dp, _dp, _dp, P, ctypes.c_double, ctypes.c_int32, _dp, _i64p]
        L.orc_step.restype = ctypes.c_int32
        L.orc_step_entropy.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, P, ctypes.c_double, ctypes.c_int32,
                                       _dp, _i64p, _dp]
        L.orc_step_entropy.restype = ctypes.c_int32
        L.orc_init_entropy.argtypes = [ctypes.c_void_p, P, _dp, _dp]
        L.orc_entropy_face.argtypes = [_dp, _dp, _dp, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_double, _dp, _dp]
        L.orc_face_velocity.argtypes = [_dp] * 6
        L.orc_moving_face_flux.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int32, _dp]
        L.orc_hll_prim.argtypes = [_dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_hllc_prim.argtypes = [_dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_dm_factor.argtypes = [ctypes.c_double] * 3
        L.orc_dm_factor.restype = ctypes.c_double
        L.orc_apply_floors.argtypes = [P, _dp]
        L.orc_apply_floors.restype = ctypes.c_int32
        L.orc_exact_riemann.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_int64, _dp, _dp, _dp]
        L.orc_exact_riemann.restype = ctypes.c_int32
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    return int(lib().orc_num_threads())


@dataclass
class Mesh:
    """Periodic Voronoi tessellation computed by the oracle.

    Faces are directed: every cell lists all its faces, ordered by
    (neighbour, image code); the face between i and image (j, k) appears in
    i's list as (j, k) and in j's list as (i, 26 - k)."""

    handle: int
    n: int
    box: tuple
    pos: np.ndarray
    V: np.ndarray
    c: np.ndarray
    vtet: np.ndarray
    rmax: np.ndarray
    nvert: np.ndarray
    off: np.ndarray
    j: np.ndarray
    code: np.ndarray
    A: np.ndarray
    f: np.ndarray
    delta_min: float
    status: int
    delta: np.ndarray

    def face_owner(self) -> np.ndarray:
        return np.repeat(np.arange(self.n), np.diff(self.off))

    def free(self):
        if self.handle:
            lib().orc_mesh_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def tessellate(pos, box, method="grid", certificate=False, exhaustive=False, subset=None) -> Mesh:
    """Oracle tessellation.  With `subset` (cell indices) only those cells
    are built (grid path, certificate included); the others have no faces."""
    pos = _f64(pos)
    n = pos.shape[0]
    b = _f64(box)
    if subset is not None:
        idx = np.ascontiguousarray(subset, dtype=np.int64)
        h = lib().orc_mesh_build_subset(n, _p(pos), _p(b), idx.ctypes.data_as(_i64p), idx.shape[0])
    else:
        h = lib().orc_mesh_build(n, _p(pos), _p(b), 1 if method == "grid" else 0,
                                 1 if certificate else 0, 1 if exhaustive else 0)
    L = lib()
    nf = int(L.orc_mesh_nfaces(h))
    V = np.empty(n); c = np.empty((n, 3)); vtet = np.empty(n); rmax = np.empty(n)
    nvert = np.empty(n, dtype=np.int32); delta = np.empty(n)
    L.orc_mesh_cells(h, _p(V), _p(c), _p(vtet), _p(rmax), nvert.ctypes.data_as(_i32p), _p(delta))
    off = np.empty(n + 1, dtype=np.int64)
    j = np.empty(nf, dtype=np.int32); code = np.empty(nf, dtype=np.int32)
    A = np.empty(nf); f = np.empty((nf, 3))
    L.orc_mesh_faces(h, off.ctypes.data_as(_i64p), j.ctypes.data_as(_i32p), code.ctypes.data_as(_i32p),
                     _p(A), _p(f))
    return Mesh(h, n, tuple(float(x) for x in box), pos, V, c, vtet, rmax, nvert, off, j, code, A, f,
                float(L.orc_mesh_delta_min(h)), int(L.orc_mesh_status(h)), delta)


def init_charges(mesh: Mesh, params: Params, prim) -> np.ndarray:
    prim = _f64(prim, (mesh.n, 5))
    Q = np.empty((mesh.n, 5))
    lib().orc_init_charges(mesh.handle, ctypes.byref(params), _p(prim), _p(Q))
    return Q


def init_entropy(mesh: Mesh, params: Params, prim) -> np.ndarray:
    """Entropy charges S = m P rho^-gamma (Sec. 4.3) of primitive states."""
    prim = _f64(prim, (mesh.n, 5))
    S = np.empty(mesh.n)
    lib().orc_init_entropy(mesh.handle, ctypes.byref(params), _p(prim), _p(S))
    return S


def cell_state(mesh: Mesh, params: Params, Q):
    Q = _f64(Q, (mesh.n, 5))
    U = np.empty((mesh.n, 5)); w = np.empty((mesh.n, 3)); dti = np.empty(mesh.n)
    hits = np.zeros(1, dtype=np.int64)
    dt = lib().orc_cell_state(mesh.handle, ctypes.byref(params), _p(Q), _p(U), _p(w), _p(dti),
                              hits.ctypes.data_as(_i64p))
    return U, w, dti, float(dt), int(hits[0])


def gradient(mesh: Mesh, params: Params, U, limit=True) -> np.ndarray:
    U = _f64(U, (mesh.n, 5))
    G = np.empty((mesh.n, 5, 3))
    lib().orc_gradient(mesh.handle, ctypes.byref(params), _p(U), _p(G), 1 if limit else 0)
    return G


def predict(mesh: Mesh, params: Params, U, G, w, dt, form=0):
    U = _f64(U, (mesh.n, 5)); G = _f64(G, (mesh.n, 5, 3)); w = _f64(w, (mesh.n, 3))
    Uh = np.empty((mesh.n, 5)); hits = np.zeros(1, dtype=np.int64)
    lib().orc_predict(mesh.handle, ctypes.byref(params), _p(U), _p(G), _p(w), float(dt), _p(Uh), int(form),
                      hits.ctypes.data_as(_i64p))
    return Uh, int(hits[0])


def fluxes(mesh: Mesh, params: Params, Uh, Gh, w, dt):
    Uh = _f64(Uh, (mesh.n, 5)); Gh = _f64(Gh, (mesh.n, 5, 3)); w = _f64(w, (mesh.n, 3))
    dQ = np.empty((mesh.n, 5)); hits = np.zeros(1, dtype=np.int64)
    rc = lib().orc_fluxes(mesh.handle, ctypes.byref(params), _p(Uh), _p(Gh), _p(w), float(dt), _p(dQ),
                          hits.ctypes.data_as(_i64p))
    if rc:
        raise RuntimeError(f"oracle fluxes failed (code {rc}): asymmetric face topology")
    return dQ, int(hits[0])


def face_states(mesh: Mesh, params: Params, Uh, Gh, w):
    """Reconstructed states of every directed face (ordered like mesh.j):
    returns (UL, UR, normal, face velocity)."""
    Uh = _f64(Uh, (mesh.n, 5)); Gh = _f64(Gh, (mesh.n, 5, 3)); w = _f64(w, (mesh.n, 3))
    nf = mesh.j.shape[0]
    UL = np.empty((nf, 5)); UR = np.empty((nf, 5)); nrm = np.empty((nf, 3)); wt = np.empty((nf, 3))
    lib().orc_face_states(mesh.handle, ctypes.byref(params), _p(Uh), _p(Gh), _p(w), _p(UL), _p(UR), _p(nrm), _p(wt))
    return UL, UR, nrm, wt


def step(pos, Q, params: Params, dt_max=1e300, method="grid"):
    """One whole step.  Returns (pos', Q', w, dt, counters)."""
    pos = _f64(pos).copy(); Q = _f64(Q).copy()
    n = pos.shape[0]
    w = np.empty((n, 3)); dt = np.zeros(1); cnt = np.zeros(4, dtype=np.int64)
    rc = lib().orc_step(n, _p(pos), _p(Q), _p(w), ctypes.byref(params), float(dt_max),
                        1 if method == "grid" else 0, _p(dt), cnt.ctypes.data_as(_i64p))
    if rc:
        raise RuntimeError(f"oracle step failed (code {rc})")
    return pos, Q, w, float(dt[0]), cnt


def step_entropy(pos, Q, S, params: Params, dt_max=1e300, method="grid"):
    """One whole step with the entropy column (Sec. 4.3).  Returns
    (pos', Q', S', w, dt, counters, mach) with mach each cell's largest face
    Mach number."""
    pos = _f64(pos).copy(); Q = _f64(Q).copy(); S = _f64(S).copy()
    n = pos.shape[0]
    w = np.empty((n, 3)); dt = np.zeros(1); cnt = np.zeros(4, dtype=np.int64); mach = np.empty(n)
    rc = lib().orc_step_entropy(n, _p(pos), _p(Q), _p(S), _p(w), ctypes.byref(params), float(dt_max),
                                1 if method == "grid" else 0, _p(dt), cnt.ctypes.data_as(_i64p), _p(mach))
    if rc:
        raise RuntimeError(f"oracle step failed (code {rc})")
    return pos, Q, S, w, float(dt[0]), cnt, mach


def face_velocity(ri, rj_img, wi, wj, f) -> np.ndarray:
    a = [_f64(x) for x in (ri, rj_img, wi, wj, f)]
    out = np.empty(3)
    lib().orc_face_velocity(*[_p(x) for x in a], _p(out))
    return out


def moving_face_flux(UL, UR, n, wt, gamma, riemann=0) -> np.ndarray:
    """Lab-frame flux across a moving face; riemann 0 is HLLC, 1 is HLL."""
    a = [_f64(x) for x in (UL, UR, n, wt)]
    F = np.empty(5)
    lib().orc_moving_face_flux(*[_p(x) for x in a], float(gamma), int(riemann), _p(F))
    return F


def hllc_prim(WL, WR, n, gamma) -> np.ndarray:
    a = [_f64(x) for x in (WL, WR, n)]
    F = np.empty(5)
    lib().orc_hllc_prim(*[_p(x) for x in a], float(gamma), _p(F))
    return F


def entropy_face(WL, WR, n, gamma, riemann, AL, AR):
    """Face-frame flux of rho A and the face's shock Mach number (Sec. 4.3)."""
    a = [_f64(x) for x in (WL, WR, n)]
    FX, mach = np.zeros(1), np.zeros(1)
    lib().orc_entropy_face(*[_p(x) for x in a], float(gamma), int(riemann), float(AL), float(AR), _p(FX), _p(mach))
    return float(FX[0]), float(mach[0])


def hll_prim(WL, WR, n, gamma) -> np.ndarray:
    a = [_f64(x) for x in (WL, WR, n)]
    F = np.empty(5)
    lib().orc_hll_prim(*[_p(x) for x in a], float(gamma), _p(F))
    return F


def dm_factor(theta, dU, D) -> float:
    return float(lib().orc_dm_factor(float(theta), float(dU), float(D)))


def apply_floors(params: Params, U):
    U = _f64(U).copy()
    hits = int(lib().orc_apply_floors(ctypes.byref(params), _p(U)))
    return U, hits


def exact_riemann(WL, WR, gamma, xi):
    """Exact Riemann solution sampled at xi = x/t; returns (W[m,3], p*, u*)."""
    WL = _f64(WL); WR = _f64(WR); xi = _f64(xi)
    m = xi.shape[0]
    W = np.empty((m, 3)); star = np.empty(2)
    rc = lib().orc_exact_riemann(_p(WL), _p(WR), float(gamma), m, _p(xi), _p(W), _p(star))
    if rc:
        raise ValueError("vacuum generated")
    return W, float(star[0]), float(star[1])
