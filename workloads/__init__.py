"""Seeded synthetic inputs for the moving-mesh finite-volume step.

This module is shared by the HIP path, the CPU oracle, the tests and the
benchmark.  It only draws point positions and primitive fields
(rho, vx, vy, vz, P); it holds none of the method's arithmetic (no volumes,
no charges, no fluxes).  Every generator is deterministic in its seed
(numpy PCG64).

The paper's own initial conditions are tiled glass files (Sec. 5
introduction), which are not available; jittered cubic lattices and Poisson
points of the same shapes and sizes stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Default scheme parameters.  eta = 1 (Lagrangian mesh), chi = 1 and
# zeta = 0.25 (Sec. 4.2), theta = 0.49 (Sec. 5.1), floors far below every
# workload's density and pressure.
DEFAULT_PARAMS = dict(
    gamma=5.0 / 3.0,
    cfl=0.3,
    eta=1.0,
    chi=1.0,
    zeta=0.25,
    theta=0.49,
    rho_floor=1e-12,
    p_floor=1e-14,
)


@dataclass
class Workload:
    """One synthetic simulation input.

    pos   : float64 [n, 3], every coordinate in [0, box).
    prim  : float64 [n, 5], columns rho, vx, vy, vz, P.
    box   : periodic box lengths.
    params: scheme parameters (gamma, cfl, eta, chi, zeta, theta, floors).
    steps : number of steps the workload is defined for.
    energy_cells / energy_amount: optional point deposit of total energy,
        added to the charge E of each listed cell after the first
        tessellation.
    """

    name: str
    pos: np.ndarray
    prim: np.ndarray
    box: tuple
    params: dict
    steps: int
    energy_cells: np.ndarray | None = None
    energy_amount: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _params(**over):
    p = dict(DEFAULT_PARAMS)
    p.update(over)
    return p


def _wrap_inside(pos: np.ndarray, box) -> np.ndarray:
    """Move coordinates into [0, L) (only ever needed for jitter at edges)."""
    L = np.asarray(box, dtype=np.float64)
    pos = np.where(pos < 0.0, pos + L, pos)
    pos = np.where(pos >= L, pos - L, pos)
    return np.ascontiguousarray(pos, dtype=np.float64)


def jittered_lattice(shape, box, jitter=1e-3, seed=0) -> np.ndarray:
    """Cubic lattice with nx*ny*nz points at ((i + 1/2) h) plus uniform
    jitter in [-jitter*h, +jitter*h] per axis (h the lattice spacing of that
    axis).  Point order is x fastest, then y, then z."""
    nx, ny, nz = (int(s) for s in shape)
    L = np.asarray(box, dtype=np.float64)
    h = L / np.array([nx, ny, nz], dtype=np.float64)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    base = (base + 0.5) * h
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter, jitter, size=base.shape) * h
    return _wrap_inside(base + jit, box)


def poisson_points(n, box, seed=0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=np.float64)
    return _wrap_inside(rng.uniform(0.0, 1.0, size=(int(n), 3)) * L, box)


def crowded_site(m=16, n_shell=36, seed=9, r_lo=0.28, r_hi=0.34, hole=1.0) -> np.ndarray:
    """Jittered m^3 lattice in the unit box with a crowded site at the box
    centre (a corner shared by eight lattice cells): the lattice points
    closer than `hole` spacings to it are removed, and a point near the
    centre is surrounded by n_shell points on a rough sphere (spiral
    directions, radii uniform in [r_lo, r_hi] spacings, all jittered so no
    five points are cospherical).  The centre's cell has about n_shell
    faces; the points spread over the eight lattice cells around the centre,
    a handful each.  Point order: the lattice (x fastest), then the centre,
    then the shell."""
    h = 1.0 / m
    rng = np.random.default_rng(seed)
    lat = jittered_lattice((m, m, m), (1.0, 1.0, 1.0), seed=seed)
    c = np.full(3, 0.5)
    lat = lat[np.linalg.norm(lat - c, axis=1) >= hole * h]
    k = np.arange(n_shell) + 0.5
    phi = np.arccos(1.0 - 2.0 * k / n_shell) + rng.uniform(-0.05, 0.05, n_shell)
    th = np.pi * (1.0 + 5.0 ** 0.5) * k + rng.uniform(-0.05, 0.05, n_shell)
    d = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)
    r = rng.uniform(r_lo, r_hi, n_shell) * h
    centre = c + rng.uniform(-0.01, 0.01, 3) * h
    shell = centre + d * r[:, None]
    return _wrap_inside(np.concatenate([lat, centre[None, :], shell]), (1.0, 1.0, 1.0))


def bcc_lattice(m, box=(1.0, 1.0, 1.0), offset=0.25) -> np.ndarray:
    """Body-centred cubic lattice: m^3 cube corners plus m^3 body centres
    (2 m^3 points), cubic side a = L/m.  `offset` (in units of a) shifts the
    whole lattice away from the box walls.  No jitter: the Voronoi cell of
    every point is the same truncated octahedron."""
    L = np.asarray(box, dtype=np.float64)
    a = L / m
    iz, iy, ix = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    base = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    corners = (base + offset) * a
    centres = (base + offset + 0.5) * a
    return _wrap_inside(np.concatenate([corners, centres], axis=0), box)


# ---------------------------------------------------------------------------
# The five workloads.  Sizes default to the full configurations; the tests
# call them with smaller shapes of the same structure.
# ---------------------------------------------------------------------------

def c1_uniform_random_velocity(n_side=16, seed=1) -> Workload:
    """Unit cube, n_side^3 jittered lattice, gamma = 5/3, rho = 1, P = 1,
    velocities uniform in [-0.1, 0.1]^3, one step at CFL 0.3."""
    box = (1.0, 1.0, 1.0)
    pos = jittered_lattice((n_side,) * 3, box, seed=seed)
    n = pos.shape[0]
    rng = np.random.default_rng(seed + 1000)
    prim = np.empty((n, 5))
    prim[:, 0] = 1.0
    prim[:, 1:4] = rng.uniform(-0.1, 0.1, size=(n, 3))
    prim[:, 4] = 1.0
    return Workload("c1_uniform_random_velocity", pos, prim, box,
                    _params(gamma=5.0 / 3.0), steps=1,
                    meta=dict(shape=(n_side,) * 3))


def c2_sod(shape=(256, 64, 64), seed=2, box=(4.0, 1.0, 1.0)) -> Workload:
    """Periodic Sod shock tube: x < L/2: rho = 1, P = 1; x >= L/2:
    rho = 0.125, P = 0.1; v = 0, gamma = 1.4, Lagrangian mesh, 50 steps."""
    pos = jittered_lattice(shape, box, seed=seed)
    n = pos.shape[0]
    prim = np.zeros((n, 5))
    left = pos[:, 0] < 0.5 * box[0]
    prim[:, 0] = np.where(left, 1.0, 0.125)
    prim[:, 4] = np.where(left, 1.0, 0.1)
    return Workload("c2_sod", pos, prim, box, _params(gamma=1.4), steps=50,
                    meta=dict(shape=tuple(shape)))


def c3_point_blast(n_side=128, seed=3, n_hot=32) -> Workload:
    """Unit cube, n_side^3 jittered lattice, rho = 1, P = 1e-5, v = 0,
    gamma = 5/3; total energy 1 shared equally by the n_hot generators
    nearest the box centre; 100 steps."""
    box = (1.0, 1.0, 1.0)
    pos = jittered_lattice((n_side,) * 3, box, seed=seed)
    n = pos.shape[0]
    prim = np.zeros((n, 5))
    prim[:, 0] = 1.0
    prim[:, 4] = 1e-5
    r2 = np.sum((pos - 0.5) ** 2, axis=1)
    hot = np.argsort(r2, kind="stable")[:n_hot]
    return Workload("c3_point_blast", pos, prim, box, _params(gamma=5.0 / 3.0),
                    steps=100, energy_cells=np.sort(hot).astype(np.int64),
                    energy_amount=1.0 / n_hot, meta=dict(shape=(n_side,) * 3))


def c4_kelvin_helmholtz(k, n_min=1000, n_max=200000, base_seed=4000) -> Workload:
    """Serving request k: unit cube, N drawn log-uniform in [n_min, n_max],
    rounded to a cube n^3; slab |y - 0.5| < 0.25 has rho = 2, vx = +0.5,
    outside rho = 1, vx = -0.5; P = 2.5; vy = 0.01 sin(4 pi x); 20 steps."""
    seed = base_seed + int(k)
    rng = np.random.default_rng(seed)
    n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
    side = max(2, int(round(n_target ** (1.0 / 3.0))))
    box = (1.0, 1.0, 1.0)
    pos = jittered_lattice((side,) * 3, box, seed=seed)
    n = pos.shape[0]
    inner = np.abs(pos[:, 1] - 0.5) < 0.25
    prim = np.zeros((n, 5))
    prim[:, 0] = np.where(inner, 2.0, 1.0)
    prim[:, 1] = np.where(inner, 0.5, -0.5)
    prim[:, 2] = 0.01 * np.sin(4.0 * np.pi * pos[:, 0])
    prim[:, 4] = 2.5
    return Workload(f"c4_kh_{k}", pos, prim, box, _params(gamma=5.0 / 3.0),
                    steps=20, meta=dict(shape=(side,) * 3, request=int(k)))


def gresho_profile(r):
    """Gresho-Chan vortex (Sec. 5 test problems): the steady pressure and
    tangential speed at cylinder radius r (rho = 1)."""
    r = np.asarray(r, dtype=np.float64)
    inner, mid = r < 0.2, (r >= 0.2) & (r < 0.4)
    P = np.full(r.shape, 3.0 + 4.0 * math.log(2.0))
    P = np.where(inner, 5.0 + 12.5 * r * r, P)
    with np.errstate(divide="ignore"):
        P = np.where(mid, 9.0 + 12.5 * r * r - 20.0 * r + 4.0 * np.log(np.maximum(5.0 * r, 1e-300)), P)
    vphi = np.where(inner, 5.0 * r, np.where(mid, 2.0 - 5.0 * r, 0.0))
    return P, vphi


def gresho(N=64, seed=6, gamma=5.0 / 3.0, jitter=0.25) -> Workload:
    """Gresho-Chan vortex at an equivalent 2D resolution N^2: an N x N x nz
    lattice with nz = round(0.2 N) in the periodic box 1 x 1 x nz/N (about
    0.2), vortex axis along z through (0.5, 0.5).  The default jitter of a
    quarter spacing breaks the lattice's alignment with the flow, as a glass
    does, while keeping the local spacing regular."""
    nz = max(1, int(round(0.2 * N)))
    box = (1.0, 1.0, nz / N)
    pos = jittered_lattice((N, N, nz), box, jitter=jitter, seed=seed)
    n = pos.shape[0]
    dx, dy = pos[:, 0] - 0.5, pos[:, 1] - 0.5
    r = np.sqrt(dx * dx + dy * dy)
    P, vphi = gresho_profile(r)
    rs = np.where(r > 0.0, r, 1.0)
    prim = np.zeros((n, 5))
    prim[:, 0] = 1.0
    prim[:, 1] = -vphi * dy / rs
    prim[:, 2] = vphi * dx / rs
    prim[:, 4] = P
    return Workload(f"gresho_{N}", pos, prim, box, _params(gamma=gamma), steps=0,
                    meta=dict(shape=(N, N, nz), t_end=2.0))


def sod_paper(k=14, seed=7, jitter=0.25, riemann="hllc", static_mesh=False) -> Workload:
    """The paper's Sod tube (Sec. 5, Sod shock-tube test): periodic box
    16 x 1 x 1, left half rho = 1, P = 1, right half rho = 0.25,
    P = 0.1795, v = 0, gamma = 1.4, run to t = 2.  Points: a 16k x k x k
    lattice jittered by a quarter spacing (k = 14: 43,904 points; the paper
    uses about 41K).  The box is shifted by half its length, so the central
    discontinuity sits at x = 8 and the periodic one at x = 0.  riemann is
    "hllc" or "hll" (stored as the solver code 0 or 1); a static mesh sets
    the generator velocity to zero (eta = chi = 0)."""
    box = (16.0, 1.0, 1.0)
    pos = jittered_lattice((16 * k, k, k), box, jitter=jitter, seed=seed)
    n = pos.shape[0]
    prim = np.zeros((n, 5))
    left = pos[:, 0] < 8.0
    prim[:, 0] = np.where(left, 1.0, 0.25)
    prim[:, 4] = np.where(left, 1.0, 0.1795)
    over = dict(gamma=1.4, riemann={"hllc": 0, "hll": 1}[riemann])
    if static_mesh:
        over.update(eta=0.0, chi=0.0)
    return Workload(f"sod_paper_{k}", pos, prim, box, _params(**over), steps=0,
                    meta=dict(shape=(16 * k, k, k), t_end=2.0, left=(1.0, 0.0, 1.0), right=(0.25, 0.0, 0.1795)))


def lane_emden(n=1.5, h=1e-4):
    """Lane-Emden solution of index n by fourth-order Runge-Kutta from the
    series start: returns (xi, theta, -xi^2 theta') sampled up to the first
    zero xi_1 (the last sample is interpolated onto the zero)."""
    def rhs(x, y):
        th, dth = y
        return np.array([dth, -max(th, 0.0) ** n - 2.0 * dth / x])
    x = 1e-6
    y = np.array([1.0 - x * x / 6.0, -x / 3.0])
    xs, ths, ms = [0.0], [1.0], [0.0]
    while True:
        k1 = rhs(x, y); k2 = rhs(x + h / 2, y + h / 2 * k1)
        k3 = rhs(x + h / 2, y + h / 2 * k2); k4 = rhs(x + h, y + h * k3)
        yn = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if yn[0] <= 0.0:
            f = y[0] / (y[0] - yn[0])
            x1 = x + f * h
            d1 = y[1] + f * (yn[1] - y[1])
            xs.append(x1); ths.append(0.0); ms.append(-x1 * x1 * d1)
            return np.array(xs), np.array(ths), np.array(ms)
        x += h
        y = yn
        xs.append(x); ths.append(y[0]); ms.append(-x * x * y[1])


def c5_polytropes(n_points=1 << 23, seed=5, m1=1.0, m2=0.7, r1=0.1, r2=0.08, sep=0.18, rho_bg=1e-6,
                  inside_fraction=0.9) -> Workload:
    """Two touching n = 1.5 polytropes in the periodic unit box (no
    gravity: a workload of strongly non-uniform density).  G = 1; masses
    m1, m2, radii r1, r2, centres sep apart along x with the centre of mass
    at the box centre; P = K_k rho^(5/3) with K_k from the Lane-Emden
    scaling; background rho_bg, P = K_1 rho_bg^(5/3), v = 0.  The stars
    translate rigidly at -+(m_other / M) sqrt(M / sep) along y (a circular
    binary's speeds).  inside_fraction of the points sample each star's mass
    (in proportion to its mass), the rest are uniform outside both stars."""
    rng = np.random.default_rng(seed)
    xi, th, mxi = lane_emden(1.5)
    xi1, mu1 = xi[-1], mxi[-1]
    M = m1 + m2
    vorb = math.sqrt(M / sep)
    stars = []
    for (m, R, cx, vy) in ((m1, r1, 0.5 - sep * m2 / M, -vorb * m2 / M),
                           (m2, r2, 0.5 + sep * m1 / M, vorb * m1 / M)):
        alpha = R / xi1
        rho_c = m / (4.0 * math.pi * alpha ** 3 * mu1)
        K = 4.0 * math.pi * alpha ** 2 * rho_c ** (1.0 / 3.0) / 2.5
        stars.append(dict(m=m, R=R, c=np.array([cx, 0.5, 0.5]), vy=vy, alpha=alpha, rho_c=rho_c, K=K))
    n_in = int(round(inside_fraction * n_points))
    counts = [int(round(n_in * st["m"] / M)) for st in stars]
    counts[1] = n_in - counts[0]
    pos_parts, prim_parts = [], []
    for st, k in zip(stars, counts):
        # radius by inverting the mass profile, direction uniform
        u = rng.uniform(0.0, mu1, size=k)
        r = np.interp(u, mxi, xi) * st["alpha"]
        d = rng.normal(size=(k, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        pos_parts.append(st["c"] + r[:, None] * d)
        rho = st["rho_c"] * np.interp(r / st["alpha"], xi, th) ** 1.5
        rho = np.maximum(rho, rho_bg)
        pr = np.zeros((k, 5))
        pr[:, 0] = rho
        pr[:, 2] = st["vy"]
        pr[:, 4] = st["K"] * rho ** (5.0 / 3.0)
        prim_parts.append(pr)
    n_out = n_points - n_in
    out = np.empty((0, 3))
    while out.shape[0] < n_out:
        cand = rng.uniform(0.0, 1.0, size=(2 * (n_out - out.shape[0]) + 16, 3))
        keep = np.ones(cand.shape[0], dtype=bool)
        for st in stars:
            keep &= np.linalg.norm(cand - st["c"], axis=1) > st["R"]
        out = np.vstack([out, cand[keep]])
    out = out[:n_out]
    pbg = np.zeros((n_out, 5))
    pbg[:, 0] = rho_bg
    pbg[:, 4] = stars[0]["K"] * rho_bg ** (5.0 / 3.0)
    pos = _wrap_inside(np.vstack(pos_parts + [out]), (1.0, 1.0, 1.0))
    prim = np.vstack(prim_parts + [pbg])
    return Workload("c5_polytropes", pos, prim, (1.0, 1.0, 1.0), _params(gamma=5.0 / 3.0), steps=20,
                    meta=dict(stars=[{k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
                                     for st in stars], xi1=xi1, mu1=mu1))


def poisson_arrivals(n, rate, seed=4) -> np.ndarray:
    """Arrival times (seconds, non-decreasing, first at 0) of n requests of a
    Poisson stream with the given rate (requests per second)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / float(rate), size=int(n))
    gaps[0] = 0.0
    return np.cumsum(gaps)


def uniform_state(pos, box, rho=1.0, vel=(0.0, 0.0, 0.0), P=1.0, gamma=5.0 / 3.0,
                  name="uniform", **over) -> Workload:
    """Uniform density, velocity and pressure on a given point set."""
    n = pos.shape[0]
    prim = np.empty((n, 5))
    prim[:, 0] = rho
    prim[:, 1:4] = np.asarray(vel, dtype=np.float64)
    prim[:, 4] = P
    return Workload(name, np.ascontiguousarray(pos), prim, tuple(box),
                    _params(gamma=gamma, **over), steps=10)


def random_smooth_state(pos, box, seed=0, amp=0.2, gamma=5.0 / 3.0, name="smooth",
                        **over) -> Workload:
    """A smooth periodic non-uniform state (sums of low sine modes) used by
    parity tests: every component varies, nothing is near a floor."""
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=np.float64)
    x = pos / L
    n = pos.shape[0]
    prim = np.empty((n, 5))
    base = [1.0, 0.0, 0.0, 0.0, 1.0]
    for c in range(5):
        acc = np.full(n, base[c])
        for _ in range(3):
            kv = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(-amp, amp) * (0.5 if c in (0, 4) else 1.0)
            acc += a * np.sin(2 * np.pi * (x @ kv) + ph)
        prim[:, c] = acc
    return Workload(name, np.ascontiguousarray(pos), prim, tuple(box),
                    _params(gamma=gamma, **over), steps=5)


def mean_spacing(n, box) -> float:
    return float((box[0] * box[1] * box[2] / n) ** (1.0 / 3.0))
