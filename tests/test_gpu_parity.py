"""Parity of the HIP path with the CPU oracle, through the C ABI.

Tessellation: the neighbour topology must match bit-exactly on certified
non-degenerate inputs; volumes, centroids, areas and face centres within
1e-10 of the cell scale.  States after whole steps (FP64): element by
element within 1e-10 of that element's own scale (the largest value of its
column over the cell and its neighbours, and at least the cell's rounding
scale: m, m(|v| + c_s), |E|).  The component calls on smooth states are
compared against each column's scale.
"""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import compare_mesh, dev, host, local_err, mesh_pair, state_scale

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _print_case(what, **kw):
    print(f"[case] {what} {kw}", flush=True)


TESS_CASES = [
    ("c1_lattice_16", lambda: (W.jittered_lattice((16, 16, 16), (1, 1, 1), seed=1), (1, 1, 1))),
    ("lattice_ragged_7x9x11", lambda: (W.jittered_lattice((7, 9, 11), (0.7, 0.9, 1.1), seed=3), (0.7, 0.9, 1.1))),
    ("sod_strip_64x8x8", lambda: (W.jittered_lattice((64, 8, 8), (4, 0.5, 0.5), seed=2), (4, 0.5, 0.5))),
    ("poisson_3001", lambda: (W.poisson_points(3001, (1, 1, 1), seed=4), (1, 1, 1))),
    ("poisson_20000", lambda: (W.poisson_points(20000, (1, 2, 0.5), seed=6), (1, 2, 0.5))),
    ("lattice_3", lambda: (W.jittered_lattice((3, 3, 3), (1, 1, 1), seed=5), (1, 1, 1))),
    ("lattice_2x3x4", lambda: (W.jittered_lattice((2, 3, 4), (1, 1, 1), seed=8), (1, 1, 1))),
]


@pytest.mark.parametrize("name,make", TESS_CASES, ids=[c[0] for c in TESS_CASES])
def test_tessellation_parity(orc, name, make):
    pos, box = make()
    _print_case("tessellation", name=name, n=pos.shape[0])
    mm, info, om = mesh_pair(orc, pos, box, method="brute" if pos.shape[0] <= 64 else "grid")
    assert om.status == 0
    om_cert = orc.tessellate(pos, box, method="grid", certificate=True)
    assert om_cert.delta_min > 1e-12, "input not certified non-degenerate"
    compare_mesh(mm, om)
    assert info["n_faces"] * 2 == len(om.j)


@pytest.mark.parametrize("hole", [1.0, 1.7], ids=["candidate_overflow", "slot_overflow"])
def test_crowded_site_cells_are_handed_on(orc, hole):
    """Cells that the two-cells-per-wavefront first pass cannot hold are built
    again by the one-cell first pass.  Around the crowded site with the small
    hole, the shell and its neighbours see more than 48 candidates; with the
    large hole the centre sees 36, and its 36 faces (68 vertices) need more
    plane and vertex slots than a half-wavefront keeps, so it is handed on in
    the middle of its cuts.  Either way the tessellation matches the
    oracle's."""
    pos = W.crowded_site(hole=hole)
    _print_case("crowded site", hole=hole, n=pos.shape[0])
    mm, info, om = mesh_pair(orc, pos, (1, 1, 1))
    assert om.status == 0
    assert om.delta_min > 1e-12, "input not certified non-degenerate"
    assert int(np.diff(om.off)[pos.shape[0] - 37]) == 36
    compare_mesh(mm, om)
    assert info["rebuilt_cells"] > 0 and info["n_faces"] * 2 == len(om.j)


def test_tessellation_parity_on_a_deformed_sod_tube(orc):
    """The mesh of a Sod tube after 30 oracle steps: shock, contact and
    rarefaction have compressed and stretched layers of the lattice, and the
    jitter has turned into sliver faces (the certificate's margin is
    7e-11).  The positions come from the oracle's own steps; the GPU
    tessellation of them matches the oracle's: the same faces, volumes,
    centroids and areas within 1e-10, face centroids within 1e-9 of the
    cell scale (a sliver's centroid comes from nearly coincident vertices,
    whose rounding the near-degeneracy amplifies in both implementations:
    up to 5e-10 h, on faces of area 1e-5 h^2, while their areas agree to
    1e-13 h^2)."""
    import paper_1707_05333_amd as M
    wl = W.c2_sod(shape=(128, 16, 16), box=(4.0, 0.5, 0.5))
    _print_case("deformed sod tube", n=wl.n, oracle_steps=30)
    p = orc.make_params(wl.box, **wl.params)
    Q = orc.init_charges(orc.tessellate(wl.pos, wl.box), p, wl.prim)
    pos = wl.pos.copy()
    for _ in range(30):
        pos, Q, _w, _dt, _cnt = orc.step(pos, Q, p)
    mm, info, om = mesh_pair(orc, pos, wl.box, **wl.params)
    assert om.status == 0
    assert om.delta_min > 1e-12, "input not certified non-degenerate"
    compare_mesh(mm, om, ftol=1e-9)
    assert info["n_faces"] * 2 == len(om.j)


def test_bcc_closed_form_on_gpu():
    # Exact body-centred cubic lattice: every cell is the truncated
    # octahedron (volume a^3/2, 6 squares a^2/8, 8 hexagons 3 sqrt(3) a^2/16,
    # centroid at the generator).  The lattice is degenerate for the
    # certificate, so only the unique geometry is compared.
    import paper_1707_05333_amd as M
    m = 5
    a = 1.0 / m
    pos = W.bcc_lattice(m)
    _print_case("bcc", n=pos.shape[0])
    mm = M.MovingMesh(pos.shape[0], M.make_params(box=(1, 1, 1)))
    info = mm.tessellate(dev(pos))
    ex = mm.mesh_export()
    np.testing.assert_allclose(host(ex.V), a ** 3 / 2, rtol=1e-12)
    assert np.abs(host(ex.centroid) - pos).max() < 1e-14
    A = np.sort(host(ex.face_A))
    assert info["n_faces"] == 7 * pos.shape[0]
    np.testing.assert_allclose(A[: 3 * pos.shape[0]], a * a / 8, rtol=1e-12)
    np.testing.assert_allclose(A[3 * pos.shape[0]:], 3 * math.sqrt(3) * a * a / 16, rtol=1e-12)


@pytest.mark.parametrize("pos,box", [(np.array([[0.3, 0.6, 0.1]]), (2, 1, 0.5)),
                                     (np.array([[0.3, 0.5, 0.5], [1.62, 0.5, 0.5]]), (2, 1, 1))],
                         ids=["one_point", "two_points"])
def test_tiny_sets_violate_box_precondition(pos, box):
    # With one or two generators twice the farthest vertex exceeds the box,
    # outside the scheme's periodic premise: the library refuses.
    import paper_1707_05333_amd as M
    _print_case("tiny", n=pos.shape[0])
    mm = M.MovingMesh(pos.shape[0], M.make_params(box=box))
    with pytest.raises(M.MMError) as e:
        mm.tessellate(dev(pos))
    assert e.value.name == "MM_EDEGENERATE"


def _setup(orc, wl, precision="fp64", **over):
    import paper_1707_05333_amd as M
    params = dict(wl.params)
    params.update(over)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision=precision, **params))
    mm.tessellate(dev(wl.pos))
    p = orc.make_params(wl.box, **params)
    om = orc.tessellate(wl.pos, wl.box)
    return mm, p, om


def _check_components(orc, wl):
    """Every component call against the oracle, element by element: charges,
    cell states, mesh velocities, timestep, gradients (limited and not),
    predictor and the per-cell face-flux sums."""
    mm, p, om = _setup(orc, wl)
    gamma = wl.params["gamma"]
    # charges (Sec. 4.3)
    Qg = host(mm.init_charges(dev(wl.prim)))
    Qo = orc.init_charges(om, p, wl.prim)
    assert local_err(Qg, Qo, om, state_scale(Qo, gamma)) < TOL
    # cell state, mesh velocity, timestep (Sec. 4.2)
    Ug, wg, dtg, hg = mm.cell_state(dev(Qo))
    Uo, wo, dti, dto, ho = orc.cell_state(om, p, Qo)
    assert hg == ho == 0
    su = state_scale(Uo, gamma)
    speed = su[:, 1] / su[:, 0]                       # |v| + c_s
    assert local_err(host(Ug), Uo, om, su) < TOL
    assert local_err(host(wg), wo, om, np.repeat(speed[:, None], 3, axis=1)) < TOL
    assert abs(dtg - dto) <= TOL * dto
    # gradients with and without the S10 limiter (Sec. 4.1): each component
    # against the size of its whole gradient vector
    for limit in (False, True):
        Gg = host(mm.gradients(dev(Uo), limit=limit))
        Go = orc.gradient(om, p, Uo, limit=limit)
        gnorm = np.repeat(np.sqrt((Go ** 2).sum(axis=2)), 3, axis=1)
        assert local_err(Gg, Go, om, gnorm) < TOL, f"limit={limit}"
    # predictor (Sec. 4.1)
    dt = 0.5 * dto
    Uhg = host(mm.predict(dev(Uo), dev(Go), dev(wo), dt))
    Uho, _ = orc.predict(om, p, Uo, Go, wo, dt)
    assert local_err(Uhg, Uho, om, state_scale(Uho, gamma)) < TOL
    # face fluxes summed per cell (Sec. 4 items 1-5): against the size of
    # one cell's face fluxes, dt (sum of its face areas) (|v| + c_s) U
    Gho = orc.gradient(om, p, Uho, limit=True)
    dQg = host(mm.fluxes(dev(Uho), dev(Gho), dev(wo), dt))
    dQo, _ = orc.fluxes(om, p, Uho, Gho, wo, dt)
    sh = state_scale(Uho, gamma)
    area = np.bincount(om.face_owner(), weights=om.A, minlength=om.n)
    fscale = dt * (area * sh[:, 1] / sh[:, 0])[:, None] * sh
    assert local_err(dQg, dQo, om, fscale) < TOL
    assert np.abs(dQg).max() > 0


def test_charges_state_gradient_predictor_flux_parity(orc):
    box = (1.0, 1.0, 1.0)
    wl = W.random_smooth_state(W.jittered_lattice((12, 12, 12), box, seed=11), box, seed=11, amp=0.3)
    _print_case("components", n=wl.n)
    _check_components(orc, wl)


SMALL_MESHES = [
    ("lattice_3", lambda: W.jittered_lattice((3, 3, 3), (1, 1, 1), seed=5)),
    ("lattice_4", lambda: W.jittered_lattice((4, 4, 4), (1, 1, 1), seed=21)),
    ("lattice_2x3x4", lambda: W.jittered_lattice((2, 3, 4), (1, 1, 1), seed=8)),
]


@pytest.mark.parametrize("name,make", SMALL_MESHES, ids=[c[0] for c in SMALL_MESHES])
def test_small_mesh_components_and_steps(orc, name, make):
    # Meshes of 24-64 cells have fewer faces than one block of the face
    # kernel per XCD range: every face's flux must still be computed.
    box = (1.0, 1.0, 1.0)
    wl = W.random_smooth_state(make(), box, seed=17, amp=0.3)
    _print_case("small mesh", name=name, n=wl.n)
    _check_components(orc, wl)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 2)
    assert _state_err(Qg, Qo, wl) < TOL
    assert np.abs(pg - po).max() < TOL


def _run_steps(orc, wl, nsteps, precision="fp64", **over):
    import paper_1707_05333_amd as M
    import torch
    params = dict(wl.params)
    params.update(over)
    p = orc.make_params(wl.box, **params)
    om = orc.tessellate(wl.pos, wl.box)
    Q0 = orc.init_charges(om, p, wl.prim)
    if wl.energy_cells is not None:
        Q0[wl.energy_cells, 4] += wl.energy_amount
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision=precision, **params))
    pos_g, Q_g = dev(wl.pos), dev(Q0)
    w_g = torch.empty_like(pos_g)
    pos_o, Q_o = wl.pos.copy(), Q0.copy()
    for k in range(nsteps):
        info = mm.step(pos_g, w_g, Q_g)
        start = pos_o
        pos_o, Q_o, w_o, dt_o, cnt = orc.step(pos_o, Q_o, p)
        assert abs(info["dt"] - dt_o) <= TOL * dt_o, f"step {k}: dt {info['dt']} vs {dt_o}"
        assert info["floor_hits"] == list(cnt)
    _run_steps.mesh = orc.tessellate(start, wl.box) if nsteps else None
    return host(pos_g), host(Q_g), host(w_g), pos_o, Q_o, w_o


def _state_err(Qg, Qo, wl):
    """Per-element error of charges after steps, against the neighbourhood
    of the last step's mesh (see the module docstring)."""
    return local_err(Qg, Qo, _run_steps.mesh, state_scale(Qo, wl.params["gamma"]))


def _vel_err(wg, wo, Qo, wl):
    """Per-element error of mesh velocities, each against the largest speed
    plus sound speed of its neighbourhood."""
    sc = state_scale(Qo, wl.params["gamma"])
    vel = np.repeat((sc[:, 1] / np.maximum(sc[:, 0], 1e-300))[:, None], 3, axis=1)
    return local_err(wg, wo, _run_steps.mesh, vel)


def test_step_parity_c1(orc):
    wl = W.c1_uniform_random_velocity()
    _print_case("step c1", n=wl.n)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 1)
    assert _state_err(Qg, Qo, wl) < TOL
    assert np.abs(pg - po).max() < TOL
    assert _vel_err(wg, wo, Qo, wl) < TOL


def test_step_parity_sod_strip(orc):
    wl = W.c2_sod(shape=(64, 8, 8), box=(4.0, 0.5, 0.5))
    _print_case("step sod strip", n=wl.n, steps=5)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 5)
    assert _state_err(Qg, Qo, wl) < TOL
    assert np.abs(pg - po).max() < TOL


def test_step_parity_poisson_smooth(orc):
    box = (1.0, 1.0, 1.0)
    wl = W.random_smooth_state(W.poisson_points(2500, box, seed=9), box, seed=9, amp=0.2)
    _print_case("step poisson", n=wl.n, steps=2)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 2)
    assert _state_err(Qg, Qo, wl) < TOL
    assert np.abs(pg - po).max() < TOL


def test_step_parity_gresho(orc):
    # The Gresho-Chan vortex (Sec. 5) at an equivalent 2D resolution of 16^2:
    # a rotating, pressure-supported state on a thin periodic slab.
    wl = W.gresho(16)
    _print_case("step gresho", n=wl.n, steps=3)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 3)
    assert _state_err(Qg, Qo, wl) < TOL
    assert np.abs(pg - po).max() < TOL


def test_step_parity_blast(orc):
    wl = W.c3_point_blast(n_side=16)
    _print_case("step blast", n=wl.n, steps=3)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 3)
    assert _state_err(Qg, Qo, wl) < TOL


def test_uniform_state_and_conservation_on_gpu(orc):
    import paper_1707_05333_amd as M
    import torch
    box = (1.0, 1.0, 1.0)
    wl = W.uniform_state(W.jittered_lattice((10, 10, 10), box, seed=4), box, vel=(0.3, -0.2, 0.1))
    _print_case("uniform", n=wl.n)
    mm = M.MovingMesh(wl.n, M.make_params(box=box, **wl.params))
    mm.tessellate(dev(wl.pos))
    Q = mm.init_charges(dev(wl.prim))
    U0 = host(Q) / host(mm.mesh_export().V)[:, None]
    pos = dev(wl.pos)
    w = torch.empty_like(pos)
    S0 = host(Q).sum(axis=0)
    for _ in range(10):
        mm.step(pos, w, Q)
    mm.tessellate(pos)
    U1 = host(Q) / host(mm.mesh_export().V)[:, None]
    assert np.abs(U1 / U0 - 1).max() < 1e-12
    assert np.all(np.abs(host(Q).sum(axis=0) - S0) <= 1e-13 * np.abs(host(Q)).sum(axis=0))


def test_deterministic_and_resumable(orc):
    # Two runs give bitwise-identical states; a run split with a copy of
    # (pos, Q) in between equals the uninterrupted run (restart, Sec. 4.3).
    import paper_1707_05333_amd as M
    import torch
    wl = W.c2_sod(shape=(32, 8, 8), box=(4.0, 1.0, 1.0))
    _print_case("determinism", n=wl.n)
    p = orc.make_params(wl.box, **wl.params)
    om = orc.tessellate(wl.pos, wl.box)
    Q0 = orc.init_charges(om, p, wl.prim)

    def run(nsteps, pos, Q):
        mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **wl.params))
        w = torch.empty_like(pos)
        for _ in range(nsteps):
            mm.step(pos, w, Q)
        return pos, Q

    a = run(6, dev(wl.pos), dev(Q0))
    b = run(6, dev(wl.pos), dev(Q0))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    c = run(2, dev(wl.pos), dev(Q0))
    c = run(4, c[0].cpu().clone().cuda(), c[1].cpu().clone().cuda())
    assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1])


def test_error_paths(orc):
    import paper_1707_05333_amd as M
    import torch
    mm = M.MovingMesh(100, M.make_params(box=(1, 1, 1)))
    bad = dev(np.array([[0.5, 0.5, 1.5]] + [[0.1 * (k % 9) + 0.05, 0.3, 0.4] for k in range(7)]))
    with pytest.raises(M.MMError) as e:
        mm.tessellate(bad)
    assert e.value.name == "MM_EINVAL"
    with pytest.raises(M.MMError) as e:
        mm.tessellate(dev(W.jittered_lattice((5, 5, 5), (1, 1, 1))))   # 125 > capacity 100
    assert e.value.name == "MM_EINVAL"
    fresh = M.MovingMesh(10, M.make_params(box=(1, 1, 1)))
    with pytest.raises(M.MMError) as e:
        fresh.gradients(torch.zeros(0, 5, dtype=torch.float64, device="cuda"))
    assert e.value.name == "MM_ESTATE"
    small = M.MovingMesh(64, M.make_params(box=(1, 1, 1)), face_capacity=10)
    with pytest.raises(M.MMError) as e:
        small.tessellate(dev(W.jittered_lattice((4, 4, 4), (1, 1, 1), seed=1)))
    assert e.value.name == "MM_ECAPACITY"


def test_step_parity_hll_sod_strip(orc):
    # HLL face fluxes (Sec. 4 item 4) on the shock-tube strip.
    wl = W.c2_sod(shape=(64, 8, 8), box=(4.0, 0.5, 0.5))
    _print_case("step sod strip hll", n=wl.n, steps=5)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 5, riemann=1)
    assert _state_err(Qg, Qo, wl) < TOL
    assert np.abs(pg - po).max() < TOL


@pytest.mark.parametrize("riemann", [0, 1], ids=["hllc", "hll"])
def test_step_parity_static_mesh_paper_sod(orc, riemann):
    # The paper's Sod tube (16 x 1 x 1, rho_R = 0.25, P_R = 0.1795) on a
    # static mesh (w = 0, Sec. 4.2): generators stay exactly in place.
    wl = W.sod_paper(k=4, static_mesh=True, riemann=("hllc", "hll")[riemann])
    _print_case("step paper sod static", n=wl.n, steps=5, riemann=riemann)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 5)
    assert _state_err(Qg, Qo, wl) < TOL
    assert np.array_equal(pg, wl.pos) and np.array_equal(po, wl.pos)
    assert not wg.any()


@pytest.mark.parametrize("name", ["gresho_16", "sod_strip"])
def test_step_parity_half_step_mesh(orc, name):
    # Fluxes on the mesh rebuilt at the half-step positions (the paper's
    # first future improvement, Sec. 6): rotating and shocked flows, so the
    # half-step mesh differs from the start-of-step one.
    wl = W.gresho(16) if name == "gresho_16" else W.c2_sod(shape=(64, 8, 8), box=(4.0, 0.5, 0.5))
    _print_case("step half-step mesh", name=name, n=wl.n, steps=4)
    pg, Qg, wg, po, Qo, wo = _run_steps(orc, wl, 4, half_step_mesh=1)
    assert _state_err(Qg, Qo, wl) < TOL
    assert np.abs(pg - po).max() < TOL
    assert _vel_err(wg, wo, Qo, wl) < TOL
