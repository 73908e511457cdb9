"""GPU checks on the two-polytrope workload (two touching n = 1.5 stars in a
background a million times thinner: cell sizes differ ~20x in length):

* 20K points: the whole tessellation against the oracle (topology bit-exact,
  geometry within 1e-10 of the cell scale), two FP64 steps against the
  oracle element by element (every charge within 1e-10 of its own scale:
  the largest value of its column over the cell and its neighbours, and at
  least m, m(|v| + c_s), |E| of those cells, so a background cell a million
  times thinner than a star's core is measured against its own
  neighbourhood; the floor and fall-back counters equal), and three mixed
  steps: finite, mass conserved to rounding, density within 1e-4 (L1,
  mass-weighted) of the oracle.
* 8,388,608 points (the workload's full size, in the benchmark's launch
  configuration): 3000 sampled cells against the oracle, the volumes tile
  the box, and two mixed steps conserve mass to rounding.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import compare_mesh, dev, host, local_err, sampled_cells_match, state_scale

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _case(what, **kw):
    print(f"[case] {what} {kw}", flush=True)


@pytest.fixture(scope="module")
def c5_small():
    return W.c5_polytropes(20000, seed=5)


def test_c5_small_tessellation_parity(orc, c5_small):
    import paper_1707_05333_amd as M
    wl = c5_small
    _case("c5 tessellation", n=wl.n)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **wl.params))
    info = mm.tessellate(dev(wl.pos))
    om = orc.tessellate(wl.pos, wl.box, certificate=True)
    assert om.status == 0 and om.delta_min > 1e-12
    compare_mesh(mm, om)
    assert info["n_faces"] * 2 == len(om.j)


def test_dense_cells_beyond_the_sized_grid(orc, c5_small):
    """The two-cells-per-wavefront dense pass launches as many wavefronts as
    the previous tessellation listed dense cells (and a quarter more); listed
    cells beyond that go to the one-cell dense pass.  The passes over the
    other lists get grids sized from the previous lists' lengths (256 blocks
    of 4 wavefronts at least) and walk longer lists with a grid stride.  A
    context that first tessellates uniform random points (no dense cell and
    no cell for the shell pass, so those grids are small) and then the
    polytropes (thousands of dense cells, and more cells for the shell pass
    than its grid has wavefronts) builds the polytropes' tessellation
    exactly as the oracle does."""
    import paper_1707_05333_amd as M
    wl = c5_small
    _case("dense cells beyond the sized grid", n=wl.n)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **wl.params))
    first = mm.tessellate(dev(W.poisson_points(wl.n, wl.box, seed=11)))
    assert first["deferred_cells"] == 0
    info = mm.tessellate(dev(wl.pos))
    assert info["deferred_cells"] > 256 * 4   # the shell pass's list outgrows its grid
    om = orc.tessellate(wl.pos, wl.box, certificate=True)
    assert om.status == 0 and om.delta_min > 1e-12
    compare_mesh(mm, om)
    assert info["n_faces"] * 2 == len(om.j)
    # and the next call, sized from this one, as well
    info = mm.tessellate(dev(wl.pos))
    compare_mesh(mm, om)


def _oracle_run(orc, wl, nsteps):
    p = orc.make_params(wl.box, **wl.params)
    om = orc.tessellate(wl.pos, wl.box)
    Q0 = orc.init_charges(om, p, wl.prim)
    pos, Q = wl.pos.copy(), Q0.copy()
    out = []
    for _ in range(nsteps):
        om = orc.tessellate(pos, wl.box)   # the step's mesh: each cell's neighbourhood
        pos, Q, w, dt, cnt = orc.step(pos, Q, p)
        out.append((pos.copy(), Q.copy(), dt, list(cnt), om))
    return Q0, out


def test_c5_small_fp64_steps_match_oracle(orc, c5_small):
    import paper_1707_05333_amd as M
    import torch
    wl = c5_small
    _case("c5 fp64 steps", n=wl.n, steps=2)
    Q0, ref = _oracle_run(orc, wl, 2)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision="fp64", **wl.params))
    pos, Q = dev(wl.pos), dev(Q0)
    w = torch.empty_like(pos)
    for k, (po, Qo, dto, cnt, om) in enumerate(ref):
        info = mm.step(pos, w, Q)
        assert abs(info["dt"] - dto) <= TOL * dto, f"step {k}"
        assert info["floor_hits"] == cnt, f"step {k}"
        assert cnt[2] > 0   # faces at the stars' edges fell back to first order
        err = local_err(host(Q), Qo, om, state_scale(Qo, wl.params["gamma"]))
        print(f"[step {k}] max element error {err:.3e}", flush=True)
        assert err < TOL, f"step {k}"
        assert np.abs(host(pos) - po).max() < TOL, f"step {k}"


def test_c5_small_mixed_steps(orc, c5_small):
    import paper_1707_05333_amd as M
    import torch
    wl = c5_small
    _case("c5 mixed steps", n=wl.n, steps=3)
    Q0, ref = _oracle_run(orc, wl, 3)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision="mixed", **wl.params))
    pos, Q = dev(wl.pos), dev(Q0)
    w = torch.empty_like(pos)
    for _ in range(3):
        mm.step(pos, w, Q)
    Qg, Qo = host(Q), ref[-1][1]
    assert np.all(np.isfinite(Qg))
    m0 = Q0[:, 0].sum()
    assert abs(Qg[:, 0].sum() - m0) <= 1e-14 * m0
    # mass-weighted L1 of the density: the cells' masses (the volumes are
    # the same function of the same positions up to the drift's rounding)
    l1 = np.abs(Qg[:, 0] - Qo[:, 0]).sum() / Qo[:, 0].sum()
    print("mixed vs FP64 mass L1", l1, flush=True)
    assert l1 < 1e-4


def test_c5_full_size_sampled_and_conservation(orc):
    import paper_1707_05333_amd as M
    import torch
    wl = W.c5_polytropes()
    _case("c5 full size", n=wl.n)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision="mixed", **wl.params))
    pos = dev(wl.pos)
    info = mm.tessellate(pos)
    ex = mm.mesh_export()
    assert abs(host(ex.V).sum() - 1.0) < 1e-12
    assert info["max_faces_cell"] <= 64
    sampled_cells_match(orc, wl, ex)
    del ex
    Q = mm.init_charges(dev(wl.prim))
    m0 = float(Q[:, 0].sum())
    w = torch.empty_like(pos)
    for k in range(2):
        info = mm.step(pos, w, Q)
        print(f"step {k}: dt {info['dt']:.3e} floors {info['floor_hits']}", flush=True)
    assert bool(torch.isfinite(Q).all())
    assert abs(float(Q[:, 0].sum()) - m0) <= 1e-13 * m0


def _cluster(n_in, n_out, width, seed, centre=0.5):
    rng = np.random.default_rng(seed)
    inner = centre + rng.normal(scale=width, size=(n_in, 3))
    outer = rng.uniform(0.0, 1.0, size=(n_out, 3))
    return np.ascontiguousarray(np.vstack([inner, outer]) % 1.0)


def test_large_sub_grids_match_oracle(orc):
    # A Gaussian cluster of 3000 points in a uniform background of 2000:
    # the grid's central buckets hold up to ~2,000 points (sub-grids up to
    # 10^3), every query crosses the boundary between the two levels.
    import paper_1707_05333_amd as M
    pos = _cluster(3000, 2000, 0.02, seed=12)
    _case("cluster tessellation", n=pos.shape[0])
    mm = M.MovingMesh(pos.shape[0], M.make_params(box=(1, 1, 1)))
    info = mm.tessellate(dev(pos))
    om = orc.tessellate(pos, (1, 1, 1), certificate=True)
    assert om.status == 0 and om.delta_min > 1e-12
    compare_mesh(mm, om)
    assert info["n_faces"] * 2 == len(om.j)


def test_bucket_beyond_sort_capacity_is_refused():
    # 5000 points within ~1e-3 of one spot among 1000 spread ones: one grid
    # bucket holds more points than the in-LDS sort of a bucket takes.
    import paper_1707_05333_amd as M
    pos = _cluster(5000, 1000, 3e-4, seed=13, centre=0.52)   # well inside one bucket
    _case("bucket over capacity", n=pos.shape[0])
    mm = M.MovingMesh(pos.shape[0], M.make_params(box=(1, 1, 1)))
    with pytest.raises(M.MMError) as e:
        mm.tessellate(dev(pos))
    assert e.value.name == "MM_ECAPACITY" and "density contrast" in str(e.value)
