"""GPU checks at the workloads' full sizes, in the launch configuration the
benchmark uses: sampled cells against the oracle (which builds just those
cells), properties that hold at any size, the Sod tube against the exact
Riemann solution, and the mixed-precision error against FP64."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import dev, host, sampled_cells_match as _sampled_cells_match

pytestmark = pytest.mark.gpu


def _case(what, **kw):
    print(f"[case] {what} {kw}", flush=True)


@pytest.mark.parametrize("name", ["sod_256x64x64", "blast_128^3"])
def test_full_size_tessellation_sampled(orc, name):
    import paper_1707_05333_amd as M
    wl = W.c2_sod() if name.startswith("sod") else W.c3_point_blast()
    _case("full tessellation", name=name, n=wl.n)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **wl.params))
    info = mm.tessellate(dev(wl.pos))
    ex = mm.mesh_export()
    V = host(ex.V)
    assert abs(V.sum() / np.prod(wl.box) - 1) < 1e-12
    assert info["max_faces_cell"] <= 64
    _sampled_cells_match(orc, wl, ex)


def test_full_size_closed_cells_and_conservation():
    # Every cell's faces close (sum A n = 0) and one step conserves mass,
    # momentum and energy to rounding, at 1M cells.
    import paper_1707_05333_amd as M
    import torch
    wl = W.c2_sod()
    _case("closure+conservation", n=wl.n)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **wl.params))
    pos = dev(wl.pos)
    mm.tessellate(pos)
    ex = mm.mesh_export()
    fi, fj, fc = ex.face_i.long(), ex.face_j.long(), ex.face_code.long()
    L = torch.tensor(wl.box, dtype=torch.float64, device="cuda")
    k = torch.stack([fc % 3 - 1, (fc // 3) % 3 - 1, fc // 9 - 1], dim=1).double()
    d = pos[fj] + k * L - pos[fi]
    an = ex.face_A[:, None] * d / d.norm(dim=1, keepdim=True)
    S = torch.zeros(wl.n, 3, dtype=torch.float64, device="cuda")
    S.index_add_(0, fi, an)
    S.index_add_(0, fj, -an)
    scale = float(ex.V.mean()) ** (2 / 3)
    assert float(S.abs().max()) < 1e-12 * scale
    Q = mm.init_charges(dev(wl.prim))
    S0 = Q.sum(dim=0)
    w = torch.empty_like(pos)
    info = mm.step(pos, w, Q)
    assert info["floor_hits"] == [0, 0, 0, 0]
    rel = ((Q.sum(dim=0) - S0).abs() / Q.abs().sum(dim=0)).max()
    assert float(rel) < 1e-13


def test_sod_full_resolution_against_exact_solution(orc):
    # The Sod workload (4 x 1 x 1, 256 x 64 x 64) run to t ~ 0.12 (about 50
    # steps): star plateaus and wave positions about x = 2 against the exact
    # Riemann solution (Sec. 5.1 test problem; exact solver of Toro 2009).
    import paper_1707_05333_amd as M
    import torch
    wl = W.c2_sod()
    _case("sod exact", n=wl.n)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **wl.params))
    pos = dev(wl.pos)
    mm.tessellate(pos)
    Q = mm.init_charges(dev(wl.prim))
    w = torch.empty_like(pos)
    t = 0.0
    for _ in range(60):
        info = mm.step(pos, w, Q)
        t += info["dt"]
        assert info["floor_hits"] == [0, 0, 0, 0]
        # The first-pass radius adapts to the deforming mesh without feeding
        # back into candidate overflow: most cells stay in the first pass.
        assert info["deferred_cells"] < 0.2 * wl.n, info
        if t >= 0.12:
            break
    mm.tessellate(pos)
    V = host(mm.mesh_export().V)
    Qh, x = host(Q), host(pos)[:, 0]
    rho, vx = Qh[:, 0] / V, Qh[:, 1] / Qh[:, 0]
    right = x > 1.0    # the interface at x = 2 (the one at x = 0 is the mirror image)
    xi = (x[right] - 2.0) / t
    Wex, ps, us = orc.exact_riemann([1, 0, 1], [0.125, 0, 0.1], 1.4, xi)
    h = 1.0 / 64
    star = (xi > -0.0703 + 3 * h / t) & (xi < us - 3 * h / t)
    assert star.sum() > 1000
    assert abs(np.median(vx[right][star]) - us) < 0.02 * us
    assert abs(np.median(rho[right][star]) - 0.42632) < 0.02 * 0.42632
    l1 = np.mean(np.abs(rho[right] - Wex[:, 0]))
    assert l1 < 0.02, l1
    shock = 2.0 + 1.75216 * t
    behind = (x > shock - 5 * h) & (x < shock - 2 * h)
    ahead = (x > shock + 2 * h) & (x < shock + 5 * h)
    assert np.median(rho[behind]) > 0.24 and np.median(rho[ahead]) < 0.14


def test_mixed_precision_blast_error():
    # FP32 gradients, predictor and fluxes with FP64 geometry and sums
    # against the FP64 path on the point blast (64^3, 40 steps): relative
    # L1 density error <= 1e-4; mass is conserved by both.
    import paper_1707_05333_amd as M
    import torch
    wl = W.c3_point_blast(n_side=64)
    _case("mixed vs fp64", n=wl.n)
    out = {}
    for prec in ("fp64", "mixed"):
        mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision=prec, **wl.params))
        pos = dev(wl.pos)
        mm.tessellate(pos)
        Q = mm.init_charges(dev(wl.prim))
        Q[torch.from_numpy(wl.energy_cells).cuda(), 4] += wl.energy_amount
        M0 = float(Q[:, 0].sum())
        w = torch.empty_like(pos)
        for _ in range(40):
            mm.step(pos, w, Q)
        mm.tessellate(pos)
        V = mm.mesh_export().V
        out[prec] = (host(Q[:, 0] / V), abs(float(Q[:, 0].sum()) - M0) / M0)
    r64, r32 = out["fp64"][0], out["mixed"][0]
    l1 = np.abs(r32 - r64).sum() / np.abs(r64).sum()
    print(f"[mixed] L1(rho) = {l1:.3e}, mass drift fp64 {out['fp64'][1]:.2e} mixed {out['mixed'][1]:.2e}")
    assert l1 < 1e-4
    assert out["fp64"][1] < 1e-13 and out["mixed"][1] < 1e-12
