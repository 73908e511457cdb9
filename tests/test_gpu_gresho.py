"""Gresho-Chan vortex on the GPU (Sec. 5 test problems): the steady vortex
run to t = 2 at equivalent 2D resolutions 32^2, 64^2 and 128^2.  The exact
solution is the initial state, so the L1 error of the tangential speed at
the generators (the paper's measure) must fall with resolution; the paper
reports L1 proportional to N^-0.88."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import dev, host

pytestmark = pytest.mark.gpu


def run_gresho(M, N, t_end=2.0, precision="fp64"):
    """Steps the vortex to t_end; returns (L1 of v_phi, steps, mass drift)."""
    import torch
    wl = W.gresho(N)
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision=precision, **wl.params))
    pos = dev(wl.pos)
    mm.tessellate(pos)
    Q = mm.init_charges(dev(wl.prim))
    m0 = float(Q[:, 0].sum())
    w = torch.empty_like(pos)
    t, steps = 0.0, 0
    while t < t_end * (1 - 1e-12):
        info = mm.step(pos, w, Q, dt_max=t_end - t)
        assert info["floor_hits"] == [0, 0, 0, 0]
        t += info["dt"]
        steps += 1
    x, q = host(pos), host(Q)
    dx, dy = x[:, 0] - 0.5, x[:, 1] - 0.5
    r = np.hypot(dx, dy)
    v = q[:, 1:3] / q[:, :1]
    vphi = (-dy * v[:, 0] + dx * v[:, 1]) / r
    l1 = float(np.mean(np.abs(vphi - W.gresho_profile(r)[1])))
    mm.close()
    return l1, steps, abs(float(q[:, 0].sum()) - m0) / m0


def test_gresho_converges():
    import paper_1707_05333_amd as M
    res = {}
    for N in (32, 64, 128):
        print(f"[case] gresho N={N}", flush=True)
        res[N] = run_gresho(M, N)
        print(f"[gresho] N={N} L1={res[N][0]:.4e} steps={res[N][1]} mass drift {res[N][2]:.1e}", flush=True)
    l1 = {N: r[0] for N, r in res.items()}
    slope = math.log(l1[32] / l1[128]) / math.log(4.0)
    print(f"[gresho] slope {slope:.3f}", flush=True)
    assert l1[32] > l1[64] > l1[128]
    assert slope > 0.5
    assert all(r[2] < 1e-12 for r in res.values())
