"""Half-step mesh on the GPU (the paper's first future improvement, Sec. 6):
the fluxes use a tessellation rebuilt at r + w dt/2.

* Static mesh: bitwise the same step as without it.
* A uniform flow on a mesh drifting relative to it (roundness correction):
  the density error after a fixed time falls at first order in the
  timestep with start-of-step areas and at second order or faster with
  half-step areas (the geometric conservation law to second order).
* Batches refuse the option.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev, host

pytestmark = pytest.mark.gpu


def _advance(M, wl, T, **over):
    import torch
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **dict(wl.params, **over)))
    pos = dev(wl.pos)
    mm.tessellate(pos)
    Q = mm.init_charges(dev(wl.prim))
    w = torch.empty_like(pos)
    t, steps = 0.0, 0
    while t < T * (1 - 1e-12):
        t += mm.step(pos, w, Q, dt_max=T - t)["dt"]
        steps += 1
    mm.tessellate(pos)
    V = host(mm.mesh_export().V)
    out = host(pos), host(Q), V, steps
    mm.close()
    return out


def test_static_mesh_bitwise_identical():
    import paper_1707_05333_amd as M
    wl = W.sod_paper(k=6, static_mesh=True)
    print(f"[case] half-step static n={wl.n}", flush=True)
    a = _advance(M, wl, 0.3)
    b = _advance(M, wl, 0.3, half_step_mesh=1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_free_stream_error_orders():
    import paper_1707_05333_amd as M
    pos = W.jittered_lattice((24, 24, 24), (1, 1, 1), jitter=0.2, seed=3)
    wl = W.uniform_state(pos, (1, 1, 1), rho=1.3, vel=(0.4, -0.2, 0.1), P=0.7)
    e = {}
    for half in (0, 1):
        for cfl in (0.4, 0.1):
            print(f"[case] free stream half={half} cfl={cfl} n={wl.n}", flush=True)
            p, Q, V, steps = _advance(M, wl, 0.05, half_step_mesh=half, cfl=cfl)
            e[half, cfl] = float(np.abs(Q[:, 0] / V - 1.3).max())
    print("[free-stream]", e, flush=True)
    assert 2.5 < e[0, 0.4] / e[0, 0.1] < 8.0
    assert e[1, 0.4] / e[1, 0.1] > 12.0
    assert e[1, 0.1] < 0.05 * e[0, 0.1]


def test_batch_refuses_half_step_mesh():
    import paper_1707_05333_amd as M
    b = M.Batch(64 << 20, max_sims=2, precision="fp64")
    wl = W.c1_uniform_random_velocity()
    print(f"[case] batch admission with half_step_mesh n={wl.n}", flush=True)
    with pytest.raises(M.MMError) as e:
        b.admit(M.make_params(box=wl.box, half_step_mesh=1, **wl.params), dev(wl.pos), dev(wl.prim))
    assert e.value.name == "MM_EINVAL" and "single simulations" in str(e.value)
    b.close()
