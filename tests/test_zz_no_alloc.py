"""The allocation-free step (mm_step_static), through the C ABI, against the
step of a context (mm_step) on the same inputs: two calls in a row on the
device's one scratch array, the second with fewer points, each bitwise
equal to the context's result (which the parity tests tie to the oracle)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev

pytestmark = pytest.mark.gpu


def _case(what, **kw):
    print(f"[case] {what} {kw}", flush=True)


def _inputs(M, wl, prec):
    """Positions, charges (from a context's first tessellation) and params."""
    params = M.make_params(box=wl.box, precision=prec, **wl.params)
    mm = M.MovingMesh(wl.n, params)
    pos = dev(wl.pos)
    mm.tessellate(pos)
    Q = mm.init_charges(dev(wl.prim))
    mm.close()
    return params, pos, Q


def _context_steps(M, params, pos, Q, steps):
    import torch
    mm = M.MovingMesh(pos.shape[0], params)
    pos, Q = pos.clone(), Q.clone()
    w = torch.empty_like(pos)
    infos = [mm.step(pos, w, Q) for _ in range(steps)]
    mm.close()
    return pos, Q, w, infos


def _static_steps(M, params, pos, Q, steps):
    import torch
    pos, Q = pos.clone(), Q.clone()
    w = torch.empty_like(pos)
    infos = [M.step_static(params, pos, w, Q) for _ in range(steps)]
    return pos, Q, w, infos


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_static_step_equals_context_step_twice(prec):
    import torch
    import paper_1707_05333_amd as M
    big = W.c2_sod(shape=(40, 12, 12), box=(4.0, 1.2, 1.2))            # 5,760 points
    small = W.random_smooth_state(W.jittered_lattice((9, 10, 11), (0.9, 1.0, 1.1), seed=31),
                                  (0.9, 1.0, 1.1), seed=31, amp=0.25)   # 990 points
    for wl, steps in ((big, 3), (small, 2)):
        _case("static step", prec=prec, n=wl.n, steps=steps)
        params, pos, Q = _inputs(M, wl, prec)
        p1, Q1, w1, i1 = _context_steps(M, params, pos, Q, steps)
        p2, Q2, w2, i2 = _static_steps(M, params, pos, Q, steps)
        assert torch.equal(p1, p2) and torch.equal(Q1, Q2) and torch.equal(w1, w2)
        assert [i["dt"] for i in i1] == [i["dt"] for i in i2]
        assert [i["n_faces"] for i in i1] == [i["n_faces"] for i in i2]
        assert bool(torch.isfinite(Q2).all())


def test_static_step_refusals():
    import torch
    import paper_1707_05333_amd as M
    _case("static step refusals")
    n = M.STATIC_MAX_POINTS + 1
    pos = torch.rand(n, 3, dtype=torch.float64, device="cuda")
    Q = torch.ones(n, 5, dtype=torch.float64, device="cuda")
    w = torch.empty_like(pos)
    with pytest.raises(M.MMError) as e:
        M.step_static(M.make_params(), pos, w, Q)
    assert e.value.name == "MM_EINVAL" and "MM_STATIC_MAX_POINTS" in str(e.value)
    wl = W.c1_uniform_random_velocity(n_side=6)
    params, pos, Q = _inputs(M, wl, "fp64")
    w = torch.empty_like(pos)
    with pytest.raises(M.MMError) as e:
        M.step_static(M.make_params(box=wl.box, half_step_mesh=1, **wl.params), pos, w, Q)
    assert e.value.name == "MM_EINVAL"
    # a failing call leaves the state, and the next call on the array works
    Q_bad = Q.clone()
    Q_bad[5, 0] = float("nan")
    before = Q_bad.clone()
    with pytest.raises(M.MMError) as e:
        M.step_static(params, pos, w, Q_bad)
    assert e.value.name == "MM_ENONFINITE"
    assert torch.equal(torch.isnan(Q_bad), torch.isnan(before))
    p1, Q1, _, _ = _context_steps(M, params, pos, Q, 1)
    p2, Q2, _, _ = _static_steps(M, params, pos, Q, 1)
    assert torch.equal(p1, p2) and torch.equal(Q1, Q2)
