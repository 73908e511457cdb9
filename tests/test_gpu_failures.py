"""Failures the host can force, through the C ABI: a step that fails leaves
the caller's positions and charges as they were, a simulation whose step
fails in a batch is parked alone while the others advance exactly as they
would without it, and the serving loop evicts it.  Every kernel exits
normally in these cases; the failures are flagged on the device and read
back with the step's status block (positivity floors and non-finite
states, Sec. 4.1)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev, host

pytestmark = pytest.mark.gpu

MM_ENONFINITE = -5   # mm_status of include/mm.h


def _case(what, **kw):
    print(f"[case] {what} {kw}", flush=True)


def _ctx_and_state(M, wl, face_capacity=0, prec="fp64"):
    import torch
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision=prec, **wl.params), face_capacity=face_capacity)
    big = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision=prec, **wl.params))
    big.tessellate(dev(wl.pos))
    Q = big.init_charges(dev(wl.prim))
    big.close()
    pos = dev(wl.pos)
    return mm, pos, Q, torch.empty_like(pos)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_face_capacity_failure_leaves_state(prec):
    import paper_1707_05333_amd as M
    wl = W.c1_uniform_random_velocity(n_side=8)
    _case("face capacity", n=wl.n, prec=prec)
    mm, pos, Q, w = _ctx_and_state(M, wl, face_capacity=2 * wl.n, prec=prec)
    pos0, Q0 = pos.clone(), Q.clone()
    with pytest.raises(M.MMError) as e:
        mm.step(pos, w, Q)
    assert e.value.name == "MM_ECAPACITY" and "face capacity" in str(e.value)
    assert np.array_equal(host(pos), host(pos0)) and np.array_equal(host(Q), host(Q0))
    # the caller's retry: a context with room for the faces takes the step
    mm2 = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision=prec, **wl.params))
    info = mm2.step(pos, w, Q)
    assert info["n_faces"] > 2 * wl.n and bool(torch_isfinite(Q))


def torch_isfinite(t):
    import torch
    return torch.isfinite(t).all()


def test_nonfinite_charge_is_refused_and_state_kept():
    import paper_1707_05333_amd as M
    wl = W.c1_uniform_random_velocity(n_side=8)
    _case("nan charge", n=wl.n)
    mm, pos, Q, w = _ctx_and_state(M, wl)
    mm.step(pos, w, Q)   # one good step first
    Q[37, 4] = float("nan")
    pos0, Q0 = host(pos).copy(), host(Q).copy()
    with pytest.raises(M.MMError) as e:
        mm.step(pos, w, Q)
    assert e.value.name == "MM_ENONFINITE"
    assert np.array_equal(host(pos), pos0)
    Qa = host(Q)
    assert np.isnan(Qa[37, 4]) and np.array_equal(np.isnan(Qa), np.isnan(Q0))
    assert np.array_equal(Qa[~np.isnan(Q0)], Q0[~np.isnan(Q0)])
    # the repaired state steps again
    Q[37, 4] = float(Q0[36, 4])
    mm.step(pos, w, Q)
    assert bool(torch_isfinite(Q))


def _mix():
    kh = W.c4_kelvin_helmholtz(1, n_min=1500, n_max=1600)
    c1 = W.c1_uniform_random_velocity(n_side=11)
    sod = W.c2_sod(shape=(32, 8, 8), box=(4.0, 1.0, 1.0))
    return [kh, c1, sod]


def _alone(M, wl, prec, steps):
    import torch
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision=prec, **wl.params))
    pos = dev(wl.pos)
    mm.tessellate(pos)
    Q = mm.init_charges(dev(wl.prim))
    w = torch.empty_like(pos)
    for _ in range(steps):
        mm.step(pos, w, Q)
    mm.close()
    return pos, Q


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_failing_simulation_is_parked_alone(prec):
    import paper_1707_05333_amd as M
    import torch
    wls = _mix()
    bad_prim = wls[1].prim.copy()
    bad_prim[50, 0] = float("nan")
    _case("batch parks a failing simulation", prec=prec, n=[w.n for w in wls])
    budget = sum(M.batch_footprint(wl.n, prec) for wl in wls) * 2
    B = M.Batch(budget, max_sims=8, precision=prec)
    ids = []
    for k, wl in enumerate(wls):
        prim = bad_prim if k == 1 else wl.prim
        ids.append(B.admit(M.make_params(box=wl.box, precision=prec, **wl.params), dev(wl.pos), dev(prim)))
    rep = {r["sim"]: r for r in B.step()}
    assert rep[ids[1]]["status"] == MM_ENONFINITE
    assert rep[ids[0]]["status"] == 0 and rep[ids[2]]["status"] == 0
    for _ in range(2):
        rep = B.step()
        assert sorted(r["sim"] for r in rep) == sorted([ids[0], ids[2]])   # the parked one is not stepped
        assert all(r["status"] == 0 for r in rep)
    for k in (0, 2):
        pos, Q = _alone(M, wls[k], prec, 3)
        p2, Q2, _ = B.read(ids[k])
        assert torch.equal(p2, pos) and torch.equal(Q2, Q)
    B.evict(ids[1])
    assert B.usage()["sims"] == 2
    B.close()


def test_serving_loop_evicts_a_failing_request():
    import paper_1707_05333_amd as M
    import torch
    prec = "mixed"
    wls = [W.c4_kelvin_helmholtz(k, n_min=1000, n_max=8000) for k in range(4)]
    prims = [wl.prim.copy() for wl in wls]
    prims[2][10, 4] = float("inf")
    _case("serve with a failing request", n=[w.n for w in wls])
    budget = int(sum(M.batch_footprint(w.n, prec) for w in wls))
    B = M.Batch(budget, max_sims=8, precision=prec)
    reqs = []
    for k, wl in enumerate(wls):
        reqs.append(dict(arrival=0.001 * k, params=M.make_params(box=wl.box, precision=prec, **wl.params),
                         pos=dev(wl.pos), prim=dev(prims[k]), steps=4,
                         pos_out=torch.empty(wl.n, 3, dtype=torch.float64, device="cuda"),
                         Q_out=torch.empty(wl.n, 5, dtype=torch.float64, device="cuda")))
    res, stats = B.serve(reqs)
    assert res[2]["status"] == MM_ENONFINITE and res[2]["steps"] == 0
    assert all(res[k]["status"] == 0 and res[k]["steps"] == 4 for k in (0, 1, 3))
    assert stats["sim_steps"] == 12 and B.usage()["sims"] == 0
    for k in (0, 1, 3):
        pos, Q = _alone(M, wls[k], prec, 4)
        assert torch.equal(reqs[k]["pos_out"], pos) and torch.equal(reqs[k]["Q_out"], Q)
    B.close()
