"""GPU checks of batched serving: simulations stepped together in shared
launches give bitwise the results they give alone (in a batch of their own
and through the one-simulation context), simulations join and leave between
steps, admission follows the device budget, and the serving loop runs a
request trace to completion with every result equal to the lone run."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import dev

pytestmark = pytest.mark.gpu


def _case(what, **kw):
    print(f"[case] {what} {kw}", flush=True)


def _mix():
    """Three simulations with different boxes, sizes, gammas and limiters."""
    kh = W.c4_kelvin_helmholtz(0, n_min=1500, n_max=1600)
    c1 = W.c1_uniform_random_velocity(n_side=11)
    sod = W.c2_sod(shape=(32, 8, 8), box=(4.0, 1.0, 1.0))
    sod.params = dict(sod.params, limit_mask=1, theta=0.3)
    return [kh, c1, sod]


def _params(M, wl, prec):
    return M.make_params(box=wl.box, precision=prec, **wl.params)


def _alone(M, wl, prec, steps):
    """The one-simulation context: tessellate, charges, `steps` steps."""
    import torch
    mm = M.MovingMesh(wl.n, _params(M, wl, prec))
    pos = dev(wl.pos)
    mm.tessellate(pos)
    Q = mm.init_charges(dev(wl.prim))
    w = torch.empty_like(pos)
    for _ in range(steps):
        mm.step(pos, w, Q)
    mm.close()
    return pos, Q


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_alone_bitwise(prec):
    import paper_1707_05333_amd as M
    import torch
    wls = _mix()
    _case("batch vs alone", prec=prec, n=[w.n for w in wls])
    steps = 4
    ref = [_alone(M, wl, prec, steps) for wl in wls]
    budget = sum(M.batch_footprint(wl.n, prec) for wl in wls) * 2
    B = M.Batch(budget, max_sims=8, precision=prec)
    ids = [B.admit(_params(M, wl, prec), dev(wl.pos), dev(wl.prim)) for wl in wls]
    for k in range(steps):
        rep = B.step()
        assert [r["status"] for r in rep] == [0, 0, 0]
        assert sorted(r["sim"] for r in rep) == sorted(ids)
    for sim, (pos, Q) in zip(ids, ref):
        p2, Q2, _ = B.read(sim)
        assert torch.equal(p2, pos) and torch.equal(Q2, Q)
    B.close()


def test_simulations_join_and_leave_between_steps():
    # A runs 2 steps alone, B joins for 3, A leaves, C takes A's room and
    # runs 2 steps: every one equals its lone run, bitwise.
    import paper_1707_05333_amd as M
    import torch
    a, b, c = _mix()
    _case("join and leave", n=[a.n, b.n, c.n])
    prec = "mixed"
    budget = (M.batch_footprint(a.n, prec) + M.batch_footprint(b.n, prec) + M.batch_footprint(c.n, prec)) * 2
    B = M.Batch(budget, max_sims=4, precision=prec)
    ia = B.admit(_params(M, a, prec), dev(a.pos), dev(a.prim))
    for _ in range(2):
        B.step()
    ib = B.admit(_params(M, b, prec), dev(b.pos), dev(b.prim))
    for _ in range(3):
        rep = B.step()
        assert len(rep) == 2
    pa, Qa, _ = B.read(ia)
    ra = _alone(M, a, prec, 5)
    assert torch.equal(pa, ra[0]) and torch.equal(Qa, ra[1])
    B.evict(ia)
    ic = B.admit(_params(M, c, prec), dev(c.pos), dev(c.prim))
    for _ in range(2):
        B.step()
    pb, Qb, _ = B.read(ib)
    rb = _alone(M, b, prec, 5)
    assert torch.equal(pb, rb[0]) and torch.equal(Qb, rb[1])
    pc, Qc, _ = B.read(ic)
    rc = _alone(M, c, prec, 2)
    assert torch.equal(pc, rc[0]) and torch.equal(Qc, rc[1])
    B.close()


def test_admission_follows_the_budget():
    import paper_1707_05333_amd as M
    wl = W.c1_uniform_random_velocity(n_side=12)
    prec = "mixed"
    _case("admission", n=wl.n)
    B = M.Batch(int(2.5 * M.batch_footprint(wl.n, prec)), max_sims=8, precision=prec)
    p = _params(M, wl, prec)
    s0 = B.admit(p, dev(wl.pos), dev(wl.prim))
    s1 = B.admit(p, dev(wl.pos), dev(wl.prim))
    assert B.try_admit(p, dev(wl.pos), dev(wl.prim)) is None
    u = B.usage()
    assert u["sims"] == 2 and u["cells"] == 2 * wl.n and u["cell_capacity"] < 3 * wl.n
    B.step()
    B.evict(s0)
    s2 = B.admit(p, dev(wl.pos), dev(wl.prim))
    rep = B.step()
    assert {r["sim"] for r in rep} == {s1, s2}
    assert {r["steps"] for r in rep} == {1, 2}
    with pytest.raises(M.MMError) as e:
        B.read(s2 + 5)
    assert e.value.name == "MM_EINVAL"
    B.close()


def test_serving_loop_runs_a_trace():
    # Ten Kelvin-Helmholtz requests of 1e3..2e4 points with Poisson arrivals,
    # 5 steps each, a budget that holds a few at once: all complete, and
    # each result equals the lone run of its request.
    import paper_1707_05333_amd as M
    import torch
    prec = "mixed"
    wls = [W.c4_kelvin_helmholtz(k, n_min=1000, n_max=20000) for k in range(10)]
    _case("serve", n=[w.n for w in wls])
    arrival = W.poisson_arrivals(len(wls), rate=200.0, seed=4)
    budget = int(sum(sorted(M.batch_footprint(w.n, prec) for w in wls)[-3:]))
    B = M.Batch(budget, max_sims=16, precision=prec)
    reqs = []
    for t, wl in zip(arrival, wls):
        reqs.append(dict(arrival=float(t), params=_params(M, wl, prec), pos=dev(wl.pos), prim=dev(wl.prim),
                         steps=5, pos_out=torch.empty(wl.n, 3, dtype=torch.float64, device="cuda"),
                         Q_out=torch.empty(wl.n, 5, dtype=torch.float64, device="cuda")))
    res, stats = B.serve(reqs)
    print("[serve]", stats, flush=True)
    assert all(r["status"] == 0 and r["steps"] == 5 for r in res)
    assert all(r["admitted"] >= t - 1e-9 for r, t in zip(res, arrival))
    assert stats["sim_steps"] == 50 and stats["cell_updates"] == 5 * sum(w.n for w in wls)
    assert 0 < stats["step_p50"] <= stats["step_p99"] and stats["max_resident"] >= 2
    assert B.usage()["sims"] == 0
    for r, wl in zip(reqs, wls):
        pos, Q = _alone(M, wl, prec, 5)
        assert torch.equal(r["pos_out"], pos) and torch.equal(r["Q_out"], Q)
    B.close()
