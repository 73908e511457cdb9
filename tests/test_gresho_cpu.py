"""CPU pins of the Gresho-Chan vortex workload (Sec. 5 test problems).

The vortex is a steady solution of the Euler equations, so its profile must
be in radial balance, dP/dr = rho v_phi^2 / r, with P continuous where the
pieces meet; the oracle's first step must leave it nearly at rest in the
co-rotating sense (small change of v_phi)."""
import math

import numpy as np

import workloads as W


def test_profile_is_in_radial_balance_and_continuous():
    r = np.linspace(1e-3, 0.7, 4001)
    P, v = W.gresho_profile(r)
    h = 1e-6
    dP = (W.gresho_profile(r + h)[0] - W.gresho_profile(r - h)[0]) / (2 * h)
    away = (np.abs(r - 0.2) > 2 * h) & (np.abs(r - 0.4) > 2 * h)
    assert np.abs(dP - v * v / r)[away].max() < 1e-7
    for rj in (0.2, 0.4):
        lo, hi = W.gresho_profile(np.array([rj - 1e-12, rj + 1e-12]))[0]
        assert abs(lo - hi) < 1e-9
    assert abs(W.gresho_profile(np.array([1.0]))[0][0] - (3 + 4 * math.log(2))) < 1e-15
    assert W.gresho_profile(np.array([0.2]))[1][0] == 1.0   # peak speed 5 r = 1 at r = 0.2


def test_workload_geometry_and_state():
    wl = W.gresho(32)
    assert wl.n == 32 * 32 * 6 and wl.box == (1.0, 1.0, 6 / 32)
    dx, dy = wl.pos[:, 0] - 0.5, wl.pos[:, 1] - 0.5
    r = np.hypot(dx, dy)
    vphi = (-dy * wl.prim[:, 1] + dx * wl.prim[:, 2]) / r
    assert np.abs(vphi - W.gresho_profile(r)[1]).max() < 1e-14
    assert np.abs(dx * wl.prim[:, 1] + dy * wl.prim[:, 2]).max() < 1e-14   # no radial velocity
    assert np.all(wl.prim[:, 0] == 1.0) and np.all(wl.prim[:, 3] == 0.0)


def test_oracle_step_keeps_the_vortex(orc):
    # One step at 16^2: the rotation profile moves by far less than its scale.
    wl = W.gresho(16)
    p = orc.make_params(wl.box, **wl.params)
    m = orc.tessellate(wl.pos, wl.box)
    Q = orc.init_charges(m, p, wl.prim)
    pos, Q1, w, dt, cnt = orc.step(wl.pos, Q, p)
    assert cnt.sum() == 0 and 0 < dt < 0.01
    dx, dy = pos[:, 0] - 0.5, pos[:, 1] - 0.5
    r = np.hypot(dx, dy)
    v = Q1[:, 1:3] / Q1[:, :1]
    vphi = (-dy * v[:, 0] + dx * v[:, 1]) / r
    err = np.mean(np.abs(vphi - W.gresho_profile(r)[1]))
    assert err < 0.02, err
