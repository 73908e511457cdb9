"""CPU pins of the two-polytrope workload (two touching n = 1.5 stars in a
thin background: a strongly non-uniform density) and of the oracle on it.

* The Lane-Emden integrator of the workload reproduces the closed forms for
  n = 0 and n = 1 (first zeros sqrt 6 and pi, mass constants 2 sqrt 6 and
  pi) and the tabulated n = 1.5 constants (3.65375 and 2.71406).
* Each star is a self-gravitating equilibrium with G = 1 of the requested
  mass and radius: checked against scipy's own integration of the
  Lane-Emden equation (mass integral and hydrostatic balance), not the
  workload's.
* Sampling: the points inside each star number in proportion to its mass,
  the background points lie outside both stars, P = K rho^(5/3) holds point
  by point, and the stars' momenta cancel with the relative speed of a
  circular binary.
* The oracle steps a 20K-point sample: every state stays finite, mass and
  energy are conserved to rounding, and faces at the stars' edges fall back
  to first order (the counter is non-zero) while no cell needs a floor
  after the update.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

import workloads as W


@pytest.mark.parametrize("n,xi1,mu1", [(0.0, math.sqrt(6.0), 2.0 * math.sqrt(6.0)),
                                      (1.0, math.pi, math.pi),
                                      (1.5, 3.65375, 2.71406)])
def test_lane_emden_constants(n, xi1, mu1):
    xi, th, m = W.lane_emden(n)
    assert abs(xi[-1] - xi1) < 2e-5
    assert abs(m[-1] - mu1) < 2e-5
    if n == 1.0:
        # theta = sin(xi) / xi
        k = slice(1, None, 997)
        assert np.allclose(th[k], np.sin(xi[k]) / xi[k], atol=1e-9)


def _scipy_lane_emden(n):
    def rhs(x, y):
        return [y[1], -max(y[0], 0.0) ** n - 2.0 * y[1] / x]

    def surface(x, y):
        return y[0]
    surface.terminal = True
    x0 = 1e-6
    sol = solve_ivp(rhs, (x0, 10.0), [1.0 - x0 * x0 / 6.0, -x0 / 3.0], events=surface,
                    rtol=1e-11, atol=1e-13, dense_output=True)
    return sol.t_events[0][0], sol.sol


@pytest.fixture(scope="module")
def c5():
    return W.c5_polytropes(20000, seed=5)


def test_stars_are_hydrostatic_with_the_requested_mass(c5):
    xi1, sol = _scipy_lane_emden(1.5)
    for st, (m, R) in zip(c5.meta["stars"], ((1.0, 0.1), (0.7, 0.08))):
        a, rc, K = st["alpha"], st["rho_c"], st["K"]
        assert abs(a * xi1 - R) < 1e-6 * R

        def rho(r):
            return rc * max(sol(r / a)[0], 0.0) ** 1.5

        def mass(r):
            return quad(lambda s: 4.0 * math.pi * s * s * rho(s), 0.0, r, limit=200, epsabs=0, epsrel=1e-10)[0]
        assert abs(mass(R * (1 - 1e-12)) - m) < 1e-6 * m
        # dP/dr = -G m(r) rho / r^2 with P = K rho^(5/3), G = 1.
        for f in (0.2, 0.5, 0.8):
            r = f * R
            h = 1e-5 * R
            dP = (K * rho(r + h) ** (5 / 3) - K * rho(r - h) ** (5 / 3)) / (2 * h)
            assert abs(dP + mass(r) * rho(r) / r ** 2) < 1e-6 * abs(dP)


def test_sampling(c5):
    stars = c5.meta["stars"]
    d = [np.linalg.norm(c5.pos - np.array(st["c"]), axis=1) for st in stars]
    inside = [di < st["R"] for di, st in zip(d, stars)]
    n_in = [int(k.sum()) for k in inside]
    assert not np.any(inside[0] & inside[1])
    assert sum(n_in) == 18000
    assert abs(n_in[0] / n_in[1] - 1.0 / 0.7) < 1e-3
    out = ~(inside[0] | inside[1])
    assert np.all(c5.prim[out, 0] == 1e-6) and np.all(c5.prim[out, 1:4] == 0.0)
    # P = K rho^(5/3) with each star's K (the background takes the first's).
    for k, st in enumerate(stars):
        sel = inside[k]
        assert np.allclose(c5.prim[sel, 4], st["K"] * c5.prim[sel, 0] ** (5 / 3), rtol=1e-14, atol=0)
        assert np.all(c5.prim[sel, 2] == st["vy"])
        assert c5.prim[sel, 0].max() <= st["rho_c"] * (1 + 1e-12)
    assert np.allclose(c5.prim[out, 4], stars[0]["K"] * 1e-6 ** (5 / 3), rtol=1e-14, atol=0)
    m = (1.0, 0.7)
    assert abs(m[0] * stars[0]["vy"] + m[1] * stars[1]["vy"]) < 1e-14
    sep = np.linalg.norm(np.array(stars[1]["c"]) - np.array(stars[0]["c"]))
    assert abs(sep - 0.18) < 1e-14
    assert abs(abs(stars[1]["vy"] - stars[0]["vy"]) - math.sqrt(1.7 / 0.18)) < 1e-12
    com = (m[0] * np.array(stars[0]["c"]) + m[1] * np.array(stars[1]["c"])) / 1.7
    assert np.allclose(com, 0.5, atol=1e-15)


def test_oracle_steps_conserve_and_fall_back_at_the_edges(orc, c5):
    p = orc.make_params(c5.box, **c5.params)
    om = orc.tessellate(c5.pos, c5.box)
    assert abs(om.V.sum() - 1.0) < 1e-12
    Q = orc.init_charges(om, p, c5.prim)
    pos = c5.pos.copy()
    m0, E0 = Q[:, 0].sum(), Q[:, 4].sum()
    for _ in range(2):
        pos, Q, w, dt, cnt = orc.step(pos, Q, p)
        assert np.all(np.isfinite(Q)) and dt > 0
        assert cnt[2] > 0 and cnt[3] == 0
    assert abs(Q[:, 0].sum() - m0) <= 1e-14 * m0
    assert abs(Q[:, 4].sum() - E0) <= 1e-14 * E0
