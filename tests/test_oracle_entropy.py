"""CPU pins of the oracle's entropy switch (Sec. 4.3; reading R-ent).

The state gains X = rho A, A = P rho^-gamma, carried by the mass flux; a
face's shock Mach number comes from the HLLC star pressure; cells whose
largest face Mach number stays below the threshold (1.1 in the paper) take
their pressure from the entropy, the others keep the energy.
"""
import numpy as np
import pytest

import workloads as W
from sod_exact import sod_paper_exact

G = 1.4
N = np.array([1.0, 0.0, 0.0])


def _shock_states(M0, u_shift=0.0):
    # Post-shock (left) and pre-shock (right, at rest) states of a shock of
    # Mach M0 moving to the right (Rankine-Hugoniot, ideal gas).
    rho1, P1 = 1.0, 1.0
    c1 = np.sqrt(G * P1 / rho1)
    P2 = P1 * (2 * G * M0 ** 2 - (G - 1)) / (G + 1)
    rho2 = rho1 * (G + 1) * M0 ** 2 / ((G - 1) * M0 ** 2 + 2)
    u2 = M0 * c1 * (1 - rho1 / rho2)
    return [rho2, u2 + u_shift, 0, 0, P2], [rho1, u_shift, 0, 0, P1]


@pytest.mark.parametrize("riemann", [0, 1])
def test_mach_estimate_on_exact_shocks(orc, riemann):
    for M0 in (1.05, 1.1, 1.2, 1.5, 2.0, 5.0):
        L, R = _shock_states(M0)
        _, m = orc.entropy_face(L, R, N, G, riemann, 1.0, 1.0)
        assert M0 * 0.995 < m < M0 * (1.02 if M0 <= 1.2 else 1.12), (M0, m)
        # Galilean: the same shock seen from a frame moving along the normal.
        _, m2 = orc.entropy_face(*_shock_states(M0, u_shift=-0.7), N, G, riemann, 1.0, 1.0)
        assert abs(m2 - m) < 1e-12 * m


def test_mach_is_one_without_a_shock(orc):
    # Equal states, a rarefaction (receding states) and a pure shear: no
    # compression, so the star pressure does not exceed either side's.
    W_ = [1.0, 0.2, -0.1, 0.3, 1.0]
    for L, R in ((W_, W_), ([1.0, -0.5, 0, 0, 1.0], [0.5, 0.5, 0, 0, 0.4]),
                 ([1.0, 0.0, 0.4, 0, 1.0], [1.0, 0.0, -0.4, 0, 1.0])):
        for r in (0, 1):
            assert orc.entropy_face(L, R, N, G, r, 1.0, 1.0)[1] == 1.0


def test_entropy_flux_is_the_mass_flux_for_uniform_A(orc):
    rng = np.random.default_rng(21)
    for _ in range(30):
        WL = [rng.uniform(0.2, 2), *rng.uniform(-1, 1, 3), rng.uniform(0.2, 2)]
        WR = [rng.uniform(0.2, 2), *rng.uniform(-1, 1, 3), rng.uniform(0.2, 2)]
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        A = rng.uniform(0.1, 3)
        FX0, _ = orc.entropy_face(WL, WR, n, G, 0, A, A)
        FX1, _ = orc.entropy_face(WL, WR, n, G, 1, A, A)
        assert abs(FX0 - A * orc.hllc_prim(WL, WR, n, G)[0]) < 1e-12 * (1 + abs(FX0))
        assert abs(FX1 - A * orc.hll_prim(WL, WR, n, G)[0]) < 1e-12 * (1 + abs(FX1))


def _start(orc, wl, **over):
    p = orc.make_params(wl.box, **dict(wl.params, **over))
    om = orc.tessellate(wl.pos, wl.box)
    return p, orc.init_charges(om, p, wl.prim), orc.init_entropy(om, p, wl.prim)


def test_threshold_zero_is_the_energy_step_bitwise(orc):
    wl = W.c2_sod(shape=(32, 4, 4), box=(4.0, 0.5, 0.5))
    p, Q, S = _start(orc, wl)
    a = orc.step(wl.pos, Q, p)
    b = orc.step_entropy(wl.pos, Q, S, p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_uniform_entropic_function_is_kept(orc):
    # A uniform flow on a mesh drifting relative to it: with the switch every
    # cell stays below the threshold and A = S/m is carried exactly (up to
    # rounding); the energy equation alone lets it wander.
    pos = W.jittered_lattice((8, 8, 8), (1, 1, 1), jitter=0.2, seed=3)
    wl = W.uniform_state(pos, (1, 1, 1), rho=1.3, vel=(0.4, -0.2, 0.1), P=0.7)
    spread = {}
    for mth in (0.0, 1.1):
        p, Q, S = _start(orc, wl, mach_threshold=mth)
        x = wl.pos.copy()
        for _ in range(10):
            x, Q, S, w, dt, cnt, mach = orc.step_entropy(x, Q, S, p, dt_max=0.01)
        A = S / Q[:, 0]
        spread[mth] = float(np.ptp(A) / A.mean())
        assert mach.max() < 1.1
    assert spread[1.1] < 1e-13 and spread[0.0] > 1e-7, spread


def test_sod_shock_cells_take_the_energy_equation(orc):
    # The paper's Sod tube at low resolution: the shock's cells exceed the
    # threshold (their energy equation captures shock heating) and the
    # result stays as close to the exact solution as with energy only.
    wl = W.sod_paper(k=3)
    res = {}
    for mth in (0.0, 1.1):
        p, Q, S = _start(orc, wl, mach_threshold=mth)
        x, t, shocked = wl.pos.copy(), 0.0, 0
        m0 = Q[:, 0].sum()
        while t < 1.0 - 1e-12:
            x, Q, S, w, dt, cnt, mach = orc.step_entropy(x, Q, S, p, dt_max=1.0 - t)
            t += dt
            shocked = max(shocked, int((mach >= 1.1).sum()))
        V = orc.tessellate(x, wl.box).V
        ex = sod_paper_exact(orc, x[:, 0], 1.0, wl.meta["left"], wl.meta["right"])
        res[mth] = float(np.mean(np.abs(Q[:, 0] / V - ex[:, 0])))
        assert abs(Q[:, 0].sum() - m0) < 1e-12 * m0
        assert shocked > 0
    assert res[1.1] < 1.1 * res[0.0], res
