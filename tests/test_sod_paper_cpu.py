"""CPU checks of the paper's Sod tube workload (Sec. 5, Sod shock-tube test)
and of the exact solution the GPU test compares with."""
import numpy as np

import workloads as W
from sod_exact import sod_paper_exact


def test_workload_geometry_states_and_options():
    wl = W.sod_paper(k=4)
    assert wl.n == 64 * 4 * 4 and wl.box == (16.0, 1.0, 1.0)
    assert (wl.pos >= 0).all() and (wl.pos < np.array(wl.box)).all()
    left = wl.pos[:, 0] < 8.0
    assert np.all(wl.prim[left, 0] == 1.0) and np.all(wl.prim[left, 4] == 1.0)
    assert np.all(wl.prim[~left, 0] == 0.25) and np.all(wl.prim[~left, 4] == 0.1795)
    assert not wl.prim[:, 1:4].any() and wl.params["gamma"] == 1.4
    assert wl.params["riemann"] == 0 and wl.params["eta"] == 1.0
    sm = W.sod_paper(k=4, riemann="hll", static_mesh=True)
    assert sm.params["riemann"] == 1 and sm.params["eta"] == 0.0 and sm.params["chi"] == 0.0


def test_exact_solution_of_the_two_interfaces(orc):
    # Far from both interfaces the initial states persist.  The two Riemann
    # problems are mirror images: rho(8 + s) at the central interface equals
    # rho(0 - s) at the periodic one, and the velocity changes sign.
    L, R = (1.0, 0.0, 1.0), (0.25, 0.0, 0.1795)
    x = np.array([4.5, 11.5, 12.5, 3.5])
    W_ = sod_paper_exact(orc, x, 2.0, L, R)
    np.testing.assert_array_equal(W_[:, 0], [1.0, 0.25, 0.25, 1.0])
    s = np.linspace(-3.5, 3.5, 141)
    a = sod_paper_exact(orc, 8.0 + s, 2.0, L, R)
    b = sod_paper_exact(orc, np.mod(-s, 16.0), 2.0, L, R)
    np.testing.assert_allclose(a[:, 0], b[:, 0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(a[:, 1], -b[:, 1], rtol=0, atol=1e-14)
