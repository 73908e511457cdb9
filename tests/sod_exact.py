"""Exact density of the paper's periodic Sod tube (two Riemann problems, at
x = 8 and at x = 0 = 16) from the oracle's exact Riemann solver."""
import numpy as np


def sod_paper_exact(orc, x, t, left, right, gamma=1.4):
    """Exact (rho, u, P) at positions x in [0, 16) and time t > 0, while the
    waves of the two interfaces have not met (t below about 2.4)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((x.size, 3))
    mid = (x >= 4.0) & (x < 12.0)
    if mid.any():
        W, _, _ = orc.exact_riemann(left, right, gamma, (x[mid] - 8.0) / t)
        out[mid] = W
    edge = ~mid
    if edge.any():
        xe = np.where(x[edge] < 4.0, x[edge], x[edge] - 16.0)
        W, _, _ = orc.exact_riemann(right, left, gamma, xe / t)
        out[edge] = W
    return out
