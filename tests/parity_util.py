"""Shared checks of the GPU parity tests.

Every oracle input is synthetic or the oracle's own: a GPU output is only
ever compared with the oracle, never fed to it.
"""
import numpy as np


def check_solved_density(h_gpu, rho_gpu, ref, rows, htol, rtol, label=""):
    """The GPU's solved h and its density there against the oracle's own
    solve (ref: h, rho, omega of oracle.density with the h solve) on `rows`:
    h within htol, relative; rho within rtol plus its first-order change
    with the difference in h, |d ln rho / d ln h| = 3 |Omega - 1| (the
    oracle's Omega), with a 1.5 margin for the second order. Returns the
    largest relative differences of h and of rho."""
    hr = ref["h"][rows]
    dh = np.abs(np.asarray(h_gpu, np.float64)[rows] - hr) / hr
    assert dh.max() < htol, f"{label} h: max rel {dh.max():.3e}"
    rr = ref["rho"][rows]
    drho = np.abs(np.asarray(rho_gpu, np.float64)[rows] - rr) / rr
    bar = rtol + 1.5 * (3.0 * np.abs(ref["omega"][rows] - 1.0) + 0.1) * dh
    assert (drho <= bar).all(), f"{label} rho: {np.sum(drho > bar)} rows beyond the bar"
    return float(dh.max()), float(drho.max())
