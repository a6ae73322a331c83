"""Pins of the oracle's Wendland C6 kernel against the mathematics.

The kernel (Dehnen & Aly 2012, table 1; compact support h) is fixed by:
unit normalisation, vanishing at and beyond the support radius together with
its low derivatives, and the derivative relations; each is checked here by
quadrature or finite differences, not by re-typing the formula."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


def W(r, h):
    return oracle.kernel(r, h)[0]


@pytest.mark.parametrize("h", [1.0, 0.37, 2.5])
def test_normalisation(h):
    val, err = integrate.quad(lambda r: 4 * math.pi * r * r * W(r, h), 0, h,
                              epsabs=1e-13, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-12


def test_central_value():
    # W(0, 1) is the 3D normalisation 1365 / (64 pi)
    assert W(0.0, 1.0) == pytest.approx(1365.0 / (64.0 * math.pi), rel=1e-15)


@pytest.mark.parametrize("q", [0.05, 0.3, 0.5, 0.77, 0.95])
@pytest.mark.parametrize("h", [1.0, 0.2])
def test_derivatives_by_finite_differences(q, h):
    r = q * h
    _, dWdr, dWdh, F = oracle.kernel(r, h)
    d = 1e-6 * h
    fd_r = (W(r + d, h) - W(r - d, h)) / (2 * d)
    fd_h = (W(r, h + d) - W(r, h - d)) / (2 * d)
    scale = W(0.0, h) / h
    assert abs(dWdr - fd_r) < 1e-7 * scale
    assert abs(dWdh - fd_h) < 1e-7 * scale
    assert F == pytest.approx(dWdr / r, rel=1e-13)


@pytest.mark.parametrize("q", [0.0, 0.1, 0.5, 0.9])
def test_scaling_identity(q):
    # W = h^-3 f(r/h)  =>  dW/dh = -(3 W + r dW/dr) / h
    h = 0.7
    r = q * h
    Wv, dWdr, dWdh, _ = oracle.kernel(r, h)
    assert dWdh == pytest.approx(-(3 * Wv + r * dWdr) / h, rel=1e-12, abs=1e-14)


def test_compact_support_and_smoothness():
    h = 1.0
    for r in [1.0, 1.0 + 1e-12, 1.5, 10.0]:
        assert oracle.kernel(r, h) == (0.0, 0.0, 0.0, 0.0)
    # C6 at the support edge: W ~ (1-q)^8, so W(1-d)/d^8 stays bounded and
    # the first derivative vanishes like d^7
    for d in [1e-2, 1e-3]:
        Wv, dWdr, _, _ = oracle.kernel(1 - d, h)
        assert 0 < Wv < 1e3 * d ** 8
        assert abs(dWdr) < 1e4 * d ** 7


def test_monotone_decreasing_in_r():
    r = np.linspace(0, 0.999, 400)
    w = np.array([W(x, 1.0) for x in r])
    assert np.all(np.diff(w) < 0)
    F = np.array([oracle.kernel(x, 1.0)[3] for x in r])
    assert np.all(F < 0)


def test_self_term_neff():
    # an isolated particle: N_eff(h) = (4 pi / 3) h^3 W(0, h) = 1365/48 for every h
    for h in [1e-3, 0.1, 0.9]:
        pos = np.array([[0.5, 0.5, 0.5]])
        t = oracle.Tree(pos, np.array([0.25]), [0, 0, 0, 1], gas_only=True)
        from paper_2003_10850_amd.inputs import Params
        d = oracle.density(t, Params(), h=np.array([h]), solve_h=False)
        neff = 4 * math.pi / 3 * h ** 3 * d["rho"][0] / 0.25
        assert neff == pytest.approx(1365.0 / 48.0, rel=1e-14)
        assert d["nngb"][0] == 1
