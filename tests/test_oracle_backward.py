"""Pins of the oracle's adjoints (no GPU).

The adjoints are derivatives of the forward modules, so they are pinned
against things that do not share their code path:
  * central finite differences of the forward oracle itself (the whole
    module output, re-run with one input moved), with neighbour and opening
    decisions in FP64 so that the tiny steps do not flip FP32 roundings;
  * exact identities of the forward maps: translation invariance (the loss
    depends on position differences only, so the position gradients sum to
    zero), linearity in the source masses (sum_j m_j dL/dm_j = L for a loss
    linear in rho, a or phi), and the scaling of the kernel
    (rho(lambda x, lambda h) = lambda^-3 rho(x, h), so
    sum x . dL/dx + sum h dL/dh = -3 L for L linear in rho);
  * a two-body closed form for gravity.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2003_10850_amd import inputs


def fp64(p):
    return dataclasses.replace(p, flags=oracle.FLAG_FP64_DECISIONS)


def clustered(n, seed, n_ngb=40.0):
    w = inputs.plummer(n=n, n_spheres=2, seed=seed, n_ngb=n_ngb, eps=0.01)
    w.type[:] = inputs.GAS
    return w


# ----------------------------------------------------------------- density

def density_loss(w, pos, mass, h, coef, act):
    t = oracle.Tree(pos, mass, w.box, type=w.type, gas_only=True)
    d = oracle.density(t, fp64(w.params), active=act, h=h, solve_h=False)
    a, b, c = coef
    return float((a * d["rho"] + b * d["drho_dh"] + c * d["omega"])[act].sum())


def density_setup(seed=1, n=400):
    w = clustered(n, seed)
    h = inputs.model_smoothing(w, 40.0)
    rng = np.random.default_rng(seed)
    coef = [rng.normal(size=w.n) for _ in range(3)]
    act = np.sort(rng.choice(w.n, size=w.n // 2, replace=False))
    return w, h, coef, act


def test_density_backward_matches_finite_differences():
    w, h, coef, act = density_setup()
    t = oracle.Tree(w.pos, w.mass, w.box, type=w.type, gas_only=True)
    g = oracle.density_backward(t, fp64(w.params), h, *coef, active=act)
    rng = np.random.default_rng(5)
    L = lambda P, M, H: density_loss(w, P, M, H, coef, act)
    for k in rng.choice(w.n, size=6, replace=False):
        for c in range(3):
            d = 1e-6
            P1, P2 = w.pos.copy(), w.pos.copy()
            P1[k, c] += d
            P2[k, c] -= d
            fd = (L(P1, w.mass, h) - L(P2, w.mass, h)) / (2 * d)
            assert abs(fd - g["pos"][k, c]) <= 1e-6 * np.abs(g["pos"]).max(), (k, c)
        d = 1e-6 * w.mass[k]
        M1, M2 = w.mass.copy(), w.mass.copy()
        M1[k] += d
        M2[k] -= d
        fd = (L(w.pos, M1, h) - L(w.pos, M2, h)) / (2 * d)
        assert abs(fd - g["mass"][k]) <= 1e-6 * np.abs(g["mass"]).max(), k
        d = 1e-6 * h[k]
        H1, H2 = h.copy(), h.copy()
        H1[k] += d
        H2[k] -= d
        fd = (L(w.pos, w.mass, H1) - L(w.pos, w.mass, H2)) / (2 * d)
        assert abs(fd - g["h"][k]) <= 1e-6 * np.abs(g["h"]).max(), k


def test_density_backward_identities():
    w, h, coef, act = density_setup(seed=2)
    t = oracle.Tree(w.pos, w.mass, w.box, type=w.type, gas_only=True)
    a = coef[0]
    zero = np.zeros(w.n)
    g = oracle.density_backward(t, fp64(w.params), h, a, zero, zero, active=act)
    L = density_loss(w, w.pos, w.mass, h, (a, zero, zero), act)
    # translation invariance
    assert np.abs(g["pos"].sum(0)).max() < 1e-10 * np.abs(g["pos"]).sum()
    # rho is linear in the masses
    assert abs((w.mass * g["mass"]).sum() - L) < 1e-10 * abs(L)
    # rho(lambda x, lambda h) = lambda^-3 rho(x, h)
    euler = (w.pos * g["pos"]).sum() + (h * g["h"]).sum()
    assert abs(euler + 3 * L) < 1e-9 * abs(L)


# ------------------------------------------- through the smoothing-length solve

def tight(p):
    """FP64 decisions and a bisection closed to 1e-13 of h, so that finite
    differences of the solved h resolve its derivative."""
    return dataclasses.replace(p, flags=oracle.FLAG_FP64_DECISIONS, h_tol=1e-13)


def solved_h(w, pos, mass, act):
    t = oracle.Tree(pos, mass, w.box, type=w.type, gas_only=True)
    d = oracle.density(t, tight(w.params), active=act, solve_h=True)
    assert d["nonconv"] == 0
    return t, d


def solve_setup(seed):
    w = clustered(400, seed)
    rng = np.random.default_rng(seed)
    coef = rng.normal(size=w.n)
    act = np.sort(rng.choice(w.n, size=w.n // 2, replace=False))
    return w, coef, act


def test_solve_backward_matches_finite_differences():
    w, coef, act = solve_setup(3)
    t, d = solved_h(w, w.pos, w.mass, act)
    g = oracle.density_solve_backward(t, w.params, d["h"], d["rho"], d["drho_dh"], coef,
                                      active=act)
    L = lambda P, M: float((coef * solved_h(w, P, M, act)[1]["h"])[act].sum())
    rng = np.random.default_rng(6)
    # moved particles both inside and outside the active set
    for k in list(rng.choice(act, 3, replace=False)) + list(
            rng.choice(np.setdiff1d(np.arange(w.n), act), 3, replace=False)):
        for c in range(3):
            dx = 1e-6
            P1, P2 = w.pos.copy(), w.pos.copy()
            P1[k, c] += dx
            P2[k, c] -= dx
            fd = (L(P1, w.mass) - L(P2, w.mass)) / (2 * dx)
            assert abs(fd - g["pos"][k, c]) <= 1e-6 * np.abs(g["pos"]).max(), (k, c, fd)
        dm = 1e-6 * w.mass[k]
        M1, M2 = w.mass.copy(), w.mass.copy()
        M1[k] += dm
        M2[k] -= dm
        fd = (L(w.pos, M1) - L(w.pos, M2)) / (2 * dm)
        assert abs(fd - g["mass"][k]) <= 1e-6 * np.abs(g["mass"]).max(), (k, fd)


def test_solve_backward_identities():
    w, coef, act = solve_setup(4)
    t, d = solved_h(w, w.pos, w.mass, act)
    g = oracle.density_solve_backward(t, w.params, d["h"], d["rho"], d["drho_dh"], coef,
                                      active=act)
    L = float((coef * d["h"])[act].sum())
    # h depends on position differences only
    assert np.abs(g["pos"].sum(0)).max() < 1e-10 * np.abs(g["pos"]).sum()
    # and on the masses only through ratios m_j / m_i: scaling every mass
    # leaves h unchanged (this needs the explicit 1/m_i of N_eff)
    mg = w.mass * g["mass"]
    assert abs(mg.sum()) < 1e-9 * np.abs(mg).sum()
    # h(lambda x) = lambda h(x)
    assert abs((w.pos * g["pos"]).sum() - L) < 1e-9 * abs(L)
    # an h that did not converge has no constraint and passes nothing
    bad = d["rho"].copy()
    bad[act[0]] *= 0.5
    g2 = oracle.density_solve_backward(t, w.params, d["h"], bad, d["drho_dh"], coef, active=act)
    only = np.zeros(w.n)
    only[act[0]] = coef[act[0]]
    g1 = oracle.density_solve_backward(t, w.params, d["h"], d["rho"], d["drho_dh"], only,
                                       active=act)
    assert np.allclose(g2["pos"], g["pos"] - g1["pos"], rtol=0, atol=1e-12 * np.abs(g["pos"]).max())


# ------------------------------------------------------------------- hydro

def hydro_fields(w, seed):
    rng = np.random.default_rng(seed)
    h = inputs.model_smoothing(w, 40.0)
    rho = inputs.model_gas_density(w) * rng.uniform(0.8, 1.2, w.n)
    om = rng.uniform(0.8, 1.2, w.n)
    u = rng.uniform(0.5, 2.0, w.n)
    return h, rho, om, u


def hydro_loss(w, X, gA, gD, act):
    pos, vel, mass, h, u, rho, om = X
    t = oracle.Tree(pos, mass, w.box, type=w.type, gas_only=True)
    r = oracle.hydro(t, fp64(w.params), vel, u, h, rho, om, active=act)
    return float((gA * r["acc"]).sum(1)[act].sum() + (gD * r["dudt"])[act].sum())


def test_hydro_backward_matches_finite_differences():
    w = clustered(300, 3)
    h, rho, om, u = hydro_fields(w, 3)
    rng = np.random.default_rng(4)
    gA, gD = rng.normal(size=(w.n, 3)), rng.normal(size=w.n)
    act = np.sort(rng.choice(w.n, size=200, replace=False))
    t = oracle.Tree(w.pos, w.mass, w.box, type=w.type, gas_only=True)
    g = oracle.hydro_backward(t, fp64(w.params), w.vel, u, h, rho, om, gA, gD, active=act)
    X = [w.pos, w.vel, w.mass, h, u, rho, om]
    names = ["pos", "vel", "mass", "h", "u", "rho", "omega"]
    for vi, name in enumerate(names):
        for k in rng.choice(w.n, size=4, replace=False):
            comps = range(3) if X[vi].ndim == 2 else [None]
            for c in comps:
                idx = (k, c) if c is not None else k
                base = X[vi][idx]
                d = 1e-6 * (1.0 if name in ("pos", "vel") else abs(base))
                X1 = [x.copy() for x in X]
                X2 = [x.copy() for x in X]
                X1[vi][idx] += d
                X2[vi][idx] -= d
                fd = (hydro_loss(w, X1, gA, gD, act) - hydro_loss(w, X2, gA, gD, act)) / (2 * d)
                scale = np.abs(g[name]).max()
                assert abs(fd - g[name][idx]) <= 2e-6 * scale, (name, idx, fd, g[name][idx])


def test_hydro_backward_translation_invariance():
    w = clustered(300, 6)
    h, rho, om, u = hydro_fields(w, 6)
    rng = np.random.default_rng(7)
    t = oracle.Tree(w.pos, w.mass, w.box, type=w.type, gas_only=True)
    g = oracle.hydro_backward(t, fp64(w.params), w.vel, u, h, rho, om,
                              rng.normal(size=(w.n, 3)), rng.normal(size=w.n))
    assert np.abs(g["pos"].sum(0)).max() < 1e-10 * np.abs(g["pos"]).sum()
    # velocities enter through differences v_i - v_j only
    assert np.abs(g["vel"].sum(0)).max() < 1e-10 * np.abs(g["vel"]).sum()


# ----------------------------------------------------------------- gravity

def gravity_loss(w, pos, mass, gA, gP, act, params):
    t = oracle.Tree(pos, mass, w.box, type=w.type)
    r = oracle.gravity(t, params, active=act)
    return float((gA * r["acc"]).sum(1)[act].sum() + (gP * r["pot"])[act].sum()), r["nterms"]


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_gravity_backward_matches_finite_differences(theta):
    w = inputs.plummer(n=300, n_spheres=2, seed=8)
    p = fp64(dataclasses.replace(w.params, theta=theta, eps=0.01))
    rng = np.random.default_rng(9)
    gA, gP = rng.normal(size=(w.n, 3)), rng.normal(size=w.n)
    act = np.sort(rng.choice(w.n, size=150, replace=False))
    t = oracle.Tree(w.pos, w.mass, w.box, type=w.type)
    g = oracle.gravity_backward(t, p, gA, gP, active=act)
    _, n0 = gravity_loss(w, w.pos, w.mass, gA, gP, act, p)
    checked = 0
    for k in rng.choice(w.n, size=8, replace=False):
        for c in range(3):
            d = 1e-7
            P1, P2 = w.pos.copy(), w.pos.copy()
            P1[k, c] += d
            P2[k, c] -= d
            (L1, n1), (L2, n2) = (gravity_loss(w, P1, w.mass, gA, gP, act, p),
                                  gravity_loss(w, P2, w.mass, gA, gP, act, p))
            if not (np.array_equal(n1, n0) and np.array_equal(n2, n0)):
                continue  # a decision flipped: the loss is not smooth here
            fd = (L1 - L2) / (2 * d)
            assert abs(fd - g["pos"][k, c]) <= 1e-5 * np.abs(g["pos"]).max(), (k, c)
            checked += 1
        d = 1e-6 * w.mass[k]
        M1, M2 = w.mass.copy(), w.mass.copy()
        M1[k] += d
        M2[k] -= d
        fd = (gravity_loss(w, w.pos, M1, gA, gP, act, p)[0] -
              gravity_loss(w, w.pos, M2, gA, gP, act, p)[0]) / (2 * d)
        assert abs(fd - g["mass"][k]) <= 1e-6 * np.abs(g["mass"]).max(), k
    assert checked >= 12


def test_gravity_backward_identities():
    w = inputs.plummer(n=500, n_spheres=3, seed=10)
    p = w.params
    rng = np.random.default_rng(11)
    gA, gP = rng.normal(size=(w.n, 3)), rng.normal(size=w.n)
    t = oracle.Tree(w.pos, w.mass, w.box, type=w.type)
    g = oracle.gravity_backward(t, p, gA, gP)
    L, _ = gravity_loss(w, w.pos, w.mass, gA, gP, np.arange(w.n), p)
    assert np.abs(g["pos"].sum(0)).max() < 1e-10 * np.abs(g["pos"]).sum()
    # a and phi are linear in the source masses (node masses included)
    assert abs((w.mass * g["mass"]).sum() - L) < 1e-10 * abs(L)


def test_gravity_backward_two_bodies():
    """Two particles, eps: phi_0 = -G m_1 / sqrt(r^2 + eps^2); with
    L = phi_0, dL/dx_0 = G m_1 x_01 / (r^2 + eps^2)^(3/2) and dL/dm_1 =
    -G / sqrt(r^2 + eps^2)."""
    pos = np.array([[0.2, 0.3, 0.4], [0.7, 0.1, 0.45]])
    m = np.array([0.3, 0.9])
    p = inputs.Params(theta=0.5, eps=0.05, G=2.0)
    t = oracle.Tree(pos, m, np.array([0, 0, 0, 1.0]))
    g = oracle.gravity_backward(t, p, g_pot=np.array([1.0, 0.0]), active=np.array([0]))
    x = pos[0] - pos[1]
    s2 = x @ x + p.eps ** 2
    np.testing.assert_allclose(g["pos"][0], p.G * m[1] * x / s2 ** 1.5, rtol=1e-13)
    np.testing.assert_allclose(g["pos"][1], -p.G * m[1] * x / s2 ** 1.5, rtol=1e-13)
    np.testing.assert_allclose(g["mass"], [0.0, -p.G / np.sqrt(s2)], rtol=1e-13)
