"""Pins of the oracle's thermal conduction (the paper's third ported module).

The paper names the module but prints no formula; the oracle follows the SPH
form of the heat equation of Brookshaw (1985) that Gadget's conduction module
uses (Jubelgas, Springel & Dolag 2004):
    du_i/dt = sum_j m_j (kappa_i + kappa_j) (u_i - u_j) / (rho_i rho_j)
              * (x_ij . grad_i Wbar_ij) / |x_ij|^2,
Wbar_ij = (W(h_i) + W(h_j)) / 2, kappa = kappa0 u^kappa_exp. The pins:

- closed forms on two and three particles, derived here in exact symbolic
  arithmetic from that equation (the kernel's gradient by symbolic
  differentiation of W(|x_i - x_j|, h), never the oracle's F), with a
  Spitzer-like kappa ~ u^(5/2) at perfect-square energies;
- total thermal energy is conserved (each pair's exchange is
  antisymmetric) and a uniform u stays uniform;
- on a cubic lattice the rate of a quadratic profile u = a + b x^2 is the
  continuum kappa (d2u/dx2) / rho = 2 b kappa / rho, to the lattice's
  discretisation error;
- a step profile diffuses as the heat equation's erf solution.
A plausible mistake (a dropped 1/2 of the kernel average, the sign, kappa_i
alone, rho_i^2 for rho_i rho_j, the wrong power of u) fails one of these.
"""
import numpy as np
import pytest
import sympy as sp

import oracle
from paper_2003_10850_amd import inputs


def _w_sym():
    xi = sp.symbols("xi0:3", real=True)
    xj = sp.symbols("xj0:3", real=True)
    h = sp.symbols("h", positive=True)
    r = sp.sqrt(sum((a - b) ** 2 for a, b in zip(xi, xj)))
    q = r / h
    C = sp.Rational(1365, 64) / sp.pi
    W = C / h ** 3 * (1 - q) ** 8 * (1 + 8 * q + 25 * q ** 2 + 32 * q ** 3)
    return xi, xj, h, [sp.diff(W, a) for a in xi]


_XI, _XJ, _H, _GRAD = _w_sym()


def x_dot_grad_over_r2(x_i, x_j, h):
    """(x_ij . grad_i W(|x_ij|, h)) / |x_ij|^2, exact (zero beyond h)."""
    xij = [a - b for a, b in zip(x_i, x_j)]
    r2 = sum(x * x for x in xij)
    if not sp.sqrt(r2) < h:
        return sp.Integer(0)
    sub = {**dict(zip(_XI, x_i)), **dict(zip(_XJ, x_j)), _H: h}
    g = [e.subs(sub) for e in _GRAD]
    return sum(a * b for a, b in zip(xij, g)) / r2


def expected(xs, us, hs, rhos, ms, kappa0, kexp, i):
    kap = [kappa0 * u ** kexp for u in us]
    du = sp.Integer(0)
    for j in range(len(xs)):
        if j == i:
            continue
        r = sp.sqrt(sum((a - b) ** 2 for a, b in zip(xs[i], xs[j])))
        if not r < max(hs[i], hs[j]):
            continue
        gbar = (x_dot_grad_over_r2(xs[i], xs[j], hs[i]) +
                x_dot_grad_over_r2(xs[i], xs[j], hs[j])) / 2
        du += ms[j] * (kap[i] + kap[j]) * (us[i] - us[j]) / (rhos[i] * rhos[j]) * gbar
    return du


def run_oracle(xs, us, hs, rhos, ms, kappa0, kexp):
    n = len(xs)
    pos = np.array([[float(c) for c in x] for x in xs])
    t = oracle.Tree(pos, np.array([float(m) for m in ms]), [0.0, 0.0, 0.0, 1.0],
                    gas_only=True)
    p = inputs.Params(flags=1)  # FP64 neighbour decisions: exact at dyadic inputs
    return oracle.conduction(t, p, [float(u) for u in us], [float(h) for h in hs],
                             [float(r) for r in rhos], float(kappa0), float(kexp),
                             active=np.arange(n))


R = sp.Rational


@pytest.mark.parametrize("kexp", [0, R(5, 2)])
def test_two_and_three_particle_closed_forms(kexp):
    xs = [(R(1, 2), R(1, 2), R(1, 2)), (R(9, 16), R(17, 32), R(1, 2)),
          (R(15, 32), R(1, 2), R(35, 64))]
    us = [R(4), R(9, 4), R(25, 16)]          # perfect squares: u^(5/2) is rational
    hs = [R(1, 8), R(3, 32), R(5, 64)]
    rhos = [R(3, 2), R(5, 4), R(7, 4)]
    ms = [R(1, 4), R(3, 8), R(1, 8)]
    kappa0 = R(3, 1024)
    for n in (2, 3):
        out = run_oracle(xs[:n], us[:n], hs[:n], rhos[:n], ms[:n], kappa0, kexp)
        for i in range(n):
            e = float(expected(xs[:n], us[:n], hs[:n], rhos[:n], ms[:n], kappa0, kexp, i))
            assert e != 0.0
            assert out["dudt"][i] == pytest.approx(e, rel=1e-12), (n, i)
        assert out["npairs"][:n].sum() > 0


def clustered(n=3000, seed=4):
    w = inputs.plummer(n=n, n_spheres=3, seed=seed, n_ngb=64.0, eps=1e-3)
    gas = np.nonzero(w.type == 0)[0]
    t = oracle.Tree(w.pos, w.mass, w.box, type=w.type, gas_only=True)
    d = oracle.density(t, w.params, active=gas)
    return w, gas, t, d


def test_energy_is_conserved_and_uniform_u_stays_uniform():
    w, gas, t, d = clustered()
    rng = np.random.default_rng(0)
    u = np.zeros(w.n)
    u[gas] = rng.uniform(0.5, 3.0, gas.size)
    c = oracle.conduction(t, w.params, u, d["h"], d["rho"], 1e-3, 2.5, active=gas)
    md = w.mass[gas] * c["dudt"][gas]
    assert np.abs(md).sum() > 0
    assert abs(md.sum()) < 1e-13 * np.abs(md).sum()
    # heat flows from hot to cold: the hottest particle cools, the coldest warms
    assert c["dudt"][gas[np.argmax(u[gas])]] < 0 < c["dudt"][gas[np.argmin(u[gas])]]
    u[gas] = 1.7
    c = oracle.conduction(t, w.params, u, d["h"], d["rho"], 1e-3, 2.5, active=gas)
    assert np.all(c["dudt"][gas] == 0.0)


def lattice_slab(nx, ny, nz, spacing):
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                 -1).reshape(-1, 3)
    return (g + 0.5) * spacing


def interior(pos, lo, hi, margin):
    return np.all((pos >= lo + margin) & (pos <= hi - margin), axis=1)


def test_quadratic_profile_gives_the_continuum_laplacian():
    """With 295 neighbours (h about 6 lattice spacings) the lattice sums are
    within a few 1e-4 of the continuum integrals; with 64 the lattice
    error is several per cent, the same on every interior particle."""
    a = 1.0 / 32
    pos = lattice_slab(20, 20, 20, a)
    n = pos.shape[0]
    m = np.full(n, 1.0 / n)
    p = inputs.Params(n_ngb=295.0)
    t = oracle.Tree(pos, m, [0.0, 0.0, 0.0, 1.0], gas_only=True)
    d = oracle.density(t, p)
    b, kappa = 3.0, 2e-3
    u = 1.0 + b * (pos[:, 0] - 0.3) ** 2
    c = oracle.conduction(t, p, u, d["h"], d["rho"], kappa, 0.0)
    core = interior(pos, 0.0, 20 * a, d["h"].max() * 1.01)
    assert core.sum() >= 512
    want = 2.0 * b * kappa / d["rho"][core]
    rel = np.abs(c["dudt"][core] - want) / want
    assert rel.max() < 2e-3, rel.max()


def test_step_profile_diffuses_as_the_heat_equation():
    """u = 1 left of x0, 2 right of it, constant kappa on a lattice slab;
    after time t the central columns follow
    u = 3/2 + (1/2) erf((x - x0) / (2 sqrt(D t))), D = kappa / rho."""
    from scipy.special import erf
    a = 1.0 / 32
    pos = lattice_slab(32, 12, 12, a)
    n = pos.shape[0]
    m = np.full(n, 1.0 / n)
    p = inputs.Params(n_ngb=64.0)
    t = oracle.Tree(pos, m, [0.0, 0.0, 0.0, 1.0], gas_only=True)
    d = oracle.density(t, p)
    x0 = 16 * a
    u = np.where(pos[:, 0] < x0, 1.0, 2.0)
    kappa = 1e-3
    rho0 = np.median(d["rho"])
    D = kappa / rho0
    T = (2.5 * a) ** 2 / D     # diffusion length sqrt(D T) = 2.5 spacings
    steps = 200
    dt = T / steps
    for _ in range(steps):     # midpoint (RK2) steps of the fixed-particle rate
        k1 = oracle.conduction(t, p, u, d["h"], d["rho"], kappa)["dudt"]
        k2 = oracle.conduction(t, p, u + 0.5 * dt * k1, d["h"], d["rho"], kappa)["dudt"]
        u = u + dt * k2
    core = interior(pos, np.array([0, 0, 0]), np.array([32 * a, 12 * a, 12 * a]),
                    np.array([0.0, 3.5 * a, 3.5 * a]))
    xs = pos[core, 0]
    want = 1.5 + 0.5 * erf((xs - x0) / (2.0 * np.sqrt(D * T)))
    err = np.abs(u[core] - want).max()
    assert err < 0.02, err  # of a jump of 1
    # total thermal energy is conserved by the exchange
    assert abs((m * u).sum() - (m * np.where(pos[:, 0] < x0, 1.0, 2.0)).sum()) < 1e-12
