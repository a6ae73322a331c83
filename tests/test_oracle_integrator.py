"""Pins of the oracle's kick-drift-kick integrator on power-of-two time bins.

Fixed by the mathematics and by the scheme's own structure, not by re-typing
it: a softened two-body circular orbit returns to its start after one
period with a second-order error; the leapfrog is time-reversible (forces
that depend on positions only, one bin); runs whose particles all sit in
one bin reduce exactly to the single-bin leapfrog at that step; energy
errors fall as the square of the step (gravity with bins, gas with one
bin); a Plummer sphere drawn in equilibrium stays in equilibrium
(Lagrangian radii, virial ratio, energy); the bin rule and its alignment
constraint on exact boundaries."""
import dataclasses

import numpy as np
import pytest

from paper_2003_10850_amd import inputs
from oracle.integrator import Integrator, IntegParams, bin_of_step, trailing_zeros

BOX = [0.0, 0.0, 0.0, 1.0]


def two_body(d=0.2, eps=1e-3):
    """Equal masses 1/2 on a circular orbit of separation d about the box
    centre: relative speed^2 = G M d^2 / (d^2 + eps^2)^(3/2), M = 1."""
    vrel = np.sqrt(d * d / (d * d + eps * eps) ** 1.5)
    pos = np.array([[0.5 - d / 2, 0.5, 0.5], [0.5 + d / 2, 0.5, 0.5]])
    vel = np.array([[0.0, -vrel / 2, 0.0], [0.0, vrel / 2, 0.0]])
    period = 2 * np.pi * d / vrel
    p = inputs.Params(theta=0.0, eps=eps)
    return pos, vel, period, p


def run(pos, vel, m, u, typ, p, ip, steps):
    it = Integrator(pos, vel, m, u, typ, BOX, p, ip)
    it.start()
    e0 = it.energy()["total"]
    for _ in range(steps):
        it.system_step()
    return it, e0


def test_two_body_orbit_returns_with_second_order_error():
    pos, vel, P, p = two_body()
    errs = []
    for k in (100, 200):
        ip = IntegParams(dt_max=P / k, bin_depth=0, eta=1e9)
        it, e0 = run(pos, vel, [0.5, 0.5], [0, 0], [1, 1], p, ip, k)
        errs.append(np.abs(it.x - pos).max())
        assert abs(it.energy()["total"] - e0) <= 1e-4 * abs(e0)
        # momentum and the centre of mass are exact
        assert np.abs(it.v.sum(0)).max() < 1e-13
    assert errs[0] < 5e-3 * 0.2
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_time_reversible():
    w = inputs.plummer_equilibrium(n=64, seed=9, eps=0.01)
    p = dataclasses.replace(w.params, theta=0.0)
    ip = IntegParams(dt_max=2e-3, bin_depth=0)
    it, _ = run(w.pos, w.vel, w.mass, w.u, w.type, p, ip, 20)
    it.v = -it.v
    for _ in range(20):
        it.system_step()
    np.testing.assert_allclose(it.x, w.pos, rtol=0, atol=1e-12)
    np.testing.assert_allclose(-it.v, w.vel, rtol=0, atol=1e-10)


def test_all_in_one_bin_reduce_to_the_single_bin_leapfrog():
    """(a) Every particle in bin 0 of B = 3: forces only at the eighth tick,
    the drift in eight equal parts, i.e. the B = 0 leapfrog at dt_max.
    (b) Every particle in bin B: the B = 0 leapfrog at dt_max / 2^B."""
    w = inputs.plummer_equilibrium(n=200, seed=4, gas_fraction=0.5, eps=0.01, n_ngb=32.0)
    p = dataclasses.replace(w.params, theta=0.0)
    args = (w.pos, w.vel, w.mass, w.u, w.type, p)
    coarse, _ = run(*args, IntegParams(dt_max=1e-3, bin_depth=3, eta=1e12, courant=1e12), 2)
    assert np.all(coarse.bin == 0)
    ref, _ = run(*args, IntegParams(dt_max=1e-3, bin_depth=0, eta=1e12, courant=1e12), 2)
    np.testing.assert_allclose(coarse.x, ref.x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(coarse.v, ref.v, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(coarse.u, ref.u, rtol=1e-11)
    assert coarse.tick_active == ([0] * 7 + [200]) * 2
    fine, _ = run(*args, IntegParams(dt_max=1e-3, bin_depth=2, eta=1e-12, courant=1e-12), 2)
    assert np.all(fine.bin == 2)
    ref, _ = run(*args, IntegParams(dt_max=2.5e-4, bin_depth=0, eta=1e-12, courant=1e-12), 8)
    np.testing.assert_allclose(fine.x, ref.x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(fine.v, ref.v, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(fine.u, ref.u, rtol=1e-11)


def test_gravity_energy_error_is_second_order_with_bins():
    w = inputs.plummer_equilibrium(n=512, seed=6, eps=0.01)
    p = dataclasses.replace(w.params, theta=0.0)
    errs = []
    for s in (1, 2, 4):
        ip = IntegParams(dt_max=4e-3 / s, bin_depth=2, eta=0.05 / s ** 2)
        it, e0 = run(w.pos, w.vel, w.mass, w.u, w.type, p, ip, 4 * s)
        assert it.bin.min() < it.bin.max()  # several bins in use
        errs.append(abs(it.energy()["total"] - e0) / abs(e0))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_gas_energy_error_is_second_order():
    """Inviscid gas (alpha = 0, G = 0) in a smooth compression: total energy
    kinetic + thermal changes only through the integration error, which
    falls as the square of the step. The hydro force's du/dt depends on the
    velocities; with the predicted velocities it keeps second order."""
    g = np.arange(8)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) * 0.02 + 0.43
    n = pos.shape[0]
    rng = np.random.default_rng(3)
    vel = -0.2 * (pos - 0.5) + rng.normal(0.0, 1e-3, (n, 3))
    p = inputs.Params(n_ngb=40.0, alpha=0.0, h_tol=1e-12, theta=0.0, G=0.0, eps=0.01)
    errs = []
    for s in (4, 8, 16):
        ip = IntegParams(dt_max=4e-3 / s, bin_depth=0)
        it, e0 = run(pos, vel, np.full(n, 1.0 / n), np.ones(n), np.zeros(n, np.uint8), p, ip,
                     4 * s)
        errs.append(abs(it.energy()["total"] - e0) / abs(e0))
    assert errs[2] < 3e-5
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def lagrangian_radii(x):
    r = np.sqrt(((x - 0.5) ** 2).sum(1))
    return np.quantile(r, [0.25, 0.5, 0.75])


def test_plummer_sphere_stays_in_equilibrium():
    """About five dynamical times (sqrt(a^3 / G M) = 0.008) of a 1024-body
    Plummer sphere drawn from its distribution function, with four bins."""
    w = inputs.plummer_equilibrium(n=1024, seed=5)
    p = w.params
    ip = IntegParams(dt_max=4e-3, bin_depth=3)
    it = Integrator(w.pos, w.vel, w.mass, w.u, w.type, BOX, p, ip)
    it.start()
    e0 = it.energy()
    r0 = lagrangian_radii(it.x)
    assert 0.85 < 2 * e0["kinetic"] / abs(e0["potential"]) < 1.15
    for _ in range(10):
        it.system_step()
        e = it.energy()
        np.testing.assert_allclose(lagrangian_radii(it.x), r0, rtol=0.1)
        assert 0.8 < 2 * e["kinetic"] / abs(e["potential"]) < 1.25
    assert abs(e["total"] - e0["total"]) < 3e-3 * abs(e0["total"])
    assert len(set(it.bin.tolist())) >= 3


def test_bin_rule_on_boundaries_and_alignment():
    ip = IntegParams(dt_max=1.0, bin_depth=4)
    dt = np.array([2.0, 1.0, 0.75, 0.5, 0.5 - 1e-12, 1 / 16, 1 / 100, np.inf])
    k, margin = bin_of_step(dt, ip)
    np.testing.assert_array_equal(k, [0, 0, 1, 1, 2, 4, 4, 0])
    assert margin[2] == pytest.approx(np.log2(4 / 3), rel=1e-12)
    assert np.isinf(margin[[0, 1, 6, 7]]).all()
    assert [trailing_zeros(T) for T in (1, 2, 3, 4, 6, 8, 12, 16)] == [0, 1, 0, 2, 1, 3, 2, 4]
    # alignment: a particle whose criterion asks for bin 0 at tick 6 of 16
    # may only take a step that 6 is a multiple of (2 ticks: bin 3)
    w = inputs.plummer_equilibrium(n=64, seed=2, eps=0.01)
    it = Integrator(w.pos, w.vel, w.mass, w.u, w.type, BOX, w.params, ip)
    it.start()
    it.acc[:] = 0.0
    act = np.arange(8)
    it._new_bins(act, 6)
    np.testing.assert_array_equal(it.bin[act], 3)
    it._new_bins(act, 16)
    np.testing.assert_array_equal(it.bin[act], 0)


def test_active_ticks_follow_the_bins():
    w = inputs.plummer_equilibrium(n=400, seed=7, eps=0.005)
    ip = IntegParams(dt_max=4e-3, bin_depth=3)
    it = Integrator(w.pos, w.vel, w.mass, w.u, w.type, BOX, w.params, ip)
    it.start()
    bins0 = it.bin.copy()
    it.system_step()
    # the first tick's active particles are exactly those that began in bin 3
    assert it.tick_active[0] == int((bins0 == 3).sum())
    assert it.tick_active[-1] == w.n
    assert len(it.tick_active) == 8
