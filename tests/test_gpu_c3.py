"""The precision workload at full size: N = 2e7 particles (256 Plummer
spheres + 20 % background, half gas) with FP64 stored positions, run on the
mixed-precision path (FP32 offsets, compensated sums, FP64 moments, FP64 h
solve, FP64 decisions near every threshold), checked against the FP64
oracle (FP64 decisions) on a random subsample of 1e4 particles.

Reported: h, rho, hydro and gravity accelerations and potential errors
(max and median, relative to the value or to the L1 sum S of the terms);
counts must be exact. The hydro force is checked at synthetic inputs both
sides read (h and gas density from a gas mass histogram, Omega = 1), so that
no oracle input comes from the GPU; the density at the GPU's solved h, after
that h is compared with the oracle's own solve.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from parity_util import check_solved_density
from paper_2003_10850_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def report(name, e):
    print(f"C3 {name}: max {e.max():.3e} median {np.median(e):.3e}", flush=True)


def test_precision_workload_full_size_subsample():
    from paper_2003_10850_amd import ops
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    w = inputs.plummer(n=20_000_000, n_spheres=256, seed=3)
    print(f"C3 workload {w.name} n={w.n}", flush=True)
    ctx = ops.Context(torch.device("cuda", 0))
    m32 = w.mass.astype(np.float32)
    tree = ops.Tree(ctx, dev_t(w.pos), dev_t(m32), dev_t(w.type), tuple(w.box), w.params)
    d = ops.density(tree)
    assert ctx.nonconverged(reset=True) == 0
    v32, u32 = w.vel.astype(np.float32), w.u.astype(np.float32)
    # the hydro force at synthetic inputs both sides read: h (FP64, the
    # tree's dtype) and gas density from a 128^3 gas mass histogram, Omega = 1
    rm64 = inputs.grid_gas_density(w, cells=128)
    hm = (3.0 * w.params.n_ngb * w.mass / (4.0 * np.pi * rm64)) ** (1.0 / 3.0)
    rm = rm64.astype(np.float32)
    del rm64
    om1 = np.ones(w.n, np.float32)
    hy = ops.hydro_force(tree, dev_t(v32), dev_t(u32), dev_t(hm), dev_t(rm), dev_t(om1))
    # the density also at that synthetic h, for exact counts on both sides
    dm = ops.density(tree, h=dev_t(hm), solve_h=False)
    g = ops.gravity(tree)
    torch.cuda.synchronize()
    h, rho = host(d["h"]), host(d["rho"])
    acc, npairs = host(hy["acc"]), host(hy["npairs"])
    rho_m, nngb_m = host(dm["rho"]), host(dm["nngb"])
    gacc, pot, nterms = host(g["acc"]), host(g["pot"]), host(g["nterms"])
    del d, dm, hy, g, tree
    torch.cuda.empty_cache()
    print("C3 GPU step done; oracle on the subsample", flush=True)

    rng = np.random.default_rng(11)
    gas = np.nonzero(w.type == 0)[0]
    sg = np.sort(rng.choice(gas, 10_000, replace=False))
    sa = np.sort(rng.choice(w.n, 10_000, replace=False))
    M = m32.astype(np.float64)
    p = dataclasses.replace(w.params, flags=oracle.FLAG_FP64_DECISIONS)
    gt = oracle.Tree(w.pos, M, w.box, type=w.type, gas_only=True)
    ref = oracle.density(gt, p, active=sg)
    eh, er = check_solved_density(h, rho, ref, sg, 2e-6, 1e-5, "C3")
    print(f"C3 h rel: max {eh:.3e}; rho at the solved h: max {er:.3e}", flush=True)
    at_h = oracle.density(gt, p, active=sg, h=hm, solve_h=False)
    np.testing.assert_array_equal(nngb_m[sg], at_h["nngb"][sg])
    e = np.abs(rho_m[sg] - at_h["rho"][sg]) / at_h["rho"][sg]
    report("rho rel (given h)", e)
    assert e.max() < 1e-5
    r = oracle.hydro(gt, p, v32, u32, hm, rm, om1, active=sg)
    np.testing.assert_array_equal(npairs[sg], r["npairs"][sg])
    e = np.linalg.norm(acc[sg] - r["acc"][sg], axis=1) / r["S"][sg]
    report("hydro acc |da|/S", e)
    assert e.max() < 1e-5
    del gt
    at = oracle.Tree(w.pos, M, w.box, type=w.type)
    rg = oracle.gravity(at, p, active=sa)
    np.testing.assert_array_equal(nterms[sa], rg["nterms"][sa])
    e = np.linalg.norm(gacc[sa] - rg["acc"][sa], axis=1) / rg["S"][sa]
    report("gravity acc |da|/S", e)
    assert e.max() < 1e-5
    e = np.linalg.norm(gacc[sa] - rg["acc"][sa], axis=1) / np.linalg.norm(rg["acc"][sa], axis=1)
    report("gravity acc |da|/|a|", e)
    e = np.abs(pot[sa] - rg["pot"][sa]) / np.abs(rg["pot"][sa])
    report("potential rel", e)
    assert e.max() < 1e-5
