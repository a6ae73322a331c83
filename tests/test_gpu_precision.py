"""GPU parity of the mixed-precision path (FP64 stored positions, FP32
group-relative offsets, compensated sums, FP64 h solve) against the oracle
with every neighbour and opening decision taken in FP64.

Bars: exact octree, neighbour counts, pair counts and interaction counts;
h within 2e-6 of the oracle's FP64 bisection; density within 1e-5; hydro and
gravity accelerations within 1e-5 of the L1 sum of their terms. A box moved
far from the origin keeps the same bars on this path, while the plain FP32
path visibly degrades there.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from parity_util import check_solved_density
from paper_2003_10850_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
HTOL = 2e-6


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2003_10850_amd import ops
    return ops.Context(torch.device("cuda", 0))


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def fp64_params(p):
    return dataclasses.replace(p, flags=oracle.FLAG_FP64_DECISIONS)


class Case64:
    def __init__(self, ctx, w, shift=0.0):
        from paper_2003_10850_amd import ops
        self.w = w
        self.pos = w.pos + shift
        self.box = np.array(w.box, float)
        self.box[:3] += shift
        self.m32 = w.mass.astype(np.float32)
        self.M = self.m32.astype(np.float64)
        self.p = w.params
        self.pr = fp64_params(w.params)
        print(f"case64 {w.name} n={w.n} shift={shift}", flush=True)
        self.tree = ops.Tree(ctx, dev_t(self.pos), dev_t(self.m32), dev_t(w.type),
                             tuple(self.box), self.p)
        self.gas = np.nonzero(w.type == 0)[0]
        self.gt = oracle.Tree(self.pos, self.M, self.box, type=w.type, gas_only=True)
        self.at = oracle.Tree(self.pos, self.M, self.box, type=w.type)


def test_tree_from_fp64_positions_is_exact(ctx):
    w = inputs.plummer(n=30000, n_spheres=5, seed=21)
    c = Case64(ctx, w, shift=0.0)
    for which, t in ((0, c.at), (1, c.gt)):
        ref = t.export()
        got = {k: host(v) for k, v in c.tree.export(which).items()}
        np.testing.assert_array_equal(got["order"], ref["order"])
        for k in ("start", "count", "level", "skip"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        np.testing.assert_allclose(got["com"], ref["com"], rtol=1e-12, atol=1e-15)


def density64(c, active=None):
    """The FP64 h solve against the oracle's (h within HTOL, rho within TOL
    plus its change with the difference in h), then counts and sums at the
    oracle's solved h given to both sides. Returns that h and the largest
    relative error of rho there."""
    from paper_2003_10850_amd import ops
    act = c.gas if active is None else np.intersect1d(active, c.gas)
    a_t = None if active is None else dev_t(active.astype(np.int32))
    d = ops.density(c.tree, active=a_t)
    assert d["h"].dtype == torch.float64
    ref = oracle.density(c.gt, c.pr, active=act)
    check_solved_density(host(d["h"]), host(d["rho"]), ref, act, HTOL, TOL)
    assert c.tree.ctx.nonconverged(reset=True) == 0
    h = np.where(np.isin(np.arange(c.w.n), act), ref["h"], 1.0)
    dg = ops.density(c.tree, h=dev_t(h), active=a_t, solve_h=False)
    at = oracle.density(c.gt, c.pr, active=act, h=h, solve_h=False)
    np.testing.assert_array_equal(host(dg["nngb"])[act], at["nngb"][act])
    r = host(dg["rho"])[act]
    err = np.abs(r - at["rho"][act]) / at["rho"][act]
    assert err.max() < TOL, f"rho: max rel {err.max():.3e}"
    return h, err.max()


@pytest.mark.parametrize("shift", [0.0, 1000.0])
def test_density_mixed_precision(ctx, shift):
    w = inputs.plummer(n=40000, n_spheres=5, seed=22, n_ngb=64.0)
    density64(Case64(ctx, w, shift=shift))


def test_density_mixed_precision_active_subset(ctx):
    w = inputs.plummer(n=30000, n_spheres=4, seed=23, n_ngb=64.0)
    density64(Case64(ctx, w, shift=100.0), active=inputs.active_subset(w.n, 0.05, seed=7))


def test_plain_path_degrades_in_a_far_box(ctx):
    """The reason for the mixed-precision path: FP32 absolute positions of a
    box at 1000 lose ~5 digits of the separations the kernels need."""
    from paper_2003_10850_amd import ops
    w = inputs.plummer(n=30000, n_spheres=4, seed=24, n_ngb=64.0)
    c = Case64(ctx, w, shift=1000.0)
    h64, err64 = density64(c)
    # the plain path on the FP32 rounding of the same positions
    t32 = ops.Tree(c.tree.ctx, dev_t(c.pos.astype(np.float32)), dev_t(c.m32), dev_t(w.type),
                   tuple(c.box), c.p)
    d32 = ops.density(t32, h=dev_t(h64.astype(np.float32)), solve_h=False)
    at = oracle.density(c.gt, c.pr, active=c.gas, h=h64, solve_h=False)
    err32 = (np.abs(host(d32["rho"])[c.gas] - at["rho"][c.gas]) / at["rho"][c.gas]).max()
    print(f"far box: rho max rel err mixed {err64:.2e}, plain FP32 {err32:.2e}")
    assert err32 > 100 * err64


@pytest.mark.parametrize("shift", [0.0, 1000.0])
def test_hydro_and_gravity_mixed_precision(ctx, shift):
    from paper_2003_10850_amd import ops
    w = inputs.plummer(n=30000, n_spheres=4, seed=25)
    c = Case64(ctx, w, shift=shift)
    # hydro on the generating model's smooth fields, h in FP64
    h = inputs.model_smoothing(w)
    rho = inputs.model_gas_density(w).astype(np.float32)
    om = np.ones(w.n, np.float32)
    v32, u32 = w.vel.astype(np.float32), w.u.astype(np.float32)
    g = ops.hydro_force(c.tree, dev_t(v32), dev_t(u32), dev_t(h), dev_t(rho), dev_t(om))
    r = oracle.hydro(c.gt, c.pr, v32, u32, h, rho, om, active=c.gas)
    np.testing.assert_array_equal(host(g["npairs"])[c.gas], r["npairs"][c.gas])
    da = np.linalg.norm(host(g["acc"])[c.gas] - r["acc"][c.gas], axis=1)
    assert (da / r["S"][c.gas]).max() < TOL
    # gravity with FP64 opening decisions
    gr = ops.gravity(c.tree)
    rg = oracle.gravity(c.at, c.pr)
    np.testing.assert_array_equal(host(gr["nterms"]), rg["nterms"])
    dg = np.linalg.norm(host(gr["acc"]) - rg["acc"], axis=1)
    assert (dg / rg["S"]).max() < TOL
    np.testing.assert_allclose(host(gr["pot"]), rg["pot"], rtol=TOL)


def test_refit_after_drift_in_a_far_box(ctx):
    """An FP64 tree of a box at 1000, refit after particles drift by up to
    3e-3 of the box per axis (some leave the box), keeps exact neighbour
    and pair counts and the same bars: the offsets are taken from each
    group's FP64 centre, and the walk's rounding pad follows the largest
    coordinate found on the device at the refit."""
    from paper_2003_10850_amd import ops
    w = inputs.plummer(n=30000, n_spheres=4, seed=26, n_ngb=64.0)
    c = Case64(ctx, w, shift=1000.0)
    rng = np.random.default_rng(27)
    moved = c.pos + rng.uniform(-3e-3, 3e-3, c.pos.shape)
    c.tree.refit(dev_t(moved), dev_t(c.m32))
    # the oracle's trees only organise its direct definitions: give them a
    # box that holds the moved particles
    lo = moved.min(0) - 1e-3
    big = np.array([*lo, (moved.max(0) - lo).max() + 1e-3])
    gt = oracle.Tree(moved, c.M, big, type=w.type, gas_only=True)
    at = oracle.Tree(moved, c.M, big, type=w.type)
    h = inputs.model_smoothing(w)
    d = ops.density(c.tree, h=dev_t(h), solve_h=False)
    r = oracle.density(gt, c.pr, active=c.gas, h=h, solve_h=False)
    np.testing.assert_array_equal(host(d["nngb"])[c.gas], r["nngb"][c.gas])
    err = (np.abs(host(d["rho"])[c.gas] - r["rho"][c.gas]) / r["rho"][c.gas]).max()
    assert err < TOL, f"rho: max rel {err:.3e}"
    rho = inputs.model_gas_density(w).astype(np.float32)
    om = np.ones(w.n, np.float32)
    v32, u32 = w.vel.astype(np.float32), w.u.astype(np.float32)
    g = ops.hydro_force(c.tree, dev_t(v32), dev_t(u32), dev_t(h), dev_t(rho), dev_t(om))
    rh = oracle.hydro(gt, c.pr, v32, u32, h, rho, om, active=c.gas)
    np.testing.assert_array_equal(host(g["npairs"])[c.gas], rh["npairs"][c.gas])
    da = np.linalg.norm(host(g["acc"])[c.gas] - rh["acc"][c.gas], axis=1)
    assert (da / rh["S"][c.gas]).max() < TOL
    # gravity at theta = 0 (no decision depends on the refit cells)
    p0 = dataclasses.replace(c.p, theta=0.0)
    gr = ops.gravity(c.tree, params=p0)
    rg = oracle.gravity(at, fp64_params(p0))
    np.testing.assert_array_equal(host(gr["nterms"]), rg["nterms"])
    dg = np.linalg.norm(host(gr["acc"]) - rg["acc"], axis=1)
    assert (dg / rg["S"]).max() < TOL
    print(f"far-box refit: rho {err:.2e}, hydro {(da / rh['S'][c.gas]).max():.2e}, "
          f"gravity {(dg / rg['S']).max():.2e}", flush=True)


@pytest.mark.parametrize("shift", [0.0, 1000.0])
def test_walk_lists_on_fp64_trees(ctx, shift):
    """g3_walk on a tree of FP64 positions: every list is the FP64-decision
    list of the oracle, as exact sets (gather, symmetric, gravity; all
    targets and a sparse active subset)."""
    from paper_2003_10850_amd import ops, g3
    w = inputs.plummer(n=8000, n_spheres=3, seed=28, n_ngb=64.0)
    c = Case64(ctx, w, shift=shift)
    h = inputs.model_smoothing(w, 64.0)
    sub = inputs.active_subset(w.n, 0.1, seed=2)
    for kind, act in ((g3.G3_GATHER, None), (g3.G3_SYMMETRIC, None), (g3.G3_GRAVITY, None),
                      (g3.G3_SYMMETRIC, sub)):
        a_t = None if act is None else dev_t(act.astype(np.int32))
        off, lst, st = ops.walk(c.tree, kind, h=None if kind == g3.G3_GRAVITY else dev_t(h),
                                active=a_t)
        assert st == g3.G3_OK
        off, lst = host(off), host(lst)
        tgt = np.arange(w.n) if act is None else act
        t = c.at if kind == g3.G3_GRAVITY else c.gt
        roff, rl = oracle.lists(t, c.pr, kind, active=tgt,
                                h=None if kind == g3.G3_GRAVITY else h)
        np.testing.assert_array_equal(np.diff(off), np.diff(roff))
        for a in range(len(tgt)):
            assert np.array_equal(np.sort(lst[off[a]:off[a + 1]]), rl[roff[a]:roff[a + 1]]), \
                (kind, a)
        print(f"fp64 walk kind {kind} shift {shift}: {off[-1]} entries exact", flush=True)
