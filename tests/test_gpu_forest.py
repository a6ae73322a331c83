"""GPU parity of forests (many snapshots in one tree object, served by one
persistent launch per kernel) against the FP64 oracle run on each snapshot
alone.

A forest must give every snapshot exactly what a tree built for it alone
gives: the same octree (offset by the earlier snapshots), the same
neighbour and interaction counts and lists, and densities, h, forces and
potentials within the single-tree bars. The snapshots here cover the edge
cases of the forest layout: an empty snapshot, a one-particle snapshot, a
snapshot without gas, boxes at different places, and active sets from a
single particle to all of them.
"""
import numpy as np
import pytest

import oracle
from parity_util import check_solved_density
from paper_2003_10850_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2003_10850_amd import ops
    return ops.Context(torch.device("cuda", 0))


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def small_forest(seed=31, n_ngb=40.0, fp64=False):
    """Seven snapshots with the layout's edge cases, boxes along x."""
    sizes = [3000, 0, 1, 700, 12000, 257, 5000]
    snaps = []
    for k, n in enumerate(sizes):
        if n == 0:
            w = inputs.uniform(n=0, seed=1)
        elif n < 10:
            w = inputs.uniform(n=n, seed=k)
        else:
            w = inputs.plummer(n=n, n_spheres=3, seed=seed + k, n_ngb=n_ngb)
        if k == 5:
            w.type[:] = inputs.COLLISIONLESS  # a snapshot without gas
        # snapshot k in a box of side 1 + k/4 at x = 10 k (positions scaled)
        side = 1.0 + 0.25 * k
        w.pos = w.pos * side + np.array([10.0 * k, 0.0, 0.0])
        w.box = np.array([10.0 * k, 0.0, 0.0, side])
        snaps.append(w)
    off = np.concatenate([[0], np.cumsum([w.n for w in snaps])]).astype(np.int64)
    cat = lambda f: np.concatenate([getattr(w, f) for w in snaps])
    F = dict(snaps=snaps, off=off, pos=cat("pos"), vel=cat("vel"), mass=cat("mass"),
             u=cat("u"), type=cat("type"), boxes=np.array([w.box for w in snaps]),
             params=inputs.Params(n_ngb=n_ngb, eps=1e-3))
    F["pos_in"] = F["pos"] if fp64 else F["pos"].astype(np.float32)
    F["P"] = F["pos_in"].astype(np.float64)
    F["m32"] = F["mass"].astype(np.float32)
    return F


class Forest:
    def __init__(self, ctx, F):
        from paper_2003_10850_amd import ops
        self.F = F
        print(f"forest n={len(F['pos'])} snapshots={len(F['snaps'])}", flush=True)
        self.tree = ops.Tree(ctx, dev_t(F["pos_in"]), dev_t(F["m32"]), dev_t(F["type"]),
                             [tuple(b) for b in F["boxes"]], F["params"], snap_off=F["off"])
        self._ot = {}

    def snap_rows(self, k):
        return np.arange(self.F["off"][k], self.F["off"][k + 1])

    def otree(self, k, gas_only):
        key = (k, gas_only)
        if key not in self._ot:
            r = self.snap_rows(k)
            self._ot[key] = oracle.Tree(self.F["P"][r], self.F["m32"][r].astype(np.float64),
                                        self.F["boxes"][k], type=self.F["type"][r],
                                        gas_only=gas_only)
        return self._ot[key]


def test_forest_octrees_are_the_snapshots_octrees(ctx):
    fo = Forest(ctx, small_forest())
    F = fo.F
    for which in (0, 1):
        got = {k: host(v) for k, v in fo.tree.export(which).items()}
        m0 = 0  # sorted members of the earlier snapshots
        n0 = 0  # nodes of the earlier snapshots
        for k in range(len(F["snaps"])):
            if F["snaps"][k].n == 0:
                continue
            ref = fo.otree(k, bool(which)).export()
            m, nn = len(ref["order"]), len(ref["start"])
            np.testing.assert_array_equal(got["order"][m0:m0 + m] - F["off"][k], ref["order"])
            np.testing.assert_array_equal(got["keys"][m0:m0 + m].view(np.uint64), ref["keys"])
            sl = slice(n0, n0 + nn)
            np.testing.assert_array_equal(got["start"][sl] - m0, ref["start"])
            np.testing.assert_array_equal(got["skip"][sl] - n0, ref["skip"])
            for f in ("count", "level"):
                np.testing.assert_array_equal(got[f][sl], ref[f], err_msg=f"{f} snapshot {k}")
            np.testing.assert_allclose(got["mass"][sl], ref["mass"], rtol=1e-12)
            np.testing.assert_allclose(got["com"][sl], ref["com"], rtol=1e-12, atol=1e-12)
            m0 += m
            n0 += nn
        assert m0 == len(got["order"]) and n0 == len(got["start"])


def forest_active(F, seed):
    """Per snapshot: everything, a ragged subset, or a single particle."""
    rng = np.random.default_rng(seed)
    act = []
    for k, w in enumerate(F["snaps"]):
        if w.n == 0:
            continue
        mode = k % 3
        if mode == 0:
            a = np.arange(w.n)
        elif mode == 1:
            a = inputs.active_subset(w.n, 0.13, seed=seed + k)
        else:
            a = rng.choice(w.n, size=1)
        act.append(a + F["off"][k])
    return np.sort(np.concatenate(act)).astype(np.int32)


def test_forest_density_solve(ctx):
    from paper_2003_10850_amd import ops
    F = small_forest()
    fo = Forest(ctx, F)
    act = forest_active(F, 5)
    d = ops.density(fo.tree, active=dev_t(act))
    h, rho = host(d["h"]).astype(np.float64), host(d["rho"])
    nonconv = 0
    # the oracle's solved h (FP32-rounded) is then given to both sides for
    # exact counts and sums at one h
    hg = np.ones(len(F["type"]), np.float32)
    checked = []
    for k, w in enumerate(F["snaps"]):
        r = fo.snap_rows(k)
        a = np.intersect1d(act, r[F["type"][r] == 0]) - F["off"][k]
        if a.size == 0:
            continue
        gt = fo.otree(k, True)
        ngas = int((F["type"][r] == 0).sum())
        if ngas * 1365.0 / 48.0 < F["params"].n_ngb * 1.5:
            nonconv += a.size  # too few gas particles for any root
            continue
        ref = oracle.density(gt, F["params"], active=a)
        check_solved_density(h[r], rho[r], ref, a, TOL, TOL, f"snapshot {k}")
        hg[a + F["off"][k]] = ref["h"][a].astype(np.float32)
        checked.append((k, a, gt))
    assert fo.tree.ctx.nonconverged(reset=True) == nonconv
    dg = ops.density(fo.tree, h=dev_t(hg), active=dev_t(act), solve_h=False)
    fo.tree.ctx.nonconverged(reset=True)
    for k, a, gt in checked:
        r = fo.snap_rows(k)
        at = oracle.density(gt, F["params"], active=a, h=hg[r].astype(np.float64), solve_h=False)
        np.testing.assert_array_equal(host(dg["nngb"])[a + F["off"][k]], at["nngb"][a])
        err = np.abs(host(dg["rho"])[a + F["off"][k]] - at["rho"][a]) / at["rho"][a]
        assert err.max() < TOL, f"snapshot {k}: rho {err.max():.3e}"


def test_forest_hydro_and_gravity(ctx):
    from paper_2003_10850_amd import ops
    F = small_forest(seed=41)
    fo = Forest(ctx, F)
    act = forest_active(F, 9)
    # smooth synthetic SPH fields per snapshot (the generating model's)
    h = np.zeros(len(F["pos"]))
    rho = np.ones(len(F["pos"]))
    for k, w in enumerate(F["snaps"]):
        if w.n == 0:
            continue
        r = fo.snap_rows(k)
        if getattr(w, "model", None) is not None:
            side = F["boxes"][k][3]
            w2 = inputs.Workload(w.name, (w.pos - F["boxes"][k][:3]) / side, w.vel, w.mass, w.u,
                                 w.type, np.array([0, 0, 0, 1.0]), w.params)
            w2.model = w.model
            h[r] = inputs.model_smoothing(w2, 40.0) * side
            rho[r] = inputs.model_gas_density(w2) / side ** 3
        else:
            h[r] = 0.5 * F["boxes"][k][3]
    h32, rho32 = h.astype(np.float32), rho.astype(np.float32)
    om = np.ones(len(h), np.float32)
    v32, u32 = F["vel"].astype(np.float32), F["u"].astype(np.float32)
    g = ops.hydro_force(fo.tree, dev_t(v32), dev_t(u32), dev_t(h32), dev_t(rho32), dev_t(om),
                        active=dev_t(act))
    gr = ops.gravity(fo.tree, active=dev_t(act))
    for k, w in enumerate(F["snaps"]):
        r = fo.snap_rows(k)
        a_all = np.intersect1d(act, r) - F["off"][k]
        if a_all.size == 0:
            continue
        a_gas = np.intersect1d(act, r[F["type"][r] == 0]) - F["off"][k]
        if a_gas.size:
            ref = oracle.hydro(fo.otree(k, True), F["params"], v32[r], u32[r],
                               h32[r].astype(np.float64), rho32[r].astype(np.float64),
                               om[r].astype(np.float64), active=a_gas)
            rows = a_gas + F["off"][k]
            np.testing.assert_array_equal(host(g["npairs"])[rows], ref["npairs"][a_gas])
            da = np.linalg.norm(host(g["acc"])[rows] - ref["acc"][a_gas], axis=1)
            S = ref["S"][a_gas]
            assert np.all(da[S == 0] == 0)
            assert (da[S > 0] / S[S > 0]).max(initial=0) < TOL, f"snapshot {k} hydro"
        rg = oracle.gravity(fo.otree(k, False), F["params"], active=a_all)
        rows = a_all + F["off"][k]
        np.testing.assert_array_equal(host(gr["nterms"])[rows], rg["nterms"][a_all])
        dg = np.linalg.norm(host(gr["acc"])[rows] - rg["acc"][a_all], axis=1)
        S = rg["S"][a_all]
        assert np.all(dg[S == 0] == 0)
        assert (dg[S > 0] / S[S > 0]).max(initial=0) < TOL, f"snapshot {k} gravity"
    # rows that are not active keep what was there
    idle = np.setdiff1d(np.arange(len(h)), act)
    assert np.all(host(gr["acc"])[idle] == 0)


def test_forest_equals_separate_trees(ctx):
    """Every snapshot of a forest gets bit-identical results to a tree built
    for it alone: the same groups, walks and tiles."""
    from paper_2003_10850_amd import ops
    F = small_forest(seed=51)
    fo = Forest(ctx, F)
    d = ops.density(fo.tree)
    gr = ops.gravity(fo.tree)
    for k, w in enumerate(F["snaps"]):
        r = fo.snap_rows(k)
        if w.n == 0:
            continue
        t = ops.Tree(fo.tree.ctx, dev_t(F["pos_in"][r]), dev_t(F["m32"][r]), dev_t(F["type"][r]),
                     tuple(F["boxes"][k]), F["params"])
        ds = ops.density(t)
        gs = ops.gravity(t)
        gas = F["type"][r] == 0
        for f in ("h", "rho", "nngb", "omega"):
            np.testing.assert_array_equal(host(d[f])[r][gas], host(ds[f])[gas], err_msg=f)
        for f in ("acc", "pot", "nterms"):
            np.testing.assert_array_equal(host(gr[f])[r], host(gs[f]), err_msg=f)
        t.close()
    fo.tree.ctx.nonconverged(reset=True)


def test_forest_walk_lists(ctx):
    from paper_2003_10850_amd import ops, g3
    F = small_forest(seed=61)
    fo = Forest(ctx, F)
    act = forest_active(F, 3)
    h = np.zeros(len(F["pos"]))
    for k, w in enumerate(F["snaps"]):
        h[fo.snap_rows(k)] = 0.06 * F["boxes"][k][3]
    h32 = h.astype(np.float32)
    node0 = {}  # first node of each snapshot in the forest's all-particle octree
    st = host(fo.tree.export(0)["start"])
    m0 = 0
    for k, w in enumerate(F["snaps"]):
        node0[k] = int(np.searchsorted(st, m0))
        m0 += w.n
    for kind in (g3.G3_GATHER, g3.G3_SYMMETRIC, g3.G3_GRAVITY):
        off, lst, s = ops.walk(fo.tree, kind, h=dev_t(h32), active=dev_t(act))
        assert s == g3.G3_OK
        off, lst = host(off), host(lst)
        for k, w in enumerate(F["snaps"]):
            r = fo.snap_rows(k)
            sel = np.nonzero((act >= r[0]) & (act <= r[-1]))[0] if w.n else []
            if len(sel) == 0:
                continue
            a = act[sel] - F["off"][k]
            ot = fo.otree(k, kind != g3.G3_GRAVITY)
            roff, rl = oracle.lists(ot, F["params"], kind, active=a,
                                    h=None if kind == g3.G3_GRAVITY else h32[r].astype(np.float64))
            np.testing.assert_array_equal(off[sel + 1] - off[sel], np.diff(roff))
            for i, row in enumerate(sel):
                got = lst[off[row]:off[row + 1]].astype(np.int64)
                got = np.where(got >= 0, got - F["off"][k], got + node0[k])
                assert np.array_equal(np.sort(got), rl[roff[i]:roff[i + 1]]), (kind, k, i)


def test_forest_mixed_precision_density(ctx):
    from paper_2003_10850_amd import ops
    import dataclasses
    F = small_forest(seed=71, fp64=True)
    fo = Forest(ctx, F)
    d = ops.density(fo.tree)
    assert d["h"].dtype == torch.float64
    h, rho = host(d["h"]), host(d["rho"])
    pr = dataclasses.replace(F["params"], flags=oracle.FLAG_FP64_DECISIONS)
    hg = np.ones(len(F["type"]))  # the oracle's solved h, given to both sides
    checked = []
    for k, w in enumerate(F["snaps"]):
        r = fo.snap_rows(k)
        ng = int((F["type"][r] == 0).sum())
        if ng * 1365.0 / 48.0 < F["params"].n_ngb * 1.5:
            continue
        a = np.nonzero(F["type"][r] == 0)[0]
        gt = fo.otree(k, True)
        ref = oracle.density(gt, pr, active=a)
        check_solved_density(h[r], rho[r], ref, a, 2e-6, 1e-5, f"snapshot {k}")
        hg[a + F["off"][k]] = ref["h"][a]
        checked.append((k, a, gt))
    fo.tree.ctx.nonconverged(reset=True)
    dg = ops.density(fo.tree, h=dev_t(hg), solve_h=False)
    fo.tree.ctx.nonconverged(reset=True)
    for k, a, gt in checked:
        r = fo.snap_rows(k)
        at = oracle.density(gt, pr, active=a, h=hg[r], solve_h=False)
        np.testing.assert_array_equal(host(dg["nngb"])[r][a], at["nngb"][a])
        err = np.abs(host(dg["rho"])[r][a] - at["rho"][a]) / at["rho"][a]
        assert err.max() < 1e-5, f"snapshot {k}: rho {err.max():.3e}"


def test_forest_argument_checks(ctx):
    from paper_2003_10850_amd import ops, g3
    F = small_forest()
    x, m = dev_t(F["pos_in"]), dev_t(F["m32"])
    boxes = [tuple(b) for b in F["boxes"]]
    bad_off = F["off"].copy()
    bad_off[2], bad_off[3] = bad_off[3], bad_off[2] - 1  # decreasing
    with pytest.raises((g3.G3Error, ValueError)):
        ops.Tree(ctx, x, m, None, boxes, F["params"], snap_off=bad_off)
    bad_box = [list(b) for b in boxes]
    bad_box[3][3] = 0.0
    with pytest.raises(g3.G3Error) as e:
        ops.Tree(ctx, x, m, None, bad_box, F["params"], snap_off=F["off"])
    assert e.value.status == g3.G3_EINVAL
