"""GPU tests of the launch tuning: the autotuner's choices (candidate tile
depth walk_leaf, group split level, fixed or per snapshot (-2), candidate
streams) may change only the order of FP32 partial sums, never a count or a
decision.

Every choice is run on a forest with time-bin (sparse, clustered) active
sets; neighbour, pair and term counts must equal those of the default
choice exactly and the sums agree to rounding; one split choice is also
checked against the oracle per snapshot.
"""
import numpy as np
import pytest

import oracle
from paper_2003_10850_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def setup():
    from paper_2003_10850_amd import ops
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = ops.Context(torch.device("cuda", 0))
    b = inputs.batch(n_snap=5, n_min=2e3, n_max=3e4, seed=9, n_ngb=64.0, shift_boxes=True)
    print(f"tuning forest n={b.n} snapshots={b.n_snap} active={b.active.size}", flush=True)
    tree = ops.Tree(ctx, dev_t(b.pos.astype(np.float32)), dev_t(b.mass.astype(np.float32)),
                    dev_t(b.type), [tuple(x) for x in b.boxes], b.params, snap_off=b.snap_off)
    h0 = np.zeros(b.n)
    for w, o0 in zip(b.snaps, b.snap_off[:-1]):
        m = dict(w.model)
        w2 = inputs.Workload(w.name, w.pos - w.box[:3], w.vel, w.mass, w.u, w.type,
                             np.array([0, 0, 0, 1.0]), w.params)
        m["centres"] = m["centres"] - w.box[:3]
        w2.model = m
        h0[o0:o0 + w.n] = inputs.model_smoothing(w2, 64.0)
    return ctx, b, tree, h0.astype(np.float32)


def run_step(ctx, b, tree, h0):
    from paper_2003_10850_amd import ops
    act = dev_t(b.active)
    d = ops.density(tree, h=dev_t(h0), active=act)
    rho = torch.where(d["rho"] > 0, d["rho"], torch.ones_like(d["rho"]))
    om = torch.where(d["omega"] > 0, d["omega"], torch.ones_like(d["omega"]))
    hy = ops.hydro_force(tree, dev_t(b.vel.astype(np.float32)), dev_t(b.u.astype(np.float32)),
                         dev_t(h0), rho, om, active=act)
    g = ops.gravity(tree, active=act)
    # the density also at the given (model) h, for the comparison with the
    # oracle at that same h
    dm = ops.density(tree, h=dev_t(h0), active=act, solve_h=False)
    torch.cuda.synchronize()
    ctx.nonconverged(reset=True)
    return {k: host(v) for k, v in dict(h=d["h"], rho=d["rho"], nngb=d["nngb"], acc=hy["acc"],
                                          npairs=hy["npairs"], gacc=g["acc"], pot=g["pot"],
                                          nterms=g["nterms"], rho_m=dm["rho"],
                                          nngb_m=dm["nngb"]).items()}


def set_all(ctx, leaf, split, streams=1):
    from paper_2003_10850_amd import g3
    for kind in (g3.G3_TUNE_DENSITY, g3.G3_TUNE_HYDRO, g3.G3_TUNE_GRAVITY):
        ctx.set_tuning(kind, leaf, split, streams=streams)


@pytest.mark.parametrize("leaf,split,streams", [(16, -1, 1), (128, -1, 1), (64, 2, 1),
                                                (32, 4, 1), (16, 6, 1), (64, -1, 4),
                                                (128, 3, 4), (16, -1, 4), (128, -2, 1),
                                                (64, -2, 4)])
def test_choices_change_no_count(setup, leaf, split, streams):
    ctx, b, tree, h0 = setup
    set_all(ctx, 64, -1)
    ref = run_step(ctx, b, tree, h0)
    set_all(ctx, leaf, split, streams)
    got = run_step(ctx, b, tree, h0)
    set_all(ctx, 64, -1)
    a = b.active
    gas = a[b.type[a] == 0]
    # h is solved to 1e-6: the solve may stop a step earlier or later
    assert (np.abs(got["h"][gas] - ref["h"][gas]) / ref["h"][gas]).max() < 2e-6
    for k in ("npairs", "nterms"):
        np.testing.assert_array_equal(got[k][a], ref[k][a], err_msg=k)
    np.testing.assert_allclose(got["pot"][a], ref["pot"][a], rtol=TOL)
    for k in ("acc", "gacc"):
        rows = gas if k == "acc" else a
        scale = np.abs(ref[k][rows]).max()
        assert np.abs(got[k][rows] - ref[k][rows]).max() <= 1e-4 * scale, k


@pytest.mark.parametrize("streams", [1, 4])
def test_split_groups_against_oracle(setup, streams):
    ctx, b, tree, h0 = setup
    set_all(ctx, 32, 3, streams)
    got = run_step(ctx, b, tree, h0)
    set_all(ctx, 64, -1)
    for k, w in enumerate(b.snaps):
        r0, r1 = int(b.snap_off[k]), int(b.snap_off[k + 1])
        a = b.active[(b.active >= r0) & (b.active < r1)] - r0
        P = b.pos[r0:r1].astype(np.float32).astype(np.float64)
        M = b.mass[r0:r1].astype(np.float32).astype(np.float64)
        at = oracle.Tree(P, M, b.boxes[k], type=w.type)
        rg = oracle.gravity(at, b.params, active=a)
        np.testing.assert_array_equal(got["nterms"][a + r0], rg["nterms"][a])
        dg = np.linalg.norm(got["gacc"][a + r0] - rg["acc"][a], axis=1)
        S = rg["S"][a]
        assert (dg[S > 0] / S[S > 0]).max(initial=0) < TOL
        ag = a[w.type[a] == 0]
        gt = oracle.Tree(P, M, b.boxes[k], type=w.type, gas_only=True)
        d = oracle.density(gt, b.params, active=ag, h=h0[r0:r1].astype(np.float64),
                           solve_h=False)
        np.testing.assert_array_equal(got["nngb_m"][ag + r0], d["nngb"][ag])
        assert (np.abs(got["rho_m"][ag + r0] - d["rho"][ag]) / d["rho"][ag]).max() < TOL


def test_autotune_picks_candidates(setup):
    from paper_2003_10850_amd import g3
    ctx, b, tree, h0 = setup
    set_all(ctx, 64, -1)
    ref = run_step(ctx, b, tree, h0)
    before = ctx.stats()
    ctx.autotune(tree, dev_t(h0), active=dev_t(b.active))
    assert ctx.stats() == before  # the tuning runs leave the statistics alone
    n = b.active.size
    leaf, split, streams = ctx.tuning(g3.G3_TUNE_DENSITY, n)
    assert leaf in (16, 32, 64, 128) and split in (-1, -2, 2, 3, 4, 5) and streams in (1, 4)
    _, gsplit, _ = ctx.tuning(g3.G3_TUNE_GRAVITY, n)
    assert gsplit in (-1, -2, 2, 3, 4, 5)
    print(f"autotuned: density leaf {leaf} split {split}, gravity split {gsplit}")
    got = run_step(ctx, b, tree, h0)
    a = b.active
    np.testing.assert_array_equal(got["nterms"][a], ref["nterms"][a])
    set_all(ctx, 64, -1)


def test_tuning_file_round_trip(setup, tmp_path):
    from paper_2003_10850_amd import g3, ops
    ctx, b, tree, h0 = setup
    ctx.set_tuning(g3.G3_TUNE_DENSITY, 32, 3, n_targets=5000, streams=4)
    ctx.set_tuning(g3.G3_TUNE_HYDRO, 16, -2, n_targets=70000)
    ctx.set_tuning(g3.G3_TUNE_GRAVITY, 64, 5, n_targets=300)
    path = str(tmp_path / "tuning.txt")
    ctx.save_tuning(path)
    fresh = ops.Context(torch.device("cuda", 0))
    fresh.load_tuning(path)
    for kind, n in ((g3.G3_TUNE_DENSITY, 5000), (g3.G3_TUNE_HYDRO, 70000),
                    (g3.G3_TUNE_GRAVITY, 300), (g3.G3_TUNE_DENSITY, 70000)):
        assert fresh.tuning(kind, n) == ctx.tuning(kind, n)
    # a malformed file is refused and leaves the choices as they were
    bad = tmp_path / "bad.txt"
    bad.write_text("g3-tuning 1\n0 12 64 99 1\n")
    with pytest.raises(g3.G3Error):
        fresh.load_tuning(str(bad))
    assert fresh.tuning(g3.G3_TUNE_DENSITY, 5000) == (32, 3, 4)
    set_all(ctx, 64, -1)
