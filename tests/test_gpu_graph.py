"""A whole interaction step (h solve and density, hydro force, gravity) over
a forest with time-bin active sets, captured once in a HIP graph and
replayed: every replay must reproduce the eager step bit for bit, with
eager work and synchronisations between the replays.

The calls allocate nothing and never wait on the host once their scratch
has been sized by an eager call of the same shape, which is what capture
needs; the output rows of inactive particles are set before each step by
fill kernels inside the graph.
"""
import numpy as np
import pytest

from paper_2003_10850_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("fork", [False, True])
def test_captured_step_replays_match_eager(fork):
    """fork: gravity on a second stream, queued after the density and
    joined at the step's end (in the graph: a fork and a join)."""
    from paper_2003_10850_amd import ops
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = ops.Context(torch.device("cuda", 0))
    b = inputs.batch(n_snap=6, n_min=1e3, n_max=2e4, seed=5, n_ngb=64.0)
    print(f"graph step: forest n={b.n} snapshots={b.n_snap} active={b.active.size} "
          f"fork={fork}", flush=True)
    tree = ops.Tree(ctx, dev_t(b.pos.astype(np.float32)), dev_t(b.mass.astype(np.float32)),
                    dev_t(b.type), [tuple(x) for x in b.boxes], b.params, snap_off=b.snap_off)
    act = dev_t(b.active)
    vel = dev_t(b.vel.astype(np.float32))
    u = dev_t(b.u.astype(np.float32))
    n = b.n
    f32 = dict(dtype=torch.float32, device="cuda:0")
    bufs = dict(h=torch.zeros(n, **f32), rho=torch.zeros(n, **f32), omega=torch.zeros(n, **f32),
                drho_dh=torch.zeros(n, **f32), nngb=torch.zeros(n, dtype=torch.int32, device="cuda:0"),
                acc=torch.zeros(n, 3, **f32), dudt=torch.zeros(n, **f32), vsig=torch.zeros(n, **f32),
                npairs=torch.zeros(n, dtype=torch.int32, device="cuda:0"),
                gacc=torch.zeros(n, 3, **f32), pot=torch.zeros(n, **f32),
                nterms=torch.zeros(n, dtype=torch.int32, device="cuda:0"))
    # every particle's rho and omega are needed as neighbour inputs of the
    # hydro force: a first full density pass provides the inactive ones
    base = ops.density(tree)
    rho_all = base["rho"].clone()
    om_all = base["omega"].clone()
    h_all = base["h"].clone()

    side = torch.cuda.Stream()  # default priority

    def gravity():
        ops.gravity(tree, active=act, out={"acc": bufs["gacc"], "pot": bufs["pot"],
                                           "nterms": bufs["nterms"]})

    def step():
        main = torch.cuda.current_stream()
        for k in bufs:
            bufs[k].zero_()
        start = torch.cuda.Event()
        start.record(main)
        bufs["h"].copy_(h_all)
        ops.density(tree, active=act, out={k: bufs[k] for k in
                                           ("h", "rho", "drho_dh", "omega", "nngb")})
        if fork:
            side.wait_event(start)
            with torch.cuda.stream(side):
                gravity()
        rho = torch.where(bufs["rho"] > 0, bufs["rho"], rho_all)
        om = torch.where(bufs["omega"] > 0, bufs["omega"], om_all)
        ops.hydro_force(tree, vel, u, bufs["h"], rho, om, active=act,
                        out={k: bufs[k] for k in ("acc", "dudt", "vsig", "npairs")})
        if fork:
            main.wait_stream(side)
        else:
            gravity()

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()  # sizes every scratch buffer before capture
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in bufs.items()}
    assert int((eager["nngb"] > 0).sum()) > 0 and float(eager["pot"].abs().max()) > 0

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        # unrelated eager work on the same buffers between replays
        for v in bufs.values():
            v.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in bufs.items():
            assert torch.equal(v, eager[k]), f"replay {rep}: {k} differs from the eager step"
    ctx.nonconverged(reset=True)
