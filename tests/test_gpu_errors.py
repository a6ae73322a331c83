"""The boundary's error contract on the GPU, observed through the C ABI.

- G3_ENOCONV: g3_density never waits on the host; g3_ctx_stats reports
  solves that did not converge, both for a target no h below the bracket
  cap can reach (fewer gas particles than the target neighbour number can
  give: the oracle reports the same particles) and for a pass limit forced
  from the host (G3_INJECT_MAX_ITER).
- G3_ENOMEM: with allocation failures forced from the host
  (G3_INJECT_ALLOC), every interaction call returns G3_ENOMEM, leaves its
  outputs untouched and its stream idle, and works again once the injection
  is off; a build that fails leaves its tree unusable (G3_ESTATE) until it
  is rebuilt.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2003_10850_amd import g3, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def stream():
    return torch.cuda.current_stream().cuda_stream


def status_name(st):
    return g3.STATUS_NAMES.get(st, st)


class Raw:
    """A ctx and a tree driven through the raw C entry points."""

    def __init__(self, w):
        self.L = g3.lib()
        self.ctx = g3.g3_ctx_create(0)
        self.w = w
        self.p = g3.g3_params.of(w.params)
        pos32, vel32, m32, u32 = w.as_f32()
        self.pos, self.mass, self.type = dev_t(pos32), dev_t(m32), dev_t(w.type)
        self.vel, self.u = dev_t(vel32), dev_t(u32)
        self.tree = ctypes.c_void_p()

    def build(self):
        box = (ctypes.c_double * 4)(*[float(x) for x in self.w.box])
        return self.L.g3_build_tree(self.ctx, self.w.n, g3.G3_F32, self.pos.data_ptr(),
                                    self.mass.data_ptr(), self.type.data_ptr(), box,
                                    ctypes.byref(self.p), ctypes.byref(self.tree), stream())

    def density(self, h, rho, nngb, active=None, solve=1):
        na = self.w.n if active is None else int(active.shape[0])
        ap = None if active is None else active.data_ptr()
        return self.L.g3_density(self.ctx, self.tree, na, ap, ctypes.byref(self.p), solve,
                                 h.data_ptr(), rho.data_ptr(), None, None, nngb.data_ptr(),
                                 stream())

    def stats(self, reset=1):
        c = (ctypes.c_int64 * 4)()
        st = self.L.g3_ctx_stats(self.ctx, c, reset)
        return st, [int(x) for x in c]

    def close(self):
        g3.g3_ctx_destroy(self.ctx)


def test_enoconv_when_no_root_below_the_cap():
    """Three equal-mass gas particles give N_eff(h) = (1365/48) sum_j w(q_j),
    which stays below 3 x 1365/48 = 85.3 at every h; with n_ngb = 90 every
    solve runs into the bracket cap."""
    import dataclasses
    w = inputs.uniform(n=3, seed=5)
    w = dataclasses.replace(w, params=dataclasses.replace(w.params, n_ngb=90.0))
    r = Raw(w)
    try:
        assert r.build() == g3.G3_OK
        assert r.stats()[0] == g3.G3_OK
        h = torch.zeros(w.n, dtype=torch.float32, device=DEV)
        rho = torch.zeros(w.n, dtype=torch.float32, device=DEV)
        nn = torch.zeros(w.n, dtype=torch.int32, device=DEV)
        assert r.density(h, rho, nn) == g3.G3_OK  # no host wait: reported later
        st, s = r.stats()
        print(f"stats {status_name(st)} {s}", flush=True)
        assert st == g3.G3_ENOCONV and s[0] == 3
        # the oracle reports the same particles
        t = oracle.Tree(w.pos.astype(np.float32).astype(np.float64), w.mass, w.box,
                        gas_only=True)
        d = oracle.density(t, w.params)
        assert d["status"] == oracle.ENOCONV and d["nonconv"] == 3
        # h stayed at or below the cap of twice the box diagonal
        assert float(h.max()) <= 2 * np.sqrt(3) * w.box[3] * (1 + 1e-6)
        # the counter was reset by the read
        assert r.stats() == (g3.G3_OK, [0, 0, 0, 0])
    finally:
        r.close()


def test_enoconv_from_a_forced_pass_limit():
    w = inputs.uniform(n=4096, seed=0)
    r = Raw(w)
    try:
        assert r.build() == g3.G3_OK
        h = torch.zeros(w.n, dtype=torch.float32, device=DEV)
        rho = torch.zeros(w.n, dtype=torch.float32, device=DEV)
        nn = torch.zeros(w.n, dtype=torch.int32, device=DEV)
        assert r.L.g3_ctx_inject(r.ctx, g3.G3_INJECT_MAX_ITER, 1) == g3.G3_OK
        assert r.density(h, rho, nn) == g3.G3_OK
        st, s = r.stats()
        print(f"pass limit 1: {status_name(st)} {s}", flush=True)
        # one pass from a cold start converges nowhere (the first guess is
        # never within the tolerance of the root on random points)
        assert st == g3.G3_ENOCONV and s[0] == w.n
        assert s[1] == s[2]  # one pass per wave
        assert r.L.g3_ctx_inject(r.ctx, g3.G3_INJECT_MAX_ITER, 0) == g3.G3_OK
        h.zero_()
        assert r.density(h, rho, nn) == g3.G3_OK
        st, s = r.stats()
        assert st == g3.G3_OK and s[0] == 0
        # a pass limit beyond the kernel's own is rejected
        assert r.L.g3_ctx_inject(r.ctx, g3.G3_INJECT_MAX_ITER, 65) == g3.G3_EINVAL
    finally:
        r.close()


def sentinel(shape, dtype=torch.float32):
    return torch.full(shape, -7, dtype=dtype, device=DEV)


def test_enomem_leaves_nothing_enqueued_and_recovers():
    w = inputs.plummer(n=6000, n_spheres=3, seed=9, n_ngb=64.0, eps=1e-3)
    r = Raw(w)
    try:
        assert r.build() == g3.G3_OK
        torch.cuda.synchronize()
        n = w.n
        act = torch.arange(0, n, 3, dtype=torch.int32, device=DEV)
        h = sentinel((n,))
        rho, nn = sentinel((n,)), sentinel((n,), torch.int32)
        acc, pot, nt = sentinel((n, 3)), sentinel((n,)), sentinel((n,), torch.int32)
        model_h = dev_t(inputs.model_smoothing(w, 64.0).astype(np.float32))
        ones = torch.ones(n, dtype=torch.float32, device=DEV)
        hacc, du, vs, npair = sentinel((n, 3)), sentinel((n,)), sentinel((n,)), \
            sentinel((n,), torch.int32)
        off = sentinel((int(act.shape[0]) + 1,), torch.int64)
        lst = sentinel((1 << 23,), torch.int32)  # room for every gravity list entry
        total = ctypes.c_int64(-1)
        P = ctypes.byref(r.p)
        calls = {
            "g3_density": lambda: r.density(h, rho, nn, active=act),
            "g3_gravity": lambda: r.L.g3_gravity(r.ctx, r.tree, int(act.shape[0]), act.data_ptr(),
                                                 P, acc.data_ptr(), pot.data_ptr(),
                                                 nt.data_ptr(), stream()),
            "g3_hydro_force": lambda: r.L.g3_hydro_force(
                r.ctx, r.tree, int(act.shape[0]), act.data_ptr(), P, r.vel.data_ptr(),
                r.u.data_ptr(), model_h.data_ptr(), ones.data_ptr(), ones.data_ptr(),
                hacc.data_ptr(), du.data_ptr(), vs.data_ptr(), npair.data_ptr(), stream()),
            "g3_walk": lambda: r.L.g3_walk(r.ctx, r.tree, g3.G3_GRAVITY, int(act.shape[0]),
                                           act.data_ptr(), None, P, int(lst.shape[0]),
                                           off.data_ptr(), lst.data_ptr(),
                                           ctypes.byref(total), stream()),
        }
        outs = [h, rho, nn, acc, pot, nt, hacc, du, vs, npair, off, lst]
        torch.cuda.synchronize()  # the sentinel fills are done before the calls
        # a fresh ctx owns no scratch yet: each call's first allocation fails
        assert r.L.g3_ctx_inject(r.ctx, g3.G3_INJECT_ALLOC, 0) == g3.G3_OK
        for name, call in calls.items():
            print(f"injected allocation failure: {name}", flush=True)
            st = call()
            assert st == g3.G3_ENOMEM, (name, status_name(st))
            # nothing enqueued: the stream is idle at once, outputs untouched
            assert torch.cuda.current_stream().query(), name
            assert "alloc" in g3.g3_last_error(r.ctx), g3.g3_last_error(r.ctx)
        torch.cuda.synchronize()
        for t in outs:
            assert bool((t == -7).all()), "an output was written by a failed call"
        # the injection off: every call works on the same ctx
        assert r.L.g3_ctx_inject(r.ctx, g3.G3_INJECT_ALLOC, -1) == g3.G3_OK
        for name, call in calls.items():
            assert call() == g3.G3_OK, (name, g3.g3_last_error(r.ctx))
        torch.cuda.synchronize()
        a = act.cpu().numpy()
        assert int(nt[act.long()].min()) > 0 and int(total.value) > 0
        gas_act = torch.from_numpy(a[w.type[a] == 0]).long().to(DEV)
        assert float(rho[gas_act].min()) > 0
    finally:
        r.close()


@pytest.mark.parametrize("budget", [0, 3, 9])
def test_failed_build_leaves_an_unusable_tree_until_rebuilt(budget):
    w = inputs.plummer(n=5000, n_spheres=2, seed=3, n_ngb=64.0, eps=1e-3)
    r = Raw(w)
    try:
        assert r.L.g3_ctx_inject(r.ctx, g3.G3_INJECT_ALLOC, budget) == g3.G3_OK
        st = r.build()
        print(f"build with {budget} allocations: {status_name(st)}", flush=True)
        assert st == g3.G3_ENOMEM
        assert torch.cuda.current_stream().query()
        assert r.tree.value, "the handle of the new tree is returned"
        h = torch.zeros(w.n, dtype=torch.float32, device=DEV)
        rho = torch.zeros(w.n, dtype=torch.float32, device=DEV)
        nn = torch.zeros(w.n, dtype=torch.int32, device=DEV)
        assert r.L.g3_ctx_inject(r.ctx, g3.G3_INJECT_ALLOC, -1) == g3.G3_OK
        assert r.density(h, rho, nn) == g3.G3_ESTATE
        assert r.build() == g3.G3_OK
        assert r.density(h, rho, nn) == g3.G3_OK
        torch.cuda.synchronize()
        gas = np.nonzero(w.type == 0)[0]
        assert float(rho[torch.from_numpy(gas).to(DEV)].min()) > 0
    finally:
        r.close()
