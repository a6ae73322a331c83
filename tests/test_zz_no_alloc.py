"""g3_gravity_noalloc, the allocation-free twin of g3_gravity, through the C
ABI: on the same tree and active set it gives g3_gravity's outputs exactly
(same kernels, same work tables, same order of every sum), on two calls in
a row whose second is smaller than the first (the region keeps the first
call's contents, which the second must not read), with and without an
active list; a call whose work tables exceed the region is refused with
G3_EINVAL, enqueues nothing and leaves its outputs untouched."""
import ctypes

import numpy as np
import pytest

from paper_2003_10850_amd import g3, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def stream():
    return torch.cuda.current_stream().cuda_stream


class Snapshot:
    def __init__(self, L, ctx, w):
        self.L, self.ctx, self.w = L, ctx, w
        self.p = g3.g3_params.of(w.params)
        pos32, _, m32, _ = w.as_f32()
        self.pos, self.mass, self.type = dev_t(pos32), dev_t(m32), dev_t(w.type)
        self.tree = ctypes.c_void_p()
        box = (ctypes.c_double * 4)(*[float(x) for x in w.box])
        st = L.g3_build_tree(ctx, w.n, g3.G3_F32, self.pos.data_ptr(), self.mass.data_ptr(),
                             self.type.data_ptr(), box, ctypes.byref(self.p),
                             ctypes.byref(self.tree), stream())
        assert st == g3.G3_OK, g3.g3_last_error(ctx)

    def gravity(self, fn, active):
        n = self.w.n
        acc = torch.full((n, 3), -7.0, dtype=torch.float32, device=DEV)
        pot = torch.full((n,), -7.0, dtype=torch.float32, device=DEV)
        nt = torch.full((n,), -7, dtype=torch.int32, device=DEV)
        torch.cuda.synchronize()  # the fills are done: the call's own work is all that follows
        na = n if active is None else int(active.shape[0])
        ap = None if active is None else active.data_ptr()
        st = getattr(self.L, fn)(self.ctx, self.tree, na, ap, ctypes.byref(self.p),
                                 acc.data_ptr(), pot.data_ptr(), nt.data_ptr(), stream())
        return st, acc, pot, nt


def same(a, b):
    """Bitwise equal float tensors (the same kernels sum in the same order)."""
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def check_pair(snap, active, label):
    print(f"no-alloc gravity: {label} n={snap.w.n} "
          f"n_act={'all' if active is None else int(active.shape[0])}", flush=True)
    st0, acc0, pot0, nt0 = snap.gravity("g3_gravity", active)
    assert st0 == g3.G3_OK, g3.g3_last_error(snap.ctx)
    st1, acc1, pot1, nt1 = snap.gravity("g3_gravity_noalloc", active)
    assert st1 == g3.G3_OK, g3.g3_last_error(snap.ctx)
    torch.cuda.synchronize()
    assert torch.equal(nt0, nt1)
    assert same(acc0, acc1) and same(pot0, pot1)
    if active is not None:
        # rows outside the active set are untouched, active rows written
        mask = torch.zeros(snap.w.n, dtype=torch.bool, device=DEV)
        mask[active.long()] = True
        assert bool((nt1[~mask] == -7).all()) and bool((nt1[mask] > 0).all())
    else:
        assert bool((nt1 > 0).all())


def test_noalloc_gravity_matches_gravity_on_two_calls_the_second_smaller():
    L = g3.lib()
    ctx = g3.g3_ctx_create(0)
    try:
        big = Snapshot(L, ctx, inputs.plummer(n=200_000, n_spheres=8, seed=21, n_ngb=64.0,
                                              eps=1e-3))
        small = Snapshot(L, ctx, inputs.plummer(n=7_001, n_spheres=2, seed=22, n_ngb=64.0,
                                                eps=1e-3))
        act_big = dev_t(inputs.active_subset(big.w.n, 0.3, seed=4).astype(np.int32))
        act_small = dev_t(inputs.active_subset(small.w.n, 0.05, seed=5).astype(np.int32))
        # an active list, then a smaller one; every particle, then fewer
        check_pair(big, act_big, "active list")
        check_pair(small, act_small, "smaller active list")
        check_pair(big, None, "every particle")
        check_pair(small, None, "fewer particles")
        # an empty active list (a valid pointer, n_act = 0) writes nothing
        one = torch.zeros(1, dtype=torch.int32, device=DEV)
        nt = torch.full((small.w.n,), -7, dtype=torch.int32, device=DEV)
        st = L.g3_gravity_noalloc(ctx, small.tree, 0, one.data_ptr(), ctypes.byref(small.p),
                                  None, None, nt.data_ptr(), stream())
        assert st == g3.G3_OK, g3.g3_last_error(ctx)
        torch.cuda.synchronize()
        assert bool((nt == -7).all())
    finally:
        g3.g3_ctx_destroy(ctx)


def test_noalloc_gravity_refuses_tables_beyond_its_region():
    """An active list over a 2^22-member octree needs about 20 bytes per
    member of work tables (mark, scan, row and target arrays), 84 MB, more
    than the 64 MiB region: G3_EINVAL before any launch; the same tree with
    every particle active fits."""
    L = g3.lib()
    ctx = g3.g3_ctx_create(0)
    try:
        w = inputs.uniform(n=1 << 22, seed=3)
        snap = Snapshot(L, ctx, w)
        act = torch.arange(0, w.n, 1000, dtype=torch.int32, device=DEV)
        torch.cuda.synchronize()
        print("no-alloc gravity: oversized active list", flush=True)
        st, acc, pot, nt = snap.gravity("g3_gravity_noalloc", act)
        assert st == g3.G3_EINVAL, g3.STATUS_NAMES.get(st, st)
        assert "region" in g3.g3_last_error(ctx)
        assert torch.cuda.current_stream().query()
        torch.cuda.synchronize()
        assert bool((nt == -7).all()) and bool((acc == -7).all())
        # the ctx is usable afterwards; every particle active fits
        print("no-alloc gravity: every particle of 2^22", flush=True)
        st0, acc0, pot0, nt0 = snap.gravity("g3_gravity", None)
        assert st0 == g3.G3_OK
        st1, acc1, pot1, nt1 = snap.gravity("g3_gravity_noalloc", None)
        assert st1 == g3.G3_OK, g3.g3_last_error(ctx)
        torch.cuda.synchronize()
        assert torch.equal(nt0, nt1) and bool((nt1 > 0).all())
        assert same(acc0, acc1) and same(pot0, pot1)
    finally:
        g3.g3_ctx_destroy(ctx)
