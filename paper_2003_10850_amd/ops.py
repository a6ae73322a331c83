"""torch-facing wrappers of the C entry points.

PyTorch provides device memory and the current stream; each call passes
``data_ptr()`` addresses and ``torch.cuda.current_stream().cuda_stream`` to
the library, which does all of the work in its HIP kernels. Output tensors are
in the caller's particle order; rows of particles that are not active keep
the values of the ``out`` tensors passed in (zeros when the wrapper
allocates them).
"""
from __future__ import annotations

import ctypes

import torch

from . import g3


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return 0 if t is None else t.data_ptr()


def _need(t, dtype, shape, name, device):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device:
        raise TypeError(f"{name} must be a {dtype} tensor on {device}")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}")
    return t


class Context:
    """A library context bound to one GPU."""

    def __init__(self, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.handle = g3.g3_ctx_create(self.device.index or 0)

    def stats(self, reset: bool = False):
        """(non-converged h solves, walk passes over all waves, waves)."""
        return g3.g3_ctx_stats(self.handle, reset)

    def nonconverged(self, reset: bool = False) -> int:
        return self.stats(reset)[0]

    def kernel_timing(self, kind: int, capacity: int) -> None:
        """Record the next `capacity` interaction kernels of `kind` (a
        G3_TUNE_* value) with HIP events on their streams; 0 turns it off."""
        g3.g3_ctx_kernel_timing(self.handle, kind, capacity)

    def kernel_times(self, kind: int) -> list:
        """Durations (ms) of the kernels recorded since enabling or the last
        read, in call order (waits for them)."""
        return g3.g3_ctx_kernel_times(self.handle, kind)

    def tuning(self, kind: int, n_targets: int):
        """(walk_leaf, split, streams) the calls of `kind` over n_targets use."""
        return g3.g3_tuning_get(self.handle, kind, n_targets)

    def set_tuning(self, kind: int, walk_leaf: int, split: int, n_targets: int = -1,
                   streams: int = 1):
        g3.g3_tuning_set(self.handle, kind, n_targets, walk_leaf, split, streams)

    def save_tuning(self, path: str) -> None:
        """Write the tuned launch choices to a text file (see g3_tuning_save)."""
        g3.g3_tuning_save(self.handle, path)

    def load_tuning(self, path: str) -> None:
        """Replace the launch choices with a saved file's (see g3_tuning_load)."""
        g3.g3_tuning_load(self.handle, path)

    def autotune(self, tree, h, vel=None, u=None, rho=None, omega=None, params=None,
                 active=None):
        """Time the launch choices on this tree and active set and keep the
        fastest (g3_autotune); h is copied, not changed."""
        na, ap = _active(tree, active)
        g3.g3_autotune(self.handle, tree.handle, na, ap, g3.g3_params.of(params or tree.params),
                       _ptr(h), _ptr(vel), _ptr(u), _ptr(rho), _ptr(omega), _stream(self.device))

    def close(self):
        if getattr(self, "handle", None):
            g3.g3_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """The octrees of one particle set (all particles, and the gas ones), or
    of a forest of snapshots: ``snap_off`` (n_snap + 1 offsets into the
    particle arrays) with one box per snapshot in ``box``."""

    def __init__(self, ctx: Context, pos, mass, type=None, box=(0.0, 0.0, 0.0, 1.0),
                 params=None, snap_off=None):
        self.ctx = ctx
        self.handle = 0
        self.params = params
        self.build(pos, mass, type, box, snap_off)

    def build(self, pos, mass, type=None, box=None, snap_off=None):
        """pos float32 (plain path) or float64 (mixed-precision path)."""
        dev = self.ctx.device
        n = int(pos.shape[0])
        if pos.dtype not in (torch.float32, torch.float64):
            raise TypeError("pos must be float32 or float64")
        _need(pos, pos.dtype, (n, 3), "pos", dev)
        _need(mass, torch.float32, (n,), "mass", dev)
        if type is not None:
            _need(type, torch.uint8, (n,), "type", dev)
        if box is not None:
            b = [[float(x) for x in row] for row in box] if snap_off is not None \
                else [[float(x) for x in box]]
            self.box = b
        self.snap_off = [0, n] if snap_off is None else [int(x) for x in snap_off]
        if self.snap_off[-1] != n:
            raise ValueError("snap_off must end at the particle count")
        self.n = n
        self.hdtype = pos.dtype  # the SPH calls' h follows the positions
        pt = g3.G3_F64 if pos.dtype == torch.float64 else g3.G3_F32
        self.handle = g3.g3_build_forest(self.ctx.handle, self.snap_off, pt, _ptr(pos),
                                         _ptr(mass), _ptr(type), self.box,
                                         g3.g3_params.of(self.params), self.handle, _stream(dev))
        return self

    def refit(self, pos, mass):
        """Move the built tree to new positions and masses (same dtype as
        built) without rebuilding it: see g3_refit_tree."""
        dev = self.ctx.device
        _need(pos, self.hdtype, (self.n, 3), "pos", dev)
        _need(mass, torch.float32, (self.n,), "mass", dev)
        g3.g3_refit_tree(self.ctx.handle, self.handle, _ptr(pos), _ptr(mass), _stream(dev))
        return self

    def info(self, which: int):
        return g3.g3_tree_info(self.handle, which)

    def export(self, which: int = 0) -> dict:
        dev = self.ctx.device
        m, k = self.info(which)
        i32 = dict(dtype=torch.int32, device=dev)
        d = dict(order=torch.zeros(m, **i32), keys=torch.zeros(m, dtype=torch.int64, device=dev),
                 start=torch.zeros(k, **i32), count=torch.zeros(k, **i32),
                 level=torch.zeros(k, **i32), skip=torch.zeros(k, **i32),
                 mass=torch.zeros(k, dtype=torch.float64, device=dev),
                 com=torch.zeros((k, 3), dtype=torch.float64, device=dev))
        g3.g3_tree_export(self.ctx.handle, self.handle, which,
                          *[_ptr(d[x]) for x in ("order", "keys", "start", "count", "level",
                                                 "skip", "mass", "com")], _stream(dev))
        return d

    def close(self):
        if self.handle and getattr(self.ctx, "handle", None):
            g3.g3_tree_destroy(self.ctx.handle, self.handle)
        self.handle = 0


def _active(tree, active):
    if active is None:
        return tree.n, 0
    _need(active, torch.int32, (active.shape[0],), "active", tree.ctx.device)
    return int(active.shape[0]), active.data_ptr()


def _zeros(tree, *shape, dtype=torch.float32):
    return torch.zeros(*shape, dtype=dtype, device=tree.ctx.device)


def density(tree: Tree, params=None, h=None, active=None, solve_h: bool = True, out=None):
    """SPH density of the active gas particles; returns a dict of tensors.

    h: first guess (solve_h) or the given h, copied; out["h"] instead is
    used in place (its values are the guess or the given h)."""
    p = g3.g3_params.of(params or tree.params)
    n = tree.n
    o = out or {}
    if "h" in o:
        hh = o["h"]
    else:
        hh = h.clone() if h is not None else _zeros(tree, n, dtype=tree.hdtype)
    _need(hh, tree.hdtype, (n,), "h", tree.ctx.device)
    res = dict(h=hh, rho=o.get("rho", _zeros(tree, n)), drho_dh=o.get("drho_dh", _zeros(tree, n)),
               omega=o.get("omega", _zeros(tree, n)),
               nngb=o.get("nngb", _zeros(tree, n, dtype=torch.int32)))
    na, ap = _active(tree, active)
    g3.g3_density(tree.ctx.handle, tree.handle, na, ap, p, int(solve_h), _ptr(hh),
                  _ptr(res["rho"]), _ptr(res["drho_dh"]), _ptr(res["omega"]), _ptr(res["nngb"]),
                  _stream(tree.ctx.device))
    return res


def hydro_force(tree: Tree, vel, u, h, rho, omega, params=None, active=None, out=None):
    p = g3.g3_params.of(params or tree.params)
    n = tree.n
    dev = tree.ctx.device
    _need(vel, torch.float32, (n, 3), "vel", dev)
    _need(h, tree.hdtype, (n,), "h", dev)
    for name, t in (("u", u), ("rho", rho), ("omega", omega)):
        _need(t, torch.float32, (n,), name, dev)
    o = out or {}
    res = dict(acc=o.get("acc", _zeros(tree, n, 3)), dudt=o.get("dudt", _zeros(tree, n)),
               vsig=o.get("vsig", _zeros(tree, n)),
               npairs=o.get("npairs", _zeros(tree, n, dtype=torch.int32)))
    na, ap = _active(tree, active)
    g3.g3_hydro_force(tree.ctx.handle, tree.handle, na, ap, p, _ptr(vel), _ptr(u), _ptr(h),
                      _ptr(rho), _ptr(omega), _ptr(res["acc"]), _ptr(res["dudt"]),
                      _ptr(res["vsig"]), _ptr(res["npairs"]), _stream(dev))
    return res


def conduction(tree: Tree, u, h, rho, kappa0: float, kappa_exp: float = 0.0, params=None,
               active=None, out=None):
    """Thermal conduction rate du/dt of the active gas particles (FP32 trees),
    kappa = kappa0 u^kappa_exp; see g3_conduction."""
    p = g3.g3_params.of(params or tree.params)
    n = tree.n
    dev = tree.ctx.device
    _need(h, torch.float32, (n,), "h", dev)
    for name, t in (("u", u), ("rho", rho)):
        _need(t, torch.float32, (n,), name, dev)
    o = out or {}
    res = dict(dudt=o.get("dudt", _zeros(tree, n)),
               npairs=o.get("npairs", _zeros(tree, n, dtype=torch.int32)))
    na, ap = _active(tree, active)
    g3.g3_conduction(tree.ctx.handle, tree.handle, na, ap, p, kappa0, kappa_exp, _ptr(u),
                     _ptr(h), _ptr(rho), _ptr(res["dudt"]), _ptr(res["npairs"]), _stream(dev))
    return res


def _switch_params(sw) -> "g3.g3_switch_params":
    return g3.g3_switch_params(alpha_min=float(sw.alpha_min), alpha_max=float(sw.alpha_max),
                               decay=float(sw.decay), balsara_eps=float(sw.balsara_eps),
                               alpha_u=float(sw.alpha_u), flags=int(sw.flags))


def velocity_gradients(tree: Tree, vel, h, rho, omega, params=None, active=None, out=None):
    """Velocity divergence [n] and curl [n, 3] of the active gas particles
    (FP32 trees); see g3_velocity_gradients."""
    p = g3.g3_params.of(params or tree.params)
    n = tree.n
    dev = tree.ctx.device
    _need(vel, torch.float32, (n, 3), "vel", dev)
    _need(h, torch.float32, (n,), "h", dev)
    for name, t in (("rho", rho), ("omega", omega)):
        _need(t, torch.float32, (n,), name, dev)
    o = out or {}
    res = dict(div=o.get("div", _zeros(tree, n)), curl=o.get("curl", _zeros(tree, n, 3)))
    na, ap = _active(tree, active)
    g3.g3_velocity_gradients(tree.ctx.handle, tree.handle, na, ap, p, _ptr(vel), _ptr(h),
                             _ptr(rho), _ptr(omega), _ptr(res["div"]), _ptr(res["curl"]),
                             _stream(dev))
    return res


def viscosity_switch(ctx: Context, sw, params, dt: float, u, h, div, curl, alpha=None,
                     balsara=None, active=None):
    """One step dt of the per-particle viscosity strength (alpha, updated in
    place when given) and the Balsara factor (returned); see
    g3_viscosity_switch."""
    dev = ctx.device
    n = int(u.shape[0])
    _need(u, torch.float32, (n,), "u", dev)
    if h.dtype not in (torch.float32, torch.float64):
        raise TypeError("h must be float32 or float64")
    _need(h, h.dtype, (n,), "h", dev)
    _need(div, torch.float32, (n,), "div", dev)
    _need(curl, torch.float32, (n, 3), "curl", dev)
    if alpha is not None:
        _need(alpha, torch.float32, (n,), "alpha", dev)
    bf = balsara if balsara is not None else torch.zeros(n, dtype=torch.float32, device=dev)
    if active is None:
        na, ap = n, 0
    else:
        _need(active, torch.int32, (active.shape[0],), "active", dev)
        na, ap = int(active.shape[0]), active.data_ptr()
    ht = g3.G3_F64 if h.dtype == torch.float64 else g3.G3_F32
    g3.g3_viscosity_switch(ctx.handle, n, ht, na, ap, g3.g3_params.of(params),
                           _switch_params(sw), dt, _ptr(u), _ptr(h), _ptr(div), _ptr(curl),
                           _ptr(alpha), _ptr(bf), _stream(dev))
    return bf


def hydro_force_switches(tree: Tree, vel, u, h, rho, omega, sw, alpha=None, balsara=None,
                         params=None, active=None, out=None):
    """The hydro force with per-particle viscosity strengths, Balsara
    factors and artificial conduction; see g3_hydro_force_switches."""
    p = g3.g3_params.of(params or tree.params)
    n = tree.n
    dev = tree.ctx.device
    _need(vel, torch.float32, (n, 3), "vel", dev)
    _need(h, tree.hdtype, (n,), "h", dev)
    for name, t in (("u", u), ("rho", rho), ("omega", omega)):
        _need(t, torch.float32, (n,), name, dev)
    for name, t in (("alpha", alpha), ("balsara", balsara)):
        if t is not None:
            _need(t, torch.float32, (n,), name, dev)
    o = out or {}
    res = dict(acc=o.get("acc", _zeros(tree, n, 3)), dudt=o.get("dudt", _zeros(tree, n)),
               vsig=o.get("vsig", _zeros(tree, n)),
               npairs=o.get("npairs", _zeros(tree, n, dtype=torch.int32)))
    na, ap = _active(tree, active)
    g3.g3_hydro_force_switches(tree.ctx.handle, tree.handle, na, ap, p, _switch_params(sw),
                               _ptr(vel), _ptr(u), _ptr(h), _ptr(rho), _ptr(omega),
                               _ptr(alpha), _ptr(balsara), _ptr(res["acc"]), _ptr(res["dudt"]),
                               _ptr(res["vsig"]), _ptr(res["npairs"]), _stream(dev))
    return res


def gravity(tree: Tree, params=None, active=None, out=None):
    p = g3.g3_params.of(params or tree.params)
    n = tree.n
    o = out or {}
    res = dict(acc=o.get("acc", _zeros(tree, n, 3)), pot=o.get("pot", _zeros(tree, n)),
               nterms=o.get("nterms", _zeros(tree, n, dtype=torch.int32)))
    na, ap = _active(tree, active)
    g3.g3_gravity(tree.ctx.handle, tree.handle, na, ap, p, _ptr(res["acc"]), _ptr(res["pot"]),
                  _ptr(res["nterms"]), _stream(tree.ctx.device))
    return res


def walk(tree: Tree, kind: int, params=None, h=None, active=None, capacity=None):
    """CSR interaction lists (offsets int64 [n_act+1], list int32)."""
    p = g3.g3_params.of(params or tree.params)
    na, ap = _active(tree, active)
    dev = tree.ctx.device
    offsets = torch.zeros(na + 1, dtype=torch.int64, device=dev)
    if h is not None:
        _need(h, tree.hdtype, (tree.n,), "h", dev)
    cap = 0 if capacity is None else int(capacity)
    lst = torch.zeros(max(cap, 1), dtype=torch.int32, device=dev)
    st, total = g3.g3_walk(tree.ctx.handle, tree.handle, kind, na, ap, _ptr(h), p, cap,
                           offsets.data_ptr(), lst.data_ptr() if cap else 0, _stream(dev))
    if st == g3.G3_EOVERFLOW and capacity is None:
        lst = torch.zeros(max(total, 1), dtype=torch.int32, device=dev)
        st, total = g3.g3_walk(tree.ctx.handle, tree.handle, kind, na, ap, _ptr(h), p, total,
                               offsets.data_ptr(), lst.data_ptr(), _stream(dev))
    return offsets, lst[:total], st


# ------------------------------------------------------------- autograd

def _grad_buf(tree, *shape):
    return torch.zeros(*shape, dtype=torch.float32, device=tree.ctx.device)


class _DensityFn(torch.autograd.Function):
    """rho, drho/dh, Omega at the given h (no solve) as a differentiable
    function of (pos, mass, h); the backward is g3_density_backward."""

    @staticmethod
    def forward(fctx, tree, params, active, pos, mass, h):
        d = density(tree, params, h=h, active=active, solve_h=False)
        fctx.tree, fctx.params, fctx.active = tree, params, active
        fctx.save_for_backward(h, d["rho"], d["drho_dh"])
        return d["rho"], d["drho_dh"], d["omega"]

    @staticmethod
    def backward(fctx, g_rho, g_drho, g_omega):
        tree = fctx.tree
        h, rho, drho = fctx.saved_tensors
        n = tree.n
        gp, gm, gh = _grad_buf(tree, n, 3), _grad_buf(tree, n), _grad_buf(tree, n)
        na, ap = _active(tree, fctx.active)
        c = lambda t: None if t is None else t.contiguous()
        g_rho, g_drho, g_omega = c(g_rho), c(g_drho), c(g_omega)
        g3.g3_density_backward(tree.ctx.handle, tree.handle, na, ap,
                               g3.g3_params.of(fctx.params or tree.params), _ptr(h), _ptr(rho),
                               _ptr(drho), _ptr(g_rho), _ptr(g_drho), _ptr(g_omega), _ptr(gp),
                               _ptr(gm), _ptr(gh), _stream(tree.ctx.device))
        return None, None, None, gp, gm, gh


class _DensitySolveFn(torch.autograd.Function):
    """h solved from N_eff(h) = N_ngb, and rho, drho/dh, Omega at that h, as
    differentiable functions of (pos, mass): the fixed-h part of the backward
    is g3_density_backward, and its dL/dh joins the upstream gradient of h in
    g3_density_solve_backward (the implicit derivative of the solve)."""

    @staticmethod
    def forward(fctx, tree, params, active, h0, pos, mass):
        d = density(tree, params, h=h0, active=active, solve_h=True)
        fctx.tree, fctx.params, fctx.active = tree, params, active
        fctx.set_materialize_grads(False)
        fctx.save_for_backward(d["h"], d["rho"], d["drho_dh"])
        return d["h"], d["rho"], d["drho_dh"], d["omega"]

    @staticmethod
    def backward(fctx, g_h, g_rho, g_drho, g_omega):
        tree = fctx.tree
        h, rho, drho = fctx.saved_tensors
        n = tree.n
        gp, gm = _grad_buf(tree, n, 3), _grad_buf(tree, n)
        # the total gradient of h: its upstream one plus what rho, drho/dh
        # and Omega owe it at fixed h (the fixed-h adjoint adds into it)
        gh = _grad_buf(tree, n) if g_h is None else g_h.contiguous().clone()
        na, ap = _active(tree, fctx.active)
        p = g3.g3_params.of(fctx.params or tree.params)
        st = _stream(tree.ctx.device)
        if g_rho is not None or g_drho is not None or g_omega is not None:
            c = lambda t: None if t is None else t.contiguous()
            g_rho, g_drho, g_omega = c(g_rho), c(g_drho), c(g_omega)
            g3.g3_density_backward(tree.ctx.handle, tree.handle, na, ap, p, _ptr(h), _ptr(rho),
                                   _ptr(drho), _ptr(g_rho), _ptr(g_drho), _ptr(g_omega),
                                   _ptr(gp), _ptr(gm), _ptr(gh), st)
        g3.g3_density_solve_backward(tree.ctx.handle, tree.handle, na, ap, p, _ptr(h), _ptr(rho),
                                     _ptr(drho), _ptr(gh), _ptr(gp), _ptr(gm), st)
        return None, None, None, None, gp, gm


class _HydroFn(torch.autograd.Function):
    """acc, du/dt as a differentiable function of (pos, vel, mass, u, h, rho,
    omega); the backward is g3_hydro_force_backward."""

    @staticmethod
    def forward(fctx, tree, params, active, pos, vel, mass, u, h, rho, omega):
        r = hydro_force(tree, vel, u, h, rho, omega, params=params, active=active)
        fctx.tree, fctx.params, fctx.active = tree, params, active
        fctx.save_for_backward(vel, u, h, rho, omega)
        return r["acc"], r["dudt"]

    @staticmethod
    def backward(fctx, g_acc, g_dudt):
        tree = fctx.tree
        vel, u, h, rho, omega = fctx.saved_tensors
        n = tree.n
        out = [_grad_buf(tree, n, 3), _grad_buf(tree, n, 3), _grad_buf(tree, n),
               _grad_buf(tree, n), _grad_buf(tree, n), _grad_buf(tree, n), _grad_buf(tree, n)]
        gpos, gvel, gmass, gh, gu, grho, gom = out
        na, ap = _active(tree, fctx.active)
        c = lambda t: None if t is None else t.contiguous()
        g3.g3_hydro_force_backward(tree.ctx.handle, tree.handle, na, ap,
                                   g3.g3_params.of(fctx.params or tree.params), _ptr(vel),
                                   _ptr(u), _ptr(h), _ptr(rho), _ptr(omega), _ptr(c(g_acc)),
                                   _ptr(c(g_dudt)), _ptr(gpos), _ptr(gvel), _ptr(gmass),
                                   _ptr(gh), _ptr(gu), _ptr(grho), _ptr(gom),
                                   _stream(tree.ctx.device))
        return None, None, None, gpos, gvel, gmass, gu, gh, grho, gom


class _GravityFn(torch.autograd.Function):
    """acc, pot as a differentiable function of (pos, mass); the backward is
    g3_gravity_backward (opening decisions of the forward held fixed)."""

    @staticmethod
    def forward(fctx, tree, params, active, pos, mass):
        r = gravity(tree, params=params, active=active)
        fctx.tree, fctx.params, fctx.active = tree, params, active
        return r["acc"], r["pot"]

    @staticmethod
    def backward(fctx, g_acc, g_pot):
        tree = fctx.tree
        n = tree.n
        gp, gm = _grad_buf(tree, n, 3), _grad_buf(tree, n)
        na, ap = _active(tree, fctx.active)
        c = lambda t: None if t is None else t.contiguous()
        g3.g3_gravity_backward(tree.ctx.handle, tree.handle, na, ap,
                               g3.g3_params.of(fctx.params or tree.params), _ptr(c(g_acc)),
                               _ptr(c(g_pot)), _ptr(gp), _ptr(gm), _stream(tree.ctx.device))
        return None, None, None, gp, gm


def density_ad(tree: Tree, pos, mass, h, params=None, active=None):
    """Differentiable (rho, drho_dh, omega) at the given h. pos and mass must
    be the tensors `tree` was built from (the kernels read the tree's sorted
    copies); gradients flow to pos, mass and h."""
    _need(h, torch.float32, (tree.n,), "h", tree.ctx.device)
    return _DensityFn.apply(tree, params, active, pos, mass, h)


def density_solve_ad(tree: Tree, pos, mass, h0=None, params=None, active=None):
    """Differentiable (h, rho, drho_dh, omega) with h solved at the active gas
    rows (h0: optional first guess, not differentiated). pos and mass must be
    the tensors `tree` was built from; gradients flow to pos and mass, also
    through the solved h. Rows whose solve did not converge hold their h
    fixed (no gradient through it)."""
    if h0 is not None:
        _need(h0, torch.float32, (tree.n,), "h0", tree.ctx.device)
    return _DensitySolveFn.apply(tree, params, active, h0, pos, mass)


def hydro_force_ad(tree: Tree, pos, vel, mass, u, h, rho, omega, params=None, active=None):
    """Differentiable (acc, dudt); gradients flow to every tensor argument."""
    return _HydroFn.apply(tree, params, active, pos, vel, mass, u, h, rho, omega)


def gravity_ad(tree: Tree, pos, mass, params=None, active=None):
    """Differentiable (acc, pot); gradients flow to pos and mass."""
    return _GravityFn.apply(tree, params, active, pos, mass)


class Integrator:
    """The kick-drift-kick leapfrog on power-of-two time bins of one particle
    set (g3_integrate_start, g3_system_step). The state tensors are updated
    in place by the library; ``pos`` (float32 or float64) and ``h`` share a
    dtype, the rest are float32 (``bin`` int32, ``type`` uint8)."""

    FIELDS = ("pos", "vel", "mass", "u", "type", "h", "rho", "omega", "acc", "dudt", "vsig",
              "pot", "bin")

    def __init__(self, ctx: Context, pos, vel, mass, u, type=None, box=(0.0, 0.0, 0.0, 1.0),
                 params=None, dt_max=1e-3, bin_depth=3, courant=0.15, eta=0.025):
        dev = ctx.device
        n = int(pos.shape[0])
        if pos.dtype not in (torch.float32, torch.float64):
            raise TypeError("pos must be float32 or float64")
        self.ctx, self.n, self.params, self.box = ctx, n, params, [float(x) for x in box]
        f32 = dict(dtype=torch.float32, device=dev)
        self.pos = _need(pos, pos.dtype, (n, 3), "pos", dev)
        self.vel = _need(vel, torch.float32, (n, 3), "vel", dev)
        self.mass = _need(mass, torch.float32, (n,), "mass", dev)
        self.u = _need(u, torch.float32, (n,), "u", dev)
        self.type = None if type is None else _need(type, torch.uint8, (n,), "type", dev)
        self.h = torch.zeros(n, dtype=pos.dtype, device=dev)
        self.rho = torch.zeros(n, **f32)
        self.omega = torch.ones(n, **f32)
        self.acc = torch.zeros(n, 3, **f32)
        self.dudt = torch.zeros(n, **f32)
        self.vsig = torch.zeros(n, **f32)
        self.pot = torch.zeros(n, **f32)
        self.bin = torch.zeros(n, dtype=torch.int32, device=dev)
        self.pos_t = g3.G3_F64 if pos.dtype == torch.float64 else g3.G3_F32
        self.iparams = g3.g3_integ_params(dt_max=float(dt_max), courant=float(courant),
                                          eta=float(eta), bin_depth=int(bin_depth), flags=0)
        self.tree = ctypes.c_void_p()
        self.started = False

    def _state(self):
        return g3.g3_state(**{f: _ptr(getattr(self, f)) for f in self.FIELDS})

    def start(self):
        """Forces and bins of the current (synchronised) state."""
        g3.g3_integrate_start(self.ctx.handle, self.tree, self.n, self.pos_t, self._state(),
                              self.box, g3.g3_params.of(self.params), self.iparams,
                              _stream(self.ctx.device))
        self.started = True

    def system_step(self, tick_active=None):
        """One system step; tick_active (int64 [2^B] on the device, optional)
        receives the number of active particles at each tick."""
        if not self.started:
            self.start()
        if tick_active is not None:
            _need(tick_active, torch.int64, (1 << self.iparams.bin_depth,), "tick_active",
                  self.ctx.device)
        g3.g3_system_step(self.ctx.handle, self.tree, self.n, self.pos_t, self._state(),
                          self.box, g3.g3_params.of(self.params), self.iparams,
                          _ptr(tick_active), _stream(self.ctx.device))
