"""FP64 CPU oracle of the Gadget3 interaction phase (ctypes front-end).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the HIP library and never loads it; the product path never imports it.

Every array is float64 (positions of the FP32 path are passed as the FP32
values widened to float64); outputs are written at the active rows of
caller-ordered arrays, like the product's.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "g3ref.cpp")

GATHER, SYMMETRIC, GRAVITY = 0, 1, 2
FLAG_FP64_DECISIONS = 1
OK, EINVAL, ENOCONV = 0, -1, -5


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-o", _SO + ".tmp", _SRC]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class Params(ctypes.Structure):
    _fields_ = [("n_ngb", ctypes.c_double), ("h_tol", ctypes.c_double),
                ("gamma", ctypes.c_double), ("alpha", ctypes.c_double),
                ("theta", ctypes.c_double), ("eps", ctypes.c_double),
                ("G", ctypes.c_double), ("leaf_size", ctypes.c_int32),
                ("flags", ctypes.c_int32)]

    @classmethod
    def of(cls, p, **over) -> "Params":
        d = {f: getattr(p, f) for f, _ in cls._fields_}
        d.update(over)
        return cls(**d)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.g3ref_threads.argtypes = []
        L.g3ref_threads.restype = i32
        L.g3ref_set_threads.argtypes = [i32]
        L.g3ref_set_threads.restype = None
        L.g3ref_kernel.argtypes = [dbl, dbl, P, P, P, P]
        L.g3ref_kernel.restype = None
        L.g3ref_key.argtypes = [P, P]
        L.g3ref_key.restype = ctypes.c_uint64
        L.g3ref_tree_build.argtypes = [i64, P, P, P, P, i32, i32]
        L.g3ref_tree_build.restype = P
        L.g3ref_tree_free.argtypes = [P]
        L.g3ref_tree_free.restype = None
        L.g3ref_tree_refit.argtypes = [P, P, P]
        L.g3ref_tree_refit.restype = ctypes.c_int
        L.g3ref_tree_nnodes.argtypes = [P]
        L.g3ref_tree_nnodes.restype = i64
        L.g3ref_tree_nmembers.argtypes = [P]
        L.g3ref_tree_nmembers.restype = i64
        L.g3ref_tree_export.argtypes = [P] * 9
        L.g3ref_tree_export.restype = None
        L.g3ref_density.argtypes = [P, i64, P, P, i32, P, P, P, P, P, P]
        L.g3ref_density.restype = ctypes.c_int
        L.g3ref_hydro.argtypes = [P, i64, P, P, P, P, P, P, P, P, P, P, P, P]
        L.g3ref_hydro.restype = ctypes.c_int
        L.g3ref_gravity.argtypes = [P, i64, P, P, P, P, P, P]
        L.g3ref_hydro_switches.restype = ctypes.c_int
        L.g3ref_hydro_switches.argtypes = [P, i64, P, P, P, P, P, P, P, P, P, dbl, P, P, P, P, P,
                                           P]
        L.g3ref_velgrad.restype = ctypes.c_int
        L.g3ref_velgrad.argtypes = [P, i64, P, P, P, P, P, P, P, P, P, P]
        L.g3ref_conduction.restype = ctypes.c_int
        L.g3ref_conduction.argtypes = [P, i64, P, P, dbl, dbl, P, P, P, P, P, P]
        L.g3ref_gravity.restype = ctypes.c_int
        L.g3ref_lists.argtypes = [P, i32, i64, P, P, P, P, P]
        L.g3ref_lists.restype = ctypes.c_int
        L.g3ref_density_backward.argtypes = [P, i64, P, P] + [P] * 8
        L.g3ref_density_backward.restype = ctypes.c_int
        L.g3ref_hydro_backward.argtypes = [P, i64, P, P] + [P] * 15
        L.g3ref_hydro_backward.restype = ctypes.c_int
        L.g3ref_gravity_backward.argtypes = [P, i64, P, P] + [P] * 5
        L.g3ref_gravity_backward.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().g3ref_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP threads of the oracle's parallel loops."""
    lib().g3ref_set_threads(int(n))


def kernel(r: float, h: float):
    """(W, dW/dr, dW/dh, F) of the Wendland C6 kernel at (r, h)."""
    out = [ctypes.c_double() for _ in range(4)]
    lib().g3ref_kernel(float(r), float(h), *[ctypes.byref(o) for o in out])
    return tuple(o.value for o in out)


def key(x, box) -> int:
    return int(lib().g3ref_key(_ptr(_f64(x, 3)), _ptr(_f64(box, 4))))


class Tree:
    """Octree over all particles (gas_only=False) or over the gas ones."""

    def __init__(self, pos, mass, box, type=None, leaf_size: int = 8, gas_only: bool = False):
        self.pos = _f64(pos, (-1, 3))
        self.mass = _f64(mass)
        self.n = self.pos.shape[0]
        self.type = None if type is None else np.ascontiguousarray(type, np.uint8)
        self.box = _f64(box, 4)
        self._h = lib().g3ref_tree_build(self.n, _ptr(self.pos), _ptr(self.mass),
                                         _ptr(self.type), _ptr(self.box),
                                         int(leaf_size), int(gas_only))
        if not self._h:
            raise ValueError("g3ref_tree_build rejected its arguments")

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        # at interpreter exit the module's globals may already be cleared;
        # the process then releases the tree itself
        L = _lib
        if h and L is not None:
            L.g3ref_tree_free(h)

    def refit(self, pos, mass) -> "Tree":
        """Drift update: new positions and masses, the build's topology and
        cells kept, node moments and bounding boxes recomputed."""
        self.pos = _f64(pos, (-1, 3)).copy()
        self.mass = _f64(mass).copy()
        if self.pos.shape[0] != self.n or self.mass.shape[0] != self.n:
            raise ValueError("refit needs the tree's particle count")
        if lib().g3ref_tree_refit(self._h, _ptr(self.pos), _ptr(self.mass)) != OK:
            raise ValueError("g3ref_tree_refit rejected its arguments")
        return self

    @property
    def nnodes(self) -> int:
        return int(lib().g3ref_tree_nnodes(self._h))

    @property
    def nmembers(self) -> int:
        return int(lib().g3ref_tree_nmembers(self._h))

    def export(self) -> dict:
        m, k = self.nmembers, self.nnodes
        d = dict(order=np.zeros(m, np.int64), keys=np.zeros(m, np.uint64),
                 start=np.zeros(k, np.int64), count=np.zeros(k, np.int64),
                 level=np.zeros(k, np.int32), skip=np.zeros(k, np.int64),
                 mass=np.zeros(k), com=np.zeros((k, 3)))
        lib().g3ref_tree_export(self._h, *[_ptr(d[x]) for x in
                                ("order", "keys", "start", "count", "level", "skip", "mass", "com")])
        return d


def _active(n, active):
    if active is None:
        return np.arange(n, dtype=np.int64)
    return np.ascontiguousarray(active, np.int64)


def density(tree: Tree, params, active=None, h=None, solve_h: bool = True) -> dict:
    act = _active(tree.n, active)
    hh = np.zeros(tree.n) if h is None else _f64(h).copy()
    out = dict(h=hh, rho=np.zeros(tree.n), drho_dh=np.zeros(tree.n),
               omega=np.zeros(tree.n), nngb=np.zeros(tree.n, np.int32))
    nonconv = ctypes.c_int64(0)
    p = Params.of(params)
    st = lib().g3ref_density(tree._h, act.size, _ptr(act), ctypes.byref(p), int(solve_h),
                             _ptr(hh), _ptr(out["rho"]), _ptr(out["drho_dh"]),
                             _ptr(out["omega"]), _ptr(out["nngb"]), ctypes.byref(nonconv))
    if st not in (OK, ENOCONV):
        raise ValueError(f"g3ref_density status {st}")
    out["nonconv"] = int(nonconv.value)
    out["status"] = st
    return out


def hydro(tree: Tree, params, vel, u, h, rho, omega, active=None) -> dict:
    act = _active(tree.n, active)
    n = tree.n
    out = dict(acc=np.zeros((n, 3)), dudt=np.zeros(n), vsig=np.zeros(n), S=np.zeros(n),
               npairs=np.zeros(n, np.int32))
    ins = [_f64(vel, (-1, 3)), _f64(u), _f64(h), _f64(rho), _f64(omega)]
    p = Params.of(params)
    st = lib().g3ref_hydro(tree._h, act.size, _ptr(act), ctypes.byref(p),
                           *[_ptr(a) for a in ins],
                           *[_ptr(out[k]) for k in ("acc", "dudt", "vsig", "S", "npairs")])
    if st != OK:
        raise ValueError(f"g3ref_hydro status {st}")
    return out


def hydro_switches(tree: Tree, params, vel, u, h, rho, omega, alpha=None, balsara=None,
                   alpha_u: float = 0.0, active=None) -> dict:
    """The hydro force with per-particle viscosity strengths and Balsara
    factors (None: params.alpha and 1) and artificial conduction alpha_u;
    see g3ref_hydro_switches."""
    act = _active(tree.n, active)
    n = tree.n
    out = dict(acc=np.zeros((n, 3)), dudt=np.zeros(n), vsig=np.zeros(n), S=np.zeros(n),
               npairs=np.zeros(n, np.int32), S_du=np.zeros(n))
    ins = [_f64(vel, (-1, 3)), _f64(u), _f64(h), _f64(rho), _f64(omega)]
    al = None if alpha is None else _f64(alpha)
    bf = None if balsara is None else _f64(balsara)
    p = Params.of(params)
    st = lib().g3ref_hydro_switches(tree._h, act.size, _ptr(act), ctypes.byref(p),
                                    *[_ptr(a) for a in ins], _ptr(al), _ptr(bf), float(alpha_u),
                                    *[_ptr(out[k]) for k in ("acc", "dudt", "vsig", "S",
                                                             "npairs", "S_du")])
    if st != OK:
        raise ValueError(f"g3ref_hydro_switches status {st}")
    return out


def balsara(div_v, curl_v, u, h, gamma: float, eps: float = 1e-4):
    """The Balsara (1995) factor f = |div v| / (|div v| + |curl v| + eps c / h),
    c = sqrt(gamma (gamma - 1) u): near 1 in compression, near 0 in shear."""
    d = np.abs(_f64(div_v))
    c = np.sqrt(gamma * (gamma - 1.0) * np.maximum(_f64(u), 0.0))
    cv = np.linalg.norm(_f64(curl_v, (-1, 3)), axis=1)
    return d / (d + cv + eps * c / _f64(h))


def alpha_step(alpha, dt, div_v, f, u, h, gamma: float, alpha_min: float, alpha_max: float,
               decay: float):
    """One step dt of the time-dependent viscosity strength (Morris &
    Monaghan 1997, with the (alpha_max - alpha) source factor of Rosswog et
    al. 2000 and the Balsara factor f in the source):
        d alpha / dt = -(alpha - alpha_min) / tau + s (alpha_max - alpha),
        tau = h / (decay c),  s = f max(-div v, 0),
    integrated exactly over the step for inputs held fixed: the equation is
    linear in alpha, so alpha relaxes to alpha_inf = (alpha_min/tau + s
    alpha_max) / (1/tau + s) at the rate 1/tau + s."""
    c = np.sqrt(gamma * (gamma - 1.0) * np.maximum(_f64(u), 0.0))
    rate_decay = decay * c / _f64(h)
    s = _f64(f) * np.maximum(-_f64(div_v), 0.0)
    k = rate_decay + s
    with np.errstate(invalid="ignore", divide="ignore"):
        a_inf = np.where(k > 0, (alpha_min * rate_decay + s * alpha_max) / k, _f64(alpha))
    return a_inf + (_f64(alpha) - a_inf) * np.exp(-k * dt)


def velgrad(tree: Tree, params, vel, h, rho, omega, active=None) -> dict:
    """Velocity divergence and curl (grad-h SPH estimates); see g3ref_velgrad."""
    act = _active(tree.n, active)
    n = tree.n
    out = dict(div=np.zeros(n), curl=np.zeros((n, 3)), S_div=np.zeros(n), S_curl=np.zeros(n))
    p = Params.of(params)
    st = lib().g3ref_velgrad(tree._h, act.size, _ptr(act), ctypes.byref(p),
                             _ptr(_f64(vel, (-1, 3))), _ptr(_f64(h)), _ptr(_f64(rho)),
                             _ptr(_f64(omega)),
                             *[_ptr(out[k]) for k in ("div", "curl", "S_div", "S_curl")])
    if st != OK:
        raise ValueError(f"g3ref_velgrad status {st}")
    return out


def conduction(tree: Tree, params, u, h, rho, kappa0: float, kappa_exp: float = 0.0,
               active=None) -> dict:
    """du/dt of thermal conduction (Brookshaw 1985; Jubelgas, Springel & Dolag
    2004) with kappa = kappa0 u^kappa_exp; see g3ref_conduction."""
    act = _active(tree.n, active)
    n = tree.n
    out = dict(dudt=np.zeros(n), S=np.zeros(n), npairs=np.zeros(n, np.int32))
    p = Params.of(params)
    st = lib().g3ref_conduction(tree._h, act.size, _ptr(act), ctypes.byref(p), float(kappa0),
                                float(kappa_exp), _ptr(_f64(u)), _ptr(_f64(h)), _ptr(_f64(rho)),
                                *[_ptr(out[k]) for k in ("dudt", "S", "npairs")])
    if st != OK:
        raise ValueError(f"g3ref_conduction status {st}")
    return out


def gravity(tree: Tree, params, active=None) -> dict:
    act = _active(tree.n, active)
    n = tree.n
    out = dict(acc=np.zeros((n, 3)), pot=np.zeros(n), S=np.zeros(n),
               nterms=np.zeros(n, np.int32))
    p = Params.of(params)
    st = lib().g3ref_gravity(tree._h, act.size, _ptr(act), ctypes.byref(p),
                             *[_ptr(out[k]) for k in ("acc", "pot", "S", "nterms")])
    if st != OK:
        raise ValueError(f"g3ref_gravity status {st}")
    return out


def lists(tree: Tree, params, kind: int, active=None, h=None):
    """CSR (offsets, list) of the interaction lists, each row sorted."""
    act = _active(tree.n, active)
    hh = None if h is None else _f64(h)
    p = Params.of(params)
    off = np.zeros(act.size + 1, np.int64)
    st = lib().g3ref_lists(tree._h, int(kind), act.size, _ptr(act), ctypes.byref(p),
                           _ptr(hh), _ptr(off), None)
    if st != OK:
        raise ValueError(f"g3ref_lists status {st}")
    lst = np.zeros(int(off[-1]), np.int64)
    lib().g3ref_lists(tree._h, int(kind), act.size, _ptr(act), ctypes.byref(p),
                      _ptr(hh), _ptr(off), _ptr(lst))
    return off, lst


def _opt(a, shape=None):
    return None if a is None else _f64(a, shape)


def density_backward(tree: Tree, params, h, g_rho=None, g_drho_dh=None, g_omega=None,
                     active=None) -> dict:
    """Gradients (pos [n,3], mass [n], h [n]) of sum_i g_rho_i rho_i +
    g_drho_dh_i drho_i/dh + g_omega_i Omega_i over the active gas i."""
    act = _active(tree.n, active)
    n = tree.n
    out = dict(pos=np.zeros((n, 3)), mass=np.zeros(n), h=np.zeros(n))
    S = np.zeros(5 * n)
    ins = [_f64(h), _opt(g_rho), _opt(g_drho_dh), _opt(g_omega)]
    st = lib().g3ref_density_backward(tree._h, act.size, _ptr(act),
                                      ctypes.byref(Params.of(params)),
                                      *[_ptr(a) for a in ins],
                                      *[_ptr(out[k]) for k in ("pos", "mass", "h")], _ptr(S))
    if st != OK:
        raise ValueError(f"g3ref_density_backward status {st}")
    out["S"] = dict(pos=S[:3 * n].reshape(n, 3), mass=S[3 * n:4 * n], h=S[4 * n:])
    return out


def density_solve_backward(tree: Tree, params, h, rho, drho_dh, g_h, active=None,
                           gate: float = 1e-3) -> dict:
    """Gradients (pos [n,3], mass [n]) of sum_i g_h_i h_i, where each active gas
    h_i is the root of the density iteration's constraint
    F_i = N_eff(h_i) - N_ngb = 0 with N_eff = (4 pi/3) h^3 rho / m_i (the
    mass-weighted neighbour number, Springel & Hernquist 2002, eq. 6).

    The paper does not differentiate the iteration; this is the implicit
    function theorem on F_i, with rho, drho/dh the module's outputs at the
    root:
        dh_i/dtheta = -(dF_i/dtheta) / (dF_i/dh_i)
        dF_i/dh_i   = (4 pi/3) (3 h_i^2 rho_i + h_i^3 drho_i/dh) / m_i
        dF_i/dtheta = (4 pi/3) h_i^3 / m_i  drho_i/dtheta
                      - [theta = m_i] N_eff_i / m_i
    The drho/dtheta terms are the oracle's density adjoint seeded with
    g_rho_i = -lambda_i (4 pi/3) h_i^3 / m_i, lambda_i = g_h_i / (dF_i/dh_i).
    A row whose N_eff misses N_ngb by more than `gate` (relative: an h that
    did not converge) has no constraint and passes nothing."""
    act = _active(tree.n, active)
    n = tree.n
    h, rho, drho_dh, g_h = _f64(h), _f64(rho), _f64(drho_dh), _f64(g_h)
    m = tree.mass
    sel = np.zeros(n, bool)
    sel[act] = True
    if tree.type is not None:
        sel &= tree.type == 0
    c = 4.0 * np.pi / 3.0 * h ** 3 / m
    N = c * rho
    sel &= np.abs(N / params.n_ngb - 1.0) <= gate
    dFdh = 4.0 * np.pi / 3.0 * (3.0 * h ** 2 * rho + h ** 3 * drho_dh) / m
    lam = np.where(sel, g_h / np.where(sel, dFdh, 1.0), 0.0)
    seed = -lam * c
    g = density_backward(tree, params, h, g_rho=seed, active=np.nonzero(sel)[0])
    mass = g["mass"] + lam * N / m
    # S: the L1 sums of the contributions to each entry
    S = dict(pos=g["S"]["pos"], mass=g["S"]["mass"] + np.abs(lam * N / m))
    return dict(pos=g["pos"], mass=mass, S=S)


def hydro_backward(tree: Tree, params, vel, u, h, rho, omega, g_acc=None, g_dudt=None,
                   active=None) -> dict:
    """Gradients (pos, vel, mass, h, u, rho, omega) of
    sum_i g_acc_i . a_i + g_dudt_i du_i/dt over the active gas i."""
    act = _active(tree.n, active)
    n = tree.n
    out = dict(pos=np.zeros((n, 3)), vel=np.zeros((n, 3)), mass=np.zeros(n), h=np.zeros(n),
               u=np.zeros(n), rho=np.zeros(n), omega=np.zeros(n))
    S = np.zeros(11 * n)
    ins = [_f64(vel, (-1, 3)), _f64(u), _f64(h), _f64(rho), _f64(omega),
           _opt(g_acc, (-1, 3)), _opt(g_dudt)]
    st = lib().g3ref_hydro_backward(tree._h, act.size, _ptr(act),
                                    ctypes.byref(Params.of(params)), *[_ptr(a) for a in ins],
                                    *[_ptr(out[k]) for k in
                                      ("pos", "vel", "mass", "h", "u", "rho", "omega")], _ptr(S))
    if st != OK:
        raise ValueError(f"g3ref_hydro_backward status {st}")
    out["S"] = dict(pos=S[:3 * n].reshape(n, 3), vel=S[3 * n:6 * n].reshape(n, 3),
                    mass=S[6 * n:7 * n], h=S[7 * n:8 * n], u=S[8 * n:9 * n],
                    rho=S[9 * n:10 * n], omega=S[10 * n:])
    return out


def gravity_backward(tree: Tree, params, g_acc=None, g_pot=None, active=None) -> dict:
    """Gradients (pos [n,3], mass [n]) of sum_i g_acc_i . a_i + g_pot_i phi_i
    over the active i (Barnes-Hut decisions fixed)."""
    act = _active(tree.n, active)
    n = tree.n
    out = dict(pos=np.zeros((n, 3)), mass=np.zeros(n))
    S = np.zeros(4 * n)
    st = lib().g3ref_gravity_backward(tree._h, act.size, _ptr(act),
                                      ctypes.byref(Params.of(params)),
                                      _ptr(_opt(g_acc, (-1, 3))), _ptr(_opt(g_pot)),
                                      _ptr(out["pos"]), _ptr(out["mass"]), _ptr(S))
    if st != OK:
        raise ValueError(f"g3ref_gravity_backward status {st}")
    out["S"] = dict(pos=S[:3 * n].reshape(n, 3), mass=S[3 * n:])
    return out
