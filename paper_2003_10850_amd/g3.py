"""Thin ctypes binding of libg3.so: the C entry points under the same names.

Argument marshalling only: every pointer argument is an integer address
(a device pointer from ``tensor.data_ptr()``, or a host address), every
stream a HIP stream handle. All work happens in the library's kernels. The
library must have been built (``paper_2003_10850_amd.build``); loading fails
loudly otherwise: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libg3.so")

G3_OK, G3_EINVAL, G3_ENOMEM, G3_EHIP, G3_EOVERFLOW, G3_ENOCONV, G3_ESTATE = 0, -1, -2, -3, -4, -5, -6
G3_F32, G3_F64 = 0, 1
G3_GATHER, G3_SYMMETRIC, G3_GRAVITY = 0, 1, 2

STATUS_NAMES = {0: "G3_OK", -1: "G3_EINVAL", -2: "G3_ENOMEM", -3: "G3_EHIP",
                -4: "G3_EOVERFLOW", -5: "G3_ENOCONV", -6: "G3_ESTATE"}

# every symbol include/g3.h declares
EXPORTS = ("g3_ctx_create", "g3_ctx_destroy", "g3_last_error", "g3_ctx_stats",
           "g3_ctx_kernel_timing", "g3_ctx_kernel_times", "g3_ctx_inject",
           "g3_build_tree", "g3_build_forest", "g3_refit_tree", "g3_tree_destroy", "g3_tree_info",
           "g3_tree_export",
           "g3_walk", "g3_density", "g3_hydro_force", "g3_gravity", "g3_gravity_noalloc",
           "g3_conduction", "g3_velocity_gradients", "g3_viscosity_switch",
           "g3_hydro_force_switches",
           "g3_density_backward", "g3_density_solve_backward", "g3_hydro_force_backward",
           "g3_gravity_backward",
           "g3_integrate_start", "g3_system_step",
           "g3_autotune", "g3_tuning_get", "g3_tuning_set", "g3_tuning_save", "g3_tuning_load")


class g3_params(ctypes.Structure):
    _fields_ = [("n_ngb", ctypes.c_double), ("h_tol", ctypes.c_double),
                ("gamma", ctypes.c_double), ("alpha", ctypes.c_double),
                ("theta", ctypes.c_double), ("eps", ctypes.c_double),
                ("G", ctypes.c_double), ("leaf_size", ctypes.c_int32),
                ("flags", ctypes.c_int32)]

    @classmethod
    def of(cls, p, **over) -> "g3_params":
        d = {f: getattr(p, f) for f, _ in cls._fields_}
        d.update(over)
        return cls(**d)


class g3_integ_params(ctypes.Structure):
    _fields_ = [("dt_max", ctypes.c_double), ("courant", ctypes.c_double),
                ("eta", ctypes.c_double), ("bin_depth", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class g3_state(ctypes.Structure):
    """Device pointers of the particle state (integers from data_ptr())."""
    _fields_ = [(f, ctypes.c_void_p) for f in
                ("pos", "vel", "mass", "u", "type", "h", "rho", "omega", "acc", "dudt",
                 "vsig", "pot", "bin")]


class g3_switch_params(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("decay", ctypes.c_double), ("balsara_eps", ctypes.c_double),
                ("alpha_u", ctypes.c_double), ("flags", ctypes.c_int32)]


class G3Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded libg3.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2003_10850_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        sig = {
            "g3_ctx_create": ([ctypes.POINTER(P), ctypes.c_int], ctypes.c_int),
            "g3_ctx_destroy": ([P], None),
            "g3_last_error": ([P], ctypes.c_char_p),
            "g3_ctx_stats": ([P, P, i32], ctypes.c_int),
            "g3_ctx_kernel_timing": ([P, i32, i32], ctypes.c_int),
            "g3_ctx_kernel_times": ([P, i32, P, P], ctypes.c_int),
            "g3_ctx_inject": ([P, i32, i64], ctypes.c_int),
            "g3_build_tree": ([P, i64, i32, P, P, P, P, P, P, P], ctypes.c_int),
            "g3_build_forest": ([P, i32, P, i32, P, P, P, P, P, P, P], ctypes.c_int),
            "g3_refit_tree": ([P, P, P, P, P], ctypes.c_int),
            "g3_tree_destroy": ([P, P], None),
            "g3_tree_info": ([P, i32, P, P], ctypes.c_int),
            "g3_tree_export": ([P, P, i32, P, P, P, P, P, P, P, P, P], ctypes.c_int),
            "g3_walk": ([P, P, i32, i64, P, P, P, i64, P, P, P, P], ctypes.c_int),
            "g3_density": ([P, P, i64, P, P, i32, P, P, P, P, P, P], ctypes.c_int),
            "g3_hydro_force": ([P, P, i64, P, P, P, P, P, P, P, P, P, P, P, P], ctypes.c_int),
            "g3_gravity": ([P, P, i64, P, P, P, P, P, P], ctypes.c_int),
            "g3_gravity_noalloc": ([P, P, i64, P, P, P, P, P, P], ctypes.c_int),
            "g3_conduction": ([P, P, i64, P, P, ctypes.c_double, ctypes.c_double, P, P, P, P, P,
                               P], ctypes.c_int),
            "g3_velocity_gradients": ([P, P, i64, P, P, P, P, P, P, P, P, P], ctypes.c_int),
            "g3_viscosity_switch": ([P, i64, i32, i64, P, P, P, ctypes.c_double, P, P, P, P, P,
                                     P, P], ctypes.c_int),
            "g3_hydro_force_switches": ([P, P, i64, P, P, P] + [P] * 12, ctypes.c_int),
            "g3_density_backward": ([P, P, i64, P, P] + [P] * 10, ctypes.c_int),
            "g3_density_solve_backward": ([P, P, i64, P, P] + [P] * 7, ctypes.c_int),
            "g3_hydro_force_backward": ([P, P, i64, P, P] + [P] * 15, ctypes.c_int),
            "g3_gravity_backward": ([P, P, i64, P, P] + [P] * 5, ctypes.c_int),
            "g3_integrate_start": ([P, P, i64, i32, P, P, P, P, P], ctypes.c_int),
            "g3_system_step": ([P, P, i64, i32, P, P, P, P, P, P], ctypes.c_int),
            "g3_autotune": ([P, P, i64, P, P] + [P] * 6, ctypes.c_int),
            "g3_tuning_get": ([P, i32, i64, P, P, P], ctypes.c_int),
            "g3_tuning_set": ([P, i32, i64, i32, i32, i32], ctypes.c_int),
            "g3_tuning_save": ([P, ctypes.c_char_p], ctypes.c_int),
            "g3_tuning_load": ([P, ctypes.c_char_p], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def g3_ctx_create(device: int) -> int:
    h = ctypes.c_void_p()
    st = lib().g3_ctx_create(ctypes.byref(h), int(device))
    if st != G3_OK:
        raise G3Error(st, f"g3_ctx_create(device={device})")
    return h.value


def g3_ctx_destroy(ctx: int) -> None:
    lib().g3_ctx_destroy(ctx)


def g3_last_error(ctx: int) -> str:
    return (lib().g3_last_error(ctx) or b"").decode()


def _check(ctx, st, name, ok=(G3_OK,)):
    if st not in ok:
        raise G3Error(st, f"{name}: {g3_last_error(ctx)}")
    return st


def g3_ctx_stats(ctx: int, reset: bool = False):
    """(non-converged particles, walk passes summed over waves, waves); the
    library's G3_ENOCONV (some solve did not converge) is not an error here:
    the first count says it."""
    return g3_ctx_stats_status(ctx, reset)[1]


def g3_ctx_stats_status(ctx: int, reset: bool = False):
    """(status, stats) with the raw status: G3_OK or G3_ENOCONV."""
    c = (ctypes.c_int64 * 4)()
    st = _check(ctx, lib().g3_ctx_stats(ctx, c, int(reset)), "g3_ctx_stats",
                ok=(G3_OK, G3_ENOCONV))
    return st, (int(c[0]), int(c[1]), int(c[2]))


G3_INJECT_ALLOC, G3_INJECT_MAX_ITER = 1, 2


def g3_ctx_inject(ctx: int, what: int, value: int) -> None:
    _check(ctx, lib().g3_ctx_inject(ctx, int(what), int(value)), "g3_ctx_inject")


def g3_build_tree(ctx, n, pos_t, pos, mass, type_, box, params, tree, stream) -> int:
    """box: 4 host doubles; tree: existing handle or 0. Returns the handle."""
    b = (ctypes.c_double * 4)(*[float(x) for x in box])
    h = ctypes.c_void_p(tree or None)
    st = lib().g3_build_tree(ctx, int(n), int(pos_t), pos, mass, type_ or None, b,
                             ctypes.byref(params), ctypes.byref(h), stream)
    _check(ctx, st, "g3_build_tree")
    return h.value


def g3_build_forest(ctx, snap_off, pos_t, pos, mass, type_, boxes, params, tree, stream) -> int:
    """snap_off: n_snap + 1 host ints; boxes: n_snap x 4 host doubles; tree:
    existing handle or 0. Returns the handle."""
    off = [int(x) for x in snap_off]
    ns = len(off) - 1
    flat = [float(x) for b in boxes for x in b]
    if ns < 1 or len(flat) != 4 * ns:
        raise ValueError("need n_snap >= 1 offsets + 1 and n_snap boxes of 4")
    o = (ctypes.c_int64 * (ns + 1))(*off)
    b = (ctypes.c_double * (4 * ns))(*flat)
    h = ctypes.c_void_p(tree or None)
    st = lib().g3_build_forest(ctx, ns, o, int(pos_t), pos, mass, type_ or None, b,
                               ctypes.byref(params), ctypes.byref(h), stream)
    _check(ctx, st, "g3_build_forest")
    return h.value


def g3_refit_tree(ctx, tree, pos, mass, stream) -> None:
    _check(ctx, lib().g3_refit_tree(ctx, tree, pos, mass, stream), "g3_refit_tree")


def g3_tree_destroy(ctx, tree) -> None:
    lib().g3_tree_destroy(ctx, tree)


def g3_tree_info(tree, which):
    m, k = ctypes.c_int64(), ctypes.c_int64()
    st = lib().g3_tree_info(tree, int(which), ctypes.byref(m), ctypes.byref(k))
    if st != G3_OK:
        raise G3Error(st, "g3_tree_info")
    return int(m.value), int(k.value)


def g3_tree_export(ctx, tree, which, order, keys, start, count, level, skip, mass, com, stream):
    st = lib().g3_tree_export(ctx, tree, int(which), order, keys, start, count, level, skip,
                              mass, com, stream)
    _check(ctx, st, "g3_tree_export")


def g3_walk(ctx, tree, kind, n_act, active, h, params, capacity, offsets, lst, stream):
    """Returns (status, total); status is G3_OK or G3_EOVERFLOW."""
    total = ctypes.c_int64()
    st = lib().g3_walk(ctx, tree, int(kind), int(n_act), active or None, h or None,
                       ctypes.byref(params), int(capacity), offsets, lst or None,
                       ctypes.byref(total), stream)
    _check(ctx, st, "g3_walk", ok=(G3_OK, G3_EOVERFLOW))
    return st, int(total.value)


def g3_density(ctx, tree, n_act, active, params, solve_h, h, rho, drho_dh, omega, nngb, stream):
    st = lib().g3_density(ctx, tree, int(n_act), active or None, ctypes.byref(params),
                          int(solve_h), h, rho or None, drho_dh or None, omega or None,
                          nngb or None, stream)
    _check(ctx, st, "g3_density")


def g3_hydro_force(ctx, tree, n_act, active, params, vel, u, h, rho, omega, acc, dudt, vsig,
                   npairs, stream):
    st = lib().g3_hydro_force(ctx, tree, int(n_act), active or None, ctypes.byref(params),
                              vel, u, h, rho, omega, acc or None, dudt or None, vsig or None,
                              npairs or None, stream)
    _check(ctx, st, "g3_hydro_force")


def g3_gravity(ctx, tree, n_act, active, params, acc, pot, nterms, stream):
    st = lib().g3_gravity(ctx, tree, int(n_act), active or None, ctypes.byref(params),
                          acc or None, pot or None, nterms or None, stream)
    _check(ctx, st, "g3_gravity")


def g3_conduction(ctx, tree, n_act, active, params, kappa0, kappa_exp, u, h, rho, dudt, npairs,
                  stream):
    st = lib().g3_conduction(ctx, tree, int(n_act), active or None, ctypes.byref(params),
                             float(kappa0), float(kappa_exp), u, h, rho, dudt or None,
                             npairs or None, stream)
    _check(ctx, st, "g3_conduction")


def g3_velocity_gradients(ctx, tree, n_act, active, params, vel, h, rho, omega, div_v, curl_v,
                          stream):
    st = lib().g3_velocity_gradients(ctx, tree, int(n_act), active or None,
                                     ctypes.byref(params), vel, h, rho, omega, div_v or None,
                                     curl_v or None, stream)
    _check(ctx, st, "g3_velocity_gradients")


def g3_viscosity_switch(ctx, n, h_type, n_act, active, params, sw, dt, u, h, div_v, curl_v,
                        alpha, balsara, stream):
    st = lib().g3_viscosity_switch(ctx, int(n), int(h_type), int(n_act), active or None,
                                   ctypes.byref(params), ctypes.byref(sw), float(dt), u, h,
                                   div_v, curl_v, alpha or None, balsara or None, stream)
    _check(ctx, st, "g3_viscosity_switch")


def g3_hydro_force_switches(ctx, tree, n_act, active, params, sw, vel, u, h, rho, omega, alpha,
                            balsara, acc, dudt, vsig, npairs, stream):
    st = lib().g3_hydro_force_switches(ctx, tree, int(n_act), active or None,
                                       ctypes.byref(params), ctypes.byref(sw), vel, u, h, rho,
                                       omega, alpha or None, balsara or None, acc or None,
                                       dudt or None, vsig or None, npairs or None, stream)
    _check(ctx, st, "g3_hydro_force_switches")


def g3_gravity_noalloc(ctx, tree, n_act, active, params, acc, pot, nterms, stream):
    st = lib().g3_gravity_noalloc(ctx, tree, int(n_act), active or None, ctypes.byref(params),
                                  acc or None, pot or None, nterms or None, stream)
    _check(ctx, st, "g3_gravity_noalloc")


def g3_density_backward(ctx, tree, n_act, active, params, h, rho, drho_dh, g_rho, g_drho_dh,
                        g_omega, g_pos, g_mass, g_h, stream):
    st = lib().g3_density_backward(ctx, tree, int(n_act), active or None, ctypes.byref(params),
                                   h or None, rho or None, drho_dh or None, g_rho or None,
                                   g_drho_dh or None, g_omega or None, g_pos or None,
                                   g_mass or None, g_h or None, stream)
    _check(ctx, st, "g3_density_backward")


def g3_density_solve_backward(ctx, tree, n_act, active, params, h, rho, drho_dh, g_h, g_pos,
                              g_mass, stream):
    st = lib().g3_density_solve_backward(ctx, tree, int(n_act), active or None,
                                         ctypes.byref(params), h or None, rho or None,
                                         drho_dh or None, g_h or None, g_pos or None,
                                         g_mass or None, stream)
    _check(ctx, st, "g3_density_solve_backward")


def g3_hydro_force_backward(ctx, tree, n_act, active, params, vel, u, h, rho, omega, g_acc,
                            g_dudt, g_pos, g_vel, g_mass, g_h, g_u, g_rho, g_omega, stream):
    st = lib().g3_hydro_force_backward(
        ctx, tree, int(n_act), active or None, ctypes.byref(params), vel or None, u or None,
        h or None, rho or None, omega or None, g_acc or None, g_dudt or None, g_pos or None,
        g_vel or None, g_mass or None, g_h or None, g_u or None, g_rho or None, g_omega or None,
        stream)
    _check(ctx, st, "g3_hydro_force_backward")


def g3_gravity_backward(ctx, tree, n_act, active, params, g_acc, g_pot, g_pos, g_mass, stream):
    st = lib().g3_gravity_backward(ctx, tree, int(n_act), active or None, ctypes.byref(params),
                                   g_acc or None, g_pot or None, g_pos or None, g_mass or None,
                                   stream)
    _check(ctx, st, "g3_gravity_backward")


def g3_integrate_start(ctx, tree_ref, n, pos_t, state, box, params, iparams, stream):
    """tree_ref: a ctypes.c_void_p holding the tree handle (None: a new one)."""
    b = (ctypes.c_double * 4)(*[float(x) for x in box])
    st = lib().g3_integrate_start(ctx, ctypes.byref(tree_ref), int(n), int(pos_t),
                                  ctypes.byref(state), b, ctypes.byref(params),
                                  ctypes.byref(iparams), stream)
    _check(ctx, st, "g3_integrate_start")


def g3_system_step(ctx, tree_ref, n, pos_t, state, box, params, iparams, tick_active, stream):
    b = (ctypes.c_double * 4)(*[float(x) for x in box])
    st = lib().g3_system_step(ctx, ctypes.byref(tree_ref), int(n), int(pos_t),
                              ctypes.byref(state), b, ctypes.byref(params),
                              ctypes.byref(iparams), tick_active or None, stream)
    _check(ctx, st, "g3_system_step")


G3_TUNE_DENSITY, G3_TUNE_HYDRO, G3_TUNE_GRAVITY = 0, 1, 2
G3_SPLIT_AUTO = -2
G3_TIMING_MAX = 4096
_timing_cap = {}


def g3_ctx_kernel_timing(ctx, kind, capacity):
    st = lib().g3_ctx_kernel_timing(ctx, int(kind), int(capacity))
    _check(ctx, st, "g3_ctx_kernel_timing")
    _timing_cap[(ctx, int(kind))] = int(capacity)


def g3_ctx_kernel_times(ctx, kind):
    """Kernel durations (ms) recorded since timing was enabled or last read."""
    cap = max(_timing_cap.get((ctx, int(kind)), 0), 1)
    ms = (ctypes.c_float * cap)()
    n = ctypes.c_int32(0)
    st = lib().g3_ctx_kernel_times(ctx, int(kind), ms, ctypes.byref(n))
    _check(ctx, st, "g3_ctx_kernel_times")
    return [float(ms[k]) for k in range(n.value)]


def g3_autotune(ctx, tree, n_act, active, params, h, vel, u, rho, omega, stream):
    st = lib().g3_autotune(ctx, tree, int(n_act), active or None, ctypes.byref(params),
                           h or None, vel or None, u or None, rho or None, omega or None, stream)
    _check(ctx, st, "g3_autotune")


def g3_tuning_get(ctx, kind, n_targets):
    """(walk_leaf, split, streams) a call of `kind` over n_targets targets uses."""
    a, b, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    st = lib().g3_tuning_get(ctx, int(kind), int(n_targets), ctypes.byref(a), ctypes.byref(b),
                             ctypes.byref(c))
    _check(ctx, st, "g3_tuning_get")
    return a.value, b.value, c.value


def g3_tuning_set(ctx, kind, n_targets, walk_leaf, split, streams=1):
    st = lib().g3_tuning_set(ctx, int(kind), int(n_targets), int(walk_leaf), int(split),
                             int(streams))
    _check(ctx, st, "g3_tuning_set")


def g3_tuning_save(ctx, path: str) -> None:
    _check(ctx, lib().g3_tuning_save(ctx, os.fsencode(path)), "g3_tuning_save")


def g3_tuning_load(ctx, path: str) -> None:
    _check(ctx, lib().g3_tuning_load(ctx, os.fsencode(path)), "g3_tuning_load")
