"""Seeded synthetic particle sets for the interaction phase.

This module only draws inputs. It holds none of the method's arithmetic
(no kernel, no tree, no force); both the HIP path and the CPU oracle read
what it returns, and neither is imported here.

The paper profiles Magneticum boxes (Box4/hr with 2e7 particles, Box3/hr,
Box2/hr; sections 1 and 3), which are not available. These generators stand
in for them with the same scale and the same kind of structure: a clustered
particle distribution (dense haloes on a smooth background, as in the
paper's first figure) made of Plummer spheres on a uniform background, with
gas and collisionless species mixed half and half.

Workloads (all in a unit box, non-periodic, G = 1, equal masses 1/N):

* ``uniform``   - N gas particles uniform in [0,1)^3, zero velocities,
  u = 1; 64 target neighbours, eps = 0.01 (the 4096-particle case the
  oracle finishes in seconds).
* ``plummer``   - N particles, half gas and half collisionless, 80 % drawn
  from ``n_spheres`` Plummer spheres (scale radius 0.02, masses log-uniform
  over one decade, centres uniform in [0.1, 0.9]^3) and 20 % uniform,
  Gaussian velocities sigma = 0.1, u = 1; 295 target neighbours,
  eps = 1e-3 (the 2^21-particle paper-like case).
* ``batch``     - a forest of independent ``plummer`` snapshots with sizes
  log-uniform in [1e3, 1e6], each with the active set of one step of a
  hierarchical (power-of-two) time-step scheme: the fraction 2^-K of its
  particles with the shortest time steps (the densest, as free-fall times
  go), K = round(-log2 f) for f log-uniform in [1e-3, 1].
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

GAS = 0
COLLISIONLESS = 1


@dataclass
class Params:
    """Result-defining parameters of one workload (plain numbers, no maths)."""
    n_ngb: float = 64.0        # target (mass-weighted) neighbour number
    h_tol: float = 1e-6        # relative bracket width of the h root solve
    gamma: float = 5.0 / 3.0   # adiabatic index
    alpha: float = 1.0         # artificial-viscosity strength
    theta: float = 0.5         # Barnes-Hut opening angle
    eps: float = 0.01          # Plummer softening length
    G: float = 1.0             # gravitational constant
    leaf_size: int = 8         # maximum particles in an octree leaf
    flags: int = 0


@dataclass
class SwitchParams:
    """Parameters of the improved-SPH switches (plain numbers)."""
    alpha_min: float = 0.025   # floor of the viscosity strength
    alpha_max: float = 1.0     # ceiling of the viscosity strength
    decay: float = 0.2         # l of the decay time h / (l c)
    balsara_eps: float = 1e-4  # eps of the Balsara factor's c/h term
    alpha_u: float = 1.0       # artificial conduction strength
    flags: int = 0


@dataclass
class Workload:
    name: str
    pos: np.ndarray            # [N,3] float64 draws (cast per precision)
    vel: np.ndarray            # [N,3] float64
    mass: np.ndarray           # [N]   float64
    u: np.ndarray              # [N]   float64 specific internal energy
    type: np.ndarray           # [N]   uint8, 0 gas / 1 collisionless
    box: np.ndarray            # [4]   lo xyz + side
    params: Params = field(default_factory=Params)
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def as_f32(self):
        """The FP32 arrays the plain path computes on (pos, vel, mass, u)."""
        return (self.pos.astype(np.float32), self.vel.astype(np.float32),
                self.mass.astype(np.float32), self.u.astype(np.float32))


def uniform(n: int = 4096, seed: int = 0) -> Workload:
    """N gas particles uniform in the unit cube, m = 1/N, v = 0, u = 1."""
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    return Workload(
        name=f"uniform_n{n}_seed{seed}", pos=pos, vel=np.zeros((n, 3)),
        mass=np.full(n, 1.0 / max(n, 1)), u=np.ones(n),
        type=np.zeros(n, np.uint8), box=np.array([0.0, 0.0, 0.0, 1.0]),
        params=Params(n_ngb=64.0, eps=0.01), seed=seed)


def _plummer_radii(rng, a, k):
    x = rng.random(k)
    x = np.clip(x, 1e-300, 1.0)
    return a / np.sqrt(np.maximum(x ** (-2.0 / 3.0) - 1.0, 1e-300))


def _directions(rng, k):
    z = rng.uniform(-1.0, 1.0, k)
    phi = rng.uniform(0.0, 2.0 * np.pi, k)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def plummer(n: int = 1 << 21, n_spheres: int = 32, seed: int = 1,
            scale_radius: float = 0.02, background: float = 0.2,
            n_ngb: float = 295.0, eps: float = 1e-3,
            sigma_v: float = 0.1) -> Workload:
    """Clustered set: Plummer spheres on a uniform background, half gas."""
    rng = np.random.default_rng(seed)
    n_bg = int(round(background * n))
    n_cl = n - n_bg
    centres = rng.uniform(0.1, 0.9, (n_spheres, 3))
    smass = 10.0 ** rng.random(n_spheres)
    share = smass / smass.sum() * n_cl
    counts = np.floor(share).astype(np.int64)
    rest = n_cl - counts.sum()
    if rest > 0:  # largest remainders get the leftover particles
        counts[np.argsort(-(share - counts), kind="stable")[:rest]] += 1
    pos = np.empty((n, 3))
    k0 = 0
    for s in range(n_spheres):
        need = int(counts[s])
        got = []
        while need > 0:
            r = _plummer_radii(rng, scale_radius, need)
            p = centres[s] + r[:, None] * _directions(rng, need)
            ok = np.all((p >= 0.0) & (p < 1.0), axis=1)
            got.append(p[ok])
            need -= int(ok.sum())
        pos[k0:k0 + counts[s]] = np.concatenate(got)[:counts[s]]
        k0 += int(counts[s])
    pos[k0:] = rng.random((n_bg, 3))
    # mix the species: exactly half gas, chosen at random
    typ = np.full(n, COLLISIONLESS, np.uint8)
    typ[rng.permutation(n)[: n // 2]] = GAS
    # shuffle the caller order so that no input order is Morton-like
    order = rng.permutation(n)
    pos = pos[order]
    typ = typ[order]
    vel = rng.normal(0.0, sigma_v, (n, 3))
    w = Workload(
        name=f"plummer_n{n}_s{n_spheres}_seed{seed}", pos=pos, vel=vel,
        mass=np.full(n, 1.0 / n), u=np.ones(n), type=typ,
        box=np.array([0.0, 0.0, 0.0, 1.0]),
        params=Params(n_ngb=n_ngb, eps=eps), seed=seed)
    w.model = dict(centres=centres, counts=counts, a=scale_radius, n_bg=n_bg)
    return w


def plummer_equilibrium(n: int = 2048, scale_radius: float = 0.04, r_max: float = 0.45,
                        seed: int = 5, gas_fraction: float = 0.0, eps: float | None = None,
                        n_ngb: float = 64.0) -> Workload:
    """One Plummer sphere of total mass 1 (G = 1) centred in the unit box,
    drawn in dynamical equilibrium: radii by the inverse mass profile and
    speeds from the isotropic distribution function by rejection on
    g(q) = q^2 (1 - q^2)^(7/2), q = v / v_esc(r), v_esc^2 = 2 / sqrt(r^2 + a^2)
    (the sampling recipe of Aarseth, Henon & Wielen 1974). Radii beyond
    r_max are redrawn. A fraction of the particles (chosen at random) is gas
    with u = 1/100 of the central potential depth; the rest is
    collisionless."""
    rng = np.random.default_rng(seed)
    a = scale_radius
    r = np.empty(0)
    while r.size < n:
        rr = _plummer_radii(rng, a, n)
        r = np.concatenate([r, rr[rr < r_max]])
    r = r[:n]
    q = np.empty(0)
    while q.size < n:
        x4, x5 = rng.random(2 * n), rng.random(2 * n)
        keep = 0.1 * x5 < x4 ** 2 * (1.0 - x4 ** 2) ** 3.5
        q = np.concatenate([q, x4[keep]])
    q = q[:n]
    vesc = np.sqrt(2.0) * (r * r + a * a) ** -0.25
    pos = 0.5 + r[:, None] * _directions(rng, n)
    vel = (q * vesc)[:, None] * _directions(rng, n)
    typ = np.full(n, COLLISIONLESS, np.uint8)
    typ[rng.permutation(n)[: int(round(gas_fraction * n))]] = GAS
    return Workload(
        name=f"plummer_eq_n{n}_a{a}_seed{seed}", pos=pos, vel=vel,
        mass=np.full(n, 1.0 / n), u=np.full(n, 0.01 / a), type=typ,
        box=np.array([0.0, 0.0, 0.0, 1.0]),
        params=Params(n_ngb=n_ngb, eps=a / 20.0 if eps is None else eps), seed=seed)


@dataclass
class Batch:
    """Snapshots concatenated in caller order: snapshot k is the rows
    [snap_off[k], snap_off[k+1]) of every array, in its own box boxes[k]."""
    name: str
    snaps: list
    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    u: np.ndarray
    type: np.ndarray
    snap_off: np.ndarray       # [S+1] int64
    boxes: np.ndarray          # [S,4]
    active: np.ndarray         # int32 caller ids over the whole forest
    level: np.ndarray          # [S] time-bin level K: active fraction 2^-K
    params: Params = field(default_factory=Params)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_snap(self) -> int:
        return len(self.snaps)


def timestep_active(w: Workload, level: int) -> np.ndarray:
    """Active set of a hierarchical time-step scheme at a step where the
    bins of time step dt_max 2^-K and shorter are due: the fraction 2^-K
    of the particles with the highest model density (shortest free-fall
    time), as sorted caller ids."""
    k = max(1, int(np.ceil(w.n * 2.0 ** -level))) if w.n else 0
    rank = np.argsort(-model_gas_density(w), kind="stable")
    return np.sort(rank[:k]).astype(np.int32)


def batch(n_snap: int = 64, n_min: float = 1e3, n_max: float = 1e6, seed: int = 2,
          f_min: float = 1e-3, n_spheres: int = 32, n_ngb: float = 295.0,
          eps: float = 1e-3, shift_boxes: bool = False) -> Batch:
    """Forest workload: n_snap Plummer snapshots (as ``plummer``) with sizes
    log-uniform in [n_min, n_max] and time-bin active sets. With shift_boxes
    snapshot k lives in the unit box at (k, 0, 0) instead of the origin."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(10.0 ** rng.uniform(np.log10(n_min), np.log10(n_max), n_snap)).astype(np.int64)
    frac = 10.0 ** rng.uniform(np.log10(f_min), 0.0, n_snap)
    level = np.clip(np.rint(-np.log2(frac)), 0, None).astype(np.int64)
    snaps, act, boxes = [], [], []
    off = [0]
    for k in range(n_snap):
        w = plummer(n=int(sizes[k]), n_spheres=n_spheres, seed=seed * 1000 + k, n_ngb=n_ngb,
                    eps=eps)
        if shift_boxes:
            w.pos = w.pos + np.array([float(k), 0.0, 0.0])
            w.box = np.array([float(k), 0.0, 0.0, 1.0])
            w.model["centres"] = w.model["centres"] + np.array([float(k), 0.0, 0.0])
        snaps.append(w)
        act.append(timestep_active(w, int(level[k])) + off[-1])
        boxes.append(w.box)
        off.append(off[-1] + w.n)
    cat = lambda f: np.concatenate([getattr(w, f) for w in snaps])
    return Batch(name=f"batch_s{n_snap}_seed{seed}", snaps=snaps, pos=cat("pos"), vel=cat("vel"),
                 mass=cat("mass"), u=cat("u"), type=cat("type"),
                 snap_off=np.array(off, np.int64), boxes=np.array(boxes),
                 active=np.concatenate(act).astype(np.int32), level=level,
                 params=Params(n_ngb=n_ngb, eps=eps))


def model_gas_density(w: Workload) -> np.ndarray:
    """Gas mass density of the generating model at every particle: the
    Plummer profiles 3M/(4 pi a^3) (1 + r^2/a^2)^(-5/2) of the spheres plus
    the uniform background, times the gas share (1/2). Input synthesis only:
    it gives smooth, realistic smoothing lengths and densities to feed the
    hydro force and the fixed-h density without solving anything."""
    m = getattr(w, "model", None)
    if m is None:  # uniform gas box
        return np.full(w.n, w.mass.sum() / w.box[3] ** 3)
    mp = 1.0 / w.n
    rho = np.full(w.n, m["n_bg"] * mp)
    a = m["a"]
    for c, k in zip(m["centres"], m["counts"]):
        r2 = ((w.pos - c) ** 2).sum(1)
        rho += 3.0 * k * mp / (4.0 * np.pi * a ** 3) * (1.0 + r2 / a ** 2) ** -2.5
    return 0.5 * rho


def model_smoothing(w: Workload, n_ngb: float | None = None) -> np.ndarray:
    """h with (4 pi/3) h^3 rho_model = n_ngb m: a synthetic smoothing field."""
    n_ngb = w.params.n_ngb if n_ngb is None else n_ngb
    return (3.0 * n_ngb * w.mass / (4.0 * np.pi * model_gas_density(w))) ** (1.0 / 3.0)


def grid_gas_density(w: Workload, cells: int = 256) -> np.ndarray:
    """Gas mass density at every particle from a cells^3 mass histogram of
    the gas particles over the box (the density of the particle's cell; the
    cell of a gas particle is never empty). Input synthesis only: a cheap
    stand-in for ``model_gas_density`` at tens of millions of particles."""
    gas = w.type == 0
    q = np.floor((w.pos - w.box[:3]) / w.box[3] * cells).astype(np.int64)
    np.clip(q, 0, cells - 1, out=q)
    flat = (q[:, 0] * cells + q[:, 1]) * cells + q[:, 2]
    mcell = np.bincount(flat[gas], weights=w.mass[gas], minlength=cells ** 3)
    rho = mcell[flat] / (w.box[3] / cells) ** 3
    rho[rho <= 0] = mcell[mcell > 0].min() / (w.box[3] / cells) ** 3
    return rho


def grid_smoothing(w: Workload, n_ngb: float | None = None, cells: int = 256) -> np.ndarray:
    """h with (4 pi/3) h^3 rho_grid = n_ngb m, from ``grid_gas_density``."""
    n_ngb = w.params.n_ngb if n_ngb is None else n_ngb
    return (3.0 * n_ngb * w.mass / (4.0 * np.pi * grid_gas_density(w, cells))) ** (1.0 / 3.0)


def lattice(side: int, spacing: float = 1.0) -> np.ndarray:
    """Integer cubic lattice points (side^3 of them) times ``spacing``."""
    g = np.arange(side, dtype=np.float64) * spacing
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def active_subset(n: int, fraction: float, seed: int) -> np.ndarray:
    """A sorted random subset of caller ids (an active set)."""
    rng = np.random.default_rng(seed)
    k = max(0, min(n, int(round(fraction * n))))
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
