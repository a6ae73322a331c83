"""FP64 oracle of the time integration around the interaction phase.

TEST INFRASTRUCTURE ONLY: loaded by the test-suite and never by the product
path. It shares no code with the HIP library; its forces are the oracle's
own density, hydro and gravity (``oracle``), its arithmetic FP64 NumPy.

The paper's code advances the particles that are active at a step with a
kick-drift-kick leapfrog on adaptive, power-of-two time steps, and between
tree rebuilds it drifts tree nodes instead of rebuilding the tree (section 1,
the paragraph on adaptive time-stepping; section 2.2). The scheme below is
that leapfrog in the hierarchical form of Springel (2005, section 5),
written out step by step:

Time line. One system step lasts dt_max and is cut into 2^B ticks of
tau = dt_max / 2^B. A particle in bin k (0 <= k <= B) has the step
dt_max / 2^k = 2^(B-k) ticks, and is active at tick T when T is a multiple of
2^(B-k).

Time-step criterion (Springel 2005, eqs. 34 and 16):
    dt_i = sqrt(2 eta eps / |a_i|)            every particle,
    dt_i = min(dt_i, C h_i / v_sig,i)         gas particles,
and the particle's bin is the smallest k in [0, B] with dt_max / 2^k <= dt_i
(B when none is). At tick T a particle may only take a step that T is a
multiple of: k >= B - min(tz(T), B), tz = the number of trailing zero bits
(any step at T = 0 and at the end of the system step).

One system step, from a synchronised state whose forces (total acceleration
a, du/dt, v_sig) and bins are known:
  1. every particle: opening half kick v += a dt_k / 2, u += (du/dt) dt_k / 2;
  2. for T = 1 .. 2^B:
     a. drift every particle: x += v tau; refit the trees to the new x;
     b. the particles active at T: the density with its smoothing-length
        solve (active gas), the hydro force (active gas), gravity (active).
        The hydro force takes every gas particle's velocity and internal
        energy predicted to T from the middle of its current step, where the
        stored (half-kicked) values belong: v + a (T - T_mid),
        u + (du/dt) (T - T_mid), T_mid = T_0 + S/2 for the step [T_0, T_0 + S]
        that contains T (Gadget's predicted quantities; with the stored
        values, whose error is first order in the step, du/dt would break
        the scheme's second order), and the stored h, rho and Omega of the
        inactive neighbours;
     c. active particles: closing half kick with the step they had,
        v += a dt_k / 2, u += (du/dt) dt_k / 2; their new bin from the
        criterion and the alignment rule; and, unless T = 2^B, the opening
        half kick of the new step;
  3. at T = 2^B every particle is active: the state is synchronised again,
     with the forces and bins of the next system step known.
The internal energy is kept non-negative (a kick that would take u below
zero leaves it at zero). The trees are built from the positions at the
start of each system step.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle


@dataclasses.dataclass
class IntegParams:
    dt_max: float          # the longest step (bin 0)
    bin_depth: int         # B: bins 0..B, 2^B ticks per system step
    courant: float = 0.15  # C of the hydrodynamic step
    eta: float = 0.025     # accuracy parameter of the gravitational step


def trailing_zeros(T: int) -> int:
    if T == 0:
        return 64
    k = 0
    while T % 2 == 0:
        T //= 2
        k += 1
    return k


def bin_of_step(dt: np.ndarray, ip: IntegParams) -> tuple[np.ndarray, np.ndarray]:
    """Smallest k in [0, B] with dt_max / 2^k <= dt (B when none is), and the
    decision's margin: the distance of log2(dt_max / dt) to the nearest
    integer, the quantity a rounding difference could flip it at."""
    with np.errstate(divide="ignore", invalid="ignore"):
        x = np.log2(ip.dt_max / dt)
        k = np.clip(np.ceil(x), 0, ip.bin_depth)
        margin = np.where(np.isfinite(x) & (x > 0) & (x < ip.bin_depth),
                          np.abs(x - np.round(x)), np.inf)
    return k.astype(np.int64), margin


class Integrator:
    """The state of one particle set and its leapfrog on power-of-two bins."""

    def __init__(self, pos, vel, mass, u, type_, box, params, ip: IntegParams):
        self.x = np.array(pos, np.float64)
        self.v = np.array(vel, np.float64)
        self.m = np.array(mass, np.float64)
        self.u = np.array(u, np.float64)
        self.type = np.ascontiguousarray(type_, np.uint8)
        self.box = np.asarray(box, np.float64)
        self.p = params
        self.ip = ip
        n = self.x.shape[0]
        self.n = n
        self.gas = self.type == 0
        self.h = np.zeros(n)
        self.rho = np.zeros(n)
        self.omega = np.ones(n)
        self.acc = np.zeros((n, 3))
        self.dudt = np.zeros(n)
        self.vsig = np.zeros(n)
        self.pot = np.zeros(n)
        self.bin = np.zeros(n, np.int64)
        self.forces_valid = False
        self.min_margin = np.inf        # closest bin decision to a boundary
        self.tick_active: list[int] = []  # active particles at every tick
        self.interactions = [0, 0, 0]   # density pairs, hydro pairs, gravity terms

    def _build(self):
        self.gt = oracle.Tree(self.x, self.m, self.box, type=self.type, gas_only=True,
                              leaf_size=self.p.leaf_size)
        self.at = oracle.Tree(self.x, self.m, self.box, type=self.type,
                              leaf_size=self.p.leaf_size)

    def _refit(self):
        self.gt.refit(self.x, self.m)
        self.at.refit(self.x, self.m)

    def _predicted(self, T: int):
        """Velocities and internal energies predicted to tick T from the
        middle of each particle's current step (stored values at T = 0)."""
        if T == 0:
            return self.v, self.u
        S = 2 ** (self.ip.bin_depth - self.bin)
        mid = S * ((T - 1) // S) + 0.5 * S
        dt = (T - mid) * self.ip.dt_max / 2.0 ** self.ip.bin_depth
        vp = self.v + self.acc * dt[:, None]
        up = np.maximum(self.u + self.dudt * dt, 0.0)
        return vp, up

    def _forces(self, act: np.ndarray, T: int):
        """Density (h solve), hydro and gravity of the active particles at
        tick T."""
        ag = act[self.gas[act]]
        acc_h = np.zeros((self.n, 3))
        if ag.size:
            d = oracle.density(self.gt, self.p, active=ag, h=self.h)
            self.h[ag], self.rho[ag], self.omega[ag] = d["h"][ag], d["rho"][ag], d["omega"][ag]
            vp, up = self._predicted(T)
            hy = oracle.hydro(self.gt, self.p, vp, up, self.h, self.rho, self.omega,
                              active=ag)
            acc_h[ag] = hy["acc"][ag]
            self.dudt[ag] = hy["dudt"][ag]
            self.vsig[ag] = hy["vsig"][ag]
            self.interactions[0] += int(d["nngb"][ag].sum())
            self.interactions[1] += int(hy["npairs"][ag].sum())
        g = oracle.gravity(self.at, self.p, active=act)
        self.acc[act] = g["acc"][act] + acc_h[act]
        self.pot[act] = g["pot"][act]
        self.interactions[2] += int(g["nterms"][act].sum())

    def _new_bins(self, act: np.ndarray, T: int):
        a = np.linalg.norm(self.acc[act], axis=1)
        dt = np.full(act.size, np.inf)
        np.divide(2.0 * self.ip.eta * self.p.eps, a, out=dt, where=a > 0)
        dt = np.sqrt(dt)
        hyd = np.full(act.size, np.inf)
        np.divide(self.ip.courant * self.h[act], self.vsig[act], out=hyd,
                  where=self.gas[act] & (self.vsig[act] > 0))
        k, margin = bin_of_step(np.minimum(dt, hyd), self.ip)
        if margin.size:
            self.min_margin = min(self.min_margin, float(margin.min()))
        kmin = self.ip.bin_depth - min(trailing_zeros(T), self.ip.bin_depth)
        self.bin[act] = np.maximum(k, kmin)

    def _kick(self, act: np.ndarray):
        """Half kick of the active particles over half their bin's step."""
        half = 0.5 * self.ip.dt_max / 2.0 ** self.bin[act]
        self.v[act] += self.acc[act] * half[:, None]
        g = act[self.gas[act]]
        hg = 0.5 * self.ip.dt_max / 2.0 ** self.bin[g]
        self.u[g] = np.maximum(self.u[g] + self.dudt[g] * hg, 0.0)

    def start(self):
        """Forces and bins of the current (synchronised) state, if not known."""
        if not self.forces_valid:
            self._build()
            every = np.arange(self.n)
            self._forces(every, 0)
            self._new_bins(every, 0)
            self.forces_valid = True

    def system_step(self):
        ip = self.ip
        B = ip.bin_depth
        every = np.arange(self.n)
        self.start()
        self._build()
        self._kick(every)  # opening
        tau = ip.dt_max / 2.0 ** B
        for T in range(1, 2 ** B + 1):
            self.x += self.v * tau
            self._refit()
            act = every[T % (2 ** (B - self.bin)) == 0]
            self.tick_active.append(int(act.size))
            if act.size == 0:
                continue
            self._forces(act, T)
            self._kick(act)  # closing, with the step the particles had
            self._new_bins(act, T)
            if T < 2 ** B:
                self._kick(act)  # opening of the new step

    def energy(self) -> dict:
        """Kinetic, thermal and potential energy of a synchronised state
        (the potential of the last force evaluation, which at the end of a
        system step covers every particle)."""
        kin = 0.5 * float((self.m * (self.v ** 2).sum(1)).sum())
        th = float((self.m * self.u)[self.gas].sum())
        pot = 0.5 * float((self.m * self.pot).sum())
        return {"kinetic": kin, "thermal": th, "potential": pot, "total": kin + th + pot}
