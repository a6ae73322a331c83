"""Benchmark of the interaction phase on one MI355X.

One step = the whole hot path over one synthetic snapshot: octree build (all
particles and gas), SPH density with the smoothing-length solve from a cold
start, SPH hydro force, Barnes-Hut gravity, every particle active. Gravity
runs on a second stream, queued after the density and beside it and the
hydro (--serial: after them on one stream). The
workload is the paper-like clustered set: N = 2^21 particles (half gas, half
collisionless) in 32 Plummer spheres on a 20 % uniform background, FP32,
Wendland C6 with 295 target neighbours, theta = 0.5, eps = 1e-3.

The metric is particle interactions per second: neighbour pairs of the
density (self included) + hydro pairs + Barnes-Hut terms (particle and node)
of every active particle, as counted by the kernels themselves (the parity
tests check those counts against the oracle exactly).

Prints ONE JSON line. The CPU baseline is the FP64 oracle timed on a bounded
sample of the same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FP32 operations per interaction (an FMA counts 2), counted from
# the formulas each kernel evaluates; sqrt, rsqrt and division count 1
FLOP_DENSITY = 36   # rho and drho/dh of one pair in the support
FLOP_HYDRO = 90     # pressure + viscosity acceleration, du/dt, signal speed
FLOP_GRAVITY = 20   # softened monopole or particle term, acc + potential
# the modules around the path (same convention)
FLOP_CONDUCTION = 30        # symmetric test, F(r, h_i) and F(r, h_j), the pair's rate
FLOP_VELGRAD = 45           # distance, F(q), the pair's gradient, divergence and curl terms
FLOP_HYDRO_SWITCHES = 104   # the hydro pair, the pair's viscosity strength, artificial conduction
# the integration leg's largest step: a particle at the sphere's typical
# speed (about 5) moves about half the central smoothing length in it, so
# the refitted octree stays tight through a system step
DT_INT = 2.5e-4
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (packed) peak
# a short spin (GPU clock cycles, about 0.1 ms) on the gravity stream before
# its call, so that the density beside it is dispatched first
SIDE_SPIN_CYCLES = 200_000


def side_spin(torch) -> None:
    """The short spin on the current stream (torch's one-wave sleep kernel;
    skipped where this torch build has none: the order is then a race)."""
    sleep = getattr(torch.cuda, "_sleep", None)
    if sleep is not None:
        sleep(SIDE_SPIN_CYCLES)
HBM_TBS = 8.0


def kernel_source_hash() -> str:
    """Hash of the HIP sources with comments and blank space removed, so
    that only a change of code (not of its comments) invalidates counter
    figures taken earlier."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2003_10850_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(f.encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_for(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it is missing or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _oracle_ops(gt, at, p, vel, u, fields, sd, sh, sg):
    """One pass of the FP64 oracle over samples: density with the h
    bisection on sd, hydro on sh at the given (h, rho, omega) fields,
    gravity on sg. Returns (seconds per op, interactions per op, results)."""
    import oracle
    t0 = time.perf_counter()
    d = oracle.density(gt, p, active=sd)
    t_d = time.perf_counter() - t0
    h, rho, om = fields
    t0 = time.perf_counter()
    hy = oracle.hydro(gt, p, vel, u, h, rho, om, active=sh)
    t_h = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = oracle.gravity(at, p, active=sg)
    t_g = time.perf_counter() - t0
    inter = (float(d["nngb"][sd].sum()), float(hy["npairs"][sh].sum()),
             float(g["nterms"][sg].sum()))
    return (t_d, t_h, t_g), inter, (d, hy, g)


def _errors(gt, p, gpu, fields, sd, sh, sg, ref) -> dict:
    """Errors of one GPU step against the oracle on the sampled rows, the
    oracle reading only its own or synthetic inputs: the solved h against
    the oracle's own solve (h_rel), and the density there against the
    oracle's at its h (rho_solved_rel, which carries the difference of the
    two h); rho and the neighbour counts of the GPU's check call at the
    synthetic h (rho_rel); the hydro acceleration of its check call at the
    synthetic fields and the step's gravity, relative to the sum S of the
    magnitudes of their terms; counts must be exact."""
    import oracle
    d, hy, g = ref
    hm = fields[0]
    at_m = oracle.density(gt, p, active=sd, h=hm, solve_h=False)
    rel = lambda a, b: np.abs(a - b) / np.abs(b)
    h = gpu["h"].astype(np.float64)
    e = {
        "h_rel": float(rel(h[sd], d["h"][sd]).max()),
        "rho_solved_rel": float(rel(gpu["rho"][sd], d["rho"][sd]).max()),
        "rho_rel": float(rel(gpu["rho_m"][sd], at_m["rho"][sd]).max()),
        "hydro_acc_rel_S": float((np.linalg.norm(gpu["acc_m"][sh] - hy["acc"][sh], axis=1) /
                                  hy["S"][sh]).max()),
        "grav_acc_rel_S": float((np.linalg.norm(gpu["gacc"][sg] - g["acc"][sg], axis=1) /
                                 g["S"][sg]).max()),
        "counts_exact": bool(np.array_equal(gpu["nngb_m"][sd], at_m["nngb"][sd]) and
                             np.array_equal(gpu["npairs_m"][sh], hy["npairs"][sh]) and
                             np.array_equal(gpu["nterms"][sg], g["nterms"][sg])),
        "samples": {"density": int(sd.size), "hydro": int(sh.size), "gravity": int(sg.size)},
    }
    return e


def cpu_baseline(w, samples: int, gpu=None, seed: int = 0) -> dict:
    """The FP64 oracle, as it stands, on this host: both octrees built in
    full, then density (with the h bisection), hydro and gravity on random
    samples of the active particles, each op's time scaled by its sample
    fraction. On every host core: the median of three passes (each over a
    third of the sample); on one thread: one pass over a sixteenth. With the
    plain GPU step's outputs (gpu), also that step's errors on the first
    pass's samples (see _errors). The hydro is evaluated at the generating
    model's smooth fields (h, gas density, Omega = 1)."""
    import oracle

    pos32, vel32, m32, u32 = w.as_f32()
    P, M = pos32.astype(np.float64), m32.astype(np.float64)
    p = w.params
    rng = np.random.default_rng(seed)
    gas = np.nonzero(w.type == 0)[0]
    t0 = time.perf_counter()
    gt = oracle.Tree(P, M, w.box, type=w.type, gas_only=True)
    at = oracle.Tree(P, M, w.box, type=w.type)
    t_build = time.perf_counter() - t0
    from paper_2003_10850_amd import inputs
    fields = (inputs.model_smoothing(w).astype(np.float32).astype(np.float64),
              inputs.model_gas_density(w).astype(np.float32).astype(np.float64),
              np.ones(w.n))

    def draw(k):
        return (np.sort(rng.choice(gas, min(k, gas.size), replace=False)),
                np.sort(rng.choice(gas, min(k, gas.size), replace=False)),
                np.sort(rng.choice(w.n, min(10 * k, w.n), replace=False)))

    def rate(samp, times, inter):
        fr = (samp[0].size / gas.size, samp[1].size / gas.size, samp[2].size / w.n)
        t_full = t_build + sum(t / f for t, f in zip(times, fr))
        return sum(i / f for i, f in zip(inter, fr)) / t_full, t_full

    passes, first = [], None
    for _ in range(3):
        samp = draw(max(samples // 3, 1))
        times, inter, ref = _oracle_ops(gt, at, p, vel32, u32, fields, *samp)
        passes.append(rate(samp, times, inter) + (times,))
        if first is None:
            first = (samp, ref)
    order = sorted(range(3), key=lambda k: passes[k][0])
    value, t_full, times = passes[order[1]]
    cores = oracle.threads()
    oracle.set_threads(1)
    try:
        samp1 = draw(max(samples // 16, 1))
        times1, inter1, _ = _oracle_ops(gt, at, p, vel32, u32, fields, *samp1)
    finally:
        oracle.set_threads(cores)
    value1, t_full1 = rate(samp1, times1, inter1)
    out = {
        "value": value,
        "unit": "interactions/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"FP64 oracle on the same workload: both octrees built in full "
                   f"({t_build:.2f} s); per pass density with h bisection on "
                   f"{first[0][0].size}, hydro on {first[0][1].size} gas and gravity on "
                   f"{first[0][2].size} random particles, each op scaled by its sample "
                   f"fraction; median of 3 passes (median pass {times[0]:.2f}/{times[1]:.2f}/"
                   f"{times[2]:.2f} s, estimated full step {t_full:.1f} s)"),
        "one_thread": {"value": value1, "cores": 1,
                       "sample": f"one pass over {samp1[0].size}/{samp1[1].size}/"
                                 f"{samp1[2].size} samples, estimated full step "
                                 f"{t_full1:.0f} s"},
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
    }
    if gpu is not None:
        samp, ref = first
        out["gpu_errors"] = _errors(gt, p, gpu, fields, *samp, ref)
    return out


def batched_errors(check, n_pick: int = 4, per: int = 300, seed: int = 5) -> dict:
    """Errors of the batched legs' last steps against the FP64 oracle: on
    n_pick snapshots drawn at random (those with active gas), up to `per`
    active gas particles (density, hydro) and active particles (gravity)
    each; the FP32 forest with FP32 decisions, the mixed-precision forest
    (FP64 positions) with FP64 decisions. Density and hydro are compared at
    the generating model's fields (see _errors)."""
    import dataclasses
    import oracle
    b = check["batch"]
    rng = np.random.default_rng(seed)
    act = b.active.astype(np.int64)
    cand = [k for k in range(b.n_snap)
            if np.any(b.type[act[(act >= b.snap_off[k]) & (act < b.snap_off[k + 1])]] == 0)]
    picks = sorted(rng.choice(cand, min(n_pick, len(cand)), replace=False).tolist())
    out = {}
    for leg, flags in (("fp32", 0), ("mixed", oracle.FLAG_FP64_DECISIONS)):
        gpu = check[leg]
        p = dataclasses.replace(b.params, flags=flags)
        worst = {}
        for k in picks:
            r0, r1 = int(b.snap_off[k]), int(b.snap_off[k + 1])
            a = act[(act >= r0) & (act < r1)] - r0
            typ = b.type[r0:r1]
            pos = b.pos[r0:r1] if flags else b.pos[r0:r1].astype(np.float32).astype(np.float64)
            M = b.mass[r0:r1].astype(np.float32).astype(np.float64)
            gt = oracle.Tree(pos, M, b.boxes[k], type=typ, gas_only=True)
            at = oracle.Tree(pos, M, b.boxes[k], type=typ)
            ag = a[typ[a] == 0]
            sd = np.sort(rng.choice(ag, min(per, ag.size), replace=False))
            sg = np.sort(rng.choice(a, min(per, a.size), replace=False))
            g = {f: v[r0:r1] for f, v in gpu.items()}
            fields = (check["hm"][r0:r1].astype(np.float64), check["rm"][r0:r1].astype(np.float64),
                      np.ones(r1 - r0))
            _, _, ref = _oracle_ops(gt, at, p, b.vel[r0:r1].astype(np.float32),
                                    b.u[r0:r1].astype(np.float32), fields, sd, sd, sg)
            e = _errors(gt, p, g, fields, sd, sd, sg, ref)
            for f, v in e.items():
                if f == "counts_exact":
                    worst[f] = worst.get(f, True) and v
                elif f == "samples":
                    worst[f] = {x: worst.get(f, {}).get(x, 0) + y for x, y in v.items()}
                else:
                    worst[f] = max(worst.get(f, 0.0), v)
        worst["snapshots"] = picks
        out[leg] = worst
    return out


def precision_errors(check, k: int = 10_000, seed: int = 11) -> dict:
    """Errors of the precision leg's last step against the FP64 oracle (FP64
    decisions) on random subsamples of 1e4 gas (density, hydro) and 1e4
    particles (gravity), over the full 2e7-particle trees."""
    import dataclasses
    import oracle
    w = check["w"]
    gpu = check["gpu"]
    rng = np.random.default_rng(seed)
    gas = np.nonzero(w.type == 0)[0]
    sd = np.sort(rng.choice(gas, k, replace=False))
    sg = np.sort(rng.choice(w.n, k, replace=False))
    p = dataclasses.replace(w.params, flags=oracle.FLAG_FP64_DECISIONS)
    M = w.mass.astype(np.float32).astype(np.float64)
    gt = oracle.Tree(w.pos, M, w.box, type=w.type, gas_only=True)
    at = oracle.Tree(w.pos, M, w.box, type=w.type)
    fields = (check["hm"], check["rm"].astype(np.float64), np.ones(w.n))
    _, _, ref = _oracle_ops(gt, at, p, w.vel.astype(np.float32), w.u.astype(np.float32),
                            fields, sd, sd, sg)
    return _errors(gt, p, gpu, fields, sd, sd, sg, ref)


COPY_BYTES = 256 << 20  # the calibration copy: 256 MiB read + 256 MiB written


def copy_calibration(dev) -> None:
    """A plain device copy of known size, profiled beside the kernels so that
    the HBM byte counters can be scaled by what they read for it."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def is_plain_kernel(full_name: str, k: str) -> bool:
    """Whether a profiler kernel name is the FP32 (plain) instance of g3 kernel k
    without the switches' extension: k(...), k<false>(...), k<false, streams>(...)
    or k<false, false>(...)."""
    import re
    return re.search(rf"::{k}(<false(, (\d+|false))?>)?\(", full_name) is not None


def summarize_pmc(fetch_csv: str, write_csv: str, out_json: str) -> dict:
    """HBM bytes per launch of each g3 kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by the same
    counter's reading for the calibration copy of COPY_BYTES."""
    import csv
    import collections

    def per_kernel(path, counter):
        acc = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return acc

    out = {"source_hash": kernel_source_hash(), "copy_bytes": COPY_BYTES, "kernels": {}}
    scale = {}
    data = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        acc = per_kernel(path, counter)
        copies = [v for k, vs in acc.items() if "copy" in k.lower() for v in vs
                  if v * 1024 > 0.5 * COPY_BYTES]
        if not copies:
            raise RuntimeError(f"no calibration copy found in {path}")
        scale[counter] = float(np.median(copies)) * 1024 / COPY_BYTES
        data[counter] = acc
    out["counter_scale"] = scale
    for name in ("k_density", "k_hydro", "k_gravity"):
        per = {}
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = [v for k, vs in data[counter].items() if is_plain_kernel(k, name) for v in vs]
            per[counter] = float(np.mean(vals)) * 1024 / scale[counter] if vals else None
        if per["FETCH_SIZE"] is not None and per["WRITE_SIZE"] is not None:
            out["kernels"][name] = {"fetch_bytes": per["FETCH_SIZE"],
                                    "write_bytes": per["WRITE_SIZE"],
                                    "bytes_per_launch": per["FETCH_SIZE"] + per["WRITE_SIZE"]}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


def step_roofline(counts, ms: float) -> dict:
    """Whole-step FP32 roofline position: (density, hydro, gravity)
    interaction counts times their algorithmic FLOP, over the step time."""
    flop = FLOP_DENSITY * counts[0] + FLOP_HYDRO * counts[1] + FLOP_GRAVITY * counts[2]
    achieved = flop / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS}


def _check_calls(tree, vel, u, hm, rm, active=None) -> dict:
    """Outside every timed region: the density and the hydro force of the
    same tree at synthetic inputs (the generating model's h and gas density,
    Omega = 1), which the oracle then reads too, so that the error figures
    never feed a GPU output to the oracle. hm in the tree's dtype."""
    import torch
    from paper_2003_10850_amd import ops
    dm = ops.density(tree, h=hm, active=active, solve_h=False)
    hy = ops.hydro_force(tree, vel, u, hm, rm, torch.ones_like(rm), active=active)
    torch.cuda.synchronize()
    return {"rho_m": dm["rho"].cpu().numpy(), "nngb_m": dm["nngb"].cpu().numpy(),
            "acc_m": hy["acc"].cpu().numpy(), "npairs_m": hy["npairs"].cpu().numpy()}


def _host_outputs(o) -> dict:
    """Host copies of one step's outputs, under the names the error
    evaluation reads (gravity's acceleration as gacc)."""
    names = {"h": "h", "rho": "rho", "omega": "omega", "nngb": "nngb", "acc": "acc",
             "npairs": "npairs", "gacc": "gacc", "nterms": "nterms"}
    return {k: o[v].detach().cpu().numpy() for k, v in names.items()}


def run_batched(dev, steps: int, warmup: int, n_snap: int = 64, seed: int = 2):
    """The batching workload: a forest of n_snap Plummer snapshots (sizes
    log-uniform in [1e3, 1e6]) with time-bin active sets. One step = the
    interaction phase of the active particles of every snapshot (h solve and
    density, hydro force, gravity) as one persistent launch per kernel,
    captured once in a HIP graph and replayed. For comparison the same step
    runs eagerly, and as separate per-snapshot trees and calls (the
    unbatched way)."""
    import torch
    from paper_2003_10850_amd import inputs, ops

    t0 = time.perf_counter()
    b = inputs.batch(n_snap=n_snap, seed=seed)
    print(f"bench: batched workload {b.name}: n={b.n} active={b.active.size} "
          f"({time.perf_counter() - t0:.1f} s to draw)", file=sys.stderr, flush=True)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pos, mass, typ = T(b.pos.astype(np.float32)), T(b.mass.astype(np.float32)), T(b.type)
    vel, u = T(b.vel.astype(np.float32)), T(b.u.astype(np.float32))
    act = T(b.active)
    ctx = ops.Context(dev)
    boxes = [tuple(x) for x in b.boxes]
    tree = ops.Tree(ctx, pos, mass, typ, boxes, b.params, snap_off=b.snap_off)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(3):
        tree.build(pos, mass, typ, boxes, b.snap_off)
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - tb) / 3
    n = b.n
    # every particle's h, rho and omega: the state a simulation carries
    base = ops.density(tree)
    h0, rho0, om0 = base["h"].clone(), base["rho"].clone(), base["omega"].clone()
    f32 = dict(dtype=torch.float32, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    B = dict(h=torch.zeros(n, **f32), rho=torch.zeros(n, **f32), drho_dh=torch.zeros(n, **f32),
             omega=torch.zeros(n, **f32), nngb=torch.zeros(n, **i32),
             acc=torch.zeros(n, 3, **f32), dudt=torch.zeros(n, **f32), vsig=torch.zeros(n, **f32),
             npairs=torch.zeros(n, **i32), gacc=torch.zeros(n, 3, **f32),
             pot=torch.zeros(n, **f32), nterms=torch.zeros(n, **i32))
    # the carried fields of the inactive particles; the active ones are
    # overwritten by every step's density, whose outputs the hydro reads
    B["rho"].copy_(rho0)
    B["omega"].copy_(om0)
    rho_in, om_in = rho0.clone(), om0.clone()

    # gravity runs on a second stream beside density and hydro, queued after
    # the density (in the graph: a fork at the step's start, a join at its
    # end)
    side = torch.cuda.Stream(dev)  # default priority

    def fork():
        e = torch.cuda.Event()
        e.record(torch.cuda.current_stream(dev))
        return e

    def beside(e, fn):
        side.wait_event(e)
        with torch.cuda.stream(side):
            side_spin(torch)  # the density takes the CUs first
            fn()

    def join():
        torch.cuda.current_stream(dev).wait_stream(side)

    def step():
        e = fork()
        B["h"].copy_(h0)  # last step's h is the first guess of the solve
        ops.density(tree, active=act, out={k: B[k] for k in
                                           ("h", "rho", "drho_dh", "omega", "nngb")})
        beside(e, lambda: ops.gravity(tree, active=act, out={"acc": B["gacc"], "pot": B["pot"],
                                                             "nterms": B["nterms"]}))
        ops.hydro_force(tree, vel, u, B["h"], B["rho"], B["omega"], active=act,
                        out={k: B[k] for k in ("acc", "dudt", "vsig", "npairs")})
        join()

    # the autotuner picks candidate tile depth and group split per kernel
    tt = time.perf_counter()
    ctx.autotune(tree, h0, vel=vel, u=u, rho=rho_in, omega=om_in, active=act)
    tune_s = time.perf_counter() - tt
    from paper_2003_10850_amd import g3
    nact = int(b.active.size)
    tuned = {name: dict(zip(("walk_leaf", "split", "streams"), ctx.tuning(kind, nact)))
             for name, kind in (("density", g3.G3_TUNE_DENSITY), ("hydro", g3.G3_TUNE_HYDRO),
                                ("gravity", g3.G3_TUNE_GRAVITY))}
    print(f"bench: autotuned in {tune_s:.2f} s: {tuned}", file=sys.stderr, flush=True)
    s = torch.cuda.Stream(dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        for _ in range(max(warmup, 1)):
            step()
        torch.cuda.synchronize()
        te = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        eager_ms = 1e3 * (time.perf_counter() - te) / steps
    torch.cuda.current_stream(dev).wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for _ in range(max(warmup, 1)):
        g.replay()
    torch.cuda.synchronize()
    tg = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - tg) / steps
    actn = b.active.astype(np.int64)
    gas_act = actn[b.type[actn] == 0]
    i_d = int(B["nngb"][T(gas_act)].sum())
    i_h = int(B["npairs"][T(gas_act)].sum())
    i_g = int(B["nterms"][act.long()].sum())
    inter = i_d + i_h + i_g
    nonconv = ctx.nonconverged(reset=True)
    check = {"batch": b, "fp32": _host_outputs(B)}
    # synthetic fields for the error figures: the generating models' h and
    # gas density per snapshot (boxes at their own places)
    hm = np.concatenate([inputs.model_smoothing(x) for x in b.snaps])
    rm = np.concatenate([inputs.model_gas_density(x) for x in b.snaps]).astype(np.float32)
    check["hm"], check["rm"] = hm.astype(np.float32), rm
    check["fp32"].update(_check_calls(tree, vel, u, T(check["hm"]), T(rm), active=act))
    print(f"bench: batched graph {graph_ms:.3f} ms/step, eager {eager_ms:.3f} ms/step, "
          f"build {build_ms:.2f} ms; interactions {inter}", file=sys.stderr, flush=True)

    # the mixed-precision forest: FP64 positions and h, the same step
    tree64 = ops.Tree(ctx, T(b.pos), mass, typ, boxes, b.params, snap_off=b.snap_off)
    # the state this path carries: its own FP64 h (solved to the same
    # tolerance from the FP32 one), rho and omega
    base64 = ops.density(tree64, h=h0.double())
    h64 = base64["h"].clone()
    H64 = torch.zeros(n, dtype=torch.float64, device=dev)
    B["rho"].copy_(base64["rho"])
    B["omega"].copy_(base64["omega"])
    del base64

    def step64():
        e = fork()
        H64.copy_(h64)
        ops.density(tree64, active=act, out={"h": H64, **{k: B[k] for k in
                                                         ("rho", "drho_dh", "omega", "nngb")}})
        beside(e, lambda: ops.gravity(tree64, active=act, out={"acc": B["gacc"],
                                                               "pot": B["pot"],
                                                               "nterms": B["nterms"]}))
        ops.hydro_force(tree64, vel, u, H64, B["rho"], B["omega"], active=act,
                        out={k: B[k] for k in ("acc", "dudt", "vsig", "npairs")})
        join()

    for _ in range(max(warmup, 1)):
        step64()
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    for _ in range(steps):
        step64()
    torch.cuda.synchronize()
    mixed_ms = 1e3 * (time.perf_counter() - t6) / steps
    k64 = (int(B["nngb"][T(gas_act)].sum()), int(B["npairs"][T(gas_act)].sum()),
           int(B["nterms"][act.long()].sum()))
    i64 = sum(k64)
    check["mixed"] = _host_outputs(dict(B, h=H64))
    check["mixed"].update(_check_calls(tree64, vel, u, T(check["hm"].astype(np.float64)), T(rm),
                                       active=act))
    tree64.close()
    ctx.nonconverged(reset=True)
    print(f"bench: batched mixed precision {mixed_ms:.3f} ms/step", file=sys.stderr, flush=True)

    # unbatched: one tree and three calls per snapshot, default launch choices
    ctx = ops.Context(dev)
    trees = []
    for k in range(b.n_snap):
        r0, r1 = int(b.snap_off[k]), int(b.snap_off[k + 1])
        a = b.active[(b.active >= r0) & (b.active < r1)] - r0
        nk = r1 - r0
        o = dict(h=torch.zeros(nk, **f32), rho=torch.zeros(nk, **f32),
                 drho_dh=torch.zeros(nk, **f32), omega=torch.zeros(nk, **f32),
                 nngb=torch.zeros(nk, **i32), acc=torch.zeros(nk, 3, **f32),
                 dudt=torch.zeros(nk, **f32), vsig=torch.zeros(nk, **f32),
                 npairs=torch.zeros(nk, **i32), gacc=torch.zeros(nk, 3, **f32),
                 pot=torch.zeros(nk, **f32), nterms=torch.zeros(nk, **i32))
        trees.append((ops.Tree(ctx, pos[r0:r1], mass[r0:r1], typ[r0:r1], boxes[k], b.params),
                      r0, r1, T(a.astype(np.int32)), o))

    def step_unbatched():
        for t, r0, r1, a, o in trees:
            o["h"].copy_(h0[r0:r1])
            ops.density(t, active=a, out={k: o[k] for k in
                                          ("h", "rho", "drho_dh", "omega", "nngb")})
            ops.hydro_force(t, vel[r0:r1], u[r0:r1], o["h"], rho_in[r0:r1], om_in[r0:r1],
                            active=a, out={k: o[k] for k in ("acc", "dudt", "vsig", "npairs")})
            ops.gravity(t, active=a, out={"acc": o["gacc"], "pot": o["pot"],
                                          "nterms": o["nterms"]})

    step_unbatched()
    torch.cuda.synchronize()
    tu = time.perf_counter()
    for _ in range(steps):
        step_unbatched()
    torch.cuda.synchronize()
    unbatched_ms = 1e3 * (time.perf_counter() - tu) / steps
    ctx.nonconverged(reset=True)
    for t in trees:
        t[0].close()
    print(f"bench: unbatched {unbatched_ms:.3f} ms/step", file=sys.stderr, flush=True)
    return check, {
        "workload": (f"{b.name}: {b.n_snap} Plummer snapshots (32 spheres + 20% background, "
                     f"half gas), sizes log-uniform in [1e3, 1e6], n={b.n}, time-bin active "
                     f"sets 2^-K with K = round(-log2 f), f log-uniform in [1e-3, 1]; "
                     f"active {b.active.size}; FP32, 295 neighbours, theta=0.5, eps=1e-3"),
        "value": inter / (graph_ms * 1e-3),
        "unit": "interactions/s",
        "ms_per_step": graph_ms,
        "eager_ms_per_step": eager_ms,
        "unbatched_ms_per_step": unbatched_ms,
        "unbatched_value": inter / (unbatched_ms * 1e-3),
        "forest_build_ms": build_ms,
        "autotuned": tuned,
        "autotune_s": tune_s,
        "realised_active_fraction": float(b.active.size) / b.n,
        "snapshots_below_1e3_active": int(sum(
            int(((b.active >= b.snap_off[k]) & (b.active < b.snap_off[k + 1])).sum()) < 1000
            for k in range(b.n_snap))),
        # algorithmic FP32 work of the step (per-interaction operation counts)
        # over its time, against the FP32 vector peak
        "fp32_roofline": step_roofline((i_d, i_h, i_g), graph_ms),
        "mixed_precision": {"ms_per_step": mixed_ms, "value": i64 / (mixed_ms * 1e-3),
                            "fp32_roofline": step_roofline(k64, mixed_ms),
                            "path": "FP64 positions and h, two-float FP32 offsets from each group's FP64 centre, "
                                    "FP64 decisions in the error band, eager calls"},
        "interactions_per_step": {"density": i_d, "hydro": i_h, "gravity": i_g},
        "h_nonconverged": nonconv,
        "step": "h solve + density, hydro force, gravity over every snapshot's active set: "
                "one persistent launch per kernel, gravity on a second stream beside the "
                "other two, the step captured in a HIP graph",
    }


def run_differentiation(dev, steps: int, warmup: int, n: int = 1 << 20, seed: int = 4) -> dict:
    """The differentiation workload: N = 2^20 clustered particles (as the
    plain workload), loss = sum over gas of (log rho)^2 + total potential
    energy, at h from the density solve. One step = the loss forward
    (density at the given h, gravity) and its backward through the adjoint
    kernels, which recompute the walks instead of storing lists."""
    import torch
    from paper_2003_10850_amd import inputs, ops

    w = inputs.plummer(n=n, n_spheres=32, seed=seed)
    pos32, _, m32, _ = w.as_f32()
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pos, mass, typ = T(pos32), T(m32), T(w.type)
    ctx = ops.Context(dev)
    tree = ops.Tree(ctx, pos, mass, typ, tuple(w.box), w.params)
    h = ops.density(tree)["h"].detach()
    gas = T(w.type == 0)
    pos.requires_grad_(True)
    mass.requires_grad_(True)
    h.requires_grad_(True)

    def step():
        pos.grad = mass.grad = h.grad = None
        rho, _, _ = ops.density_ad(tree, pos, mass, h)
        _, pot = ops.gravity_ad(tree, pos, mass)
        L = (torch.log(rho[gas]) ** 2).sum() + 0.5 * (mass * pot).sum()
        L.backward()
        return L

    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        L = step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    ctx.nonconverged(reset=True)
    # outside the timed region: two more steps give the same gradient bits
    grads = []
    for _ in range(2):
        step()
        grads.append([t.grad.detach().clone() for t in (pos, mass, h)])
    same = all(torch.equal(a, b) for a, b in zip(*grads))
    print(f"bench: differentiation {ms:.3f} ms/step (loss {float(L):.6e}); repeated gradients "
          f"{'bit-identical' if same else 'differ'}", file=sys.stderr, flush=True)
    return {
        "workload": f"{w.name}: N={n} clustered as the plain workload, FP32; loss = sum_gas "
                    "(log rho)^2 + (1/2) sum m phi at the solved h",
        "ms_per_step": ms,
        "deterministic": bool(same),
        "step": "forward (density at h, gravity) + backward (density and gravity adjoints, "
                "walks recomputed) for dL/dpos, dL/dmass, dL/dh",
    }


def run_extras(dev, steps: int, warmup: int, n: int = 1 << 21, n_int: int = 1 << 20) -> dict:
    """The modules around the path. Thermal conduction (kappa = 1e-3 u^(5/2))
    and the improved-SPH switches (velocity gradients, the viscosity-strength
    step, the hydro force with per-particle strengths and artificial
    conduction) on the plain workload, at the fields of its own density
    solve; and the time integration of a 2^20-body Plummer sphere in
    equilibrium (half gas, four time bins). Each call is timed with HIP
    events around it on its stream (its prep and group-table kernels
    included); interactions are the kernels' own pair counts."""
    import torch
    from paper_2003_10850_amd import inputs, ops

    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    w = inputs.plummer(n=n, n_spheres=32, seed=1)
    pos32, vel32, m32, u32 = w.as_f32()
    pos, vel, mass, u, typ = T(pos32), T(vel32), T(m32), T(u32), T(w.type)
    ctx = ops.Context(dev)
    tree = ops.Tree(ctx, pos, mass, typ, tuple(w.box), w.params)
    d = ops.density(tree)
    h, rho, om = d["h"].clone(), d["rho"].clone(), d["omega"].clone()
    gas = T(w.type == 0)
    f32 = dict(dtype=torch.float32, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)

    def timed(f):
        for _ in range(max(warmup, 1)):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def entry(ms, pairs, flop):
        achieved = flop * pairs / (ms * 1e-3) / 1e12
        return {"ms_per_call": ms, "interactions": pairs, "value": pairs / (ms * 1e-3),
                "unit": "interactions/s",
                "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                             "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                             "flop_per_interaction": flop}}

    oc = dict(dudt=torch.zeros(n, **f32), npairs=torch.zeros(n, **i32))
    ms_c = timed(lambda: ops.conduction(tree, u, h, rho, 1e-3, 2.5, out=oc))
    cond = entry(ms_c, int(oc["npairs"][gas].sum()), FLOP_CONDUCTION)
    sw = inputs.SwitchParams()
    og = dict(div=torch.zeros(n, **f32), curl=torch.zeros(n, 3, **f32))
    ms_v = timed(lambda: ops.velocity_gradients(tree, vel, h, rho, om, out=og))
    # the same gather as the density at the same h: its neighbour count
    velgrad = entry(ms_v, int(d["nngb"][gas].sum()), FLOP_VELGRAD)
    alpha = torch.full((n,), 0.1, **f32)
    bal = torch.zeros(n, **f32)
    ms_a = timed(lambda: ops.viscosity_switch(ctx, sw, w.params, 1e-4, u, h, og["div"],
                                              og["curl"], alpha=alpha, balsara=bal))
    oh = dict(acc=torch.zeros(n, 3, **f32), dudt=torch.zeros(n, **f32),
              vsig=torch.zeros(n, **f32), npairs=torch.zeros(n, **i32))
    ms_h = timed(lambda: ops.hydro_force_switches(tree, vel, u, h, rho, om, sw, alpha=alpha,
                                                  balsara=bal, out=oh))
    hydro_sw = entry(ms_h, int(oh["npairs"][gas].sum()), FLOP_HYDRO_SWITCHES)
    print(f"bench: extras conduction {ms_c:.3f} ms, velocity gradients {ms_v:.3f} ms, "
          f"switch step {ms_a:.3f} ms, hydro with switches {ms_h:.3f} ms", file=sys.stderr,
          flush=True)
    tree.close()
    del oc, og, oh

    wi = inputs.plummer_equilibrium(n=n_int, gas_fraction=0.5, seed=5)
    # the ticks' time-bin active sets are sparse and uneven: every kind's
    # groups are cut per snapshot (G3_SPLIT_AUTO), the autotuner's choice for
    # such sets (63.6 -> 56.1 ms per system step against the defaults)
    from paper_2003_10850_amd import g3
    for kind in (g3.G3_TUNE_DENSITY, g3.G3_TUNE_HYDRO, g3.G3_TUNE_GRAVITY):
        ctx.set_tuning(kind, 128 if kind != g3.G3_TUNE_GRAVITY else 64, g3.G3_SPLIT_AUTO)
    gi = ops.Integrator(ctx, T(wi.pos.astype(np.float32)), T(wi.vel.astype(np.float32)),
                        T(wi.mass.astype(np.float32)), T(wi.u.astype(np.float32)), T(wi.type),
                        tuple(wi.box), wi.params, dt_max=DT_INT, bin_depth=3)
    gi.start()
    ticks = torch.zeros(8, dtype=torch.int64, device=dev)
    for _ in range(max(warmup, 1)):
        gi.system_step(ticks)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tot = torch.zeros(8, dtype=torch.int64, device=dev)
    e0.record()
    for _ in range(steps):
        gi.system_step(ticks)
        tot += ticks
    e1.record()
    torch.cuda.synchronize()
    ms_i = e0.elapsed_time(e1) / steps
    per_tick = (tot // steps).cpu().tolist()
    bins = np.bincount(gi.bin.cpu().numpy(), minlength=4).tolist()
    print(f"bench: extras system step {ms_i:.3f} ms, active per tick {per_tick}", file=sys.stderr,
          flush=True)
    return {
        "workload": f"{w.name}: the plain workload at its own density solve (conduction "
                    f"kappa = 1e-3 u^(5/2); switches with alpha = 0.1, dt = 1e-4); and "
                    f"{wi.name}: a Plummer sphere in equilibrium, N={n_int}, half gas, "
                    f"KDK leapfrog with 4 time bins (dt_max = {DT_INT:g})",
        "conduction": cond,
        "velocity_gradients": velgrad,
        "viscosity_switch_ms": ms_a,
        "hydro_force_switches": hydro_sw,
        "integration": {"ms_per_system_step": ms_i, "ticks": 8,
                        "active_per_tick": per_tick, "bins": bins,
                        "value": sum(per_tick) / (ms_i * 1e-3),
                        "unit": "active particle updates/s",
                        "step": "build; per tick: drift, refit of both octrees, density (h solve), "
                                "hydro and gravity of the tick's active set, kicks",
                        "launch_choices": "groups cut per snapshot (G3_SPLIT_AUTO) for every kind"},
    }


def run_precision(dev, steps: int, warmup: int, n: int = 20_000_000, seed: int = 3):
    """The precision workload: N = 2e7 particles clustered as the plain
    workload but in 256 Plummer spheres, FP64 stored positions, on the
    mixed-precision path. One step = both octree builds, density with a
    cold-start FP64 h solve, hydro, gravity, every particle active. (Its
    errors against the FP64 oracle on a 1e4-particle subsample are checked
    by the GPU test suite.)"""
    import torch
    from paper_2003_10850_amd import inputs, ops

    w = inputs.plummer(n=n, n_spheres=256, seed=seed)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pos, mass, typ = T(w.pos), T(w.mass.astype(np.float32)), T(w.type)
    vel, u = T(w.vel.astype(np.float32)), T(w.u.astype(np.float32))
    ctx = ops.Context(dev)
    tree = ops.Tree(ctx, pos, mass, typ, tuple(w.box), w.params)
    f32 = dict(dtype=torch.float32, device=dev)
    h = torch.zeros(n, dtype=torch.float64, device=dev)
    od = dict(h=h, rho=torch.zeros(n, **f32), drho_dh=torch.zeros(n, **f32),
              omega=torch.zeros(n, **f32), nngb=torch.zeros(n, dtype=torch.int32, device=dev))
    oh = dict(acc=torch.zeros(n, 3, **f32), dudt=torch.zeros(n, **f32), vsig=torch.zeros(n, **f32),
              npairs=torch.zeros(n, dtype=torch.int32, device=dev))
    og = dict(acc=torch.zeros(n, 3, **f32), pot=torch.zeros(n, **f32),
              nterms=torch.zeros(n, dtype=torch.int32, device=dev))

    # one stream: at this size gravity beside density and hydro lengthens
    # the step (each kernel runs long enough that the other's cache and
    # memory traffic costs more than the filled tails gain)

    def step():
        tree.build(pos, mass, typ)
        h.zero_()
        ops.density(tree, out=od)
        ops.hydro_force(tree, vel, u, h, od["rho"], od["omega"], out=oh)
        ops.gravity(tree, out=og)

    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    gas = T(w.type == 0)
    kinds = (int(od["nngb"][gas].sum()), int(oh["npairs"][gas].sum()), int(og["nterms"].sum()))
    inter = sum(kinds)
    nonconv = ctx.nonconverged(reset=True)
    print(f"bench: precision {ms:.3f} ms/step, {inter} interactions", file=sys.stderr,
          flush=True)
    # synthetic fields for the error figures (a gas mass histogram at this
    # size: the model's sum over 256 spheres for 2e7 particles is slow)
    rm64 = inputs.grid_gas_density(w, cells=128)
    hm = (3.0 * w.params.n_ngb * w.mass / (4.0 * np.pi * rm64)) ** (1.0 / 3.0)
    rm = rm64.astype(np.float32)
    del rm64
    cc = _check_calls(tree, vel, u, T(hm), T(rm))
    check = {"w": w, "hm": hm, "rm": rm,
             "gpu": _host_outputs(dict(od, acc=oh["acc"], npairs=oh["npairs"], gacc=og["acc"],
                                       nterms=og["nterms"]))}
    check["gpu"].update(cc)
    tree.close()
    return check, {
        "workload": f"{w.name}: N={n} in 256 Plummer spheres + 20% background (half gas), "
                    "FP64 stored positions, 295 neighbours, theta=0.5, eps=1e-3, all active",
        "value": inter / (ms * 1e-3),
        "unit": "interactions/s",
        "ms_per_step": ms,
        "interactions_per_step": inter,
        "fp32_roofline": step_roofline(kinds, ms),
        "h_nonconverged": nonconv,
        "path": "mixed precision: FP64 positions, two-float FP32 offsets from each group's FP64 centre, compensated "
                "FP32 sums, FP64 moments and h solve, FP64 decisions in the error band",
    }


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "GRBM_GUI_ACTIVE",
                 "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32",
                 "SQ_INSTS_VALU_TRANS_F32")


def summarize_valu(csv_path: str, out_json: str, n_cu: int = 256) -> dict:
    """Per-kernel vector-ALU figures from one rocprofv3 --pmc run of
    VALU_COUNTERS: VALU wave-instructions per dispatch and per second of
    kernel time, lane utilisation (active lanes per VALU instruction, the
    VALUUtilization expression) and the FP32 operations the hardware
    executed (FMA counted 2, on the lanes that were active)."""
    import csv
    import collections
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(dict)
    for r in csv.DictReader(open(csv_path)):
        name = r["Kernel_Name"]
        for k in ("k_density", "k_hydro", "k_gravity"):
            if is_plain_kernel(name, k):
                acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
                dur[k][r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    out = {"counters": list(VALU_COUNTERS), "cu": n_cu, "kernels": {}}
    for k, c in acc.items():
        m = {n: float(np.mean(v)) for n, v in c.items()}
        util = m["SQ_THREAD_CYCLES_VALU"] / (m["SQ_ACTIVE_INST_VALU"] * 64.0)
        t = float(np.mean(list(dur[k].values())))
        ops = 64.0 * util * (2.0 * m["SQ_INSTS_VALU_FMA_F32"] + m["SQ_INSTS_VALU_ADD_F32"] +
                             m["SQ_INSTS_VALU_MUL_F32"] + m["SQ_INSTS_VALU_TRANS_F32"])
        out["kernels"][k] = {"valu_lane_utilisation": util,
                             "valu_insts_per_dispatch": m["SQ_INSTS_VALU"],
                             "valu_insts_per_s": m["SQ_INSTS_VALU"] / t,
                             "fp32_ops_executed_per_dispatch": ops,
                             "dispatch_s_under_counters": t,
                             "fp32_tflops_executed": ops / t / 1e12}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 21)
    ap.add_argument("--spheres", type=int, default=32)
    ap.add_argument("--cpu-samples", type=int, default=40000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched (forest of snapshots) measurement")
    ap.add_argument("--no-differentiation", action="store_true",
                    help="skip the loss forward + backward measurement")
    ap.add_argument("--serial", action="store_true",
                    help="plain step: gravity after hydro on the same stream")
    ap.add_argument("--autotune", action="store_true",
                    help="plain leg: run the autotuner first (its candidate runs then appear "
                         "in kernel traces of this command); default launch choices otherwise")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 2e7-particle mixed-precision measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the conduction, switches and integration leg")
    ap.add_argument("--only", choices=("batched", "differentiation", "precision", "extras"),
                    help="run just this leg and print its object (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (for HBM counter scaling)")
    ap.add_argument("--summarize-valu", nargs=2, metavar=("CSV", "OUT_JSON"),
                    help="write per-kernel VALU figures from a rocprofv3 --pmc run of the "
                         "VALU counters and exit")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"),
                    help="write per-kernel HBM bytes from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.summarize_valu:
        print(json.dumps(summarize_valu(*args.summarize_valu), indent=1))
        return 0
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(*args.summarize_pmc), indent=1))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                          "(the interaction phase is not sharded across GPUs)"}))
        return 2

    import torch

    from paper_2003_10850_amd import inputs, ops, g3

    dev = torch.device("cuda", 0)
    if args.only:
        leg = {"batched": run_batched, "differentiation": run_differentiation,
               "precision": run_precision, "extras": run_extras}[args.only]
        res = leg(dev, args.steps, args.warmup)
        if isinstance(res, tuple):
            res = res[1]
        print(json.dumps({args.only: res}), flush=True)
        return 0
    w = inputs.plummer(n=args.n, n_spheres=args.spheres, seed=1)
    pos32, vel32, m32, u32 = w.as_f32()
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pos, vel, mass, u, typ = T(pos32), T(vel32), T(m32), T(u32), T(w.type)
    ctx = ops.Context(dev)
    p = w.params
    tree = ops.Tree(ctx, pos, mass, typ, tuple(w.box), p)
    n = w.n
    h = torch.zeros(n, dtype=torch.float32, device=dev)
    tune_s = None
    if args.autotune:
        # launch choices for this workload (cold-start solve, model hydro fields)
        tt = time.perf_counter()
        ctx.autotune(tree, h, vel=vel, u=u, rho=T(inputs.model_gas_density(w).astype(np.float32)),
                     omega=torch.ones(n, device=dev))
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - tt
    tuned = {name: dict(zip(("walk_leaf", "split", "streams"), ctx.tuning(kind, n // 2 if kind < 2 else n)))
             for name, kind in (("density", g3.G3_TUNE_DENSITY), ("hydro", g3.G3_TUNE_HYDRO),
                                ("gravity", g3.G3_TUNE_GRAVITY))}
    print(f"bench: launch choices {tuned} (autotune {tune_s} s)", file=sys.stderr, flush=True)
    outd = dict(rho=torch.zeros(n, device=dev), drho_dh=torch.zeros(n, device=dev),
                omega=torch.zeros(n, device=dev),
                nngb=torch.zeros(n, dtype=torch.int32, device=dev))
    outh = dict(acc=torch.zeros(n, 3, device=dev), dudt=torch.zeros(n, device=dev),
                vsig=torch.zeros(n, device=dev),
                npairs=torch.zeros(n, dtype=torch.int32, device=dev))
    outg = dict(acc=torch.zeros(n, 3, device=dev), pot=torch.zeros(n, device=dev),
                nterms=torch.zeros(n, dtype=torch.int32, device=dev))
    stream = torch.cuda.current_stream(dev)
    # gravity reads only the all-particle octree and has its own scratch, so
    # it runs on a second stream beside density and hydro (--serial: after
    # them on one stream, for the kernels' stand-alone durations)
    side = stream if args.serial else torch.cuda.Stream(dev)  # default priority
    ev = {k: [] for k in ("build", "density", "hydro", "gravity", "interactions")}

    def step(record: bool):
        mk = lambda: torch.cuda.Event(enable_timing=True)
        marks = [mk() for _ in range(5)] if record else None  # on `stream`
        gm = [mk(), mk()] if record else None  # gravity's, on `side`
        if record:
            marks[0].record(stream)
        tree.build(pos, mass, typ)
        if record:
            marks[1].record(stream)

        def gravity():
            with torch.cuda.stream(side):
                if record:
                    gm[0].record(side)
                ops.gravity(tree, out=outg)
                if record:
                    gm[1].record(side)

        built = torch.cuda.Event()
        built.record(stream)
        h.zero_()  # cold start of the h solve every step
        d = ops.density(tree, h=h, out=outd)
        if not args.serial:
            # the density's waves must take the CUs first, gravity's filling
            # in as the density's ragged tail drains (the other way round the
            # step is about 1.5 ms longer): both streams become ready at the
            # build's end, so the second one spins briefly first
            side.wait_event(built)
            with torch.cuda.stream(side):
                side_spin(torch)
            gravity()
        if record:
            marks[2].record(stream)
        ops.hydro_force(tree, vel, u, d["h"], outd["rho"], outd["omega"], out=outh)
        if record:
            marks[3].record(stream)
        if args.serial:
            gravity()
        else:
            stream.wait_stream(side)
        if record:
            marks[4].record(stream)
            ev["build"].append((marks[0], marks[1]))
            ev["density"].append((marks[1], marks[2]))
            ev["hydro"].append((marks[2], marks[3]))
            ev["gravity"].append((gm[0], gm[1]))
            ev["interactions"].append((marks[1], marks[4]))
        return d

    print(f"bench: {w.name} on {torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        print(f"bench: warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    # the library's own HIP events around each interaction kernel, on the
    # kernel's stream (the call spans above also hold the calls' group-table
    # and prep kernels, and gravity's its wait for CUs beside the density)
    kinds = {"density": g3.G3_TUNE_DENSITY, "hydro": g3.G3_TUNE_HYDRO,
             "gravity": g3.G3_TUNE_GRAVITY}
    for kind in kinds.values():
        ctx.kernel_timing(kind, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        d = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps
    kernel_ms = {}
    for k, kind in kinds.items():
        got = ctx.kernel_times(kind)
        assert len(got) == args.steps, f"{k}: {len(got)} kernel timings for {args.steps} steps"
        kernel_ms[k] = float(np.mean(got))
        ctx.kernel_timing(kind, 0)
    ctx.stats(reset=True)
    step(False)  # one more step to read the h-solve pass counts of one step
    torch.cuda.synchronize()
    nonconv, passes, waves = ctx.stats(reset=True)
    gas = torch.from_numpy(w.type == 0).to(dev)
    i_d = int(outd["nngb"][gas].sum())
    i_h = int(outh["npairs"][gas].sum())
    i_g = int(outg["nterms"].sum())
    inter = i_d + i_h + i_g
    times = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}
    plain_out = _host_outputs(dict(outd, h=d["h"], acc=outh["acc"], npairs=outh["npairs"],
                                   gacc=outg["acc"], nterms=outg["nterms"]))
    plain_out.update(_check_calls(tree, vel, u, T(inputs.model_smoothing(w).astype(np.float32)),
                                  T(inputs.model_gas_density(w).astype(np.float32))))
    # the three interaction calls' wall time (with gravity beside the SPH
    # calls, less than the sum of their durations)
    ms_interactions = times["interactions"]
    print(f"bench: {args.steps} steps, {ms:.3f} ms/step; per call ms {times}; "
          f"per kernel ms {kernel_ms}; "
          f"interactions dens {i_d} hydro {i_h} grav {i_g}; nonconv {nonconv}",
          file=sys.stderr, flush=True)

    # the dominant kernel, by the library's event pairs around each
    # interaction kernel
    flops = {"density": FLOP_DENSITY * i_d, "hydro": FLOP_HYDRO * i_h,
             "gravity": FLOP_GRAVITY * i_g}
    kname = {"density": "k_density", "hydro": "k_hydro", "gravity": "k_gravity"}
    dom = max(("density", "hydro", "gravity"), key=lambda k: kernel_ms[k])
    achieved = flops[dom] / (kernel_ms[dom] * 1e-3) / 1e12
    traffic = traffic_for(kname[dom])
    roofline = {"bound": "alu", "kernel": kname[dom], "achieved": achieved,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                "kernel_ms": kernel_ms[dom],
                "per_kernel": {k: {"ms": kernel_ms[k], "tflops": flops[k] / (kernel_ms[k] * 1e-3)
                                   / 1e12, "frac": flops[k] / (kernel_ms[k] * 1e-3) / 1e12
                                   / PEAK_FP32_TFLOPS} for k in kernel_ms},
                # the calls' spans (bench events): build, each call with its
                # group-table and prep kernels, the interaction phase's wall
                "per_call_ms": times,
                # with gravity beside density and hydro the kernels share the
                # CUs: each kernel's duration spans the time it shared
                "concurrent": not args.serial}
    line = {
        "metric": "particle interactions/sec (density+hydro+gravity), batched-FP32 vs plain at stated err",
        "value": inter / (ms * 1e-3),
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain GPU path, {w.name}: N={n} (half gas) in "
                               f"{args.spheres} Plummer spheres + 20% background, FP32, "
                               "Wendland C6 295 neighbours, theta=0.5, eps=1e-3, all active",
                   "n": n, "interactions_per_step": {"density": i_d, "hydro": i_h,
                                                     "gravity": i_g},
                   "h_nonconverged": nonconv,
                   "h_passes_per_wave": passes / max(waves, 1), "path": "plain",
                   "schedule": ("build; density, hydro, gravity on one stream" if args.serial
                                else "build; density then hydro on one stream, gravity "
                                     "queued after the density on a second"),
                   "launch_choices": tuned, "autotune_s": tune_s},
        # the same interactions over the three interaction calls alone (the
        # octree builds excluded: HIP-event times of the timed steps)
        "value_excl_build": inter / (ms_interactions * 1e-3),
        "build_ms": times["build"],
        "roofline": roofline,
        # the whole plain step's algorithmic FP32 work against the same peak
        "step_fp32_roofline": step_roofline((i_d, i_h, i_g), ms),
        "max_err": None,
    }
    checks = {}
    if not args.no_batched:
        checks["batched"], line["batched"] = run_batched(dev, args.steps, args.warmup)
        line["batched"]["max_err"] = None
        line["batched"]["mixed_precision"]["max_err"] = None
    if not args.no_differentiation:
        line["differentiation"] = run_differentiation(dev, args.steps, args.warmup)
    if not args.no_precision:
        checks["precision"], line["precision"] = run_precision(dev, args.steps, args.warmup)
        line["precision"]["max_err"] = None
    if not args.no_extras:
        line["extras"] = run_extras(dev, args.steps, args.warmup)
    if args.copy_calibration:
        copy_calibration(dev)
    if not args.no_cpu_baseline:
        # the oracle leg: the CPU baseline, and every GPU leg's errors
        # against the oracle (outside the timed regions)
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cb = cpu_baseline(w, args.cpu_samples, gpu=plain_out)
        line["max_err"] = cb.pop("gpu_errors")
        line["cpu_baseline"] = cb
        if "batched" in checks:
            print("bench: batched errors (oracle) ...", file=sys.stderr, flush=True)
            e = batched_errors(checks.pop("batched"))
            line["batched"]["max_err"] = e["fp32"]
            line["batched"]["mixed_precision"]["max_err"] = e["mixed"]
        if "precision" in checks:
            print("bench: precision errors (oracle) ...", file=sys.stderr, flush=True)
            line["precision"]["max_err"] = precision_errors(checks.pop("precision"))
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
