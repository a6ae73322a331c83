"""The differentiation workload at full size: N = 2^20 clustered particles
(FP32), loss = sum over gas of (log rho)^2 + (1/2) sum m phi at a given h
(the generating model's: an input both sides read, where the benchmark
takes the GPU's solved h), gradients with respect to positions, masses and
h through the autograd functions (walks recomputed in the backward),
checked against the oracle's adjoints on a random subset of 4096 particles.

The bar is the adjoint bar (1e-5 of the oracle's L1 sum of the
contributions to each entry, floored at 1e-7 of the array's median).
"""
import numpy as np
import pytest

import oracle
from paper_2003_10850_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev_t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def check(name, got, ref, S, tol=1e-5):
    err = np.abs(got - ref)
    floor = 1e-7 * np.median(S[S > 0])
    worst = (err / np.maximum(S, 1e-300)).max()
    print(f"C4 {name}: max |err|/S = {worst:.2e}", flush=True)
    assert not (err > tol * S + floor).any(), name


def test_loss_gradient_full_size_subset():
    from paper_2003_10850_amd import ops
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    w = inputs.plummer(n=1 << 20, n_spheres=32, seed=4)
    print(f"C4 workload {w.name} n={w.n}", flush=True)
    pos32, _, m32, _ = w.as_f32()
    ctx = ops.Context(torch.device("cuda", 0))
    tree = ops.Tree(ctx, dev_t(pos32), dev_t(m32), dev_t(w.type), tuple(w.box), w.params)
    h = dev_t(inputs.model_smoothing(w).astype(np.float32))
    pos = dev_t(pos32).requires_grad_(True)
    mass = dev_t(m32).requires_grad_(True)
    h.requires_grad_(True)
    rho, _, _ = ops.density_ad(tree, pos, mass, h)
    gas_t = dev_t(w.type == 0)
    _, pot = ops.gravity_ad(tree, pos, mass)
    L = (torch.log(rho[gas_t]) ** 2).sum() + 0.5 * (mass * pot).sum()
    L.backward()
    gp, gm, gh = host(pos.grad), host(mass.grad), host(h.grad)
    H = host(h).astype(np.float64)
    del tree
    print("C4 GPU gradient done; oracle adjoints", flush=True)

    P, M = pos32.astype(np.float64), m32.astype(np.float64)
    gas = np.nonzero(w.type == 0)[0]
    gt = oracle.Tree(P, M, w.box, type=w.type, gas_only=True)
    at = oracle.Tree(P, M, w.box, type=w.type)
    d = oracle.density(gt, w.params, active=gas, h=H, solve_h=False)
    g_rho = np.zeros(w.n)
    g_rho[gas] = 2.0 * np.log(d["rho"][gas]) / d["rho"][gas]
    phi = oracle.gravity(at, w.params)["pot"]
    rd = oracle.density_backward(gt, w.params, H, g_rho=g_rho, active=gas)
    rg = oracle.gravity_backward(at, w.params, g_pot=0.5 * M)
    sub = np.sort(np.random.default_rng(5).choice(w.n, 4096, replace=False))
    check("g_pos", gp[sub], (rd["pos"] + rg["pos"])[sub], (rd["S"]["pos"] + rg["S"]["pos"])[sub])
    check("g_mass", gm[sub], (rd["mass"] + rg["mass"] + 0.5 * phi)[sub],
          (rd["S"]["mass"] + rg["S"]["mass"] + 0.5 * np.abs(phi))[sub])
    check("g_h", gh[sub], rd["h"][sub], rd["S"]["h"][sub])
