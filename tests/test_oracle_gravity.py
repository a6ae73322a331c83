"""Pins of the oracle's Barnes-Hut gravity.

theta = 0 reduces the method to the direct sum (checked against an
independent O(N^2) sum); every interaction list partitions the other
particles exactly once; accepted nodes meet the opening test; the monopole
error against the direct sum shrinks with theta; two-body closed form."""
import numpy as np
import pytest

import oracle
from paper_2003_10850_amd import inputs
from brute import direct_gravity


def clustered(n=1500, seed=2):
    w = inputs.plummer(n=n, n_spheres=4, seed=seed, eps=1e-3)
    return w, w.pos.astype(np.float32).astype(np.float64)


def test_theta_zero_is_direct_sum():
    w, pos = clustered()
    t = oracle.Tree(pos, w.mass, w.box)
    p = inputs.Params(theta=0.0, eps=1e-3)
    g = oracle.gravity(t, p)
    acc, pot = direct_gravity(pos, w.mass, 1e-3)
    assert np.abs(g["acc"] - acc).max() <= 1e-12 * np.abs(acc).max()
    np.testing.assert_allclose(g["pot"], pot, rtol=1e-12)
    np.testing.assert_array_equal(g["nterms"], w.n - 1)
    ma = (w.mass[:, None] * g["acc"]).sum(0)
    assert np.abs(ma).max() <= 1e-12 * np.abs(w.mass[:, None] * g["acc"]).sum()


def test_two_body():
    pos = np.array([[0.2, 0.3, 0.4], [0.5, 0.3, 0.4]])
    m = np.array([2.0, 3.0])
    t = oracle.Tree(pos, m, [0, 0, 0, 1])
    g = oracle.gravity(t, inputs.Params(eps=0.1, G=1.5))
    s2 = 0.3 ** 2 + 0.1 ** 2
    assert g["acc"][0, 0] == pytest.approx(1.5 * 3.0 * 0.3 / s2 ** 1.5, rel=1e-14)
    assert g["acc"][1, 0] == pytest.approx(-1.5 * 2.0 * 0.3 / s2 ** 1.5, rel=1e-14)
    assert g["pot"][0] == pytest.approx(-1.5 * 3.0 / s2 ** 0.5, rel=1e-14)
    assert g["acc"][0, 1] == 0 and g["acc"][0, 2] == 0


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8, 1.2])
def test_lists_partition_the_other_particles(theta):
    w, pos = clustered(n=1200, seed=5)
    t = oracle.Tree(pos, w.mass, w.box)
    p = inputs.Params(theta=theta, eps=1e-3)
    off, lst = oracle.lists(t, p, oracle.GRAVITY)
    d = t.export()
    for i in range(0, w.n, 7):
        covered = []
        for e in lst[off[i]:off[i + 1]]:
            if e >= 0:
                covered.append(int(e))
            else:
                k = -int(e) - 1
                mem = d["order"][d["start"][k]:d["start"][k] + d["count"][k]]
                assert i not in set(mem.tolist())
                # geometric opening test, FP64 up to FP32 rounding of the decision
                dist = np.linalg.norm(pos[i] - d["com"][k])
                l = w.box[3] / 2.0 ** d["level"][k]
                assert l < theta * dist * (1 + 1e-6)
                covered.extend(mem.tolist())
        assert sorted(covered) == [j for j in range(w.n) if j != i]
    g = oracle.gravity(t, p)
    np.testing.assert_array_equal(g["nterms"], np.diff(off))


def test_monopole_error_shrinks_with_theta():
    w, pos = clustered(n=2000, seed=6)
    t = oracle.Tree(pos, w.mass, w.box)
    acc, _ = direct_gravity(pos, w.mass, 1e-3)
    errs = []
    for theta in [0.7, 0.5, 0.3]:
        g = oracle.gravity(t, inputs.Params(theta=theta, eps=1e-3))
        e = np.linalg.norm(g["acc"] - acc, axis=1) / np.linalg.norm(acc, axis=1)
        errs.append(np.sqrt((e ** 2).mean()))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 2e-2


def test_active_subset():
    w, pos = clustered(n=1000, seed=8)
    t = oracle.Tree(pos, w.mass, w.box)
    p = inputs.Params(eps=1e-3)
    full = oracle.gravity(t, p)
    act = inputs.active_subset(w.n, 0.05, seed=3)
    sub = oracle.gravity(t, p, active=act)
    np.testing.assert_array_equal(sub["acc"][act], full["acc"][act])
    rest = np.setdiff1d(np.arange(w.n), act)
    assert np.all(sub["pot"][rest] == 0)
