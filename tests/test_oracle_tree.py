"""Pins of the oracle's Morton keys and octree against an independent
geometric construction (recursive cube subdivision), FP64 moments and the
Barnes-Hut tree definition: nodes are key prefixes, subdivided while they
hold more than B members, chains kept."""
import numpy as np
import pytest

import oracle
from paper_2003_10850_amd import inputs
from brute import geometric_tree


def deinterleave(k):
    ix = iy = iz = 0
    for b in range(21):
        digit = (k >> (3 * b)) & 7
        ix |= ((digit >> 2) & 1) << b
        iy |= ((digit >> 1) & 1) << b
        iz |= (digit & 1) << b
    return ix, iy, iz


def test_key_decodes_to_cell():
    rng = np.random.default_rng(5)
    box = [0.0, 0.0, 0.0, 1.0]
    for x in rng.random((200, 3)):
        ix, iy, iz = deinterleave(oracle.key(x, box))
        assert (ix, iy, iz) == tuple(int(np.floor(v * 2 ** 21)) for v in x)
    # clamping at the box faces
    ix, iy, iz = deinterleave(oracle.key([1.0, -0.5, 0.999999999], box))
    assert ix == 2 ** 21 - 1 and iy == 0 and iz == int(np.floor(0.999999999 * 2 ** 21))


def test_key_in_shifted_box():
    box = [10.0, -3.0, 2.0, 4.0]
    x = np.array([11.0, -1.0, 5.5])
    ix, iy, iz = deinterleave(oracle.key(x, box))
    assert (ix, iy, iz) == (2 ** 19, 2 ** 20, int(3.5 / 4 * 2 ** 21))


def _oracle_nodes(t):
    d = t.export()
    return [(int(d["level"][k]), frozenset(int(i) for i in
             d["order"][d["start"][k]:d["start"][k] + d["count"][k]]))
            for k in range(t.nnodes)], d


@pytest.mark.parametrize("n,leaf,seed", [(1, 8, 0), (8, 8, 0), (9, 8, 1), (200, 8, 2),
                                         (300, 1, 3), (500, 4, 4)])
def test_tree_equals_geometric_subdivision(n, leaf, seed):
    pos = np.random.default_rng(seed).random((n, 3))
    t = oracle.Tree(pos, np.full(n, 1.0 / n), [0, 0, 0, 1], leaf_size=leaf)
    nodes, d = _oracle_nodes(t)
    assert nodes == geometric_tree(pos, [0, 0, 0, 1], leaf)


def test_clustered_tree_and_chains():
    w = inputs.plummer(n=3000, n_spheres=3, seed=7)
    pos = w.pos.astype(np.float32).astype(np.float64)
    # 12 coincident particles force a single-child chain down to level 21
    pos[:12] = pos[12]
    t = oracle.Tree(pos, w.mass, w.box)
    nodes, d = _oracle_nodes(t)
    assert nodes == geometric_tree(pos, w.box, 8)
    assert d["level"].max() == 21
    deep = d["count"][d["level"] == 21]
    assert deep.max() == 13  # the coincident group stays one level-21 leaf


def test_preorder_skip_and_moments():
    w = inputs.plummer(n=2000, n_spheres=4, seed=3)
    pos, m = w.pos, np.random.default_rng(1).random(w.n) + 0.5
    t = oracle.Tree(pos, m, w.box)
    d = t.export()
    nn = t.nnodes
    for k in range(nn):
        s, c, sk = d["start"][k], d["count"][k], d["skip"][k]
        mem = d["order"][s:s + c]
        assert d["mass"][k] == pytest.approx(m[mem].sum(), rel=1e-13)
        np.testing.assert_allclose(d["com"][k], (m[mem, None] * pos[mem]).sum(0) / m[mem].sum(),
                                   rtol=1e-12, atol=1e-14)
        # the subtree of k is exactly the preorder range (k, skip): members nest
        sub = range(k + 1, sk)
        assert all(d["start"][j] >= s and d["start"][j] + d["count"][j] <= s + c for j in sub)
        assert sk == nn or d["start"][sk] == s + c
    assert d["mass"][0] == pytest.approx(m.sum(), rel=1e-13)
    # keys are sorted, ties by caller id
    ks = d["keys"].astype(object)
    assert all((ks[a], d["order"][a]) < (ks[a + 1], d["order"][a + 1]) for a in range(len(ks) - 1))


def test_gas_only_tree_members():
    w = inputs.plummer(n=1000, n_spheres=2, seed=9)
    t = oracle.Tree(w.pos, w.mass, w.box, type=w.type, gas_only=True)
    d = t.export()
    assert set(d["order"].tolist()) == set(np.nonzero(w.type == 0)[0].tolist())
    nodes, _ = _oracle_nodes(t)
    assert nodes == geometric_tree(w.pos, w.box, 8, ids=np.nonzero(w.type == 0)[0])


def test_empty_tree():
    t = oracle.Tree(np.zeros((0, 3)), np.zeros(0), [0, 0, 0, 1])
    assert t.nnodes == 0
