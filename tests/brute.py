"""Brute-force references used to pin the oracle (tests only).

Nothing here is shared with the oracle or the HIP path: O(N^2) loops, exact
rational arithmetic for the FP32 neighbour predicate, a geometric (not
key-based) recursive octree and the direct-summation gravity.
"""
from fractions import Fraction

import numpy as np


def round_f32(x: Fraction) -> float:
    """Round an exact rational to the nearest float32 (ties to even)."""
    if x == 0:
        return 0.0
    s = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    # normalise so that 2^23 <= a / 2^(e-23) < 2^24
    while a >= Fraction(2) ** (e + 1):
        e += 1
    while a < Fraction(2) ** e:
        e -= 1
    scale = Fraction(2) ** (e - 23)
    q = round(a / scale)  # Fraction.__round__ rounds half to even
    return float(np.float32(s * q * scale))


def fmaf(a, b, c) -> float:
    return round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def pred_f32(xi, xj, H) -> bool:
    """Exact FP32 neighbour predicate: fl32 differences, two fmaf, r2 < fl32(H*H)."""
    d = [np.float32(np.float32(xj[a]) - np.float32(xi[a])) for a in range(3)]
    dxx = np.float32(d[0] * d[0])
    r2 = fmaf(d[2], d[2], fmaf(d[1], d[1], dxx))
    hf = np.float32(H)
    return r2 < float(np.float32(hf * hf))


def neighbour_sets(pos, h, targets, candidates, symmetric=False, exclude_self=False):
    """{i: set(j)} under the FP32 predicate; exact arithmetic near the boundary."""
    p32 = pos.astype(np.float32)
    h32 = np.asarray(h, np.float32)
    out = {}
    cand = np.asarray(candidates)
    for i in targets:
        d = (p32[cand] - p32[i]).astype(np.float64)
        r2 = (d * d).sum(1)
        H = np.maximum(h32[i], h32[cand]) if symmetric else np.full(cand.size, h32[i])
        H2 = (H.astype(np.float32) * H.astype(np.float32)).astype(np.float64)
        clear_in = r2 < H2 * (1 - 1e-5)
        border = np.abs(r2 - H2) <= H2 * 1e-5
        s = set(int(j) for j in cand[clear_in])
        for k in np.nonzero(border)[0]:
            j = int(cand[k])
            if pred_f32(pos[i], pos[j], H[k]):
                s.add(j)
        if exclude_self:
            s.discard(int(i))
        out[int(i)] = s
    return out


def geometric_tree(pos, box, leaf, ids=None, max_level=21):
    """Preorder [(level, frozenset(ids))] of the recursive cube subdivision.

    A cube [lo, lo + l)^3 is split into its 8 half-open octants, octant
    order = 4*(x upper) + 2*(y upper) + (z upper); a cube is split while it
    holds more than ``leaf`` particles and its level is below max_level."""
    if ids is None:
        ids = np.arange(pos.shape[0])
    out = []

    def rec(lo, l, level, members):
        out.append((level, frozenset(int(i) for i in members)))
        if len(members) <= leaf or level >= max_level:
            return
        half = l / 2.0
        for o in range(8):
            off = np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1], float) * half
            clo = lo + off
            x = pos[members]
            inside = np.all((x >= clo) & (x < clo + half), axis=1)
            sub = members[inside]
            if sub.size:
                rec(clo, half, level + 1, sub)

    if len(ids):
        rec(np.asarray(box[:3], float), float(box[3]), 0, np.asarray(ids))
    return out


def direct_gravity(pos, mass, eps, G=1.0, targets=None):
    """Direct O(N^2) softened gravity: acc [N,3], pot [N] (j != i)."""
    n = pos.shape[0]
    targets = np.arange(n) if targets is None else np.asarray(targets)
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    for i in targets:
        x = pos[i] - pos
        s2 = (x * x).sum(1) + eps * eps
        inv = 1.0 / np.sqrt(s2)
        inv[i] = 0.0
        acc[i] = -(G * mass * inv ** 3) @ x
        pot[i] = -(G * mass * inv).sum()
    return acc, pot
