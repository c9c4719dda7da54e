"""Test-side helpers written independently of both the oracle and the GPU path.

They work on explicit height fields, the form in which the octahedron model is
stated (Sec. I-A): neighbouring heights differ by exactly 1 and the
generalized Kawasaki rules of Eq. (2) lift a site lying below all four
neighbours by 2 (probability p) and lower a site lying above all four by 2
(probability q).
"""
from __future__ import annotations

import numpy as np


def slopes_from_heights(h: np.ndarray):
    """sx[y,x] = 1 iff h(x,y) - h(x-1,y) = +1; sy likewise along y (periodic)."""
    dx = h - np.roll(h, 1, axis=-1)
    dy = h - np.roll(h, 1, axis=-2)
    assert np.all(np.abs(dx) == 1) and np.all(np.abs(dy) == 1), "not a valid octahedron surface"
    return (dx == 1).astype(np.uint8), (dy == 1).astype(np.uint8)


def heights_by_walk(sx: np.ndarray, sy: np.ndarray, h0: int) -> np.ndarray:
    """Heights from slopes by cumulative sums (down column 0, then along rows)."""
    ey = 2 * sy.astype(np.int64) - 1
    ex = 2 * sx.astype(np.int64) - 1
    col = np.concatenate([[0], np.cumsum(ey[1:, 0])]) + h0
    row = np.concatenate([np.zeros((sx.shape[0], 1), np.int64), np.cumsum(ex[:, 1:], axis=1)], axis=1)
    return col[:, None] + row


def height_rule_halfstep(h: np.ndarray, parity: int, acc: np.ndarray) -> np.ndarray:
    """Eq. (2) on explicit heights for the sites with (x+y)&1 == parity.

    h: [..., Y, X] int; acc: [..., Y, X] bool acceptance per site (the same bit
    serves a minimum with p and a maximum with q).  Returns new heights.
    """
    Y, X = h.shape[-2:]
    yy, xx = np.meshgrid(np.arange(Y), np.arange(X), indexing="ij")
    on = ((xx + yy) & 1) == parity
    nb = [np.roll(h, s, axis=a) for s, a in ((1, -1), (-1, -1), (1, -2), (-1, -2))]
    is_min = np.all([n == h + 1 for n in nb], axis=0)
    is_max = np.all([n == h - 1 for n in nb], axis=0)
    out = h.copy()
    out = np.where(on & is_min & acc, h + 2, out)
    out = np.where(on & is_max & acc, h - 2, out)
    return out


def enumerate_torus_surfaces(X: int, Y: int) -> np.ndarray:
    """All height fields on the X x Y torus with h(0,0) = 0 and |dh| = 1 on
    every bond, by depth-first search in row-major order."""
    sites = [(y, x) for y in range(Y) for x in range(X)]
    h = np.zeros((Y, X), np.int64)
    out = []

    def consistent(y, x, v, assigned):
        for yy, xx in (((y, (x - 1) % X)), (y, (x + 1) % X), ((y - 1) % Y, x), ((y + 1) % Y, x)):
            if (yy, xx) in assigned and abs(h[yy, xx] - v) != 1:
                return False
        return True

    def dfs(i, assigned):
        if i == len(sites):
            out.append(h.copy())
            return
        y, x = sites[i]
        ref = h[y, x - 1] if x > 0 else h[y - 1, x]
        for v in (ref - 1, ref + 1):
            if consistent(y, x, v, assigned):
                h[y, x] = v
                assigned.add((y, x))
                dfs(i + 1, assigned)
                assigned.discard((y, x))

    h[0, 0] = 0
    dfs(1, {(0, 0)})
    return np.array(out)


def site_word_bit(X: int, x, y):
    """Canonical acceptance word g and bit b of site (x,y): k = x>>1,
    g = y*W + (k>>6), b = k&63 with W = max(1, X/128)."""
    W = max(1, X // 128)
    k = np.asarray(x) >> 1
    return np.asarray(y) * W + (k >> 6), k & 63


def acceptance_grid(X: int, Y: int, xi: np.ndarray) -> np.ndarray:
    """Per-site acceptance bits [Y, X] (bool) from canonical words xi[g]."""
    yy, xx = np.meshgrid(np.arange(Y), np.arange(X), indexing="ij")
    g, b = site_word_bit(X, xx, yy)
    return ((xi[g] >> b.astype(np.uint64)) & np.uint64(1)).astype(bool)


def pattern_to_words(X: int, Y: int, parity: int, bits: np.ndarray) -> np.ndarray:
    """Canonical words whose site bits for the parity sublattice are `bits`
    [Y, X/2] (bool); bits of the other sublattice are irrelevant and left 0."""
    W = max(1, X // 128)
    xi = np.zeros(Y * W, np.uint64)
    for y in range(Y):
        for k in range(X // 2):
            if bits[y, k]:
                xi[y * W + (k >> 6)] |= np.uint64(1) << np.uint64(k & 63)
    return xi
