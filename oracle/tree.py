"""Octree decomposition (oracle).

Sec. 2 of the paper groups the unknowns with an oct-tree, splitting each box
until it holds no more than the leaf size, and Sec. 4 counts leaves as
8^L boxes of a recursively bisected cube. The paper does not fix the root
box, the split plane or how ties are broken, so this module takes the
following reading (also used by the GPU library's host code):

* Root cube: per axis lo = min, hi = max; E = max over axes of (hi - lo);
  centre c = (lo + hi) / 2; origin o = c - E / 2.
* Quantisation to 21 bits per axis in IEEE double without fused
  multiply-add: q = clamp(floor((p - o) * (2^21 / E)), 0, 2^21 - 1).
* Morton key: bit i of qx, qy, qz goes to key bit 3i, 3i+1, 3i+2.
* Tree order: stable sort by (key, original index).
* A box is split iff it holds more than ``leaf_max`` points and its level
  is below 21; children come in octant order (the next three key bits) and
  empty children are dropped. Boxes are numbered in depth-first preorder,
  leaves in the same order.

Pinned in the tests by brute force: every point lies in exactly one leaf,
every leaf holds at most ``leaf_max`` points (or sits at depth 21), and each
box's points all share its Morton prefix. The bit order of the key and the
centring of the root cube are pinned by hand-computed values.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LEVELS = 21
QMAX = (1 << LEVELS) - 1


@dataclass
class Tree:
    perm: np.ndarray        # tree position -> user index (int64, N)
    keys: np.ndarray        # Morton keys in tree order (int64)
    q: np.ndarray           # quantised coordinates in tree order (N x 3 int64)
    level: np.ndarray       # per box (preorder)
    start: np.ndarray       # first tree position of each box
    count: np.ndarray       # number of points of each box
    anchor: np.ndarray      # integer anchor (nbox x 3) = q >> (21 - level)
    parent: np.ndarray      # preorder id of the parent (-1 for the root)
    children: list          # list of child-id lists per box
    leaf_id: np.ndarray     # leaf number of a box, -1 for internal boxes
    leaf_box: np.ndarray    # box id of each leaf (nb)

    @property
    def nbox(self) -> int:
        return int(self.level.shape[0])

    @property
    def nb(self) -> int:
        return int(self.leaf_box.shape[0])

    def leaf_offsets(self) -> np.ndarray:
        """Tree-order offsets of the leaves, length nb + 1."""
        s = self.start[self.leaf_box]
        return np.concatenate([s, [self.start[0] + self.count[0]]]).astype(np.int64)


def quantise(points: np.ndarray) -> np.ndarray:
    """Integer coordinates on the 2^21 grid of the root cube."""
    p = np.asarray(points, dtype=np.float64)
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    ext = float(np.max(hi - lo))
    if not ext > 0.0:
        raise ValueError("points span no volume: the root box has zero extent")
    c = (lo + hi) / 2.0
    o = c - ext / 2.0
    scale = float(1 << LEVELS) / ext
    t = (p - o[None, :]) * scale
    q = np.floor(t)
    q = np.clip(q, 0, QMAX).astype(np.int64)
    return q


def morton(q: np.ndarray) -> np.ndarray:
    """Interleave the 21 bits of each coordinate into a 63-bit key."""
    key = np.zeros(q.shape[0], dtype=np.int64)
    for i in range(LEVELS):
        for ax in range(3):
            bit = (q[:, ax] >> i) & 1
            key |= bit << (3 * i + ax)
    return key


def build_tree(points: np.ndarray, leaf_max: int) -> Tree:
    if leaf_max < 1:
        raise ValueError("leaf_max must be >= 1")
    q_user = quantise(points)
    key_user = morton(q_user)
    n = key_user.shape[0]
    perm = np.lexsort((np.arange(n), key_user))   # key first, index breaks ties
    keys = key_user[perm]
    q = q_user[perm]

    level, start, count, anchor, parent, children, leaf_id, leaf_box = ([] for _ in range(8))

    def visit(lvl: int, s: int, c: int, par: int) -> int:
        bid = len(level)
        level.append(lvl)
        start.append(s)
        count.append(c)
        anchor.append(tuple(int(x) >> (LEVELS - lvl) for x in q[s]))
        parent.append(par)
        children.append([])
        leaf_id.append(-1)
        if c > leaf_max and lvl < LEVELS:
            shift = 3 * (LEVELS - lvl - 1)
            oct_ = (keys[s:s + c] >> shift) & 7
            for o in range(8):
                lo = int(np.searchsorted(oct_, o, side="left"))
                hi = int(np.searchsorted(oct_, o, side="right"))
                if hi > lo:
                    cid = visit(lvl + 1, s + lo, hi - lo, bid)
                    children[bid].append(cid)
        else:
            leaf_id[bid] = len(leaf_box)
            leaf_box.append(bid)
        return bid

    visit(0, 0, n, -1)
    return Tree(perm=perm.astype(np.int64), keys=keys, q=q,
                level=np.array(level, dtype=np.int64),
                start=np.array(start, dtype=np.int64),
                count=np.array(count, dtype=np.int64),
                anchor=np.array(anchor, dtype=np.int64).reshape(-1, 3),
                parent=np.array(parent, dtype=np.int64),
                children=children,
                leaf_id=np.array(leaf_id, dtype=np.int64),
                leaf_box=np.array(leaf_box, dtype=np.int64))
