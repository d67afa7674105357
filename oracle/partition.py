"""Near / far block partition (oracle).

Sec. 2 (Eq. 8 and the text after it, Fig. 1): block pairs that satisfy the
admissibility condition are compressed (far field); the rest, at leaf level,
form the dense near field, and a pair made far at a coarse level is not
visited again below it. The workloads fix the admissibility as "near field =
adjacent leaves", so the reading here is:

* adjacent(t, s): the closed boxes touch or overlap on every axis (face, edge
  and corner contact count; a box is adjacent to itself);
* symmetric dual traversal T(t, s) from (root, root): a non-adjacent pair is
  far; two adjacent leaves are near; otherwise split both boxes if both are
  internal, else only the internal one;
* each unordered pair is kept once, oriented so that t precedes s in
  preorder (self pairs appear as (t, t)); the other orientation is its
  transpose (the point kernel is symmetric).

Output order is canonical: near pairs sorted by (leaf i, leaf j), far pairs
by (box t, box s).

Pinned in the tests by brute force: every (m, n) entry of the N x N matrix
is covered exactly once by a kept block or its transpose, and a leaf pair is
near iff the two leaves are adjacent.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .tree import LEVELS, Tree


@dataclass
class Partition:
    near: np.ndarray   # (n_near, 2) leaf ids (i <= j)
    far: np.ndarray    # (n_far, 2) box ids (t < s in preorder)


def box_bounds(tree: Tree, b: int):
    side = 1 << (LEVELS - int(tree.level[b]))
    lo = tree.anchor[b] * side
    return lo, lo + side


def adjacent(tree: Tree, t: int, s: int) -> bool:
    lt, ut = box_bounds(tree, t)
    ls, us = box_bounds(tree, s)
    return bool(np.all(lt <= us) and np.all(ls <= ut))


def build_partition(tree: Tree) -> Partition:
    near, far = [], []

    def is_leaf(b):
        return tree.leaf_id[b] >= 0

    def T(t: int, s: int):
        if t == s:
            if is_leaf(t):
                near.append((int(tree.leaf_id[t]), int(tree.leaf_id[t])))
                return
            ch = tree.children[t]
            for a in range(len(ch)):
                for b in range(a, len(ch)):
                    T(ch[a], ch[b])
            return
        if not adjacent(tree, t, s):
            far.append((t, s))
            return
        lt, ls = is_leaf(t), is_leaf(s)
        if lt and ls:
            near.append((int(tree.leaf_id[t]), int(tree.leaf_id[s])))
        elif not lt and not ls:
            for c in tree.children[t]:
                for d in tree.children[s]:
                    T(c, d)
        elif not lt:
            for c in tree.children[t]:
                T(c, s)
        else:
            for d in tree.children[s]:
                T(t, d)

    T(0, 0)
    near_a = np.array(sorted(near), dtype=np.int64).reshape(-1, 2)
    far_a = np.array(sorted(far), dtype=np.int64).reshape(-1, 2)
    return Partition(near=near_a, far=far_a)
