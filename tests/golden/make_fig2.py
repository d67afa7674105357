"""Writes fig2_four_leaves.txt: a point set whose octree has four leaves with
the near-field pattern of the paper's Fig. 2 / Eq. 12 (exactly one pair of
leaves is far, all other pairs are near).

Construction: in the unit cube, leaf A sits in the octant that shares the
x = 1/2 face with octant B = [1/2, 1]^3; B holds three sub-octant groups, one
of them on B's far x side, which therefore does not touch A. The seed loop
only jitters the points inside those regions until the oracle's octree
(leaf size 4) shows the pattern. Run from the repository root.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle.partition import build_partition  # noqa: E402
from oracle.tree import build_tree  # noqa: E402


def main():
    for seed in range(5000):
        rng = np.random.default_rng(seed)
        A = np.c_[rng.uniform(0.05, 0.45, 3), rng.uniform(0.55, 0.95, 3), rng.uniform(0.55, 0.95, 3)]
        b1 = rng.uniform(0.52, 0.73, (3, 3))
        b2 = np.c_[rng.uniform(0.52, 0.73, 3), rng.uniform(0.77, 0.98, 3), rng.uniform(0.77, 0.98, 3)]
        b3 = np.c_[rng.uniform(0.77, 0.98, 3), rng.uniform(0.52, 0.73, 3), rng.uniform(0.52, 0.73, 3)]
        pts = np.concatenate([A, b1, b2, b3, [[0.0, 0.99, 0.99]], [[0.99, 1.0, 1.0]]])
        t = build_tree(pts, 4)
        p = build_partition(t)
        off = [tuple(x) for x in p.near if x[0] != x[1]]
        if t.nb == 4 and len(off) == 5:
            out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fig2_four_leaves.txt")
            np.savetxt(out, pts, fmt="%.17g",
                       header="Fig. 2 / Eq. 12 four-leaf structure (leaf size 4); seed %d" % seed)
            return
    raise SystemExit("no configuration found")


if __name__ == "__main__":
    main()
