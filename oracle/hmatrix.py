"""H-matrix build and matvec (oracle).

Eq. 11 splits Z into the dense leaf-level near field Z_N and the compressed
far field Z_F. This module assembles Z_N on the kept near pairs (i <= j; the
lower blocks are transposes, the kernel being symmetric) and compresses
every kept far pair with ACA plus re-compression (Eq. 9-10). Vectors are in
tree order.

The matvec is the plain definition of Z_H x on the stored blocks:
near y_i += Z_ij x_j and, for i != j, y_j += Z_ij^T x_i; far
y_t += U (V x_s) and y_s += V^T (U^T x_t).

Pinned in the tests: with a tiny ACA tolerance, Z_H x equals the dense
kernel matrix times x; u^T Z_H v = v^T Z_H u (complex symmetry, Sec. 3.2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .aca import aca, recompress
from .kernel import kernel_block, kernel_row
from .partition import Partition, build_partition
from .tree import Tree, build_tree


@dataclass
class HMatrix:
    tree: Tree
    part: Partition
    pts: np.ndarray          # points in tree order
    k: float
    h: float
    near_blocks: list        # dense Z_ij for each near pair (i <= j)
    far_u: list              # U factors per far pair
    far_v: list              # V factors per far pair
    far_piv: list            # ACA pivot logs per far pair
    far_rank_aca: list       # ACA rank before re-compression

    @property
    def n(self) -> int:
        return int(self.pts.shape[0])

    def leaf_range(self, leaf: int):
        b = self.tree.leaf_box[leaf]
        s = int(self.tree.start[b])
        return s, s + int(self.tree.count[b])

    def box_range(self, box: int):
        s = int(self.tree.start[box])
        return s, s + int(self.tree.count[box])


def h_build(points: np.ndarray, k: float, h: float, leaf_max: int, aca_tol: float,
            with_far: bool = True) -> HMatrix:
    """Build Z_H; ``with_far=False`` assembles the near field only (Z_N)."""
    tree = build_tree(points, leaf_max)
    part = build_partition(tree)
    pts = np.asarray(points, dtype=np.float64)[tree.perm]
    hm = HMatrix(tree=tree, part=part, pts=pts, k=k, h=h, near_blocks=[], far_u=[],
                 far_v=[], far_piv=[], far_rank_aca=[])
    for i, j in part.near:
        a0, a1 = hm.leaf_range(int(i))
        b0, b1 = hm.leaf_range(int(j))
        hm.near_blocks.append(kernel_block(pts[a0:a1], pts[b0:b1], k, h, same=(i == j)))
    for t, s in (part.far if with_far else []):
        a0, a1 = hm.box_range(int(t))
        b0, b1 = hm.box_range(int(s))
        pt, ps = pts[a0:a1], pts[b0:b1]
        U, V, piv, _ = aca(lambda i: kernel_row(pt[i], ps, k),
                           lambda j: kernel_row(ps[j], pt, k),
                           a1 - a0, b1 - b0, aca_tol)
        hm.far_rank_aca.append(U.shape[1])
        U, V = recompress(U, V, aca_tol)
        hm.far_u.append(U)
        hm.far_v.append(V)
        hm.far_piv.append(piv)
    return hm


def near_matvec(hm: HMatrix, x: np.ndarray) -> np.ndarray:
    """Z_N x in tree order (x may be N or N x s)."""
    y = np.zeros_like(x, dtype=np.complex128)
    for (i, j), Z in zip(hm.part.near, hm.near_blocks):
        a0, a1 = hm.leaf_range(int(i))
        b0, b1 = hm.leaf_range(int(j))
        y[a0:a1] += Z @ x[b0:b1]
        if i != j:
            y[b0:b1] += Z.T @ x[a0:a1]
    return y


def far_matvec(hm: HMatrix, x: np.ndarray) -> np.ndarray:
    """Z_F x in tree order."""
    y = np.zeros_like(x, dtype=np.complex128)
    for (t, s), U, V in zip(hm.part.far, hm.far_u, hm.far_v):
        a0, a1 = hm.box_range(int(t))
        b0, b1 = hm.box_range(int(s))
        y[a0:a1] += U @ (V @ x[b0:b1])
        y[b0:b1] += V.T @ (U.T @ x[a0:a1])
    return y


def matvec(hm: HMatrix, x: np.ndarray) -> np.ndarray:
    """Z_H x = Z_N x + Z_F x (Eq. 11), tree order."""
    return near_matvec(hm, x) + far_matvec(hm, x)


def dense_near(hm: HMatrix) -> np.ndarray:
    """Z_N as a dense N x N matrix in tree order (tiny N only)."""
    n = hm.n
    Z = np.zeros((n, n), dtype=np.complex128)
    for (i, j), B in zip(hm.part.near, hm.near_blocks):
        a0, a1 = hm.leaf_range(int(i))
        b0, b1 = hm.leaf_range(int(j))
        Z[a0:a1, b0:b1] = B
        Z[b0:b1, a0:a1] = B.T
    return Z


def dense_h(hm: HMatrix) -> np.ndarray:
    """Z_H as a dense matrix in tree order (tiny N only)."""
    Z = dense_near(hm)
    for (t, s), U, V in zip(hm.part.far, hm.far_u, hm.far_v):
        a0, a1 = hm.box_range(int(t))
        b0, b1 = hm.box_range(int(s))
        B = U @ V
        Z[a0:a1, b0:b1] = B
        Z[b0:b1, a0:a1] = B.T
    return Z


def dense_kernel(pts: np.ndarray, k: float, h: float) -> np.ndarray:
    """The full dense kernel matrix on points in the given order (tiny N only)."""
    return kernel_block(pts, pts, k, h, same=True)
