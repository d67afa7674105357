"""Symmetric near-field Schur-complement elimination and its apply (oracle).

Sec. 3.1 scales the near field Z_N to block-diagonal form one leaf row at a
time: the right scaling coefficients of row k are alpha_kj = -Z_kk^-1 Z_kj
(Eq. 14), the left ones alpha'_ik = -Z_ik Z_kk^-1 (Eq. 16), and one step
leaves the Schur complement Z_ij - Z_ik Z_kk^-1 Z_kj on the later blocks
(Eq. 19). Repeating it for every row gives the block-diagonal
Z~_N = alpha'^T ... Z_N ... alpha (Eq. 20-21). Sec. 3.2: for a complex
symmetric Z_N, alpha'_k is the plain transpose of alpha_k, so only alpha is
computed and the update reads W_ij += W_ki^T alpha_kj.

The elimination runs in the order of Algorithm 1 over the filled pattern S_k
(module ``symbolic``). Fill-in blocks of alpha (pairs that are not near-field
neighbours, Sec. 3.4) are compressed afterwards with ACA + re-compression
at ``fill_tol`` and kept low-rank iff r (b_k + b_j) < b_k b_j; the Schur
updates themselves always use the dense alpha.

Apply (Eq. 23, 24 and 28 used as a right preconditioner):
P^-1 v = alpha D^-1 alpha^T v, i.e. a forward sweep y_j += alpha_kj^T y_k
(k ascending), the block-diagonal solve z_k = D_k^-1 y_k, and a backward
sweep z_k += sum_j alpha_kj z_j (k descending).

Pinned in the tests: D_k and alpha_kj equal the dense block elimination of
the dense Z_N; with fill_tol = 0, P^-1 v equals Z_N^-1 v for every ordering
(the block LDL^T identity Z_N = alpha^-T D alpha^-1); the non-symmetric
variant's alpha' equals alpha^T; D_k is symmetric.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .aca import aca_dense
from .hmatrix import HMatrix
from .symbolic import Symbolic


@dataclass
class Precond:
    sym: Symbolic
    seg: np.ndarray            # tree-order offset of block k (new numbering), nb + 1 entries
    # per block k: tree-order start and size
    start: np.ndarray
    size: np.ndarray
    D: list                    # final W_kk (the scaled block-diagonal Z~_N)
    Dlu: list                  # LU factors of D_k
    alpha: dict                # (k, j) -> dense alpha_kj
    lowrank: dict = field(default_factory=dict)   # (k, j) -> (U, V) for compressed fill-ins
    fill_piv: dict = field(default_factory=dict)  # (k, j) -> ACA pivot log of fill-in compression

    @property
    def nb(self) -> int:
        return self.sym.nb


def _near_lookup(hm: HMatrix):
    return {(int(i), int(j)): B for (i, j), B in zip(hm.part.near, hm.near_blocks)}


def initial_blocks(hm: HMatrix, sym: Symbolic):
    """W_kj (k <= j, new numbering) from Z_N; fill blocks start at zero."""
    near = _near_lookup(hm)
    order = sym.order
    size = np.array([hm.tree.count[hm.tree.leaf_box[int(o)]] for o in order], dtype=np.int64)
    W = {}
    for k in range(sym.nb):
        ok = int(order[k])
        W[(k, k)] = near[(ok, ok)].copy()
        for j in sym.rows[k]:
            oj = int(order[j])
            if (ok, oj) in near:
                W[(k, j)] = near[(ok, oj)].copy()
            elif (oj, ok) in near:
                W[(k, j)] = near[(oj, ok)].T.copy()
            else:
                W[(k, j)] = np.zeros((size[k], size[j]), dtype=np.complex128)
    return W, size


def precond_setup(hm: HMatrix, sym: Symbolic, fill_tol: float) -> Precond:
    W, size = initial_blocks(hm, sym)
    nb = sym.nb
    start = np.array([hm.tree.start[hm.tree.leaf_box[int(o)]] for o in sym.order], dtype=np.int64)
    D, Dlu, alpha = [], [], {}
    for k in range(nb):
        Wkk = W.pop((k, k))
        lu = sla.lu_factor(Wkk, check_finite=True)
        D.append(Wkk)
        Dlu.append(lu)
        S = sym.rows[k]
        for j in S:
            alpha[(k, j)] = -sla.lu_solve(lu, W[(k, j)])
        for a, i in enumerate(S):
            Wki_T = W[(k, i)].T
            for j in S[a:]:
                W[(i, j)] += Wki_T @ alpha[(k, j)]
        for j in S:
            del W[(k, j)]
    pc = Precond(sym=sym, seg=None, start=start, size=size, D=D, Dlu=Dlu, alpha=alpha)
    if fill_tol > 0:
        compress_fill(pc, fill_tol)
    return pc


def compress_fill(pc: Precond, fill_tol: float) -> None:
    """ACA + re-compression of the fill-in blocks of alpha (Sec. 3.4)."""
    for k in range(pc.nb):
        for j, o in zip(pc.sym.rows[k], pc.sym.orig[k]):
            if o:
                continue
            A = pc.alpha[(k, j)]
            U, V, piv = aca_dense(A, fill_tol)
            r = U.shape[1]
            bk, bj = A.shape
            pc.fill_piv[(k, j)] = piv
            if r * (bk + bj) < bk * bj:
                pc.lowrank[(k, j)] = (U, V)


def _alpha_T_mul(pc: Precond, k: int, j: int, y: np.ndarray) -> np.ndarray:
    if (k, j) in pc.lowrank:
        U, V = pc.lowrank[(k, j)]
        return V.T @ (U.T @ y)
    return pc.alpha[(k, j)].T @ y


def _alpha_mul(pc: Precond, k: int, j: int, z: np.ndarray) -> np.ndarray:
    if (k, j) in pc.lowrank:
        U, V = pc.lowrank[(k, j)]
        return U @ (V @ z)
    return pc.alpha[(k, j)] @ z


def apply(pc: Precond, v: np.ndarray) -> np.ndarray:
    """P^-1 v = alpha D^-1 alpha^T v, vectors in tree order (N or N x s)."""
    y = np.array(v, dtype=np.complex128, copy=True)
    st, sz = pc.start, pc.size

    def seg(k):
        return slice(int(st[k]), int(st[k] + sz[k]))

    for k in range(pc.nb):
        yk = y[seg(k)]
        for j in pc.sym.rows[k]:
            y[seg(j)] += _alpha_T_mul(pc, k, j, yk)
    z = np.empty_like(y)
    for k in range(pc.nb):
        z[seg(k)] = sla.lu_solve(pc.Dlu[k], y[seg(k)])
    for k in range(pc.nb - 1, -1, -1):
        acc = z[seg(k)].copy()
        for j in pc.sym.rows[k]:
            acc += _alpha_mul(pc, k, j, z[seg(j)])
        z[seg(k)] = acc
    return z


def nonsymmetric_alpha_prime(hm: HMatrix, sym: Symbolic) -> dict:
    """Non-symmetric Schur elimination computing the left coefficients
    alpha'_ik = -W_ik W_kk^-1 separately (the comparator of Table 2); used
    only to check that alpha' = alpha^T for a symmetric near field."""
    Wu, size = initial_blocks(hm, sym)
    W = {}
    for (k, j), B in Wu.items():
        W[(k, j)] = B
        if k != j:
            W[(j, k)] = B.T.copy()
    ap = {}
    for k in range(sym.nb):
        Wkk = W[(k, k)]
        inv = np.linalg.inv(Wkk)
        S = sym.rows[k]
        al = {j: -inv @ W[(k, j)] for j in S}
        for i in S:
            ap[(i, k)] = -W[(i, k)] @ inv
        for i in S:
            for j in S:
                W[(i, j)] = W[(i, j)] + W[(i, k)] @ al[j]
    return ap
