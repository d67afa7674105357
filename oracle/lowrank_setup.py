"""Setup-side low-rank arithmetic for the fill-in blocks (oracle).

Test infrastructure: only the tests and the benchmark's CPU study call it;
the GPU path never does.

Sec. 3.4 compresses the fill-in blocks of the scaling coefficients, and the
setup-cost argument (abstract; Sec. 4, Eq. 41-42) counts them as compressed.
This module moves the compression into the elimination. When step k is
reached, every fill-in block W_kj of row k (j in S_k, not a near-field pair)
has received all its updates. It is compressed by ACA + re-compression at
fill_tol. If the low-rank form saves storage (r (b_k + b_j) < b_k b_j), the
block is replaced by U V for everything that follows:

* its coefficient is alpha_kj = (-W_kk^-1 U) V, kept in that factored form;
* the Schur updates of step k read U V.

The arithmetic here is the plain definition: dense products of the replaced
blocks. ``factored_flops`` counts what the factored evaluation of the same
products costs.

Exactness. Z_kj enters the elimination only through W_kj, because the
pivot rows of earlier steps never read it. For a fill-in pair, Z_kj = 0.
Replacing W_kj by W_kj + Delta_kj at step k is therefore the exact
elimination of Z_N + Delta, where Delta holds Delta_kj at (k, j) and
Delta_kj^T at (j, k) for every replaced block. So P^-1 = (Z_N + Delta)^-1
holds exactly, and the tests pin it.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .aca import aca_dense
from .hmatrix import HMatrix
from .schur import Precond, initial_blocks
from .symbolic import Symbolic


def precond_setup_lowrank(hm: HMatrix, sym: Symbolic, fill_tol: float):
    """The elimination with fill-in blocks compressed as they become final.

    Returns (pc, delta): pc holds D, the dense alpha (alpha of the replaced
    blocks included) and pc.lowrank[(k, j)] = (-W_kk^-1 U, V) for every
    replaced block; delta[(k, j)] = U V - W_kj, in the new numbering."""
    W, size = initial_blocks(hm, sym)
    nb = sym.nb
    start = np.array([hm.tree.start[hm.tree.leaf_box[int(o)]] for o in sym.order], dtype=np.int64)
    D, Dlu, alpha, lowrank, piv, delta = [], [], {}, {}, {}, {}
    for k in range(nb):
        Wkk = W.pop((k, k))
        lu = sla.lu_factor(Wkk, check_finite=True)
        D.append(Wkk)
        Dlu.append(lu)
        S = sym.rows[k]
        if fill_tol > 0:
            for j, orig in zip(S, sym.orig[k]):
                if orig:
                    continue
                A = W[(k, j)]
                U, V, p = aca_dense(A, fill_tol)
                piv[(k, j)] = p
                bk, bj = A.shape
                if U.shape[1] * (bk + bj) < bk * bj:
                    At = U @ V
                    delta[(k, j)] = At - A
                    W[(k, j)] = At
                    lowrank[(k, j)] = (-sla.lu_solve(lu, U), V)
        for j in S:
            alpha[(k, j)] = -sla.lu_solve(lu, W[(k, j)])
        for a, i in enumerate(S):
            Wki_T = W[(k, i)].T
            for j in S[a:]:
                W[(i, j)] += Wki_T @ alpha[(k, j)]
        for j in S:
            del W[(k, j)]
    pc = Precond(sym=sym, seg=None, start=start, size=size, D=D, Dlu=Dlu, alpha=alpha,
                 lowrank=lowrank, fill_piv=piv)
    return pc, delta


def perturbation_matvec(pc: Precond, delta: dict, v: np.ndarray) -> np.ndarray:
    """Delta v for vectors in tree order (N or N x s): Delta_kj at block
    (k, j) and Delta_kj^T at (j, k)."""
    out = np.zeros_like(v, dtype=np.complex128)
    st, sz = pc.start, pc.size

    def seg(k):
        return slice(int(st[k]), int(st[k] + sz[k]))

    for (k, j), E in delta.items():
        out[seg(k)] += E @ v[seg(j)]
        out[seg(j)] += E.T @ v[seg(k)]
    return out


def factored_flops(pc: Precond) -> dict:
    """Real flops of the elimination (complex multiply-add = 8).

    dense: every block dense. Per step: (8/3) b_k^3 for the inversion,
      8 b_k^2 b_j per coefficient block, 8 b_i b_k b_j per update pair i <= j.
    factored: the replaced blocks enter in factored form. Let w_j = r_j for a
      replaced block and b_j otherwise.
      * A coefficient block costs 8 b_k^2 w_j.
      * Compressing a fill-in block is counted as 8 (2 r^2 (b_k + b_j) + r^3),
        whether or not it is replaced.
      * An update pair costs a core product of 8 w_i b_k w_j. When a replaced
        operand takes part, it also costs the cheaper expansion order back to
        b_i x b_j.
    """
    nb = pc.nb
    b = [int(x) for x in pc.size]
    dense = fact = 0.0
    for k in range(nb):
        bk = b[k]
        S = pc.sym.rows[k]
        r = {}
        for j, orig in zip(S, pc.sym.orig[k]):
            if (k, j) in pc.lowrank:
                r[j] = pc.lowrank[(k, j)][0].shape[1]
            if not orig and (k, j) in pc.fill_piv:
                rc = len(pc.fill_piv[(k, j)])
                fact += 8.0 * (2.0 * rc * rc * (bk + b[j]) + rc ** 3)
        w = {j: r.get(j, b[j]) for j in S}
        dense += 8.0 / 3.0 * bk ** 3
        fact += 8.0 / 3.0 * bk ** 3
        for j in S:
            dense += 8.0 * bk * bk * b[j]
            fact += 8.0 * bk * bk * w[j]
        for a, i in enumerate(S):
            for j in S[a:]:
                dense += 8.0 * b[i] * bk * b[j]
                fact += 8.0 * w[i] * bk * w[j]
                li, lj = i in r, j in r
                if li and lj:
                    fact += 8.0 * min(b[i] * r[i] * r[j] + b[i] * r[j] * b[j],
                                      r[i] * r[j] * b[j] + b[i] * r[i] * b[j])
                elif li:
                    fact += 8.0 * b[i] * r[i] * b[j]
                elif lj:
                    fact += 8.0 * b[i] * r[j] * b[j]
    return {"dense": dense, "factored": fact}
