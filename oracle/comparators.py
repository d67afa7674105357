"""Comparators for the solve (oracle): a block-Jacobi preconditioner and a
coupled block GMRES.

The paper compares its preconditioner with Null-Field and ILUT
preconditioners (Sec. 5.2, Table 7) and solves the right-hand sides one by
one (Eq. 46). Neither comparator is available here, so two plain stand-ins
are used:

* block Jacobi: P^-1 = blockdiag(Z_kk)^-1 over the leaves' own near blocks
  (no coupling between leaves), the preconditioner the Schur method reduces
  to when no leaf has a near neighbour;
* coupled block GMRES(m): one Krylov space shared by the s right-hand sides,
  right-preconditioned. Reading of its steps: R = B - Z X, R = V_0 S (QR);
  per step W = Z P^-1 V_j, block classical Gram-Schmidt applied twice
  against V_0 .. V_j (H_ij = V_i^H W), W = V_{j+1} H_{j+1,j} (QR); the block
  Hessenberg least-squares problem min || E_1 S - H Y ||_F is solved column
  by column; inside a cycle it stops once every column's least-squares
  residual is within tol of its ||b||; at the end of a cycle
  X += P^-1 (V Y) and the true residual is recomputed. Steps count block
  steps (each applies Z and P^-1 to s vectors).

Pinned in the tests: block Jacobi equals the dense solve with the block
diagonal of Z_N; block GMRES with s = 1 gives the oracle GMRES's iterates,
and on a small system it reaches the dense solution within ceil(N / s)
block steps.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla


@dataclass
class BlockJacobi:
    seg: list          # (start, stop) of each leaf in tree order
    lu: list


def block_jacobi_setup(hm) -> BlockJacobi:
    diag = {int(i): B for (i, j), B in zip(hm.part.near, hm.near_blocks) if i == j}
    segs, lus = [], []
    for leaf in range(hm.tree.nb):
        segs.append(hm.leaf_range(leaf))
        lus.append(sla.lu_factor(diag[leaf]))
    return BlockJacobi(seg=segs, lu=lus)


def block_jacobi_apply(bj: BlockJacobi, v: np.ndarray) -> np.ndarray:
    out = np.empty_like(np.asarray(v, dtype=np.complex128))
    for (a, b), lu in zip(bj.seg, bj.lu):
        out[a:b] = sla.lu_solve(lu, v[a:b])
    return out


@dataclass
class BlockStats:
    steps: int
    relres: np.ndarray     # true relative residual per column
    converged: bool


def _block_qr(W: np.ndarray):
    Q, R = np.linalg.qr(W)
    return Q, R


def block_gmres(matvec, precond, B: np.ndarray, restart: int, tol: float, max_steps: int = 5000,
                fixed_steps: int | None = None):
    """Coupled block GMRES(restart) for Z X = B (N x s); returns (X, BlockStats)."""
    B = np.asarray(B, dtype=np.complex128)
    n, s = B.shape
    bn = np.linalg.norm(B, axis=0)
    X = np.zeros_like(B)
    budget = max_steps if fixed_steps is None else fixed_steps
    steps = 0
    R = B.copy()
    while True:
        V0, S = _block_qr(R)
        Vs = [V0]
        Hb = np.zeros(((restart + 1) * s, restart * s), dtype=np.complex128)
        k = 0
        Y = None
        while k < restart and steps < budget:
            W = matvec(precond(Vs[k]))
            Vall = np.concatenate(Vs, axis=1)
            h = Vall.conj().T @ W
            W = W - Vall @ h
            h2 = Vall.conj().T @ W
            W = W - Vall @ h2
            h = h + h2
            Vn, Hn = _block_qr(W)
            Hb[:(k + 1) * s, k * s:(k + 1) * s] = h
            Hb[(k + 1) * s:(k + 2) * s, k * s:(k + 1) * s] = Hn
            Vs.append(Vn)
            k += 1
            steps += 1
            rhs = np.zeros(((k + 1) * s, s), dtype=np.complex128)
            rhs[:s] = S
            Hk = Hb[:(k + 1) * s, :k * s]
            Y, *_ = np.linalg.lstsq(Hk, rhs, rcond=None)
            ls = np.linalg.norm(rhs - Hk @ Y, axis=0)
            if fixed_steps is None and np.all(ls <= tol * bn):
                break
        if Y is None:
            break
        Vall = np.concatenate(Vs[:k], axis=1)
        X = X + precond(Vall @ Y)
        R = B - matvec(X)
        rel = np.linalg.norm(R, axis=0) / np.where(bn > 0, bn, 1.0)
        if steps >= budget or (fixed_steps is None and np.all(rel <= tol)):
            return X, BlockStats(steps, rel, bool(np.all(rel <= tol)))
