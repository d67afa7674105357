"""The paper's literal transformed system (oracle), Sec. 3.1, Eq. 22-28.

With alpha = alpha_1 alpha_2 ... the product of the right scaling steps and
alpha' = alpha^T its left counterpart (Sec. 3.2), the system Z x = b becomes
alpha^T Z alpha x~ = alpha^T b (Eq. 22-23), x = alpha x~ (Eq. 24). Split
Z = Z_N + Z_F (Eq. 25-26): alpha^T Z_N alpha is the scaled block-diagonal
D (Eq. 20-21), so the operator is D + alpha^T Z_F alpha (Eq. 27), and D is
the preconditioner applied on the left (Eq. 28):

    x~ + D^-1 alpha^T Z_F alpha x~ = D^-1 alpha^T b.

The dense near-field matvec disappears from the iteration (the saving the
paper points out after Eq. 27). The factors are applied as sweeps:

* alpha^T v: forward, y_j += alpha_kj^T y_k for k ascending (Eq. 23);
* alpha u: backward, u_k += sum_{j in S_k} alpha_kj u_j for k descending
  (Eq. 24);
* D^-1 per block from the LU factors of D_k.

Reading: the iteration is the oracle's GMRES (CGS2, Givens, restarts) with
the identity as right preconditioner, so it monitors the residual of the
transformed left-preconditioned system; the true residual ||b - Z x|| /
||b|| of x = alpha x~ is computed at the end. alpha^T Z_N alpha = D holds
exactly only when every fill-in block is kept dense (fill_tol = 0); with
compressed fill-ins the transformed system is a perturbation of Z x = b,
and its true residual is what is reported.

Pinned in the tests: with fill_tol = 0, alpha^T Z_N alpha equals the block
diagonal of D (dense brute force on small inputs), alpha^T and alpha are the
transposes of each other as operators, and the solution equals that of the
right-preconditioned form within the residual bound.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import gmres as _gmres
from . import hmatrix as _hm
from .schur import Precond, _alpha_T_mul, _alpha_mul


def _seg(pc: Precond, k: int) -> slice:
    return slice(int(pc.start[k]), int(pc.start[k] + pc.size[k]))


def alpha_T(pc: Precond, v: np.ndarray) -> np.ndarray:
    """alpha^T v (tree order)."""
    y = np.array(v, dtype=np.complex128, copy=True)
    for k in range(pc.nb):
        yk = y[_seg(pc, k)]
        for j in pc.sym.rows[k]:
            y[_seg(pc, j)] += _alpha_T_mul(pc, k, j, yk)
    return y


def alpha(pc: Precond, u: np.ndarray) -> np.ndarray:
    """alpha u (tree order)."""
    z = np.array(u, dtype=np.complex128, copy=True)
    for k in range(pc.nb - 1, -1, -1):
        acc = z[_seg(pc, k)].copy()
        for j in pc.sym.rows[k]:
            acc += _alpha_mul(pc, k, j, z[_seg(pc, j)])
        z[_seg(pc, k)] = acc
    return z


def d_solve(pc: Precond, v: np.ndarray) -> np.ndarray:
    """D^-1 v block by block."""
    out = np.empty_like(np.asarray(v, dtype=np.complex128))
    for k in range(pc.nb):
        out[_seg(pc, k)] = sla.lu_solve(pc.Dlu[k], v[_seg(pc, k)])
    return out


def d_mul(pc: Precond, v: np.ndarray) -> np.ndarray:
    """D v block by block."""
    out = np.empty_like(np.asarray(v, dtype=np.complex128))
    for k in range(pc.nb):
        out[_seg(pc, k)] = pc.D[k] @ v[_seg(pc, k)]
    return out


def operator(hm, pc: Precond, xt: np.ndarray) -> np.ndarray:
    """x~ + D^-1 alpha^T Z_F alpha x~ (Eq. 28, left side)."""
    return xt + d_solve(pc, alpha_T(pc, _hm.far_matvec(hm, alpha(pc, xt))))


def solve(hm, pc: Precond, b: np.ndarray, restart: int = 30, tol: float = 1e-6, max_iters: int = 5000,
          fixed_iters: int | None = None):
    """Solve Eq. 28 for one right-hand side in the caller's order; returns
    (x in the caller's order, GMRES stats of the transformed system, true
    relative residual ||b - Z x|| / ||b||)."""
    perm = hm.tree.perm
    bt = np.asarray(b, dtype=np.complex128)[perm]
    rhs = d_solve(pc, alpha_T(pc, bt))
    xt, st = _gmres.gmres(lambda v: operator(hm, pc, v), lambda v: v, rhs, restart, tol, max_iters, fixed_iters)
    x_tree = alpha(pc, xt)
    res = np.linalg.norm(bt - _hm.matvec(hm, x_tree)) / max(np.linalg.norm(bt), 1e-300)
    x = np.empty_like(x_tree)
    x[perm] = x_tree
    return x, st, float(res)
