"""Adaptive cross approximation and SVD re-compression (oracle).

Sec. 2, Eq. 9-10: an m x n block is approximated by U (m x r) V (r x n)
with || Z_sub - U V ||_F <= eps || Z_sub ||_F; the ACA factors are then
re-compressed by extracting the orthogonal parts of U and V and applying an
SVD (the text after Eq. 10). The cited ACA papers are not available, so the
standard partial-pivoting ACA is used, with this reading:

* first row pivot: local row 0;
* residual row R = A[i, :] - sum_l U[i, l] V[l, :];
* column pivot j = argmax over unused columns of |R[j]|^2 (computed as
  re*re + im*im; ties go to the lowest index);
* if that maximum is exactly zero, row i is marked used and the lowest
  unused row is tried next; with no rows left the loop ends;
* v = R / R[j]; u = A[:, j] - sum_l U[:, l] V[l, j];
* ||A_k||_F^2 is updated with the cross terms 2 Re((u_l^H u)(v v_l^H));
* stop when ||u|| ||v|| <= eps ||A_k||_F or k = min(m, n);
* next row pivot = argmax over unused rows of |u[i]|^2.

Re-compression: QR(U) = Q_U R_U, QR(V^T) = Q_V R_V, SVD of R_U R_V^T =
W S X^H; keep the smallest r' with sqrt(sum_{i > r'} s_i^2) <= eps ||s||_2;
U' = Q_U W_r' S_r', V' = X_r'^H Q_V^T.

Pinned in the tests: an exactly rank-r matrix is recovered at rank r to
rounding; on kernel blocks the stop rule holds exactly at the last term, and
the true error against the dense block is within eps for the median block
and within 5 eps for all (the stop test only estimates the Eq. 10 error);
the re-compressed product equals the truncated SVD of U V computed directly.
"""
from __future__ import annotations

from typing import Callable

import numpy as np


def _abs2(z: np.ndarray) -> np.ndarray:
    return z.real * z.real + z.imag * z.imag


def aca(get_row: Callable[[int], np.ndarray], get_col: Callable[[int], np.ndarray],
        m: int, n: int, eps: float, max_rank: int | None = None):
    """Partial-pivoting ACA.

    Returns (U m x r, V r x n, pivots list of (i, j), ||U V||_F^2 estimate
    accumulated by the incremental update)."""
    rmax = min(m, n) if max_rank is None else min(m, n, max_rank)
    us, vs, piv = [], [], []
    row_used = np.zeros(m, dtype=bool)
    col_used = np.zeros(n, dtype=bool)
    norm2 = 0.0
    i = 0
    while len(us) < rmax:
        row = np.array(get_row(i), dtype=np.complex128)
        for u_l, v_l in zip(us, vs):
            row -= u_l[i] * v_l
        row_used[i] = True
        mag = np.where(col_used, -1.0, _abs2(row))
        j = int(np.argmax(mag))
        if mag[j] <= 0.0:
            free = np.flatnonzero(~row_used)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = row / row[j]
        u = np.array(get_col(j), dtype=np.complex128)
        for u_l, v_l in zip(us, vs):
            u -= v_l[j] * u_l
        col_used[j] = True
        nu2 = float(np.vdot(u, u).real)
        nv2 = float(np.vdot(v, v).real)
        cross = 0.0
        for u_l, v_l in zip(us, vs):
            cross += (np.vdot(u_l, u) * np.vdot(v_l, v)).real
        norm2 += nu2 * nv2 + 2.0 * cross
        us.append(u)
        vs.append(v)
        piv.append((i, j))
        if np.sqrt(nu2 * nv2) <= eps * np.sqrt(max(norm2, 0.0)):
            break
        if len(us) >= rmax:
            break
        magu = np.where(row_used, -1.0, _abs2(u))
        if not np.any(~row_used):
            break
        i = int(np.argmax(magu))
    r = len(us)
    U = np.stack(us, axis=1) if r else np.zeros((m, 0), dtype=np.complex128)
    V = np.stack(vs, axis=0) if r else np.zeros((0, n), dtype=np.complex128)
    return U, V, piv, norm2


def recompress(U: np.ndarray, V: np.ndarray, eps: float):
    """QR + SVD re-compression of U V at relative Frobenius tolerance eps."""
    m, r = U.shape
    if r == 0:
        return U, V
    qu, ru = np.linalg.qr(U)
    qv, rv = np.linalg.qr(V.T)
    core = ru @ rv.T
    w, s, xh = np.linalg.svd(core)
    tot = float(np.sqrt(np.sum(s * s)))
    # tail[i] = sqrt(sum_{l >= i} s_l^2); keep the smallest r' with tail[r'] <= eps * tot
    tail = np.sqrt(np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]]))
    rp = int(np.argmax(tail <= eps * tot))
    Un = qu @ (w[:, :rp] * s[None, :rp])
    Vn = xh[:rp, :] @ qv.T
    return Un, Vn


def aca_dense(A: np.ndarray, eps: float):
    """ACA plus re-compression of a stored dense matrix (fill-in blocks)."""
    m, n = A.shape
    U, V, piv, _ = aca(lambda i: A[i, :], lambda j: A[:, j], m, n, eps)
    Un, Vn = recompress(U, V, eps)
    return Un, Vn, piv
