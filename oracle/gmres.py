"""Right-preconditioned restarted GMRES (oracle).

The paper solves with GMRES to a relative tolerance of 1e-6 (Sec. 5) and
allows the preconditioner on either side (Eq. 1-2). This oracle runs the
right-preconditioned form Z P^-1 x~ = b, x = P^-1 x~ (Eq. 2) with
P^-1 = alpha D^-1 alpha^T, so the residual it monitors is the true one of
Z x = b. Reading of the unstated details:

* x0 = 0, r0 = b; Arnoldi with classical Gram-Schmidt applied twice
  (h = V^H w; w -= V h; h2 = V^H w; w -= V h2; h += h2), Hermitian inner
  products;
* complex Givens rotations with real cosine: for (a, b) with d = sqrt(|a|^2
  + |b|^2), c = |a| / d and s = (a / |a|) conj(b) / d (c = 0, s = 1 when
  a = 0); the rotation maps (a, b) to ((a / |a|) d, 0) and g_{j+1} =
  -conj(s) g_j, g_j = c g_j;
* inside a cycle stop when |g_{j+1}| / ||b|| <= tol; at the end of each
  cycle x += P^-1 V y and the true residual b - Z x is recomputed;
* stop when the true relative residual <= tol or after ``max_iters`` inner
  steps in total; with ``fixed_iters`` the inner test is skipped so that
  both sides run the same number of steps.

Each right-hand side is an independent column. Pinned in the tests: for
P = Z (all leaves mutually near) it converges in one step; with exact
operators it reproduces numpy.linalg.solve.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class SolveStats:
    iters: int
    relres: float
    converged: bool


def givens(a: complex, b: complex):
    aa = abs(a)
    if aa == 0.0:
        return 0.0, 1.0 + 0.0j
    d = np.sqrt(aa * aa + abs(b) * abs(b))
    c = aa / d
    s = (a / aa) * np.conj(b) / d
    return c, s


def gmres(matvec, precond, b: np.ndarray, restart: int, tol: float,
          max_iters: int = 5000, fixed_iters: int | None = None):
    """Solve Z x = b for one column; returns (x, SolveStats)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n, dtype=np.complex128)
    if bnorm == 0.0:
        return x, SolveStats(0, 0.0, True)
    budget = max_iters if fixed_iters is None else fixed_iters
    total = 0
    r = b.copy()
    beta = bnorm
    relres = 1.0
    while True:
        m = restart
        V = np.zeros((n, m + 1), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        steps = 0
        for j in range(m):
            w = matvec(precond(V[:, j]))
            Vj = V[:, :j + 1]
            h = Vj.conj().T @ w
            w = w - Vj @ h
            h2 = Vj.conj().T @ w
            w = w - Vj @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            c, s = givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j] = c * H[j, j] + s * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            steps = j + 1
            total += 1
            if hn != 0.0:
                V[:, j + 1] = w / hn
            if fixed_iters is None and abs(g[j + 1]) / bnorm <= tol:
                break
            if total >= budget or hn == 0.0:
                break
        y = np.zeros(steps, dtype=np.complex128)
        for i in range(steps - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:steps] @ y[i + 1:steps]) / H[i, i]
        x = x + precond(V[:, :steps] @ y)
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        relres = beta / bnorm
        if fixed_iters is None and relres <= tol:
            return x, SolveStats(total, relres, True)
        if total >= budget or beta == 0.0:
            return x, SolveStats(total, relres, relres <= tol)
