"""End-to-end oracle: h_build, precond_setup, solve.

Z x = b with Z the complex-symmetric H-matrix of Eq. 11 and the symmetric
near-field Schur-complement preconditioner of Sec. 3 as P^-1 in
right-preconditioned GMRES. Vectors come and go in the user's point order;
the permutation to tree order is internal.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import gmres as _gmres
from . import hmatrix as _hm
from . import ordering as _ord
from . import schur as _schur
from . import symbolic as _sym


@dataclass
class Solved:
    x: np.ndarray
    stats: list


def h_build(points, k, h, leaf_max, aca_tol=1e-4):
    return _hm.h_build(points, k, h, leaf_max, aca_tol)


def precond_setup(hm, ordering="rcm", fill_tol=1e-2):
    order = _ord.make_order(ordering, hm.tree.nb, hm.part.near)
    sym = _sym.symbolic(hm.tree.nb, hm.part.near, order)
    return _schur.precond_setup(hm, sym, fill_tol)


def solve(hm, pc, b, restart=30, tol=1e-6, max_iters=5000, fixed_iters=None):
    """Solve for each column of b (user order). pc=None: unpreconditioned."""
    b = np.asarray(b, dtype=np.complex128)
    single = b.ndim == 1
    B = b[:, None] if single else b
    perm = hm.tree.perm
    X = np.zeros_like(B)
    stats = []
    mv = lambda v: _hm.matvec(hm, v)  # noqa: E731
    pre = (lambda v: _schur.apply(pc, v)) if pc is not None else (lambda v: v)  # noqa: E731
    for c in range(B.shape[1]):
        bt = B[perm, c]
        xt, st = _gmres.gmres(mv, pre, bt, restart, tol, max_iters, fixed_iters)
        X[perm, c] = xt
        stats.append(st)
    return Solved(x=X[:, 0] if single else X, stats=stats)
