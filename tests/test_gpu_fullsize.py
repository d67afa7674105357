"""The HIP path at the full benchmark size: sphere + ellipsoid, N = 20,000,
leaves <= 64, ten points per wavelength (the configuration bench.py times),
checked on outputs the oracle computes one row at a time:

* H-matrix matvec: sampled rows against the dense kernel rows (Eq. 5-7); the
  error is bounded by the ACA tolerance of the far blocks (Eq. 10);
* preconditioner at fill_tol = 0: P^-1 = alpha D^-1 alpha^T is the exact
  inverse of the near-field operator Z_N (Eq. 23-24), so v - Z_N P^-1 v
  vanishes on sampled rows, with Z_N's rows from the kernel and the near
  leaf pairs;
* the benchmark solve (fill_tol = 1e-2, GMRES(50) to 1e-6) converges, with
  the true residual recomputed through a separate matvec.
"""
import numpy as np
import pytest

import workloads as W
from oracle import kernel as okern

pytestmark = pytest.mark.gpu

NS = 48   # sampled rows


@pytest.fixture(scope="module")
def full():
    import torch
    import paper_2111_13483_amd as hsl
    assert torch.cuda.is_available()
    hsl.load()
    ctx = hsl.Context(0)
    wl = W.make_config("c2", nrhs=1)
    wl.restart = 50
    H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol)
    rows = np.random.default_rng(7).choice(wl.n, NS, replace=False)
    return hsl, torch, ctx, wl, H, rows


def _dense_row(wl, i):
    """Row i of the dense operator: kernel off the diagonal, self term on it."""
    pts = wl.points
    row = np.empty(wl.n, dtype=np.complex128)
    others = np.arange(wl.n) != i
    row[others] = okern.kernel_row(pts[i], pts[others], wl.k)
    row[i] = okern.self_term(wl.k, wl.self_h)
    return row


def _near_cols(H, wl):
    """Caller-order point indices of the near field of each leaf."""
    perm = H.export("perm")
    loff = H.export("leaf_off")
    near = H.export("near").reshape(-1, 2)
    nb = len(loff) - 1
    adj = [[leaf] for leaf in range(nb)]
    for a, b in near:
        if a != b:
            adj[a].append(b)
            adj[b].append(a)
    leaf_of = np.empty(wl.n, dtype=np.int64)
    for leaf in range(nb):
        leaf_of[perm[loff[leaf]:loff[leaf + 1]]] = leaf
    cols = [np.concatenate([perm[loff[m]:loff[m + 1]] for m in adj[leaf]]) for leaf in range(nb)]
    return leaf_of, cols


def test_fullsize_matvec_sampled_rows(full):
    hsl, torch, ctx, wl, H, rows = full
    rng = np.random.default_rng(11)
    x = rng.normal(size=wl.n) + 1j * rng.normal(size=wl.n)
    y = H.matvec(torch.as_tensor(x, device="cuda")).cpu().numpy()
    leaf_of, cols = _near_cols(H, wl)
    for i in rows:
        zi = _dense_row(wl, i)
        exact = zi @ x
        # near blocks are exact; the far blocks carry a relative Frobenius
        # error <= aca_tol (Eq. 10), so the row error stays within a small
        # multiple of aca_tol ||Z_i,far|| ||x_far||; a wrong block or sign
        # gives an error of the order of |y_i|, about sqrt(N) times larger
        far = np.ones(wl.n, dtype=bool)
        far[cols[leaf_of[i]]] = False
        bound = 10 * wl.aca_tol * np.linalg.norm(zi[far]) * np.linalg.norm(x[far])
        assert abs(y[i] - exact) <= bound, (i, abs(y[i] - exact), bound)


def test_fullsize_exact_near_inverse(full):
    hsl, torch, ctx, wl, H, rows = full
    P = hsl.Precond(ctx, H, "rcm", 0.0)
    rng = np.random.default_rng(13)
    v = rng.normal(size=wl.n) + 1j * rng.normal(size=wl.n)
    z = P.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    leaf_of, cols = _near_cols(H, wl)
    worst = 0.0
    for i in rows:
        c = cols[leaf_of[i]]
        pts_c = wl.points[c]
        row = np.empty(len(c), dtype=np.complex128)
        own = c == i
        row[~own] = okern.kernel_row(wl.points[i], pts_c[~own], wl.k)
        row[own] = okern.self_term(wl.k, wl.self_h)
        res = v[i] - row @ z[c]
        worst = max(worst, abs(res) / (np.linalg.norm(row) * np.linalg.norm(z[c])))
    assert worst <= 1e-9


def test_fullsize_benchmark_solve(full):
    hsl, torch, ctx, wl, H, rows = full
    P = hsl.Precond(ctx, H, "rcm", wl.fill_tol)
    b = torch.as_tensor(np.ascontiguousarray(wl.rhs[:, 0]), device="cuda")
    x, st = hsl.solve(ctx, H, P, b, restart=wl.restart, tol=wl.tol)
    assert all(s.converged for s in st)
    r = b - H.matvec(x)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(b)) <= wl.tol * 1.01
