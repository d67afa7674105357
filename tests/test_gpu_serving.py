"""Serving layer (resident geometries, per-geometry batching of request
columns): each column's solution must not depend on the batch it was served
in (independent Krylov spaces sharing matrix reads), batches follow the
oldest-request-first rule, and admission respects the device budget."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_13483_amd as hsl
    assert torch.cuda.is_available()
    hsl.load()
    ctx = hsl.Context(0)
    geos = []
    for name, n in (("c1", None), ("plate", 1500)):
        wl = W.make_config(name, n=n)
        H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol)
        P = hsl.Precond(ctx, H, "rcm", wl.fill_tol)
        geos.append((wl, H, P))
    return hsl, torch, ctx, geos


def _rhs(torch, wl, ncols, seed):
    rng = np.random.default_rng(seed)
    cols = []
    for c in range(ncols):
        if c % 2 == 0:
            cols.append(W.plane_wave(wl.points, wl.k, rng))
        else:
            cols.append(W.port_vector(wl.n, rng))
    return torch.as_tensor(np.stack(cols, axis=1), device="cuda")


def test_batches_and_column_independence(env):
    hsl, torch, ctx, geos = env
    srv = hsl.Server(ctx, 1 << 40, max_batch_cols=4, restart=30, tol=1e-8)
    g = [srv.admit(H, P) for (_, H, P) in geos]
    plan = [(0, 1), (1, 2), (0, 3), (0, 2), (1, 1)]
    t0 = hsl.Server.clock()
    reqs, rhs = [], []
    for i, (gi, nc) in enumerate(plan):
        b = _rhs(torch, geos[gi][0], nc, 100 + i)
        rhs.append(b)
        reqs.append(srv.submit(g[gi], b, t0 + 0.001 * i))
    assert srv.pending() == (5, 9)
    served = []
    while srv.pending()[0]:
        before = {r for r in reqs if not srv.request(r)["done"]}
        served.append((srv.step(), sorted(r for r in before if srv.request(r)["done"])))
    # oldest first: geometry 0 with requests 0 and 2 (4 columns), then geometry 1
    # (requests 1 and 4), then request 3
    assert served == [(4, [reqs[0], reqs[2]]), (3, [reqs[1], reqs[4]]), (2, [reqs[3]])]
    for i, r in enumerate(reqs):
        st = srv.request(r)
        assert st["done"] and st["converged"] and st["relres"] <= 1e-8
        assert st["t_done"] >= st["t_arrival"]
        wl, H, P = geos[plan[i][0]]
        x = srv.result(r).cpu().numpy()
        for c in range(plan[i][1]):
            xa, _ = hsl.solve(ctx, H, P, rhs[i][:, c].contiguous(), restart=30, tol=1e-8)
            xa = xa.cpu().numpy()
            assert np.linalg.norm(x[:, c] - xa) <= 1e-10 * np.linalg.norm(xa)


def test_admission_by_footprint(env):
    hsl, torch, ctx, geos = env
    (_, H0, P0), (_, H1, P1) = geos
    f0 = H0.info()["bytes_device"] + P0.info()["bytes_device"]
    srv = hsl.Server(ctx, f0 + 1)
    assert srv.admit(H0, P0) == 0
    with pytest.raises(hsl.HschurError) as ei:
        srv.admit(H1, P1)
    assert ei.value.status == hsl.HS_ENOMEM
    # the same H-matrix again, unpreconditioned: its bytes are already counted
    assert srv.admit(H0, None) == 1
    # nothing pending: a step serves no column
    assert srv.step() == 0
