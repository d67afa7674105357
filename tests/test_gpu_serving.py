"""Serving: resident geometries admitted by footprint, continuous batching.

Each step runs one restart cycle of every geometry with live columns; at
the cycle boundary finished columns leave their slots and pending requests
take free slots (oldest first per geometry). Checked here: requests that
arrive while others run join the running solve, a column's x is the same
as when it is solved alone (independent Krylov spaces, 1e-10), and a
geometry whose plan estimate exceeds the budget is refused before any
device memory is allocated."""
import gc

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
    wl0 = W.make_config("c1")
    H0 = hsl.HMatrix(ctx, wl0.points, wl0.k, wl0.self_h, wl0.leaf_max, wl0.aca_tol)
    P0 = hsl.Precond(ctx, H0, "rcm", wl0.fill_tol)
    wl1 = W.make_config("plate", n=1500)
    wl1.leaf_max = 24
    return hsl, torch, ctx, (wl0, H0, P0), wl1


def _rhs(torch, wl, ncols, seed):
    rng = np.random.default_rng(seed)
    cols = []
    for c in range(ncols):
        cols.append(W.plane_wave(wl.points, wl.k, rng) if c % 2 == 0 else W.port_vector(wl.n, rng))
    return torch.as_tensor(np.stack(cols, axis=1), device="cuda")


def _borrow(hsl, ctx, hh, ph, n):
    H = hsl.HMatrix.__new__(hsl.HMatrix)
    H.ctx, H.n, H._h = ctx, n, hsl.ctypes.c_void_p(hh)
    P = None
    if ph:
        P = hsl.Precond.__new__(hsl.Precond)
        P.ctx, P.H, P._h = ctx, H, hsl.ctypes.c_void_p(ph)
    return H, P


def test_continuous_batching_and_column_independence(env):
    hsl, torch, ctx, (wl0, H0, P0), wl1 = env
    srv = hsl.Server(ctx, 1 << 40, slots=4, restart=30, tol=1e-8)
    g0 = srv.admit(H0, P0)
    g1, est = srv.add_geometry(wl1.points, wl1.k, wl1.self_h, wl1.leaf_max, 1e-4, "rcm", 1e-2)
    assert est > 0
    wls = {g0: wl0, g1: wl1}
    t0 = hsl.Server.clock()
    plan = [(g0, 2), (g1, 1)]
    reqs, rhs = [], []
    for i, (g, nc) in enumerate(plan):
        rhs.append(_rhs(torch, wls[g], nc, 100 + i))
        reqs.append(srv.submit(g, rhs[-1], t0 + 0.001 * i))
    assert srv.step() >= 0           # first cycle of both geometries
    assert not srv.request(reqs[0])["done"]
    # two more requests for geometry 0 arrive while request 0 runs: the first
    # takes the two free slots, the second waits for a slot to free up
    for i, (g, nc) in enumerate([(g0, 2), (g0, 1)], start=len(plan)):
        plan.append((g, nc))
        rhs.append(_rhs(torch, wls[g], nc, 100 + i))
        reqs.append(srv.submit(g, rhs[-1], hsl.Server.clock()))
    assert srv.pending() == (4, 6)
    steps = 0
    while srv.pending()[0]:
        srv.step()
        steps += 1
        assert steps < 400
    st = [srv.request(r) for r in reqs]
    assert all(s["done"] and s["converged"] and s["relres"] <= 1e-8 for s in st)
    # request 2 joined while request 0 was still running; request 3 took a
    # slot only after one of the earlier columns of geometry 0 had finished
    assert st[2]["t_start"] < st[0]["t_done"]
    assert st[3]["t_start"] > st[2]["t_start"]
    assert all(s["t_done"] >= s["t_start"] >= s["t_arrival"] - 1e-3 for s in st)
    hh1, ph1, _ = srv.geometry(g1)
    H1, P1 = _borrow(hsl, ctx, hh1, ph1, wl1.n)
    geo = {g0: (H0, P0), g1: (H1, P1)}
    try:
        for i, r in enumerate(reqs):
            H, P = geo[plan[i][0]]
            x = srv.result(r).cpu().numpy()
            for c in range(plan[i][1]):
                xa, _ = hsl.solve(ctx, H, P, rhs[i][:, c].contiguous(), restart=30, tol=1e-8)
                xa = xa.cpu().numpy()
                assert np.linalg.norm(x[:, c] - xa) <= 1e-10 * np.linalg.norm(xa)
    finally:
        H1._h = None
        if P1 is not None:
            P1._h = None


def test_admission_by_footprint_before_allocation(env):
    hsl, torch, ctx, (wl0, H0, P0), wl1 = env
    plan_est = hsl.Plan(wl1.points, wl1.leaf_max).info()["bytes_estimate"]
    srv = hsl.Server(ctx, plan_est // 2, slots=2)
    gc.collect()              # earlier tests' handles go first, not during the measurement
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    with pytest.raises(hsl.HschurError) as ei:
        srv.add_geometry(wl1.points, wl1.k, wl1.self_h, wl1.leaf_max, 1e-4, "rcm", 1e-2)
    assert ei.value.status == hsl.HS_ENOMEM and "before allocation" in str(ei.value)
    assert srv.last_estimate == plan_est
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before
    # caller-built handles over the budget are refused too; nothing pending, nothing runs
    with pytest.raises(hsl.HschurError) as ei:
        srv.admit(H0, P0)
    assert ei.value.status == hsl.HS_ENOMEM
    assert srv.step() == 0
    # a budget that holds the geometry: the charge is its actual bytes, and the
    # plan's estimate is within a small factor of them
    big = hsl.Server(ctx, 1 << 40, slots=2)
    g, est = big.add_geometry(wl1.points, wl1.k, wl1.self_h, wl1.leaf_max, 1e-4, "rcm", 1e-2)
    _, _, charged = big.geometry(g)
    assert charged > 0 and 0.2 * charged <= est <= 10 * charged, (est, charged)
