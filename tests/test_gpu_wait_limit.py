"""Bounded device waits of the preconditioner sweeps and their library-wide
ordering across streams.

The host forces a give-up with a wait limit of 0 (a wait that is not
satisfied at its first check gives up); every kernel still ends normally,
the call reports HS_ETIMEOUT, and the next call with the default limit
gives the same result as before, bit for bit (the sweeps are
deterministic). No kernel is made to fault or hang."""
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
    wl = W.make_config("c2", n=2500)      # several sweep chunks: the chain waits
    wl.leaf_max = 32
    H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    P = hsl.Precond(ctx, H, "rcm", 1e-2)
    return hsl, torch, ctx, wl, H, P


def test_give_up_reports_timeout_and_recovers(env):
    hsl, torch, ctx, wl, H, P = env
    rng = np.random.default_rng(4)
    v = torch.as_tensor(rng.normal(size=(wl.n, 2)) + 1j * rng.normal(size=(wl.n, 2)), device="cuda")
    z_ref = P.apply(v).cpu().numpy()
    try:
        ctx.set_wait_limit(0.0)
        with pytest.raises(hsl.HschurError) as ei:
            P.apply(v)
        assert ei.value.status == hsl.HS_ETIMEOUT
        b = torch.as_tensor(wl.rhs[:, 0], device="cuda")
        with pytest.raises(hsl.HschurError) as ei:
            hsl.solve(ctx, H, P, b, restart=30, tol=1e-6)
        assert ei.value.status == hsl.HS_ETIMEOUT
    finally:
        ctx.set_wait_limit(5.0)
    torch.cuda.synchronize()
    assert np.array_equal(P.apply(v).cpu().numpy(), z_ref)
    x, st = hsl.solve(ctx, H, P, torch.as_tensor(wl.rhs[:, 0], device="cuda"), restart=30, tol=1e-6)
    assert st[0].converged
    with pytest.raises(hsl.HschurError) as ei:
        ctx.set_wait_limit(-1.0)
    assert ei.value.status == hsl.HS_EINVAL


def test_applies_on_two_streams_are_ordered(env):
    # Two contexts on two streams issue applies back to back; the library
    # orders them (an apply waits for the other stream's earlier ones), so
    # each result equals the single-stream one.
    hsl, torch, ctx, wl, H, P = env
    rng = np.random.default_rng(5)
    v = torch.as_tensor(rng.normal(size=wl.n) + 1j * rng.normal(size=wl.n), device="cuda")
    z_ref = P.apply(v).cpu().numpy()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ca, cb = hsl.Context(0, stream=s1), hsl.Context(0, stream=s2)
    Pa = hsl.Precond.__new__(hsl.Precond)
    Pa.ctx, Pa.H, Pa._h = ca, H, P._h
    Pb = hsl.Precond.__new__(hsl.Precond)
    Pb.ctx, Pb.H, Pb._h = cb, H, P._h
    torch.cuda.synchronize()
    try:
        outs = []
        for _ in range(3):
            with torch.cuda.stream(s1):      # the binding's copies run on the context's stream
                outs.append(Pa.apply(v))
            with torch.cuda.stream(s2):
                outs.append(Pb.apply(v))
        # a context moving to another stream keeps the order too
        ca.set_stream(s2)
        with torch.cuda.stream(s2):
            outs.append(Pa.apply(v))
        torch.cuda.synchronize()
        for z in outs:
            assert np.array_equal(z.cpu().numpy(), z_ref)
    finally:
        Pa._h = None   # borrowed handle: destroyed with P
        Pb._h = None
