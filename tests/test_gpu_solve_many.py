"""hs_solve_many: several geometries' systems solved together (restart
cycles in lockstep, items on separate streams). Each column's x must be the
same as when it is solved alone (independent Krylov spaces; 1e-10), a
fixed-step run must match the oracle's GMRES on one geometry, and use_x0
must start from the caller's guess."""
import numpy as np
import pytest

import workloads as W
from oracle import hmatrix as ohm
from oracle import pipeline as opl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_13483_amd as hsl
    assert torch.cuda.is_available()
    hsl.load()
    ctx = hsl.Context(0)
    cases = [W.make_config("c1"), W.make_config("plate", n=1500), W.make_config("c2", n=2500)]
    cases[1].leaf_max = 24
    cases[2].leaf_max = 32
    geos = []
    for wl in cases:
        H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
        P = hsl.Precond(ctx, H, "rcm", 1e-2)
        geos.append((wl, H, P))
    return hsl, torch, ctx, geos


def _rhs(wl, kinds, seed):
    rng = np.random.default_rng(seed)
    return np.stack([W.plane_wave(wl.points, wl.k, rng) if k == "pw" else W.port_vector(wl.n, rng)
                     for k in kinds], axis=1)


def test_columns_same_alone_and_in_mixed_batch(env):
    hsl, torch, ctx, geos = env
    # port vectors only on the resolved geometries (the 2,500-point two-body
    # case has about one point per wavelength)
    kinds = [["pw"], ["pw", "port", "pw"], ["pw", "pw"]]
    B = [_rhs(wl, k, 30 + i) for i, ((wl, _, _), k) in enumerate(zip(geos, kinds))]
    items = [(H, P, torch.as_tensor(b, device="cuda")) for (wl, H, P), b in zip(geos, B)]
    out = hsl.solve_many(ctx, items, restart=30, tol=1e-8)
    for i, ((H, P, b), (x, st)) in enumerate(zip(items, out)):
        x = x.cpu().numpy()
        for c in range(b.shape[1]):
            assert st[c].converged and st[c].relres <= 1e-8, (i, c, st[c])
            xa, sa = hsl.solve(ctx, H, P, b[:, c].contiguous(), restart=30, tol=1e-8)
            xa = xa.cpu().numpy()
            assert sa[0].iters == st[c].iters, (i, c, sa[0], st[c])
            assert np.linalg.norm(x[:, c] - xa) <= 1e-10 * np.linalg.norm(xa), (i, c)


def test_fixed_steps_match_the_oracle(env):
    hsl, torch, ctx, geos = env
    wl, H, P = geos[0]
    b = wl.rhs[:, 0]
    hm = opl.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    pc = opl.precond_setup(hm, "rcm", 1e-2)
    ref = opl.solve(hm, pc, b, restart=30, fixed_iters=37)
    other = geos[2]
    bt = torch.as_tensor(b, device="cuda")
    # with an unpreconditioned item (P = NULL) in the same batch
    items = [(H, P, bt), (other[1], other[2], torch.as_tensor(other[0].rhs[:, 0], device="cuda")), (H, None, bt)]
    (x, st), _, (xu, stu) = hsl.solve_many(ctx, items, restart=30, fixed_iters=37)
    x = x.cpu().numpy()
    assert st[0].iters == 37 and stu[0].iters == 37
    assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    refu = opl.solve(hm, None, b, restart=30, fixed_iters=37)
    assert np.linalg.norm(xu.cpu().numpy() - refu.x) <= 1e-10 * np.linalg.norm(refu.x)


def test_initial_guess(env):
    hsl, torch, ctx, geos = env
    wl, H, P = geos[0]
    b = torch.as_tensor(wl.rhs[:, 0], device="cuda")
    x, st = hsl.solve(ctx, H, P, b, restart=30, tol=1e-9)
    # from the converged x: no further step is needed
    x1, st1 = hsl.solve(ctx, H, P, b, restart=30, tol=1e-6, x0=x)
    assert st1[0].converged and st1[0].iters <= 1
    assert np.linalg.norm((x1 - x).cpu().numpy()) <= 1e-6 * np.linalg.norm(x.cpu().numpy())
    # from a rough guess: converges, and the true residual (oracle operator) meets tol
    rng = np.random.default_rng(3)
    g = x.cpu().numpy() + 1e-2 * (rng.normal(size=wl.n) + 1j * rng.normal(size=wl.n))
    x2, st2 = hsl.solve(ctx, H, P, b, restart=30, tol=1e-6, x0=torch.as_tensor(g, device="cuda"))
    hm = ohm.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    perm = hm.tree.perm
    bb = wl.rhs[:, 0]
    res = np.linalg.norm(bb[perm] - ohm.matvec(hm, x2.cpu().numpy()[perm])) / np.linalg.norm(bb)
    assert st2[0].converged and res <= 1.0001e-6
    assert st2[0].iters < st[0].iters
    with pytest.raises(hsl.HschurError) as ei:
        hsl.solve(ctx, H, P, b, mixed=True, x0=x)
    assert ei.value.status == hsl.HS_EINVAL
