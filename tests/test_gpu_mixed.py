"""Mixed-precision solve: FP64 flexible GMRES on the FP64 operator whose
preconditioning steps are inner GMRES solves on complex64 copies of the
operator and of the preconditioner. Pinned by the oracle operator: the true
residual of the mixed solution, measured with the FP64 oracle H-matrix,
meets the tolerance."""
import numpy as np
import pytest

import workloads as W
from oracle import hmatrix as ohm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_13483_amd as hsl
    assert torch.cuda.is_available()
    hsl.load()
    return hsl, torch, hsl.Context(0)


@pytest.mark.parametrize("case", ["c1", "plate"])
def test_mixed_solve_true_residual(env, case):
    hsl, torch, ctx = env
    wl = W.make_config(case, n=1500 if case == "plate" else None, nrhs=3)
    hm = ohm.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol)
    H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol, store_c64=True)
    P = hsl.Precond(ctx, H, "rcm", wl.fill_tol, mixed=True)
    b = torch.as_tensor(np.ascontiguousarray(wl.rhs), device="cuda")
    x, st = hsl.solve(ctx, H, P, b, restart=20, tol=1e-6, mixed=True)
    x = x.cpu().numpy()
    perm = hm.tree.perm
    for c in range(wl.rhs.shape[1]):
        assert st[c].converged and st[c].relres <= 1e-6
        xt = x[perm, c]
        r = wl.rhs[perm, c] - ohm.matvec(hm, xt)
        assert np.linalg.norm(r) <= 1.01e-6 * np.linalg.norm(wl.rhs[:, c])
    # the same system in plain FP64: the solutions agree to the residual level
    x64, st64 = hsl.solve(ctx, H, P, b, restart=30, tol=1e-6)
    x64 = x64.cpu().numpy()
    assert np.linalg.norm(x - x64) <= 1e-3 * np.linalg.norm(x64)


def test_mixed_solve_needs_copies(env):
    hsl, torch, ctx = env
    wl = W.make_config("c1")
    b = torch.as_tensor(wl.rhs[:, 0], device="cuda")
    H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol)
    P = hsl.Precond(ctx, H, "rcm", wl.fill_tol, mixed=True)
    with pytest.raises(hsl.HschurError) as ei:
        hsl.solve(ctx, H, P, b, mixed=True)
    assert ei.value.status == hsl.HS_EINVAL
    H2 = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, wl.aca_tol, store_c64=True)
    P2 = hsl.Precond(ctx, H2, "rcm", wl.fill_tol)
    with pytest.raises(hsl.HschurError) as ei:
        hsl.solve(ctx, H2, P2, b, mixed=True)
    assert ei.value.status == hsl.HS_EINVAL
    # unpreconditioned mixed solve: the inner solves run on the complex64 operator alone
    x, st = hsl.solve(ctx, H2, None, b, restart=20, tol=1e-6, mixed=True, inner_steps=10)
    assert st[0].converged
