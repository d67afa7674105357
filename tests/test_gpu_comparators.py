"""Comparators of the solve on the GPU against the oracle: the block-Jacobi
preconditioner blockdiag(Z_kk)^-1 and the coupled block GMRES (one Krylov
space shared by the right-hand sides). They stand in for the Null-Field and
ILUT preconditioners of the paper's Table 7, which are not available."""
import numpy as np
import pytest

import workloads as W
from oracle import comparators as ocmp
from oracle import gmres as ogm
from oracle import hmatrix as ohm
from oracle import pipeline as opl
from oracle import schur as osch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_13483_amd as hsl
    assert torch.cuda.is_available()
    hsl.load()
    ctx = hsl.Context(0)
    wl = W.make_config("c1", nrhs=4)
    hm = ohm.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    return hsl, torch, ctx, wl, hm, H


def test_block_jacobi_apply_and_solve(env):
    hsl, torch, ctx, wl, hm, H = env
    bj = ocmp.block_jacobi_setup(hm)
    P = hsl.Precond(ctx, H, kind="block_jacobi")
    perm = hm.tree.perm
    rng = np.random.default_rng(6)
    v = rng.normal(size=wl.n) + 1j * rng.normal(size=wl.n)
    z = P.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    ref = np.empty_like(v)
    ref[perm] = ocmp.block_jacobi_apply(bj, v[perm])
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    b = wl.rhs[:, 0]
    xr, _ = ogm.gmres(lambda u: ohm.matvec(hm, u), lambda u: ocmp.block_jacobi_apply(bj, u), b[perm], 30, 1e-6,
                      fixed_iters=25)
    x, st = hsl.solve(ctx, H, P, torch.as_tensor(b, device="cuda"), restart=30, fixed_iters=25)
    assert np.linalg.norm(x.cpu().numpy()[perm] - xr) <= 1e-10 * np.linalg.norm(xr)
    with pytest.raises(hsl.HschurError) as ei:
        hsl.solve(ctx, H, P, torch.as_tensor(b, device="cuda"), transformed=True)
    assert ei.value.status == hsl.HS_EINVAL


def test_block_gmres_fixed_steps_parity(env):
    hsl, torch, ctx, wl, hm, H = env
    pc = opl.precond_setup(hm, "rcm", 1e-2)
    perm = hm.tree.perm
    B = wl.rhs
    Xr, _ = ocmp.block_gmres(lambda u: ohm.matvec(hm, u), lambda u: osch.apply(pc, u), B[perm], 10, 1e-6,
                             fixed_steps=14)
    P = hsl.Precond(ctx, H, "rcm", 1e-2)
    X, st = hsl.solve(ctx, H, P, torch.as_tensor(B, device="cuda"), restart=10, fixed_iters=14, block=True)
    X = X.cpu().numpy()[perm]
    assert all(s.iters == 14 for s in st)
    # the two QR factorisations (Householder, Cholesky QR) differ by column
    # phases and rounding; X does not depend on the basis
    assert np.linalg.norm(X - Xr) <= 1e-9 * np.linalg.norm(Xr)


def test_block_gmres_converges(env):
    hsl, torch, ctx, wl, hm, H = env
    P = hsl.Precond(ctx, H, "rcm", 1e-2)
    B = torch.as_tensor(wl.rhs, device="cuda")
    X, st = hsl.solve(ctx, H, P, B, restart=30, tol=1e-6, block=True)
    Xi, sti = hsl.solve(ctx, H, P, B, restart=30, tol=1e-6)
    perm = hm.tree.perm
    for c in range(B.shape[1]):
        assert st[c].converged
        r = wl.rhs[perm, c] - ohm.matvec(hm, X.cpu().numpy()[perm, c])
        assert np.linalg.norm(r) <= 1.01e-6 * np.linalg.norm(wl.rhs[:, c])
    # one shared space: fewer block steps than the independent columns' steps
    assert st[0].iters <= max(s.iters for s in sti)
    X0, s0 = hsl.solve(ctx, H, None, B, restart=30, tol=1e-6, block=True, max_iters=400)
    assert s0[0].iters >= st[0].iters
