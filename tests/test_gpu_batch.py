"""Batched setup: the elimination steps of several geometries share
launches; each preconditioner must equal the one set up alone (same
per-block arithmetic), and the apply must match the oracle."""
import numpy as np
import pytest

import workloads as W
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
    return hsl, torch, hsl.Context(0)


def _cases():
    out = [W.make_config("c1"), W.make_config("plate", n=1500)]
    wl = W.make_config("c2", n=2500)
    wl.leaf_max = 48
    out.append(wl)
    rng = np.random.default_rng(9)
    pts = W.fibonacci_sphere(40, rng)   # a single leaf: one elimination step
    wl1 = W.make_config("c1")
    wl1.points, wl1.leaf_max = pts, 64
    out.append(wl1)
    return out


@pytest.mark.parametrize("fill_tol", [0.0, 1e-2])
def test_batched_setup_equals_single(env, fill_tol):
    hsl, torch, ctx = env
    cases = _cases()
    Hs = [hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4) for wl in cases]
    Ps = hsl.Precond.many(ctx, Hs, "rcm", fill_tol)
    for wl, H, Pb in zip(cases, Hs, Ps):
        P1 = hsl.Precond(ctx, H, "rcm", fill_tol)
        for what in ("d", "alpha_kind", "alpha_off", "alpha"):
            a, b = Pb.export(what), P1.export(what)
            assert a.shape == b.shape and np.array_equal(a, b), what
        rng = np.random.default_rng(8)
        n = len(wl.points)
        v = rng.normal(size=(n, 2)) + 1j * rng.normal(size=(n, 2))
        vt = torch.as_tensor(v, device="cuda")
        assert np.array_equal(Pb.apply(vt).cpu().numpy(), P1.apply(vt).cpu().numpy())
    # and the batched result against the oracle on one of the geometries
    wl, H, Pb = cases[1], Hs[1], Ps[1]
    hm = ohm.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    pc = opl.precond_setup(hm, "rcm", fill_tol)
    rng = np.random.default_rng(10)
    v = rng.normal(size=len(wl.points)) + 1j * rng.normal(size=len(wl.points))
    z = Pb.apply(torch.as_tensor(v, device="cuda")).cpu().numpy()
    perm = hm.tree.perm
    ref = np.empty_like(v)
    ref[perm] = osch.apply(pc, v[perm])
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
