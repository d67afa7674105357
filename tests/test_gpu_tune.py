"""The apply-layout autotuner (hs_precond_tune): every candidate layout gives
the same preconditioner up to the order of its triangular solves, the tuner
returns one of the grid's layouts with its measured times, and the layout it
picks applies P^-1 as the default one does (1e-12)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_tuner_picks_a_grid_layout_with_the_same_operator():
    import torch
    import paper_2111_13483_amd as hsl
    hsl.load()
    ctx = hsl.Context(0)
    wl = W.make_config("c2", n=4000)
    H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    (chunk, fold), times = hsl.Precond.tune(ctx, H, "rcm", 1e-2, nrhs=1, reps=5)
    grid = [(c, f) for c in (384, 256, 192) for f in (3072, 2048, 1536) if f >= c]
    assert len(times) == len(grid) and all(t > 0 for t in times)
    assert (chunk, fold) == grid[int(np.argmin(times))]
    P0 = hsl.Precond(ctx, H, "rcm", 1e-2)
    P1 = hsl.Precond(ctx, H, "rcm", 1e-2, sweep_chunk=chunk, sweep_fold_cols=fold)
    rng = np.random.default_rng(2)
    v = torch.as_tensor(rng.normal(size=(wl.n, 2)) + 1j * rng.normal(size=(wl.n, 2)), device="cuda")
    z0, z1 = P0.apply(v).cpu().numpy(), P1.apply(v).cpu().numpy()
    assert np.linalg.norm(z1 - z0) <= 1e-12 * np.linalg.norm(z0)
    with pytest.raises(hsl.HschurError) as ei:
        hsl.Precond.tune(ctx, H, "rcm", 1e-2, nrhs=0)
    assert ei.value.status == hsl.HS_EINVAL
