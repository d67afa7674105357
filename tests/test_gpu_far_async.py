"""The far field compressed beside the caller's next work.

hs_h_build returns once the near field is in; a host thread compresses the
far field on the H-matrix's own streams, and every entry point that reads
the far field joins it first. An error of the far compression (here an ACA
rank cap that the blocks need to exceed) is therefore reported by the first
call that reads the far field, and again by every later one, while the
preconditioner setup, which reads only the near field, still works. A build
that succeeds gives the same matvec whether or not a setup ran beside its
far compression."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_far_field_error_reported_where_the_far_field_is_read():
    import torch
    import paper_2111_13483_amd as hsl
    assert torch.cuda.is_available()
    hsl.load()
    ctx = hsl.Context(0)
    wl = W.make_config("c2", n=2500)
    H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4, rank_cap=2)
    P = hsl.Precond(ctx, H, "rcm", 1e-2)   # near field only: unaffected
    assert P.info()["n_pattern"] > 0
    for _ in range(2):
        with pytest.raises(hsl.HschurError) as ei:
            H.info()
        assert ei.value.status == hsl.HS_ENUMERIC
    x = torch.zeros(wl.n, dtype=torch.complex128, device="cuda")
    with pytest.raises(hsl.HschurError) as ei:
        H.matvec(x)
    assert ei.value.status == hsl.HS_ENUMERIC
    del P, H


def test_matvec_same_with_and_without_a_setup_beside_the_far_field():
    import torch
    import paper_2111_13483_amd as hsl
    hsl.load()
    ctx = hsl.Context(0)
    wl = W.make_config("c2", n=5000)
    rng = np.random.default_rng(8)
    x = torch.as_tensor(rng.normal(size=wl.n) + 1j * rng.normal(size=wl.n), device="cuda")
    H1 = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    H1.info()                                   # joined before anything else runs
    y1 = H1.matvec(x).cpu().numpy()
    H2 = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    P2 = hsl.Precond(ctx, H2, "rcm", 1e-2)      # beside H2's far compression
    y2 = H2.matvec(x).cpu().numpy()
    assert np.array_equal(y1, y2)
    del P2
