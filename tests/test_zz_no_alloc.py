"""The allocation-free matvec (hs_matvec_noalloc) against hs_matvec: the same
kernels on the library's fixed device scratch, so the products agree to the
FP64 parity bar (they are in fact bit-identical: the same per-element
arithmetic in the same order). Two calls in a row, the second on a smaller
input, show that the shared scratch carries nothing over between calls."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2111_13483_amd as hsl
    assert torch.cuda.is_available()
    L = hsl.load()
    return hsl, torch, L, hsl.Context(0)


def _noalloc(hsl, torch, L, ctx, H, x):
    # caller-order N x nrhs column-major device buffers, as for hs_matvec
    xc = x.t().contiguous()
    y = torch.empty_like(xc)
    need = ctypes.c_int64(0)
    st = L.hs_matvec_noalloc(ctx._h, H._h, ctypes.c_void_p(xc.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                             x.shape[1], ctypes.byref(need))
    torch.cuda.synchronize()
    return st, y.t(), need.value


def test_noalloc_matvec_matches_allocating_matvec(env):
    hsl, torch, L, ctx = env
    big = W.make_config("c2", n=6000)
    small = W.make_config("c1", n=700)
    Hb = hsl.HMatrix(ctx, big.points, big.k, big.self_h, big.leaf_max, 1e-4)
    Hs = hsl.HMatrix(ctx, small.points, small.k, small.self_h, small.leaf_max, 1e-4)
    rng = np.random.default_rng(11)
    for H, wl, nrhs in ((Hb, big, 3), (Hs, small, 1)):
        x = torch.as_tensor(rng.normal(size=(wl.n, nrhs)) + 1j * rng.normal(size=(wl.n, nrhs)), device="cuda")
        st, y, need = _noalloc(hsl, torch, L, ctx, H, x)
        assert st == hsl.HS_OK, hsl.load().hs_last_error()
        assert need > 0
        ref = H.matvec(x).cpu().numpy()
        got = y.cpu().numpy()
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
        # segment by segment too: no part of the result may come from stale scratch
        for c in range(nrhs):
            for a in range(0, wl.n, 256):
                seg, rs = got[a:a + 256, c], ref[a:a + 256, c]
                assert np.linalg.norm(seg - rs) <= 1e-10 * np.linalg.norm(rs)


def test_noalloc_matvec_rejects_oversized_requests(env):
    hsl, torch, L, ctx = env
    wl = W.make_config("c1", n=700)
    H = hsl.HMatrix(ctx, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    x = torch.zeros((wl.n, 400), dtype=torch.complex128, device="cuda")
    st, _, need = _noalloc(hsl, torch, L, ctx, H, x)
    assert st == hsl.HS_EINVAL and need > (64 << 20)
    assert b"64 MiB" in L.hs_last_error() or b"67108864" in L.hs_last_error()
    # the library still serves a fitting request afterwards
    x1 = torch.ones((wl.n, 1), dtype=torch.complex128, device="cuda")
    st, y, _ = _noalloc(hsl, torch, L, ctx, H, x1)
    assert st == hsl.HS_OK
    ref = H.matvec(x1).cpu().numpy()
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
