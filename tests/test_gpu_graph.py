"""The allocation-free matvec (hs_matvec_noalloc) under HIP graph capture.

It launches kernels only (no allocation, no memset node, no host sync), so a
caller can record it into a graph on its own stream and replay it. The
graph is replayed several times on new inputs, with eager library work and
synchronisations between the replays, and every replay is checked against
the eager hs_matvec of the same input (the same kernels: bit-identical)."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_matvec_replays_from_a_captured_graph():
    import torch
    import paper_2111_13483_amd as hsl
    assert torch.cuda.is_available()
    L = hsl.load()
    wl = W.make_config("c2", n=5000)
    ctx0 = hsl.Context(0)
    H = hsl.HMatrix(ctx0, wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    nrhs = 2
    s = torch.cuda.Stream()
    ctx = hsl.Context(0, stream=s)
    # caller-order N x nrhs column-major buffers, fixed for the graph
    xbuf = torch.zeros((nrhs, wl.n), dtype=torch.complex128, device="cuda")
    ybuf = torch.zeros_like(xbuf)
    need = ctypes.c_int64(0)

    def call():
        return L.hs_matvec_noalloc(ctx._h, H._h, ctypes.c_void_p(xbuf.data_ptr()), ctypes.c_void_p(ybuf.data_ptr()),
                                   nrhs, ctypes.byref(need))

    rng = np.random.default_rng(21)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):   # one eager call on the capture stream first
        assert call() == hsl.HS_OK, L.hs_last_error()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        st = call()
    assert st == hsl.HS_OK, L.hs_last_error()
    torch.cuda.synchronize()
    for rep in range(4):
        x = rng.normal(size=(wl.n, nrhs)) + 1j * rng.normal(size=(wl.n, nrhs))
        xbuf.copy_(torch.as_tensor(x.T.copy(), device="cuda"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = ybuf.cpu().numpy().T
        # eager work of the library between replays: the allocating matvec
        ref = H.matvec(torch.as_tensor(x, device="cuda")).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got, ref), (rep, np.abs(got - ref).max())
    del g
