"""Host-side tests of libhschur (no GPU): symbols, argument checks, and the
integer phases (octree, partition, ordering, symbolic fill) bit-exact against
the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2111_13483_amd as hsl
import workloads as W
from oracle import ordering as oord
from oracle import partition as opart
from oracle import symbolic as osym
from oracle import tree as otree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hschur.h")

pytestmark = pytest.mark.skipif(not os.path.exists(hsl.LIB_PATH), reason="libhschur.so not built")


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(hs_[a-z_]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_library_exports_every_declared_symbol():
    L = hsl.load()
    decl = _declared_symbols()
    assert len(decl) >= 18
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(hsl.EXPORTED)


def test_status_strings_and_no_device():
    L = hsl.load()
    assert L.hs_status_string(0) == b"ok"
    assert L.hs_status_string(-5) == b"singular leaf block"
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = L.hs_context_create(ctypes.byref(h), 0, None, hsl.ALLOC_FN(), hsl.FREE_FN(), None)
    assert st == hsl.HS_ENODEVICE and not h.value
    assert L.hs_last_error()


def test_plan_argument_validation():
    L = hsl.load()
    h = ctypes.c_void_p()
    pts = np.zeros((4, 3))
    assert L.hs_plan_create(None, 4, 8, 1, ctypes.byref(h)) == hsl.HS_EINVAL
    assert L.hs_plan_create(pts.ctypes.data_as(ctypes.c_void_p), 0, 8, 1, ctypes.byref(h)) == hsl.HS_EINVAL
    assert L.hs_plan_create(pts.ctypes.data_as(ctypes.c_void_p), 4, 0, 1, ctypes.byref(h)) == hsl.HS_EINVAL
    assert L.hs_plan_create(pts.ctypes.data_as(ctypes.c_void_p), 4, 8, 7, ctypes.byref(h)) == hsl.HS_EINVAL
    # all points equal: zero extent
    assert L.hs_plan_create(pts.ctypes.data_as(ctypes.c_void_p), 4, 8, 1, ctypes.byref(h)) == hsl.HS_EINVAL
    assert b"volume" in L.hs_last_error()
    bad = np.array([[0.0, 0, 0], [np.nan, 1, 1]])
    assert L.hs_plan_create(bad.ctypes.data_as(ctypes.c_void_p), 2, 8, 1, ctypes.byref(h)) == hsl.HS_EINVAL


def _oracle_plan(pts, leaf, kind):
    t = otree.build_tree(pts, leaf)
    p = opart.build_partition(t)
    order = oord.make_order(kind, t.nb, p.near)
    s = osym.symbolic(t.nb, p.near, order)
    return t, p, s


CASES = [
    ("sphere", lambda: W.fibonacci_sphere(1200, np.random.default_rng(1)), 32),
    ("c1", lambda: W.make_config("c1").points, 32),
    ("ellipsoid_pair", lambda: W.sphere_ellipsoid(3000, np.random.default_rng(2))[0], 64),
    ("cube", lambda: W.cube_surface(2500, np.random.default_rng(3))[0], 24),
    ("plate", lambda: W.plate_box(2000, np.random.default_rng(4))[0], 16),
    ("clusters", lambda: W.tiny_cluster_points(np.random.default_rng(5), 9), 4),
    ("tiny_leaf1", lambda: np.random.default_rng(6).normal(size=(60, 3)), 1),
    ("single_leaf", lambda: np.random.default_rng(7).normal(size=(20, 3)), 64),
]


@pytest.mark.parametrize("name,gen,leaf", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("kind", ["natural", "rcm", "cm", "sloan", "king"])
def test_plan_bit_exact_with_oracle(name, gen, leaf, kind):
    pts = gen()
    t, p, s = _oracle_plan(pts, leaf, kind)
    plan = hsl.Plan(pts, leaf, kind)
    assert np.array_equal(plan.export("perm"), t.perm)
    assert np.array_equal(plan.export("leaf_off"), t.leaf_offsets())
    boxes = plan.export("boxes").reshape(-1, 7)
    assert np.array_equal(boxes[:, 0], t.level)
    assert np.array_equal(boxes[:, 1], t.start)
    assert np.array_equal(boxes[:, 2], t.count)
    assert np.array_equal(boxes[:, 3:6], t.anchor)
    assert np.array_equal(boxes[:, 6], t.leaf_id)
    assert np.array_equal(plan.export("near").reshape(-1, 2), p.near)
    assert np.array_equal(plan.export("far").reshape(-1, 2), p.far)
    assert np.array_equal(plan.export("order"), s.order)
    rowptr = plan.export("rowptr")
    cols = plan.export("cols")
    orig = plan.export("orig")
    assert np.array_equal(rowptr, np.concatenate([[0], np.cumsum([len(r) for r in s.rows])]))
    assert np.array_equal(cols, np.array([j for r in s.rows for j in r], dtype=np.int64))
    assert np.array_equal(orig, np.array([int(o) for r in s.orig for o in r], dtype=np.int64))
    info = plan.info()
    assert info["nb"] == t.nb and info["n_near"] == len(p.near) and info["n_far"] == len(p.far)
    assert info["n_pattern"] == s.nnz_blocks()


@pytest.mark.slow
def test_plan_bit_exact_c2_rcm():
    wl = W.make_config("c2")
    t, p, s = _oracle_plan(wl.points, wl.leaf_max, "rcm")
    plan = hsl.Plan(wl.points, wl.leaf_max, "rcm")
    assert np.array_equal(plan.export("perm"), t.perm)
    assert np.array_equal(plan.export("near").reshape(-1, 2), p.near)
    assert np.array_equal(plan.export("far").reshape(-1, 2), p.far)
    assert np.array_equal(plan.export("order"), s.order)
    assert np.array_equal(plan.export("cols"), np.array([j for r in s.rows for j in r], dtype=np.int64))


def test_plan_flop_count_matches_pattern():
    pts = W.fibonacci_sphere(800, np.random.default_rng(8))
    t, p, s = _oracle_plan(pts, 16, "rcm")
    plan = hsl.Plan(pts, 16, "rcm")
    b = np.array([t.count[t.leaf_box[o]] for o in s.order], dtype=float)
    fl = 0.0
    for k in range(t.nb):
        fl += 8 / 3 * b[k] ** 3
        S = s.rows[k]
        fl += sum(8 * b[k] ** 2 * b[j] for j in S)
        fl += sum(8 * b[i] * b[k] * b[j] for a, i in enumerate(S) for j in S[a:])
    assert abs(plan.info()["flops_setup"] - fl) <= 1e-9 * fl


def test_timing_argument_validation():
    L = hsl.load()
    assert L.hs_timing_begin(None) == hsl.HS_EINVAL
    assert L.hs_timing_begin_every(None, 4) == hsl.HS_EINVAL
    assert L.hs_timing_end(None, None) == hsl.HS_EINVAL
