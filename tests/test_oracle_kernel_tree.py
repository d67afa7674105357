"""Pins of the oracle's kernel, octree and partition (CPU only)."""
import cmath
import math

import numpy as np
import pytest

import workloads as W
from oracle import kernel, partition, tree


def test_kernel_entries_match_complex_exponential():
    # Closed form of the Green's function of Eq. 5-6 evaluated independently with cmath.
    rng = np.random.default_rng(0)
    pa = rng.normal(size=(7, 3))
    pb = rng.normal(size=(5, 3)) + 3.0
    k = 7.3
    B = kernel.kernel_block(pa, pb, k, 0.1)
    for i in range(7):
        for j in range(5):
            r = math.dist(pa[i], pb[j])
            ref = cmath.exp(-1j * k * r) / (4 * math.pi * r)
            assert abs(B[i, j] - ref) <= 1e-13 * abs(ref)  # phase error ~ k r eps
    row = kernel.kernel_row(pa[2], pb, k)
    assert np.allclose(row, B[2], rtol=1e-15, atol=0)


def test_kernel_modulus_phase_and_symmetry():
    rng = np.random.default_rng(1)
    p = rng.normal(size=(20, 3))
    k = 3.0
    B = kernel.kernel_block(p, p, k, 0.05, same=True)
    # complex symmetric, not Hermitian (Sec. 3.2 relies on Z = Z^T)
    assert np.array_equal(B, B.T)
    off = ~np.eye(20, dtype=bool)
    r = np.linalg.norm(p[:, None] - p[None], axis=2)
    assert np.allclose(np.abs(B[off]), 1 / (4 * np.pi * r[off]), rtol=1e-14)
    # k = 0 reduces to the Laplace kernel 1/(4 pi r)
    B0 = kernel.kernel_block(p, p, 0.0, 0.05, same=True)
    assert np.allclose(B0[off], 1 / (4 * np.pi * r[off]), rtol=1e-14)


def test_self_term_is_disk_average_of_kernel():
    # The self term equals the mean of G over a flat disk of radius h, whose leading
    # omitted term is -k^2 h / (12 pi), i.e. (kh)^2 / 6 relative to 1/(2 pi h).
    # Integrate exp(-jkr)/(4 pi r) over the disk by Gauss-Legendre in r.
    for k, h in [(12.566, 0.02), (5.0, 0.05), (1.0, 0.01)]:
        xg, wg = np.polynomial.legendre.leggauss(40)
        r = 0.5 * h * (xg + 1)
        w = 0.5 * h * wg
        integral = np.sum(w * np.exp(-1j * k * r) / (4 * np.pi * r) * 2 * np.pi * r)
        mean = integral / (np.pi * h * h)
        st = kernel.self_term(k, h)
        assert abs(st - mean) <= 0.2 * (k * h) ** 2 / (2 * np.pi * h)


def test_coincident_points_rejected():
    p = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 0, 0]])
    with pytest.raises(ValueError):
        kernel.kernel_block(p, p, 1.0, 0.1, same=True)


@pytest.mark.parametrize("leaf_max", [1, 4, 32])
def test_tree_leaves_partition_points(leaf_max):
    rng = np.random.default_rng(leaf_max)
    pts = W.fibonacci_sphere(700, rng)
    t = tree.build_tree(pts, leaf_max)
    n = pts.shape[0]
    assert sorted(t.perm.tolist()) == list(range(n))
    seen = np.zeros(n, dtype=int)
    for lb in t.leaf_box:
        s, c = int(t.start[lb]), int(t.count[lb])
        assert c >= 1 and (c <= leaf_max or t.level[lb] == tree.LEVELS)
        seen[s:s + c] += 1
    assert np.all(seen == 1)
    # every box's points share its Morton prefix and lie in its cube
    for b in range(t.nbox):
        s, c, lv = int(t.start[b]), int(t.count[b]), int(t.level[b])
        pref = t.q[s:s + c] >> (tree.LEVELS - lv)
        assert np.all(pref == t.anchor[b][None, :])
        # children cover the parent exactly, in order
        if t.children[b]:
            cs = [(int(t.start[ch]), int(t.count[ch])) for ch in t.children[b]]
            assert cs[0][0] == s and sum(x[1] for x in cs) == c
            for (s0, c0), (s1, _) in zip(cs, cs[1:]):
                assert s0 + c0 == s1
    # tree order is sorted by key and, within equal keys, by user index
    k = t.keys
    assert np.all(k[:-1] <= k[1:])
    eq = k[:-1] == k[1:]
    assert np.all(t.perm[:-1][eq] < t.perm[1:][eq])


def test_quantisation_grid():
    rng = np.random.default_rng(5)
    pts = rng.uniform(-3, 2, size=(500, 3))
    q = tree.quantise(pts)
    assert q.min() >= 0 and q.max() <= tree.QMAX
    # monotone per axis and the longest axis spans the full grid
    for ax in range(3):
        o = np.argsort(pts[:, ax], kind="stable")
        assert np.all(np.diff(q[o, ax]) >= 0)
    ext = pts.max(0) - pts.min(0)
    ax = int(np.argmax(ext))
    assert q[:, ax].min() <= 1 and q[:, ax].max() >= tree.QMAX - 1


def _cube(t, b):
    side = 1 << (tree.LEVELS - int(t.level[b]))
    centre = (t.anchor[b] * side + side / 2.0)
    return centre, side


@pytest.mark.parametrize("leaf_max,n", [(8, 400), (32, 1500)])
def test_partition_covers_matrix_exactly_once(leaf_max, n):
    rng = np.random.default_rng(n)
    pts = W.fibonacci_sphere(n, rng)
    t = tree.build_tree(pts, leaf_max)
    p = partition.build_partition(t)
    cover = np.zeros((n, n), dtype=np.int32)
    leaf_rng = lambda lf: (int(t.start[t.leaf_box[lf]]), int(t.start[t.leaf_box[lf]] + t.count[t.leaf_box[lf]]))  # noqa
    box_rng = lambda b: (int(t.start[b]), int(t.start[b] + t.count[b]))  # noqa
    for i, j in p.near:
        a0, a1 = leaf_rng(i)
        b0, b1 = leaf_rng(j)
        assert i <= j
        cover[a0:a1, b0:b1] += 1
        if i != j:
            cover[b0:b1, a0:a1] += 1
    for tt, s in p.far:
        a0, a1 = box_rng(tt)
        b0, b1 = box_rng(s)
        assert tt < s
        cover[a0:a1, b0:b1] += 1
        cover[b0:b1, a0:a1] += 1
    assert np.all(cover == 1)
    # near <=> adjacent over all leaf pairs (adjacency from cube centres in max norm)
    nb = t.nb
    nearset = {(int(i), int(j)) for i, j in p.near}
    for a in range(nb):
        ca, sa = _cube(t, t.leaf_box[a])
        for b in range(a, nb):
            cb, sb = _cube(t, t.leaf_box[b])
            adj = np.max(np.abs(ca - cb)) <= (sa + sb) / 2.0
            assert adj == ((a, b) in nearset)
    # far pairs are not adjacent, but their parents are (admissible at the coarsest level)
    for tt, s in p.far:
        ct, st_ = _cube(t, tt)
        cs, ss = _cube(t, s)
        assert np.max(np.abs(ct - cs)) > (st_ + ss) / 2.0
        pt, ps = t.parent[tt], t.parent[s]
        cpt, spt = _cube(t, pt)
        cps, sps = _cube(t, ps)
        assert np.max(np.abs(cpt - cps)) <= (spt + sps) / 2.0


def test_single_leaf_has_no_far_field():
    rng = np.random.default_rng(9)
    pts = W.fibonacci_sphere(30, rng)
    t = tree.build_tree(pts, 64)
    p = partition.build_partition(t)
    assert t.nb == 1 and p.far.shape[0] == 0 and p.near.tolist() == [[0, 0]]


def test_fig2_fixture_has_the_four_leaf_pattern():
    # Fig. 2 / Eq. 12: four leaf cubes, exactly one pair far, all other pairs near.
    import os
    pts = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "fig2_four_leaves.txt"))
    t = tree.build_tree(pts, 4)
    p = partition.build_partition(t)
    off = [tuple(map(int, x)) for x in p.near if x[0] != x[1]]
    assert t.nb == 4 and len(off) == 5


def test_morton_keys_hand_computed():
    # The interleave puts bit i of qx, qy, qz at key bits 3i, 3i+1, 3i+2 (x lowest).
    # Values worked out by hand, so a permuted axis or a shifted bit fails.
    q = np.array([
        [1, 0, 0],          # -> 1
        [0, 1, 0],          # -> 2
        [0, 0, 1],          # -> 4
        [3, 0, 0],          # bits 0,1 of x -> key bits 0,3 -> 9
        [0, 2, 0],          # bit 1 of y -> key bit 4 -> 16
        [5, 6, 1],          # x bits 0,2 -> 0,6; y bits 1,2 -> 4,7; z bit 0 -> 2 -> 1+64+16+128+4
        [0, 0, 1 << 20],    # top bit of z -> key bit 62
        [(1 << 21) - 1] * 3,  # all ones -> 2^63 - 1
    ], dtype=np.int64)
    want = [1, 2, 4, 9, 16, 213, 1 << 62, (1 << 63) - 1]
    assert tree.morton(q).tolist() == want


def test_quantisation_centres_the_root_cube():
    # Box x in [0, 4], y and z in [0, 1]: E = 4, centre (2, .5, .5), cube origin
    # (0, -1.5, -1.5). With 2^21 / E = 2^19 the short axes start at 1.5 * 2^19,
    # not at 0 (which an origin at the box corner would give).
    pts = np.array([[0.0, 0.0, 0.0], [4.0, 1.0, 1.0], [1.0, 0.25, 0.75], [3.0, 0.5, 0.0]])
    q = tree.quantise(pts)
    s = 1 << 19
    want = np.array([
        [0, 3 * s // 2, 3 * s // 2],
        [tree.QMAX, 5 * s // 2, 5 * s // 2],     # x clamps at 2^21 - 1
        [s, 7 * s // 4, 9 * s // 4],
        [3 * s, 2 * s, 3 * s // 2],
    ], dtype=np.int64)
    assert np.array_equal(q, want)
