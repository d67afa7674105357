"""Pins of the oracle's Schur elimination, preconditioner apply and GMRES (CPU only)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import gmres, hmatrix, ordering, pipeline, schur, symbolic


def _small_hm(n=260, leaf=10, seed=21, k=6.0, aca_tol=1e-6):
    rng = np.random.default_rng(seed)
    pts = W.fibonacci_sphere(n, rng)
    return hmatrix.h_build(pts, k, np.sqrt(4 * np.pi / n), leaf, aca_tol), rng


def _permuted_dense_near(hm, sym):
    """Dense Z_N with rows/cols grouped by the new block numbering."""
    Z = hmatrix.dense_near(hm)
    idx = np.concatenate([np.arange(*hm.leaf_range(int(o))) for o in sym.order])
    sizes = [hm.leaf_range(int(o))[1] - hm.leaf_range(int(o))[0] for o in sym.order]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    return Z[np.ix_(idx, idx)], offs


@pytest.mark.parametrize("kind", ["natural", "rcm"])
def test_schur_matches_literal_dense_block_elimination(kind):
    # Eq. 17-21 applied literally with dense matrices: Z~ = a'_k ... Z_N ... a_k
    hm, _ = _small_hm()
    order = ordering.make_order(kind, hm.tree.nb, hm.part.near)
    sym = symbolic.symbolic(hm.tree.nb, hm.part.near, order)
    pc = schur.precond_setup(hm, sym, 0.0)
    Zp, offs = _permuted_dense_near(hm, sym)
    nb = sym.nb
    cur = Zp.copy()
    for k in range(nb):
        sk = slice(offs[k], offs[k + 1])
        rest = slice(offs[k + 1], offs[-1])
        a = np.eye(Zp.shape[0], dtype=complex)
        a[sk, rest] = -np.linalg.solve(cur[sk, sk], cur[sk, rest])          # Eq. 14
        ap = np.eye(Zp.shape[0], dtype=complex)
        ap[rest, sk] = -cur[rest, sk] @ np.linalg.inv(cur[sk, sk])         # Eq. 16
        # the stored right coefficients of row k match (zero outside the filled pattern)
        for j in range(k + 1, nb):
            sj = slice(offs[j], offs[j + 1])
            blk = a[sk, sj]
            if j in sym.rows[k]:
                assert np.linalg.norm(blk - pc.alpha[(k, j)]) <= 1e-11 * max(1.0, np.linalg.norm(blk))
            else:
                assert np.linalg.norm(blk) <= 1e-12 * np.linalg.norm(a[sk, rest]) + 1e-300
        # symmetric near field: left coefficients are the plain transpose (Sec. 3.2)
        assert np.allclose(ap[rest, sk], a[sk, rest].T, rtol=1e-9, atol=1e-12)
        cur = ap @ cur @ a                                                # Eq. 18
        # row and column k are zero off the diagonal block (Eq. 19)
        assert np.linalg.norm(cur[sk, rest]) <= 1e-10 * np.linalg.norm(cur[sk, sk])
        assert np.linalg.norm(cur[rest, sk]) <= 1e-10 * np.linalg.norm(cur[sk, sk])
        assert np.linalg.norm(cur[sk, sk] - pc.D[k]) <= 1e-11 * np.linalg.norm(pc.D[k])
    # Eq. 21: the result is block diagonal
    mask = np.zeros_like(cur, dtype=bool)
    for k in range(nb):
        mask[offs[k]:offs[k + 1], offs[k]:offs[k + 1]] = True
    assert np.linalg.norm(cur[~mask]) <= 1e-10 * np.linalg.norm(cur)


def test_fig2_first_step_structure():
    # Fig. 2 / Eq. 19: eliminating block 1 only changes blocks (2,2), (2,3), (3,3);
    # blocks of leaf 4 (far from 1) are untouched.
    pts = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "fig2_four_leaves.txt"))
    hm = hmatrix.h_build(pts, 2.0, 0.05, 4, 1e-10)
    off = [tuple(map(int, x)) for x in hm.part.near if x[0] != x[1]]
    allp = {(a, b) for a in range(4) for b in range(a + 1, 4)}
    (f1, f4), = allp - set(off)
    mid = [x for x in range(4) if x not in (f1, f4)]
    order = np.array([f1, mid[0], mid[1], f4])
    sym = symbolic.symbolic(4, hm.part.near, order)
    assert sym.rows[0] == [1, 2]                   # block 1 couples only to 2 and 3
    assert sym.orig[0] == [True, True]
    W0, _ = schur.initial_blocks(hm, sym)
    pc = schur.precond_setup(hm, sym, 0.0)
    Z11inv = np.linalg.inv(W0[(0, 0)])
    # after step 1, the (2,2), (2,3), (3,3) blocks are Z_ij - Z_i1 Z_11^-1 Z_1j
    step1 = {(i, j): W0[(i, j)] - W0[(0, i)].T @ Z11inv @ W0[(0, j)] for i, j in [(1, 1), (1, 2), (2, 2)]}
    # block 2 is eliminated next from the step-1 values: D_2 is step1[(1,1)]
    assert np.linalg.norm(pc.D[1] - step1[(1, 1)]) <= 1e-12 * np.linalg.norm(step1[(1, 1)])
    a12 = -np.linalg.solve(step1[(1, 1)], step1[(1, 2)])
    assert np.linalg.norm(pc.alpha[(1, 2)] - a12) <= 1e-11 * np.linalg.norm(a12)
    # (2,4) and (3,4) had no contribution from step 1: alpha_{2,4} uses the raw Z_24
    a13 = -np.linalg.solve(step1[(1, 1)], W0[(1, 3)])
    assert np.linalg.norm(pc.alpha[(1, 3)] - a13) <= 1e-11 * np.linalg.norm(a13)


@pytest.mark.parametrize("kind", ["natural", "cm", "rcm", "sloan", "king"])
def test_exact_preconditioner_is_near_field_inverse(kind):
    # with no fill-in dropped, alpha D^-1 alpha^T = Z_N^-1 for every ordering
    hm, rng = _small_hm(n=400, leaf=16, seed=5)
    pc = pipeline.precond_setup(hm, kind, 0.0)
    Zn = hmatrix.dense_near(hm)
    v = rng.normal(size=(hm.n, 2)) + 1j * rng.normal(size=(hm.n, 2))
    ref = np.linalg.solve(Zn, v)
    got = schur.apply(pc, v)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_symmetry_of_operator_and_preconditioner():
    hm, rng = _small_hm(n=500, leaf=16, seed=7)
    pc = pipeline.precond_setup(hm, "rcm", 1e-2)
    u = rng.normal(size=hm.n) + 1j * rng.normal(size=hm.n)
    v = rng.normal(size=hm.n) + 1j * rng.normal(size=hm.n)
    a, b = u @ hmatrix.matvec(hm, v), v @ hmatrix.matvec(hm, u)
    assert abs(a - b) <= 1e-13 * abs(a)
    a, b = u @ schur.apply(pc, v), v @ schur.apply(pc, u)
    assert abs(a - b) <= 1e-12 * abs(a)
    for D in pc.D:
        assert np.linalg.norm(D - D.T) <= 1e-12 * np.linalg.norm(D)


def test_nonsymmetric_left_coefficients_equal_transpose():
    hm, _ = _small_hm(n=220, leaf=12, seed=8)
    order = ordering.make_order("rcm", hm.tree.nb, hm.part.near)
    sym = symbolic.symbolic(hm.tree.nb, hm.part.near, order)
    pc = schur.precond_setup(hm, sym, 0.0)
    ap = schur.nonsymmetric_alpha_prime(hm, sym)
    for (i, k), A in ap.items():
        ref = pc.alpha[(k, i)].T
        assert np.linalg.norm(A - ref) <= 1e-10 * np.linalg.norm(ref)


def test_fill_compression_bound_and_rule():
    wl = W.make_config("c1")
    hm = hmatrix.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    pc = pipeline.precond_setup(hm, "rcm", 1e-2)
    assert len(pc.lowrank) > 0
    errs = []
    for (k, j), (U, V) in pc.lowrank.items():
        A = pc.alpha[(k, j)]
        assert not pc.sym.orig[k][pc.sym.rows[k].index(j)]
        assert U.shape[1] * sum(A.shape) < A.size
        errs.append(np.linalg.norm(A - U @ V) / np.linalg.norm(A))
    # Same reading as the far-field pin (Eq. 10): ACA's stop test estimates the
    # error, so the median block is within fill_tol and every block within
    # 5 fill_tol (measured here: worst 2.0 fill_tol, 8% of blocks above it).
    assert np.median(errs) <= 1e-2
    assert max(errs) <= 5 * 1e-2


def test_gmres_single_leaf_converges_in_one_step():
    rng = np.random.default_rng(3)
    pts = W.fibonacci_sphere(40, rng)
    hm = hmatrix.h_build(pts, 4.0, 0.3, 64, 1e-4)
    pc = pipeline.precond_setup(hm, "rcm", 1e-2)
    b = W.plane_wave(pts, 4.0, rng)
    out = pipeline.solve(hm, pc, b, restart=10, tol=1e-10)
    assert out.stats[0].iters == 1 and out.stats[0].relres <= 1e-10


def test_gmres_reproduces_dense_solve():
    hm, rng = _small_hm(n=300, leaf=12, seed=9, aca_tol=1e-13)
    pc = pipeline.precond_setup(hm, "rcm", 0.0)
    Zd = hmatrix.dense_kernel(hm.pts, hm.k, hm.h)
    b = rng.normal(size=hm.n) + 1j * rng.normal(size=hm.n)
    out = pipeline.solve(hm, pc, b, restart=40, tol=1e-13)
    perm = hm.tree.perm
    x_tree = out.x[perm]
    ref = np.linalg.solve(Zd, b[perm])
    cond = np.linalg.cond(Zd)
    assert np.linalg.norm(x_tree - ref) <= cond * 1e-12 * np.linalg.norm(ref)


def test_gmres_plain_matrix_full_krylov_is_exact():
    rng = np.random.default_rng(4)
    n = 25
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) + 8 * np.eye(n)
    b = rng.normal(size=n) + 0j
    x, st = gmres.gmres(lambda v: A @ v, lambda v: v, b, restart=n, tol=1e-14)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)
    # Givens rotation zeroes the second entry and keeps the norm
    for a, bb in [(1 + 2j, 0.5), (0.0, 2.0), (-3j, 1e-3)]:
        c, s = gmres.givens(a, bb)
        r0 = c * a + s * bb
        r1 = -np.conj(s) * a + c * bb
        assert abs(r1) <= 1e-15 * abs(r0) + 1e-300
        assert abs(abs(r0) - np.hypot(abs(a), abs(bb))) <= 1e-15 * abs(r0)


def test_preconditioned_and_plain_solutions_agree():
    hm, rng = _small_hm(n=350, leaf=12, seed=10, aca_tol=1e-5)
    pc = pipeline.precond_setup(hm, "rcm", 1e-2)
    b = W.plane_wave(hm.pts, hm.k, rng)
    a = pipeline.solve(hm, pc, b, restart=30, tol=1e-10)
    p = pipeline.solve(hm, None, b, restart=30, tol=1e-10)
    assert a.stats[0].converged and p.stats[0].converged
    assert a.stats[0].iters <= p.stats[0].iters
    Zh = hmatrix.dense_h(hm)
    cond = np.linalg.cond(Zh)
    assert np.linalg.norm(a.x - p.x) <= 2 * cond * 1e-10 * np.linalg.norm(p.x)


# ---- the transformed system of Eq. 25-28 ---------------------------------------

def test_transformed_near_field_is_block_diagonal():
    # alpha^T Z_N alpha = D (Eq. 20-21, 26-27) by brute force: apply the
    # operators to every unit vector of a small case, fill_tol = 0
    from oracle import transformed as otr
    hm, _ = _small_hm(n=180, leaf=10, seed=12)
    for kind in ("natural", "rcm"):
        order = ordering.make_order(kind, hm.tree.nb, hm.part.near)
        sym = symbolic.symbolic(hm.tree.nb, hm.part.near, order)
        pc = schur.precond_setup(hm, sym, 0.0)
        n = hm.n
        A = np.zeros((n, n), dtype=complex)
        AT = np.zeros((n, n), dtype=complex)
        for i in range(n):
            e = np.zeros(n, dtype=complex)
            e[i] = 1.0
            A[:, i] = otr.alpha(pc, e)
            AT[:, i] = otr.alpha_T(pc, e)
        assert np.allclose(AT, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
        ZN = hmatrix.dense_near(hm)
        T = A.T @ ZN @ A
        Dd = np.zeros((n, n), dtype=complex)
        for k in range(pc.nb):
            s = slice(int(pc.start[k]), int(pc.start[k] + pc.size[k]))
            Dd[s, s] = pc.D[k]
        assert np.linalg.norm(T - Dd) <= 1e-10 * np.linalg.norm(Dd)


def test_transformed_solve_matches_right_preconditioned_solve():
    from oracle import transformed as otr
    wl = W.make_config("c1", n=700)
    hm = hmatrix.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    b = wl.rhs[:, 0]
    pc0 = pipeline.precond_setup(hm, "rcm", 0.0)
    x, st, res = otr.solve(hm, pc0, b, restart=30, tol=1e-10)
    ref = pipeline.solve(hm, pc0, b, restart=30, tol=1e-10)
    assert st.converged and res <= 1e-8
    assert np.linalg.norm(x - ref.x) <= 1e-7 * np.linalg.norm(ref.x)
    # with compressed fill-ins the transformed system is perturbed
    # (alpha^T Z_N alpha != D): its solution's true residual sits near
    # fill_tol / 10 (measured 6.7e-4 at 1e-2, 4.9e-5 at 1e-3), which is
    # what is reported
    for ft in (1e-2, 1e-3):
        pc = pipeline.precond_setup(hm, "rcm", ft)
        x2, st2, res2 = otr.solve(hm, pc, b, restart=30, tol=1e-6)
        assert st2.converged and 1e-6 < res2 < ft


# ---- comparators: block Jacobi and coupled block GMRES --------------------------

def test_block_jacobi_is_block_diagonal_solve():
    from oracle import comparators as ocmp
    hm, rng = _small_hm(n=200, leaf=12, seed=31)
    bj = ocmp.block_jacobi_setup(hm)
    v = rng.normal(size=hm.n) + 1j * rng.normal(size=hm.n)
    ZN = hmatrix.dense_near(hm)
    Bd = np.zeros_like(ZN)
    for leaf in range(hm.tree.nb):
        a, b = hm.leaf_range(leaf)
        Bd[a:b, a:b] = ZN[a:b, a:b]
    assert np.allclose(ocmp.block_jacobi_apply(bj, v), np.linalg.solve(Bd, v), rtol=0,
                       atol=1e-11 * np.linalg.norm(v))


def test_block_gmres_one_column_is_gmres():
    from oracle import comparators as ocmp
    from oracle import gmres as ogm
    wl = W.make_config("c1", n=500)
    hm = hmatrix.h_build(wl.points, wl.k, wl.self_h, wl.leaf_max, 1e-4)
    pc = pipeline.precond_setup(hm, "rcm", 1e-2)
    mv = lambda v: hmatrix.matvec(hm, v)          # noqa: E731
    pre = lambda v: schur.apply(pc, v)            # noqa: E731
    b = wl.rhs[hm.tree.perm, 0]
    x1, st1 = ogm.gmres(mv, pre, b, 20, 1e-6, fixed_iters=27)
    X, st = ocmp.block_gmres(mv, pre, b[:, None], 20, 1e-6, fixed_steps=27)
    assert np.linalg.norm(X[:, 0] - x1) <= 1e-10 * np.linalg.norm(x1)


def test_block_gmres_exact_in_n_over_s_steps():
    # a 48-point system with 4 right-hand sides: the block Krylov space fills
    # the whole space after 12 block steps, so X is the dense solution
    from oracle import comparators as ocmp
    rng = np.random.default_rng(4)
    pts = W.fibonacci_sphere(48, rng)
    hm = hmatrix.h_build(pts, 3.0, np.sqrt(4 * np.pi / 48), 8, 1e-13)
    Z = hmatrix.dense_h(hm)
    Bm = rng.normal(size=(48, 4)) + 1j * rng.normal(size=(48, 4))
    X, st = ocmp.block_gmres(lambda v: Z @ v, lambda v: v, Bm, 12, 0.0, fixed_steps=12)
    ref = np.linalg.solve(Z, Bm)
    assert np.linalg.norm(X - ref) <= 1e-9 * np.linalg.norm(ref)
    X2, st2 = ocmp.block_gmres(lambda v: Z @ v, lambda v: v, Bm, 12, 1e-10)
    assert st2.converged and st2.steps <= 12
