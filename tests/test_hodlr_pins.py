"""Pins for the dense-based HODLR oracle (Section 2.4, Fig. 1)."""
import numpy as np

from oracle import hodlr as HD
from oracle import lsop_oracle as O
from paper_2005_01372_amd import synth


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def small(n=24, freq=15.0):
    w = synth.model_layered_salt(n=n, h=10.0, freq=freq, seed=2, nsrc=1)
    return w, O.Problem(w.vel, w.h, w.freq, w.c0)


def test_tree_is_column_strips():
    """Nodes are ranges of whole grid columns (multiples of nz cells), halved at each level."""
    t = HD.split_tree(ncols=13, nz=5, levels=3)
    leaves = []

    def walk(node, depth):
        assert node.lo % 5 == 0 and node.hi % 5 == 0
        if hasattr(node, "children_cols"):
            assert node.c1.lo == node.lo and node.c2.hi == node.hi and node.c1.hi == node.c2.lo
            walk(node.c1, depth + 1)
            walk(node.c2, depth + 1)
        else:
            leaves.append((node.lo, node.hi, depth))
    walk(t, 0)
    assert leaves[0][0] == 0 and leaves[-1][1] == 65 and max(d for *_, d in leaves) == 3


def test_full_rank_hodlr_is_exact_and_inverts():
    """With rank >= block size the HODLR approximation equals A and both inverses equal A^{-1} (P11)."""
    w, prob = small(12)
    A = O.operator_matrix(prob.K, prob.chi)
    tree = HD.split_tree(prob.nx, prob.nz, levels=2)
    H = HD.build(A, tree, r=prob.n, seed=1)
    assert rel(H.to_dense(), A) < 1e-12
    Ai = np.linalg.inv(A)
    assert rel(HD.invert(H, r=prob.n).to_dense(), Ai) < 1e-10
    x = synth.random_vectors((prob.n, 3), 3)
    hs = HD.HodlrSolve(prob, rank=prob.n, levels=2, seed=1)
    assert rel(hs.solve_node(hs.approx, x), Ai @ x) < 1e-10


def test_matvec_and_adjoint_match_dense():
    w, prob = small(16)
    A = O.operator_matrix(prob.K, prob.chi)
    H = HD.build(A, HD.split_tree(prob.nx, prob.nz, levels=3), r=6, seed=2)
    D = H.to_dense()
    x = synth.random_vectors((prob.n, 2), 4)
    assert rel(H.matvec(x), D @ x) < 1e-13
    assert rel(H.rmatvec(x), D.conj().T @ x) < 1e-13


def test_truncation_is_best_rank_r():
    """Recompression returns the SVD-optimal rank-r approximation of the factored sum (Eckart-Young)."""
    rng = np.random.default_rng(0)
    U = rng.standard_normal((40, 8)) + 1j * rng.standard_normal((40, 8))
    V = rng.standard_normal((30, 8)) + 1j * rng.standard_normal((30, 8))
    Ut, Vt = HD.truncate(U, V, 3)
    s = np.linalg.svd(U @ V.conj().T, compute_uv=False)
    assert abs(np.linalg.norm(U @ V.conj().T - Ut @ Vt.conj().T, 2) - s[3]) <= 1e-10 * s[0]


def test_solve_variant_inverts_its_own_hodlr_matrix():
    """The nested-SMW solve applies the exact inverse of the (truncated-rank) HODLR approximation."""
    w, prob = small(16)
    hs = HD.HodlrSolve(prob, rank=5, levels=3, seed=3)
    D = hs.approx.to_dense()
    x = synth.random_vectors((prob.n, 2), 5)
    assert rel(D @ hs.solve_node(hs.approx, x), x) < 1e-11


def test_hodlr_series_reaches_lu_solution():
    """The HODLR-preconditioned series converges to the dense-LU solution where rank-r simple H does not."""
    w, prob = small(48)
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    ref = O.solve_direct(prob, psi0)
    for H in (HD.HodlrPreconditioner(prob, 20, 3, seed=4), HD.HodlrSolve(prob, 20, 3, seed=4)):
        psi, it, r, st = O.series_solve(prob, H.apply, psi0, 1e-12, 60)
        assert st == O.OK and rel(psi, ref) < 1e-10


def test_explicit_probes_match_seeded_draws():
    """Passing the probe rows explicitly reproduces the same approximation as drawing them per node."""
    w, prob = small(16)
    r, L, n = 5, 2, prob.n
    rng = np.random.default_rng(11)
    blocks = {d: rng.standard_normal((r, n)) for d in range(L)}
    hs = HD.HodlrSolve(prob, r, L, probes=lambda d: blocks[d])
    A = O.operator_matrix(prob.K, prob.chi)
    # the root's upper block is sampled by the level-0 probes on its second half
    root = hs.approx
    i1, i2 = slice(root.a11.lo, root.a11.hi), slice(root.a22.lo, root.a22.hi)
    Y = A[i1, i2] @ blocks[0][:, i2].T
    P = root.u12 @ root.u12.conj().T
    assert np.linalg.norm(P @ Y - Y) <= 1e-12 * np.linalg.norm(Y)
    assert rel(root.u12 @ root.v12.conj().T, P @ A[i1, i2]) < 1e-13


def test_power_iteration_improves_block_and_keeps_fixed_point():
    """q = 1 (Alg. 1 step 4) tightens each off-diagonal block; the series still reaches the LU solution."""
    w, prob = small(32)
    A = O.operator_matrix(prob.K, prob.chi)
    hs0 = HD.HodlrSolve(prob, 6, 2, seed=3)
    hs1 = HD.HodlrSolve(prob, 6, 2, seed=3, q=1)
    e0 = np.linalg.norm(hs0.approx.to_dense() - A, 2)
    e1 = np.linalg.norm(hs1.approx.to_dense() - A, 2)
    assert e1 < e0
    psi0 = prob.incident(w.src_i, w.src_j)[0]
    psi, it, r, st = O.series_solve(prob, hs1.apply, psi0, 1e-12, 80)
    assert st == O.OK and rel(psi, O.solve_direct(prob, psi0)) < 1e-10


def test_strip_operator_blocks_equal_dense_blocks():
    """The matrix-free strip operator reproduces the dense matrix's diagonal strip blocks and its off-diagonal
    blocks and their adjoints (FFT convolution on a strip against direct slices of I - G0 V), on a
    non-square grid and strips that do not start at column 0."""
    rng = np.random.default_rng(5)
    vel = 2000.0 * (1.0 + 0.3 * synth.smoothed_field((14, 9), 2.0, rng))
    prob = O.Problem(vel, 10.0, 15.0, 2000.0)
    A = O.operator_matrix(prob.K, prob.chi)
    S = HD.StripOperator(prob)
    nz = prob.nz
    assert np.allclose(S.diag(3, 7), A[3 * nz:7 * nz, 3 * nz:7 * nz], rtol=0, atol=1e-15)
    for c0, cin, cout in ((2, (6, 11), (2, 6)), (2, (2, 6), (6, 11)), (0, (0, 7), (7, 14)), (5, (9, 10), (5, 9))):
        B = A[cout[0] * nz:cout[1] * nz, cin[0] * nz:cin[1] * nz]
        mv, rmv = S.block(c0, cin, cout)
        x = rng.standard_normal((B.shape[1], 3)) + 1j * rng.standard_normal((B.shape[1], 3))
        y = rng.standard_normal((B.shape[0], 2)) + 1j * rng.standard_normal((B.shape[0], 2))
        assert rel(mv(x), B @ x) <= 1e-12
        assert rel(rmv(y), B.conj().T @ y) <= 1e-12


def test_matrix_free_build_equals_dense_build():
    """With the same probes, the HODLR matrix sampled through the strip operator equals the one sampled
    from the dense matrix (q = 0 and q = 1), and so do the nested solves."""
    w, prob = small(16)
    A = O.operator_matrix(prob.K, prob.chi)
    rng = np.random.default_rng(8)
    om = rng.standard_normal((3 * 5, prob.n))
    probes = lambda d: om[d * 5:(d + 1) * 5]
    for q in (0, 1):
        hd = HD.build(A, HD.split_tree(prob.nx, prob.nz, 3), 5, probes=probes, q=q).to_dense()
        hm = HD.build(HD.StripOperator(prob), HD.split_tree(prob.nx, prob.nz, 3), 5, probes=probes, q=q).to_dense()
        assert rel(hm, hd) <= 1e-11
    sd = HD.HodlrSolve(prob, 5, 3, probes=probes, q=1)
    sm = HD.HodlrSolve(prob, 5, 3, probes=probes, q=1, matrix_free=True)
    x = synth.random_vectors((2, prob.nx, prob.nz), 1)
    assert rel(sm.apply(x), sd.apply(x)) <= 1e-11


def test_power_iterations_from_a_level():
    """q_from_level selects per tree depth between the q = 0 block construction and the q-iteration one: from
    level 0 it is the q-iteration HODLR matrix, from a level past the deepest it is the q = 0 one, and in
    between the top blocks are those of q = 0 and the deep ones those of q = 1 (same probes)."""
    w, prob = small(16)
    A = O.operator_matrix(prob.K, prob.chi)
    om = np.random.default_rng(3).standard_normal((3 * 4, prob.n))
    probes = lambda d: om[d * 4:(d + 1) * 4]
    tree = lambda: HD.split_tree(prob.nx, prob.nz, 3)
    h0 = HD.build(A, tree(), 4, probes=probes, q=0)
    h1 = HD.build(A, tree(), 4, probes=probes, q=1)
    assert rel(HD.build(A, tree(), 4, probes=probes, q=1, q_from_level=0).to_dense(), h1.to_dense()) == 0
    assert rel(HD.build(A, tree(), 4, probes=probes, q=1, q_from_level=3).to_dense(), h0.to_dense()) == 0
    hm = HD.build(A, tree(), 4, probes=probes, q=1, q_from_level=1)
    assert rel(hm.u12 @ hm.v12.conj().T, h0.u12 @ h0.v12.conj().T) == 0           # depth 0: q = 0
    assert rel(hm.a11.u12 @ hm.a11.v12.conj().T, h1.a11.u12 @ h1.a11.v12.conj().T) == 0   # depth 1: q = 1
    assert rel(hm.a11.u12 @ hm.a11.v12.conj().T, h0.a11.u12 @ h0.a11.v12.conj().T) > 0
