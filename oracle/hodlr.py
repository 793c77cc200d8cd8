"""Dense-based HODLR preconditioner of Section 2.4 (FP64, small grids).

TEST INFRASTRUCTURE ONLY (see ``oracle/lsop_oracle.py``).

The matrix A = I - G0 V (eq. 5), with cells ordered column-wise (vertical
strips), is approximated by a hierarchically off-diagonal low-rank (HODLR)
matrix (Fig. 1): the index range of a node is a range of grid columns (a
multiple of N_z cells), split in two halves; both off-diagonal blocks are
low-rank, with the same rank r at all levels; the diagonal blocks below the
last level are kept dense.  Off-diagonal blocks are found with the
randomized range finder (Alg. 1 with q = 0): B ~= Q (B^H Q)^H with
Q = orth(B Omega).  The approximate inverse is built with the 2x2 block
formula applied recursively (Section 2.4), the top-right block read as
-A^{-1} B S^{-1}; sums of low-rank terms are brought back to rank r.

Readings (where Section 2.4 is not specific):
* split: node [c0, c1) of grid columns splits at c0 + (c1 - c0) // 2; stop at
  ``levels`` or when a node is narrower than 2 * ``min_width`` columns.
* recompression of a rank-2r sum to rank r: deterministic truncated SVD of
  the factored form (QR of both factors, SVD of the small core); the paper
  allows either SVD or a randomized variant and uses the latter for speed.
* the blocks are exact submatrices of A = I - G0 V, either sliced from the
  dense matrix (small grids) or, for grids whose dense matrix does not fit
  in memory, given by `StripOperator`: a dense leaf block formed from the
  kernel table of its own strip, an off-diagonal block applied as the FFT
  convolution of the node's strip with the input and output restricted to
  the two halves (the same Toeplitz block, since a strip of whole grid
  columns is a grid of its own with the same lags).
* two inverses are given: `HodlrPreconditioner` follows the paper (block
  formula in HODLR arithmetic with recompression to rank r); `HodlrSolve`
  applies the exact inverse of the same HODLR approximation by nested
  Sherman-Morrison-Woodbury solves (no recompression) -- the form the device
  path computes.

Pins: tests/test_hodlr_pins.py (full rank reproduces A and A^{-1}; the
truncation is SVD-optimal; the nested solve inverts its own HODLR matrix;
preconditioned series reaches the dense LU solution; the strip operator's
blocks equal those of the dense matrix).
"""
from __future__ import annotations

import numpy as np

from .lsop_oracle import apply_fft, operator_matrix, orth, range_finder_generic, spectrum


class Node:
    """HODLR node: either a dense leaf or two children and two low-rank off-diagonal blocks."""

    def __init__(self, lo, hi):
        self.lo, self.hi = lo, hi          # cell index range [lo, hi)
        self.dense = None
        self.a11 = self.a22 = None
        self.u12 = self.v12 = None         # A[I1, I2] ~= u12 v12^H
        self.u21 = self.v21 = None         # A[I2, I1] ~= u21 v21^H

    @property
    def size(self):
        return self.hi - self.lo

    @property
    def is_leaf(self):
        return self.dense is not None

    def to_dense(self):
        if self.is_leaf:
            return self.dense.copy()
        m = self.a11.size
        out = np.empty((self.size, self.size), np.complex128)
        out[:m, :m] = self.a11.to_dense()
        out[m:, m:] = self.a22.to_dense()
        out[:m, m:] = self.u12 @ self.v12.conj().T
        out[m:, :m] = self.u21 @ self.v21.conj().T
        return out

    def matvec(self, x):
        """y = H x for x[size, k]."""
        if self.is_leaf:
            return self.dense @ x
        m = self.a11.size
        y = np.empty_like(x)
        y[:m] = self.a11.matvec(x[:m]) + self.u12 @ (self.v12.conj().T @ x[m:])
        y[m:] = self.a22.matvec(x[m:]) + self.u21 @ (self.v21.conj().T @ x[:m])
        return y

    def rmatvec(self, x):
        """y = H^H x."""
        if self.is_leaf:
            return self.dense.conj().T @ x
        m = self.a11.size
        y = np.empty_like(x)
        y[:m] = self.a11.rmatvec(x[:m]) + self.v21 @ (self.u21.conj().T @ x[m:])
        y[m:] = self.a22.rmatvec(x[m:]) + self.v12 @ (self.u12.conj().T @ x[:m])
        return y


def split_tree(ncols, nz, levels, min_width=1):
    """Column-strip tree of Section 2.4 / Fig. 1 (ranges in cells)."""
    def build(c0, c1, depth):
        node = Node(c0 * nz, c1 * nz)
        if depth == levels or (c1 - c0) < 2 * min_width:
            node.leaf_cols = (c0, c1)
            return node
        cm = c0 + (c1 - c0) // 2
        node.children_cols = (c0, cm, c1)
        node.c1 = build(c0, cm, depth + 1)
        node.c2 = build(cm, c1, depth + 1)
        return node
    return build(0, ncols, 0)


def lowrank_from_block(B, r, rng, om=None, q=0):
    """Alg. 1 on an explicit block (q = 0 in Section 2.4): B ~= Q (B^H Q)^H with r Gaussian probes (or om)."""
    if om is None:
        om = rng.standard_normal((B.shape[1], r))
    if q:
        return range_finder_generic(B, om, q)
    Q, _ = np.linalg.qr(B @ om)
    return Q, B.conj().T @ Q


def truncate(U, V, r):
    """Best rank-r approximation of U V^H (QR of both factors, SVD of the core)."""
    if U.shape[1] <= r:
        return U, V
    qu, ru = np.linalg.qr(U)
    qv, rv = np.linalg.qr(V)
    w, s, zh = np.linalg.svd(ru @ rv.conj().T)
    return qu @ (w[:, :r] * s[:r]), qv @ zh.conj().T[:, :r]


class StripOperator:
    """Blocks of A = I - G0 V on column strips without the dense matrix (grids too large for it).

    A strip of whole grid columns [c0, c1) is a grid of its own: its diagonal
    block of A is the operator matrix of the kernel table's first c1 - c0 rows
    and the strip's contrast.  For disjoint index sets the off-diagonal block
    is -(G0 V)[I_out, I_in], applied as the strip's FFT convolution (eq. 11's
    product) with the input zero outside I_in and the output read on I_out.
    """

    def __init__(self, prob):
        self.prob = prob
        self._spec = {}

    def _ghat(self, w):
        if w not in self._spec:
            self._spec[w] = spectrum(self.prob.K[:w, :])
        return self._spec[w]

    def diag(self, c0, c1):
        return operator_matrix(self.prob.K[:c1 - c0, :], self.prob.chi[c0:c1])

    def block(self, c0, c_in, c_out):
        """(matvec, rmatvec) of A[I_out, I_in] within the strip starting at column c0; c_in, c_out are the
        (first, last + 1) columns of the input and output index sets."""
        nz = self.prob.nz
        w = max(c_in[1], c_out[1]) - c0
        chi = self.prob.chi[c0:c0 + w]
        gh = self._ghat(w)
        si = slice((c_in[0] - c0) * nz, (c_in[1] - c0) * nz)
        so = slice((c_out[0] - c0) * nz, (c_out[1] - c0) * nz)

        def run(x, src, dst, mode):
            k = x.shape[1]
            e = np.zeros((k, w * nz), np.complex128)
            e[:, src] = x.T
            y = apply_fft(gh, chi, e.reshape(k, w, nz), mode).reshape(k, w * nz)
            return -y[:, dst].T
        return (lambda x: run(x, si, so, "G0V")), (lambda y: run(y, so, si, "VHG0H"))


def range_finder_ops(matvec, rmatvec, omega, q=0):
    """Alg. 1 for a block given by its products with a block of vectors and with its adjoint."""
    Q = orth(matvec(omega))
    for _ in range(q):
        Qt = orth(rmatvec(Q))
        Q = orth(matvec(Qt))
    return Q, rmatvec(Q)


def build(A, tree, r, seed=0, probes=None, q=0, q_from_level=0):
    """HODLR approximation of A on the given tree (off-diagonal blocks by Alg. 1, q = 0 in Section 2.4).

    A: the dense matrix, or a `StripOperator`.
    q_from_level: the q power iterations are taken on the blocks of tree depth >= q_from_level only (not in
    the paper, which uses q = 0 throughout; 0 applies them everywhere).
    probes: optional callable depth -> real [r, n] block; a node at that depth
    samples its upper block A[I1, I2] with the probe rows restricted to I2 and
    its lower block A[I2, I1] with them restricted to I1.  Without it, the
    probes are drawn from numpy's PCG64 with `seed`.
    """
    rng = np.random.default_rng(seed)
    strips = A if isinstance(A, StripOperator) else None

    def fill(node, depth):
        if not hasattr(node, "children_cols"):
            if strips is not None:
                node.dense = strips.diag(*node.leaf_cols)
            else:
                node.dense = A[node.lo:node.hi, node.lo:node.hi].copy()
            return node
        node.a11, node.a22 = fill(node.c1, depth + 1), fill(node.c2, depth + 1)
        i1 = slice(node.a11.lo, node.a11.hi)
        i2 = slice(node.a22.lo, node.a22.hi)
        om = probes(depth) if probes is not None else None
        qd = q if depth >= q_from_level else 0
        if strips is None:
            node.u12, node.v12 = lowrank_from_block(A[i1, i2], r, rng, None if om is None else om[:, i2].T, qd)
            node.u21, node.v21 = lowrank_from_block(A[i2, i1], r, rng, None if om is None else om[:, i1].T, qd)
            return node
        c0, cm, c1 = node.children_cols
        o12 = rng.standard_normal((i2.stop - i2.start, r)) if om is None else om[:, i2].T
        node.u12, node.v12 = range_finder_ops(*strips.block(c0, (cm, c1), (c0, cm)), o12, qd)
        o21 = rng.standard_normal((i1.stop - i1.start, r)) if om is None else om[:, i1].T
        node.u21, node.v21 = range_finder_ops(*strips.block(c0, (c0, cm), (cm, c1)), o21, qd)
        return node
    return fill(tree, 0)


def add_lowrank(H, P, Q, r):
    """H + P Q^H kept in the HODLR structure of H (dense leaves updated, off-diagonal blocks truncated to r)."""
    out = Node(H.lo, H.hi)
    if H.is_leaf:
        out.dense = H.dense + P @ Q.conj().T
        return out
    m = H.a11.size
    out.a11 = add_lowrank(H.a11, P[:m], Q[:m], r)
    out.a22 = add_lowrank(H.a22, P[m:], Q[m:], r)
    out.u12, out.v12 = truncate(np.hstack([H.u12, P[:m]]), np.hstack([H.v12, Q[m:]]), r)
    out.u21, out.v21 = truncate(np.hstack([H.u21, P[m:]]), np.hstack([H.v21, Q[:m]]), r)
    return out


def invert(H, r):
    """Approximate inverse by the recursive 2x2 block formula (Section 2.4) in HODLR arithmetic."""
    out = Node(H.lo, H.hi)
    if H.is_leaf:
        out.dense = np.linalg.inv(H.dense)
        return out
    X = invert(H.a11, r)                                       # A^{-1}
    # S = D - C A^{-1} B = A22 - u21 (v21^H X u12) v12^H
    core = H.v21.conj().T @ X.matvec(H.u12)
    S = add_lowrank(H.a22, -H.u21 @ core, H.v12, r)
    Y = invert(S, r)                                           # S^{-1}
    XU = X.matvec(H.u12)                                       # A^{-1} B = XU v12^H
    YU = Y.matvec(H.u21)
    # top-right: -A^{-1} B S^{-1} = (-XU)(Y^H v12)^H ; bottom-left: -S^{-1} C A^{-1} = (-YU)(X^H v21)^H
    out.u12, out.v12 = -XU, Y.rmatvec(H.v12)
    out.u21, out.v21 = -YU, X.rmatvec(H.v21)
    # top-left: A^{-1} + A^{-1} B S^{-1} C A^{-1} = X + XU (v12^H Y u21) (X^H v21)^H
    mid = H.v12.conj().T @ YU
    out.a11 = add_lowrank(X, XU @ mid, X.rmatvec(H.v21), r)
    out.a22 = Y
    return out


class HodlrPreconditioner:
    """H = (HODLR approximation of I - G0 V)^{-1}, used in eq. (11) (Section 2.4)."""

    def __init__(self, prob, rank, levels, min_width=1, seed=0, probes=None):
        A = operator_matrix(prob.K, prob.chi)
        self.tree = split_tree(prob.nx, prob.nz, levels, min_width)
        self.approx = build(A, self.tree, rank, seed, probes)
        self.inv = invert(self.approx, rank)
        self.n = prob.n

    def apply(self, x):
        x = np.asarray(x, np.complex128)
        shp = x.shape
        y = self.inv.matvec(x.reshape(-1, self.n).T)
        return y.T.reshape(shp)


class HodlrSolve:
    """Exact inverse of the HODLR approximation, applied by nested Sherman-Morrison-Woodbury solves.

    For a node with diagonal children A11, A22 and A12 = u12 v12^H,
    A21 = u21 v21^H: A = D + Ut Vt^H with D = diag(A11, A22),
    Ut = diag(u12, u21), Vt^H = [[0, v12^H], [v21^H, 0]], so
    A^{-1} b = D^{-1} b - diag(W1, W2) K^{-1} Vt^H D^{-1} b with
    W1 = A11^{-1} u12, W2 = A22^{-1} u21 and K = I + Vt^H diag(W1, W2).
    This is the same HODLR approximation of I - G0 V as `HodlrPreconditioner`,
    inverted without the rank truncation of the H-arithmetic inverse.
    """

    def __init__(self, prob, rank, levels, min_width=1, seed=0, probes=None, q=0, matrix_free=False,
                 q_from_level=0):
        A = StripOperator(prob) if matrix_free else operator_matrix(prob.K, prob.chi)
        self.tree = split_tree(prob.nx, prob.nz, levels, min_width)
        self.approx = build(A, self.tree, rank, seed, probes, q, q_from_level)
        self.n = prob.n
        self._prepare(self.approx)

    def _prepare(self, node):
        if node.is_leaf:
            node.inv_dense = np.linalg.inv(node.dense)
            return
        self._prepare(node.a11)
        self._prepare(node.a22)
        node.w1 = self.solve_node(node.a11, node.u12)
        node.w2 = self.solve_node(node.a22, node.u21)
        r1, r2 = node.u12.shape[1], node.u21.shape[1]
        K = np.eye(r1 + r2, dtype=np.complex128)
        K[:r1, r1:] = node.v12.conj().T @ node.w2
        K[r1:, :r1] = node.v21.conj().T @ node.w1
        node.kinv = np.linalg.inv(K)

    def solve_node(self, node, b):
        if node.is_leaf:
            return node.inv_dense @ b
        m = node.a11.size
        y1 = self.solve_node(node.a11, b[:m])
        y2 = self.solve_node(node.a22, b[m:])
        r1 = node.u12.shape[1]
        t = np.vstack([node.v12.conj().T @ y2, node.v21.conj().T @ y1])
        s = node.kinv @ t
        return np.vstack([y1 - node.w1 @ s[:r1], y2 - node.w2 @ s[r1:]])

    def apply(self, x):
        x = np.asarray(x, np.complex128)
        shp = x.shape
        y = self.solve_node(self.approx, x.reshape(-1, self.n).T)
        return y.T.reshape(shp)
