"""Pins of the oracle-on-H (oracle/hmatrix.py) against the dense oracle.

The module applies an H-matrix given by its parts (cluster orders, dense
blocks, low-rank factors) in FP64, block by block (Section "Compression").
Here the parts are built from the oracle's own dense matrices over the
oracle's block tree, so the products can be checked against plain dense
products: with lossless factors (U = A, V = I) the H product must equal the
dense one to rounding, with truncated SVD factors its error must stay within
the sum of the blocks' truncation errors, and the fixed point of a lossless H
operator must be the dense fixed point.  A wrong permutation direction, a
transposed factor, a dropped block or a block applied twice fails one of
these.  No GPU is used."""
import numpy as np
import pytest

from oracle import hmatrix, solve
from oracle.core import Grid, Problem
from oracle.htree import block_tree, cluster_tree

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.fixture(scope="module")
def reflect9():
    """9^3 box with random kappa, a reflective wall and two emitting faces, its dense
    G and S from the oracle, and the oracle's trees (leaf 16, eta 2)."""
    g = Grid((9, 9, 9), (0, 0, 0), (1.0, 0.9, 0.8))
    kap = np.random.default_rng(3).uniform(0.2, 2.0, g.N)
    P = Problem(g, kap, emit_faces=1 | 8, wall_axis=2, wall_side=0, R=0.5)
    G, S = P.dense_G(), P.dense_S()
    pts = g.positions()
    em = P.emitting
    tperm, troot = cluster_tree(pts, 16)
    sperm, sroot = cluster_tree(pts[em], 16)
    gd, gl = block_tree(troot, troot, 2.0)
    sd, sl = block_tree(troot, sroot, 2.0)
    assert len(gl) > 4 and len(sl) > 0
    return P, G, S, tperm, sperm, (gd, gl), (sd, sl)


def test_lossless_H_equals_the_dense_operator(reflect9):
    P, G, S, tperm, sperm, (gd, gl), (sd, sl) = reflect9
    H = hmatrix.from_dense(G, tperm, tperm, gd, gl, hmatrix.full_rank)
    assert np.array_equal(H.to_dense(), G)
    X = np.random.default_rng(1).standard_normal((3, G.shape[1]))
    Y = H.matvec(X)
    scale = H.abs_matvec(X)
    assert np.all(np.abs(Y - X @ G.T) <= 1e-13 * scale)
    # single right-hand side, and the @ form used by the fixed point
    assert np.all(np.abs(H @ X[0] - G @ X[0]) <= 1e-13 * scale[0])
    # the rounding scale bounds the product and equals it for nonnegative data
    assert np.all(np.abs(Y) <= scale * (1 + 1e-12))
    xp = np.abs(X[0])
    assert np.allclose(H.abs_matvec(xp), H.matvec(xp), rtol=1e-13, atol=0)


def test_lossless_surface_H_maps_emitting_positions(reflect9):
    """Rectangular N x L operator: the source order is a permutation of the
    emitting-vertex positions 0..L-1."""
    P, G, S, tperm, sperm, _, (sd, sl) = reflect9
    H = hmatrix.from_dense(S, tperm, sperm, sd, sl, hmatrix.full_rank)
    assert H.shape == S.shape
    q = np.random.default_rng(2).uniform(0.5, 2.0, S.shape[1])
    assert np.all(np.abs(H @ q - S @ q) <= 1e-13 * H.abs_matvec(q))


def test_truncated_H_error_within_the_blocks_truncation(reflect9):
    """Factors from truncated SVDs at relative Frobenius error 1e-5: the product's
    error is bounded by sum over blocks of ||A - U V^T||_F ||x_block||, and the
    truncation drops singular values."""
    P, G, S, tperm, sperm, (gd, gl), _ = reflect9
    eps = 1e-5
    H = hmatrix.from_dense(G, tperm, tperm, gd, gl, hmatrix.truncated_svd(eps))
    assert any(U.shape[1] < min(U.shape[0], V.shape[0]) for *_, U, V in H.lowrank)
    x = np.random.default_rng(4).uniform(0.0, 1.0, G.shape[1])
    err = np.zeros(G.shape[0])
    xc = x[tperm]
    for t0, t1, s0, s1, U, V in H.lowrank:
        A = G[np.ix_(tperm[t0:t1], tperm[s0:s1])]
        e = np.linalg.norm(A - U @ V.T)
        assert e <= eps * np.linalg.norm(A) * (1 + 1e-9)
        err[tperm[t0:t1]] += e * np.linalg.norm(xc[s0:s1])
    d = np.abs(H @ x - G @ x)
    # per row, |(H - G) x|_i <= sum over the row's blocks of ||A_b - U_b V_b^T||_F ||x_b||
    assert np.all(d <= err * (1 + 1e-9) + 1e-15 * H.abs_matvec(x))
    assert d.max() > 0


def test_fixed_point_of_lossless_H_is_the_dense_fixed_point(reflect9):
    """The oracle's fixed point (Algorithm, eq. algo) run on lossless H operators
    reaches the fixed point of the dense operators."""
    P, G, S, tperm, sperm, (gd, gl), (sd, sl) = reflect9
    HG = hmatrix.from_dense(G, tperm, tperm, gd, gl, hmatrix.full_rank)
    HS = hmatrix.from_dense(S, tperm, sperm, sd, sl, hmatrix.full_rank)
    q = solve.SIGMA * np.ones(S.shape[1])
    ref = solve.fixed_point([G], (S @ q)[None], grey=True, tol=1e-14)
    got = solve.fixed_point([HG], (HS @ q)[None], grey=True, tol=1e-14)
    assert np.max(np.abs(got.T - ref.T) / ref.T) < 1e-12
    assert got.iterations == ref.iterations


def test_dropped_or_doubled_block_is_detected(reflect9):
    """A plausible mistake in assembling the parts changes the product far above
    the rounding scale: one block left out, or one block applied twice."""
    P, G, S, tperm, sperm, (gd, gl), _ = reflect9
    x = np.random.default_rng(6).uniform(0.5, 1.0, G.shape[1])
    H = hmatrix.from_dense(G, tperm, tperm, gd, gl, hmatrix.full_rank)
    drop = hmatrix.HOperator(H.tgt_perm, H.src_perm, H.dense, H.lowrank[1:])
    twice = hmatrix.HOperator(H.tgt_perm, H.src_perm, H.dense + H.dense[:1], H.lowrank)
    swapped = hmatrix.HOperator(H.src_perm[::-1].copy(), H.src_perm, H.dense, H.lowrank)
    for bad in (drop, twice, swapped):
        assert np.max(np.abs(bad @ x - G @ x) / H.abs_matvec(x)) > 1e-6


# ---------------------------------------------------------------- recompression of low-rank factors

def _factors(rng, m, n, k, decay):
    """Factors of a k-term product whose terms fall off like decay^l, with
    non-orthogonal columns (as the ACA's are)."""
    U = rng.standard_normal((m, k)) * decay ** np.arange(k)
    V = rng.standard_normal((n, k)) + 0.3 * rng.standard_normal((n, 1))
    return U, V


def test_recompression_is_the_truncated_svd_of_the_product():
    """Eckart-Young: the recompressed product is the best approximation of U V^T
    of its rank, the dense truncated SVD of the product (same rank, same matrix)."""
    rng = np.random.default_rng(31)
    cut = 0
    for m, n, k in ((120, 90, 30), (64, 200, 41), (300, 300, 12)):
        U, V = _factors(rng, m, n, k, 0.6)
        A = U @ V.T
        for eps in (1e-5, 1e-3):
            Ur, Vr, _ = hmatrix.recompress(U, V, eps)
            Ud, Vd = hmatrix.truncated_svd(eps)(A)
            assert Ur.shape[1] == Ud.shape[1] <= k
            cut += Ur.shape[1] < k
            assert np.linalg.norm(Ur @ Vr.T - Ud @ Vd.T) < 1e-12 * np.linalg.norm(A)
    assert cut >= 4


def test_recompression_error_is_the_dropped_tail():
    """||U V^T - U' V'^T||_F equals the norm of the dropped singular values and
    stays within eps of ||U V^T||_F; a product of planted rank r is recompressed
    to rank r exactly."""
    rng = np.random.default_rng(32)
    U, V = _factors(rng, 150, 110, 40, 0.7)
    A = U @ V.T
    Ur, Vr, sv = hmatrix.recompress(U, V, 1e-4)
    r = Ur.shape[1]
    err = np.linalg.norm(A - Ur @ Vr.T)
    assert abs(err - np.linalg.norm(sv[r:])) < 1e-10 * np.linalg.norm(A)
    assert err <= 1e-4 * np.linalg.norm(A)
    assert np.linalg.norm(sv[r - 1:]) > 1e-4 * np.linalg.norm(A)     # the shortest such
    # planted rank: 40 columns spanning a 9-dimensional space
    B = rng.standard_normal((150, 9)) @ rng.standard_normal((9, 40))
    Ur, Vr, _ = hmatrix.recompress(B, V, 1e-10)
    assert Ur.shape[1] == 9
    assert np.linalg.norm(B @ V.T - Ur @ Vr.T) < 1e-12 * np.linalg.norm(B @ V.T)

