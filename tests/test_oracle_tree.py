"""Invariants of the oracle's cluster and block trees (Section "Compression").

These hold for any correct H-matrix partition: the permutation is a
bijection, leaves partition the points, the blocks cover the matrix exactly
once, admissible blocks are separated and satisfy the admissibility test,
and dense blocks join two leaves."""
import numpy as np
import pytest

from oracle.core import Grid
from oracle.htree import MIN_LOW_RANK, admissible, block_tree, cluster_tree, leaves


@pytest.mark.parametrize("n,leaf", [((9, 9, 9), 32), ((13, 7, 7), 64), ((11, 11, 11), 64)])
def test_cluster_and_block_tree_invariants(n, leaf):
    g = Grid(n, (0, 0, 0), (n[0] / n[1], 1, 1))
    pts = g.positions()
    perm, root = cluster_tree(pts, leaf)
    assert np.array_equal(np.sort(perm), np.arange(g.N))
    lv = leaves(root)
    assert lv[0][0] == 0 and lv[-1][1] == g.N
    assert all(a[1] == b[0] for a, b in zip(lv, lv[1:]))
    assert all(0 < b - a <= leaf for a, b in lv)
    dense, low = block_tree(root, root, 2.0)
    cover = np.zeros((g.N, g.N), dtype=np.int32)
    for t0, t1, s0, s1 in dense + low:
        cover[t0:t1, s0:s1] += 1
    assert np.all(cover == 1)
    leafset = set(lv)
    for t0, t1, s0, s1 in dense:
        assert (t0, t1) in leafset and (s0, s1) in leafset
    for t0, t1, s0, s1 in low:
        a, b = pts[perm[t0:t1]], pts[perm[s0:s1]]
        gap = np.maximum(0, np.maximum(b.min(0) - a.max(0), a.min(0) - b.max(0)))
        d = np.linalg.norm(gap)
        assert d > 0
        r = 0.5 * max(np.linalg.norm(a.max(0) - a.min(0)), np.linalg.norm(b.max(0) - b.min(0)))
        assert r < 2.0 * d * (1 + 1e-12)
    assert len(low) > 0


def test_rectangular_surface_tree_covers_once():
    g = Grid((9, 9, 9))
    pts = g.positions()
    em = g.emitting_vertices(1 | 8)
    tperm, troot = cluster_tree(pts, 32)
    sperm, sroot = cluster_tree(pts[em], 32)
    dense, low = block_tree(troot, sroot, 2.0)
    cover = np.zeros((g.N, len(em)), dtype=np.int32)
    for t0, t1, s0, s1 in dense + low:
        cover[t0:t1, s0:s1] += 1
    assert np.all(cover == 1)


def test_split_rule_midpoint_longest_axis_lower_child_takes_the_plane():
    # 5 x 3 x 1 points: the longest axis is x; the midpoint plane x = 2 holds a column
    g = Grid((5, 3, 1 + 1), (0, 0, 0), (4, 2, 1))
    pts = g.positions()
    perm, root = cluster_tree(pts, 20)
    lo, hi = root.children
    assert np.all(pts[perm[lo.start:lo.stop], 0] <= 2.0)
    assert np.all(pts[perm[hi.start:hi.stop], 0] > 2.0)
    assert lo.size == 18 and hi.size == 12
    # within a child the parent's (natural) order is kept
    assert np.all(np.diff(perm[lo.start:lo.stop]) > 0)


def test_low_rank_blocks_pay_for_their_rank():
    """Every compressed block can hold a rank of at least MIN_LOW_RANK below its
    storage break-even floor(m n / (m + n)); smaller admissible blocks are split
    or kept dense, and the partition still covers the matrix once."""
    g = Grid((13, 13, 13))
    pts = g.positions()
    perm, root = cluster_tree(pts, 32)
    dense, low = block_tree(root, root, 2.0)
    assert low and all((t1 - t0) * (s1 - s0) // ((t1 - t0) + (s1 - s0)) >= MIN_LOW_RANK for t0, t1, s0, s1 in low)
    cover = np.zeros((g.N, g.N), dtype=np.int32)
    for t0, t1, s0, s1 in dense + low:
        cover[t0:t1, s0:s1] += 1
    assert np.all(cover == 1)

