"""Cluster tree and block tree of the H-matrix, written plainly in Python.

TEST INFRASTRUCTURE: part of the FP64 CPU oracle (see the package docstring).
It is index work, so the GPU library's host trees must reproduce it exactly.

Section "Compression": the matrix is viewed as a hierarchical tree of blocks
of interactions between clusters of points; one descends the tree until a
block satisfies max(R1, R2) < eta |x1 - x2| and compresses it, and a block
reached at the leaves is kept dense.  Readings used here:
  - cluster split: the tight bounding box of the cluster's points is halved at
    its midpoint along its longest axis (ties: lowest axis); a point on the
    plane goes to the lower child; the order within each child is the parent's
    order; a cluster with at most leaf_size points is a leaf;
  - R is half the diagonal of the tight bounding box, and the distance is the
    gap between the two bounding boxes (0 when they touch or overlap), so
    touching blocks are never admissible; the test is evaluated as
    R^2 < eta^2 * dist^2 in FP64;
  - a block whose storage break-even rank floor(m n / (m + n)) is below
    MIN_LOW_RANK is not admissible (it is split or kept dense);
  - if exactly one side of a non-admissible block is a leaf, the other side
    is split; if both are leaves the block is dense.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Cluster:
    start: int            # range [start, stop) in the permuted order
    stop: int
    bmin: np.ndarray      # tight bounding box
    bmax: np.ndarray
    children: list = field(default_factory=list)

    @property
    def size(self):
        return self.stop - self.start


def cluster_tree(points: np.ndarray, leaf_size: int):
    """Returns (perm, root): perm[k] is the original index of the k-th point in cluster order."""
    points = np.asarray(points, dtype=np.float64)
    perm = np.arange(len(points), dtype=np.int64)

    def build(start, stop):
        idx = perm[start:stop]
        pts = points[idx]
        bmin, bmax = pts.min(axis=0), pts.max(axis=0)
        node = Cluster(start, stop, bmin, bmax)
        if stop - start <= leaf_size:
            return node
        ext = bmax - bmin
        axis = int(np.argmax(ext))          # first maximum = lowest axis on ties
        mid = 0.5 * (bmin[axis] + bmax[axis])
        low = pts[:, axis] <= mid
        perm[start:stop] = np.concatenate([idx[low], idx[~low]])
        cut = start + int(low.sum())
        node.children = [build(start, cut), build(cut, stop)]
        return node

    root = build(0, len(points))
    return perm, root


MIN_LOW_RANK = 24


def _separated(tmin, tmax, smin, smax, eta: float) -> bool:
    ht = 0.5 * (tmax - tmin)
    hs = 0.5 * (smax - smin)
    rt2 = ht[0] * ht[0] + ht[1] * ht[1] + ht[2] * ht[2]
    rs2 = hs[0] * hs[0] + hs[1] * hs[1] + hs[2] * hs[2]
    gap = np.maximum(0.0, np.maximum(smin - tmax, tmin - smax))
    d2 = gap[0] * gap[0] + gap[1] * gap[1] + gap[2] * gap[2]
    return max(rt2, rs2) < eta * eta * d2


def admissible(t: Cluster, s: Cluster, eta: float) -> bool:
    m, n = t.size, s.size
    if m * n // (m + n) < MIN_LOW_RANK:
        return False
    return _separated(t.bmin, t.bmax, s.bmin, s.bmax, eta)


def block_tree(troot: Cluster, sroot: Cluster, eta: float):
    """Returns (dense, lowrank): lists of (t0, t1, s0, s1) ranges in cluster order."""
    dense, lowrank = [], []

    def rec(t, s):
        if admissible(t, s, eta):
            lowrank.append((t.start, t.stop, s.start, s.stop))
        elif not t.children and not s.children:
            dense.append((t.start, t.stop, s.start, s.stop))
        elif not t.children:
            for sc in s.children:
                rec(t, sc)
        elif not s.children:
            for tc in t.children:
                rec(tc, s)
        else:
            for tc in t.children:
                for sc in s.children:
                    rec(tc, sc)

    rec(troot, sroot)
    return dense, lowrank


def leaves(root: Cluster):
    out = []

    def rec(c):
        if not c.children:
            out.append((c.start, c.stop))
        for ch in c.children:
            rec(ch)

    rec(root)
    return out
