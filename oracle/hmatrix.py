"""Oracle-on-H: the FP64 product and fixed point of a given compressed operator.

TEST INFRASTRUCTURE: part of the FP64 CPU oracle (see the package docstring).

Section "Compression": once the matrix is compressed, the fixed-point
iterations only need matrix-vector products with the H-matrix.  Its blocks
are interactions between a cluster of targets and a cluster of sources; a
block that is not admissible is kept dense and contributes A x[cols], an
admissible block is approximated by a low-rank product U V^T and contributes
U (V^T x[cols]).  The blocks partition the matrix, in the cluster order of the
targets and of the sources.

This module applies such an operator in FP64 with plain numpy products, one
block at a time, from its parts only: the two cluster orders, the dense
blocks and the low-rank factors.  Where the parts come from is the caller's
business: the tests build them from the oracle's own dense matrix (to pin
this module), or read them back from the GPU library's assembled operator,
upcast to FP64, so that the library's arithmetic (matvec, fixed point) is
checked against the same compressed operator; compression error is then a
separate figure, measured against the dense oracle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class HOperator:
    """An H-matrix given by its blocks.

    tgt_perm[k] is the row (natural order) of the k-th target in cluster
    order; src_perm[k] the column of the k-th source.  dense: list of
    (t0, t1, s0, s1, A) with A of shape (t1 - t0, s1 - s0); lowrank: list of
    (t0, t1, s0, s1, U, V) with U (t1 - t0, k) and V (s1 - s0, k); ranges are
    half-open, in cluster order."""
    tgt_perm: np.ndarray
    src_perm: np.ndarray
    dense: list = field(default_factory=list)
    lowrank: list = field(default_factory=list)

    @property
    def shape(self):
        return (len(self.tgt_perm), len(self.src_perm))

    def _apply(self, x, absolute: bool):
        x = np.asarray(x, dtype=np.float64)
        single = x.ndim == 1
        X = x[None, :] if single else x                     # [nrhs, n_src] natural order
        Xc = X[:, self.src_perm]                            # cluster order of the sources
        Yc = np.zeros((X.shape[0], len(self.tgt_perm)))
        for t0, t1, s0, s1, A in self.dense:
            Ab = np.abs(A) if absolute else A
            Yc[:, t0:t1] += Xc[:, s0:s1] @ Ab.T
        for t0, t1, s0, s1, U, V in self.lowrank:
            if absolute:
                U, V = np.abs(U), np.abs(V)
            Yc[:, t0:t1] += (Xc[:, s0:s1] @ V) @ U.T          # U (V^T x) per right-hand side
        Y = np.empty_like(Yc)
        Y[:, self.tgt_perm] = Yc
        return Y[0] if single else Y

    def matvec(self, x):
        """y = H x; x: [n_src] or [nrhs, n_src] in natural order."""
        return self._apply(x, False)

    def abs_matvec(self, x):
        """sum over blocks of |A| |x| and |U| (|V|^T |x|): the scale that bounds the
        rounding error of any summation order of H x, element by element."""
        return self._apply(np.abs(np.asarray(x, dtype=np.float64)), True)

    def __matmul__(self, x):
        return self.matvec(x)

    def to_dense(self) -> np.ndarray:
        out = np.zeros(self.shape)
        rows, cols = self.tgt_perm, self.src_perm
        for t0, t1, s0, s1, A in self.dense:
            out[np.ix_(rows[t0:t1], cols[s0:s1])] = A
        for t0, t1, s0, s1, U, V in self.lowrank:
            out[np.ix_(rows[t0:t1], cols[s0:s1])] = U @ V.T
        return out

    def stored_entries(self) -> int:
        """Entries of the stored operator: m n per dense block, (m + n) k per low-rank one."""
        return int(sum(A.size for *_, A in self.dense) + sum(U.size + V.size for *_, U, V in self.lowrank))


def from_dense(M, tgt_perm, src_perm, dense_blocks, lowrank_blocks, factor) -> HOperator:
    """An HOperator over a given block partition whose dense blocks are the
    corresponding blocks of the matrix M (rows and columns in natural order) and
    whose admissible blocks are factor(A) -> (U, V)."""
    tgt_perm = np.asarray(tgt_perm, dtype=np.int64)
    src_perm = np.asarray(src_perm, dtype=np.int64)
    H = HOperator(tgt_perm, src_perm)
    for t0, t1, s0, s1 in dense_blocks:
        H.dense.append((t0, t1, s0, s1, M[np.ix_(tgt_perm[t0:t1], src_perm[s0:s1])]))
    for t0, t1, s0, s1 in lowrank_blocks:
        U, V = factor(M[np.ix_(tgt_perm[t0:t1], src_perm[s0:s1])])
        H.lowrank.append((t0, t1, s0, s1, U, V))
    return H


def truncated_svd(eps: float):
    """factor(A): the shortest truncated SVD with relative Frobenius error <= eps
    (the error measure of the ACA in Section "Compression")."""
    def factor(A):
        u, s, vt = np.linalg.svd(A, full_matrices=False)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])     # tail[k] = ||s[k:]||
        total = tail[0] if len(s) else 0.0
        k = next((k for k in range(1, len(s) + 1) if k == len(s) or tail[k] <= eps * total), len(s))
        return u[:, :k] * s[:k], vt[:k].T
    return factor


def full_rank(A):
    """factor(A) = (A, I): the low-rank form of a block that loses nothing."""
    return A.copy(), np.eye(A.shape[1])


def recompress(U, V, eps: float):
    """The shortest truncation of the SVD of U V^T whose relative Frobenius error
    is <= eps (at least rank 1): the recompression of an ACA block's factors
    (Section "Compression": the ACA approximates the first terms of a block's
    SVD; its factors are not orthogonal and usually longer than the SVD needs).
    Written as the definition: U = Qu Ru and V = Qv Rv (QR), the SVD of the
    small Ru Rv^T = W S Z^T, then U' = Qu W_r S_r and V' = Qv Z_r."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    w, sv, zt = np.linalg.svd(Ru @ Rv.T)
    tail = np.sqrt(np.cumsum((sv ** 2)[::-1])[::-1])      # tail[r] = ||s[r:]||
    total = tail[0] if len(sv) else 0.0
    r = next((r for r in range(1, len(sv) + 1) if r == len(sv) or tail[r] <= eps * total), len(sv))
    return Qu @ (w[:, :r] * sv[:r]), Qv @ zt[:r].T, sv

