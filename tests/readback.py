"""Read an assembled operator back from the GPU library into the oracle's
H-operator form (oracle/hmatrix.py), for the tests that check the library's
arithmetic against the FP64 product and fixed point of the same compressed
operator.

Everything here is marshalling: the cluster orders come from the host plan
(rte_plan_export), the dense blocks and low-rank factors from the library's
read-back calls (rte_hmat_dense_block, rte_hmat_block_factors_op), widened to
FP64 exactly.  No arithmetic of the method is done here."""
from __future__ import annotations

import numpy as np

from oracle.hmatrix import HOperator
from paper_2306_05789_amd import rte


def gpu_operator(mesh, H, opts, band: int = 0, op: int = rte.RTE_OP_ACCURATE) -> HOperator:
    """The stored operator of one band of H as an HOperator in natural order
    (surface operators: sources are positions in the ascending emitting-id list)."""
    plan = rte.rte_plan_create(mesh, opts)
    try:
        tp, sp, blocks = rte.rte_plan_export(plan)
    finally:
        rte.rte_plan_destroy(plan)
    if opts.kind == rte.RTE_SURFACE:
        em = rte.rte_mesh_emitting_ids(mesh)
        pos = np.searchsorted(em, sp)
        assert np.array_equal(em[pos], sp), "surface sources must be emitting vertices"
        sp = pos
    out = HOperator(tp.astype(np.int64), sp.astype(np.int64))
    for d in range(rte.rte_hmat_dense_count(H, band)):
        (t0, t1, s0, s1), A = rte.rte_hmat_dense_block(H, band, d, op)
        out.dense.append((t0, t1, s0, s1, A))
    low = blocks[blocks[:, 4] == 1]
    covered = sum((t1 - t0) * (s1 - s0) for t0, t1, s0, s1, _ in out.dense)
    for b in range(len(low)):
        k, U, V = rte.rte_hmat_block_factors_op(H, band, b, op)
        if k <= 0:
            continue      # stored dense: among the dense blocks above
        t0, t1, s0, s1 = (int(v) for v in low[b][:4])
        out.lowrank.append((t0, t1, s0, s1, U, V))
        covered += (t1 - t0) * (s1 - s0)
    assert covered == len(tp) * len(sp), "the read-back blocks do not cover the matrix"
    return out
