"""GPU: mixed precision (FP32 entries and ACA, BF16 hi + lo low-rank factors,
inner sweeps on the BF16-hi operator, FP64 defect correction) on a reflective
multi-band case, against the FP64 oracle and the FP64 GPU path."""
import numpy as np
import pytest
import torch

from oracle import solve as osolve
from oracle.core import Grid, Problem
from paper_2306_05789_amd import inputs, rte

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NU = np.array([0.5, 1.4, 4.0])
N3 = (17, 9, 9)
HI = (2.0, 1.0, 1.0)


@pytest.fixture(scope="module")
def reflect_small():
    """Box [0,2]x[0,1]^2, wall z = 0 with R = 0.5, x = 0 at T = 1, kappa_nu = kappa(x) nu^-1.5."""
    g = Grid(N3, (0, 0, 0), HI)
    kb = inputs.smooth_kappa(g.positions())[None, :] * NU[:, None] ** -1.5
    Gs, SEs = [], []
    for b in range(len(NU)):
        P = Problem(g, kb[b], emit_faces=1, wall_axis=2, wall_side=0, R=0.5)
        Gs.append(P.dense_G())
        SEs.append(P.dense_S() @ osolve.planck(NU[b], np.ones(len(P.emitting))))
    ref = osolve.fixed_point(Gs, np.array(SEs), grey=False, nu=NU, kappa_v=kb, tol=1e-13)
    mesh = rte.rte_mesh_create(N3, (0, 0, 0), HI, reflect_axis=2, reflect_side=0, R=0.5, emit_faces=1)
    return g, kb, Gs, ref, mesh


def _solve(mesh, kb, precision, solve_precision, tol, leaf=32):
    kt = torch.tensor(kb, device=DEV)
    G = rte.rte_hmat_assemble(mesh, kt, rte.hmat_opts(kind=rte.RTE_VOLUME, leaf_size=leaf, precision=precision))
    S = rte.rte_hmat_assemble(mesh, kt, rte.hmat_opts(kind=rte.RTE_SURFACE, leaf_size=leaf, precision=precision))
    T = torch.empty((1, mesh.N), device=DEV, dtype=torch.float64)
    J = torch.empty((1, len(NU), mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, G, S, torch.ones((1, mesh.L), device=DEV, dtype=torch.float64), T, J,
                                   grey=False, nu=NU, tol=tol, max_iter=2000, precision=solve_precision)
    return G, S, T.cpu().numpy()[0], J.cpu().numpy()[0], st


def test_mixed_solve_reaches_fp64_residual_and_matches_oracle(reflect_small):
    g, kb, Gs, ref, mesh = reflect_small
    G, S, T, J, st = _solve(mesh, kb, rte.RTE_MIXED_BF16, rte.RTE_MIXED_BF16, 1e-6)
    assert st["converged"] and st["residual"] <= 1e-6
    assert st["outer_steps"] >= 2 and st["iterations"] > st["outer_steps"]
    # compression (ACA 1e-5) dominates the difference from the dense oracle
    assert np.max(np.abs(T - ref.T) / ref.T) < 3e-4
    _, _, T64, _, st64 = _solve(mesh, kb, rte.RTE_FP64, rte.RTE_FP64, 1e-10)
    assert np.max(np.abs(T - T64) / T64) < 3e-4
    assert rte.rte_hmat_stats(G)["bytes"] < rte.rte_hmat_stats(_solve_bytes(mesh, kb))["bytes"]


def _solve_bytes(mesh, kb):
    kt = torch.tensor(kb, device=DEV)
    return rte.rte_hmat_assemble(mesh, kt, rte.hmat_opts(kind=rte.RTE_VOLUME, leaf_size=32, precision=rte.RTE_FP64))


def test_mixed_solution_is_a_fixed_point_of_the_stored_operator(reflect_small):
    """J_out = S^E + G S(T_out) up to the stopping tolerance, with G applied through
    the library's accurate (hi + lo) matvec."""
    g, kb, Gs, ref, mesh = reflect_small
    G, S, T, J, st = _solve(mesh, kb, rte.RTE_MIXED_BF16, rte.RTE_MIXED_BF16, 1e-7)
    for b in range(len(NU)):
        q = torch.tensor(osolve.planck(NU[b], np.ones(mesh.L)), device=DEV)
        se = torch.empty(mesh.N, device=DEV, dtype=torch.float64)
        rte.rte_hmat_matvec(S, b, q, se)
        src = torch.tensor(osolve.planck(NU[b], T), device=DEV)
        gj = torch.empty(mesh.N, device=DEV, dtype=torch.float64)
        rte.rte_hmat_matvec(G, b, src, gj)
        pred = (se + gj).cpu().numpy()
        assert np.linalg.norm(pred - J[b]) / np.linalg.norm(J[b]) < 2e-6


def test_fp32_solve_close_to_fp64(reflect_small):
    g, kb, Gs, ref, mesh = reflect_small
    _, _, T32, _, st = _solve(mesh, kb, rte.RTE_FP32, rte.RTE_FP32, 1e-8)
    assert st["converged"]
    assert np.max(np.abs(T32 - ref.T) / ref.T) < 3e-4


def test_mixed_factors_meet_the_tolerance():
    n = 13
    g = Grid((n, n, n))
    kap = inputs.smooth_kappa(g.positions())
    P = Problem(g, kap, emit_faces=1)
    Gd = P.dense_G()
    mesh = rte.rte_mesh_create((n, n, n), emit_faces=1)
    H = rte.rte_hmat_assemble(mesh, torch.tensor(kap[None, :], device=DEV),
                              rte.hmat_opts(leaf_size=32, precision=rte.RTE_MIXED_BF16))
    plan = rte.rte_plan_create(mesh, rte.hmat_opts(leaf_size=32))
    tp, sp, blocks = rte.rte_plan_export(plan)
    low = blocks[blocks[:, 4] == 1]
    errs = []
    for b in range(len(low)):
        t0, t1, s0, s1, _ = low[b]
        k, U, V = rte.rte_hmat_block_factors(H, 0, b)
        if k < 0:
            continue
        A = Gd[np.ix_(tp[t0:t1], sp[s0:s1])]
        errs.append(np.linalg.norm(A - U @ V.T) / np.linalg.norm(A))
    errs = np.array(errs)
    assert len(errs) > 10
    # FP32 ACA at 1e-5 plus the 16-bit hi + lo representation of each factor element
    assert errs.max() < 1e-3 and np.median(errs) < 1e-4, (errs.max(), np.median(errs))
