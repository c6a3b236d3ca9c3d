"""GPU: several planar reflective walls (the three reflective planes of Section
"An Academic Test"; each ray reflects at most once, Hypothesis 1, so every
wall adds its own mirror-image term), against the FP64 oracle: dense solves
against the oracle's fixed point, compressed solves against the oracle's
fixed point of the same read-back operators."""
import numpy as np
import pytest
import torch

import readback
from oracle import solve as osolve
from oracle.core import Grid, Problem
from paper_2306_05789_amd import inputs, rte

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# the three planes through the origin reflect perfectly (R = 1), as in the academic test;
# the opposite faces x = 1 and y = 1 emit
THREE = [(0, 0, 1.0), (1, 0, 1.0), (2, 0, 1.0)]
EMIT = inputs.FACE_X_HI | inputs.FACE_Y_HI


def _mesh(n, hi, walls, emit):
    return rte.rte_mesh_create(n, (0, 0, 0), hi, emit_faces=emit, walls=walls)


def test_three_walls_dense_grey_solve_matches_oracle():
    n, hi = (9, 9, 9), (1.0, 1.0, 1.0)
    g = Grid(n, (0, 0, 0), hi)
    kap = inputs.smooth_kappa(g.positions())
    P = Problem(g, kap, emit_faces=EMIT, walls=THREE)
    ref = osolve.fixed_point([P.dense_G()], (P.dense_S() @ np.full(len(P.emitting), osolve.SIGMA))[None],
                             grey=True, tol=1e-14)
    mesh = _mesh(n, hi, THREE, EMIT)
    kt = torch.tensor(kap[None, :], device=DEV)
    G = rte.rte_hmat_assemble(mesh, kt, rte.hmat_opts(kind=rte.RTE_VOLUME, dense=True))
    S = rte.rte_hmat_assemble(mesh, kt, rte.hmat_opts(kind=rte.RTE_SURFACE, dense=True))
    T = torch.empty((1, mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, G, S, torch.ones((1, mesh.L), device=DEV, dtype=torch.float64), T,
                                   grey=True, tol=1e-14, max_iter=1000)
    assert st["converged"] and st["monotone_violations"] == 0
    assert np.max(np.abs(T.cpu().numpy()[0] - ref.T) / ref.T) < 1e-10
    # the walls matter: without them the solution is colder near the walls
    P0 = Problem(g, kap, emit_faces=EMIT)
    ref0 = osolve.fixed_point([P0.dense_G()], (P0.dense_S() @ np.full(len(P0.emitting), osolve.SIGMA))[None],
                              grey=True, tol=1e-12)
    assert np.max(np.abs(ref0.T - ref.T) / ref.T) > 1e-2


def test_two_walls_band_solve_matches_oracle():
    """Band formulation, walls x = 0 (R = 0.6) and z = 1 (R = 0.5), dense operators."""
    nu = np.array([0.5, 1.4, 4.0])
    walls = [(0, 0, 0.6), (2, 1, 0.5)]
    n, hi = (9, 7, 7), (1.5, 1.0, 1.0)
    g = Grid(n, (0, 0, 0), hi)
    kb = inputs.smooth_kappa(g.positions())[None, :] * nu[:, None] ** -1.5
    Gs, SEs = [], []
    for b in range(3):
        P = Problem(g, kb[b], emit_faces=inputs.FACE_X_HI, walls=walls)
        Gs.append(P.dense_G())
        SEs.append(P.dense_S() @ osolve.planck(nu[b], np.ones(len(P.emitting))))
    ref = osolve.fixed_point(Gs, np.array(SEs), grey=False, nu=nu, kappa_v=kb, tol=1e-14)
    mesh = _mesh(n, hi, walls, inputs.FACE_X_HI)
    kt = torch.tensor(kb, device=DEV)
    G = rte.rte_hmat_assemble(mesh, kt, rte.hmat_opts(kind=rte.RTE_VOLUME, dense=True))
    S = rte.rte_hmat_assemble(mesh, kt, rte.hmat_opts(kind=rte.RTE_SURFACE, dense=True))
    T = torch.empty((1, mesh.N), device=DEV, dtype=torch.float64)
    J = torch.empty((1, 3, mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, G, S, torch.ones((1, mesh.L), device=DEV, dtype=torch.float64), T, J,
                                   grey=False, nu=nu, tol=1e-14, max_iter=1000)
    assert st["converged"]
    assert np.max(np.abs(T.cpu().numpy()[0] - ref.T) / ref.T) < 1e-10
    assert np.max(np.abs(J.cpu().numpy()[0] - ref.J)) / np.max(ref.J) < 1e-10


@pytest.mark.parametrize("precision,gpu_tol,tol", [(rte.RTE_FP64, 1e-14, 1e-10), (rte.RTE_MIXED_BF16, 1e-9, 1e-6)])
def test_three_walls_hmatrix_solve_matches_oracle_on_the_same_operator(precision, gpu_tol, tol):
    n, hi = (15, 15, 15), (1.0, 1.0, 1.0)
    g = Grid(n, (0, 0, 0), hi)
    kap = inputs.smooth_kappa(g.positions())
    mesh = _mesh(n, hi, THREE, EMIT)
    kt = torch.tensor(kap[None, :], device=DEV)
    oG = rte.hmat_opts(kind=rte.RTE_VOLUME, leaf_size=32, precision=precision)
    oS = rte.hmat_opts(kind=rte.RTE_SURFACE, leaf_size=32, precision=precision)
    Gh, Sh = rte.rte_hmat_assemble(mesh, kt, oG), rte.rte_hmat_assemble(mesh, kt, oS)
    HG, HS = readback.gpu_operator(mesh, Gh, oG), readback.gpu_operator(mesh, Sh, oS)
    assert len(HG.lowrank) > 0
    ref = osolve.fixed_point([HG], (HS @ np.full(mesh.L, osolve.SIGMA))[None], grey=True, tol=1e-14)
    T = torch.empty((1, mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, Gh, Sh, torch.ones((1, mesh.L), device=DEV, dtype=torch.float64), T,
                                   grey=True, tol=gpu_tol, max_iter=2000, precision=precision)
    assert st["converged"]
    Tg = T.cpu().numpy()[0]
    assert np.max(np.abs(Tg - ref.T) / ref.T) < tol
    # the compressed operator against the oracle's dense one, on sampled rows
    P = Problem(g, kap, emit_faces=EMIT, walls=THREE)
    rows = np.random.default_rng(2).choice(g.N, 40, replace=False)
    x = np.random.default_rng(3).uniform(0.5, 1.5, g.N)
    Grows = P.volume_block(rows, np.arange(g.N))
    assert np.max(np.abs(HG.matvec(x)[rows] - Grows @ x) / (Grows @ x)) < 3e-4


def test_wall_descriptions_are_validated():
    with pytest.raises(rte.RteError):   # a reflective face cannot emit
        rte.rte_mesh_create((5, 5, 5), emit_faces=inputs.FACE_X_LO, walls=[(0, 0, 1.0)])
    with pytest.raises(rte.RteError):   # the same face twice
        rte.rte_mesh_create((5, 5, 5), reflect_axis=1, reflect_side=1, R=0.5, walls=[(1, 1, 0.5)])
    with pytest.raises(rte.RteError):   # R outside [0, 1]
        rte.rte_mesh_create((5, 5, 5), walls=[(2, 0, 1.5)])


def test_zero_coefficient_walls_are_the_plain_operator():
    """Walls with R = 0 add nothing: the entries equal those of the mesh without walls, bit for bit."""
    n = (7, 6, 5)
    g = Grid(n)
    kap = torch.tensor(np.random.default_rng(1).uniform(0.2, 2.0, g.N), device=DEV)
    m0 = rte.rte_mesh_create(n, emit_faces=2)
    mw = rte.rte_mesh_create(n, emit_faces=2, walls=[(0, 0, 0.0), (2, 1, 0.0)])
    rows = torch.tensor(np.random.default_rng(2).integers(0, g.N, 500), device=DEV)
    cols = torch.tensor(np.random.default_rng(3).integers(0, g.N, 500), device=DEV)
    a, b = torch.empty(500, device=DEV, dtype=torch.float64), torch.empty(500, device=DEV, dtype=torch.float64)
    rte.rte_entries(m0, rte.RTE_VOLUME, kap, rows, cols, a)
    rte.rte_entries(mw, rte.RTE_VOLUME, kap, rows, cols, b)
    assert torch.equal(a, b)
