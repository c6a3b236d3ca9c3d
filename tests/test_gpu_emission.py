"""GPU: the cosine-weighted wall source of Section "Example" (Q = [omega.n]_- Q0,
kernel ([(x-y).n]_+)^2 / |x-y|^4, half the isotropic in-plane limit) against
the FP64 oracle with the same option: surface entries one by one on the
single-wall, one-wall, several-wall and hole code paths, a dense solve
element by element, and compressed solves against the oracle's fixed point
of the read-back operators."""
import numpy as np
import pytest
import torch

from oracle import solve as osolve
from oracle.core import Grid, Problem
from paper_2306_05789_amd import inputs, rte

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [
    dict(n=(9, 8, 7), hi=(1.0, 0.9, 0.8), emit=1 | 8),
    dict(n=(9, 8, 7), hi=(1.0, 0.9, 0.8), emit=1 | 8, wall=(2, 0, 0.5)),
    dict(n=(8, 7, 6), hi=(1.0, 0.9, 0.7), emit=2 | 8, walls=[(0, 0, 0.6), (1, 0, 0.4), (2, 1, 1.0)]),
    dict(n=(9, 8, 8), hi=(1.0, 0.9, 0.9), emit=1 | 8, hole=((3, 2, 2), (6, 5, 5)), hole_emit=63),
]


def _case(n, hi, emit, wall=None, walls=None, hole=None, hole_emit=0, seed=0):
    g = Grid(tuple(n), (0.0, 0.0, 0.0), tuple(float(v) for v in hi))
    kap = np.random.default_rng(seed).uniform(0.2, 2.0, g.N)
    if wall is not None:
        a, s, R = wall
        P = Problem(g, kap, emit_faces=emit, wall_axis=a, wall_side=s, R=R, emission=1)
        mesh = rte.rte_mesh_create(n, (0, 0, 0), hi, reflect_axis=a, reflect_side=s, R=R, emit_faces=emit,
                                   emission=1)
    else:
        P = Problem(g, kap, emit_faces=emit, walls=walls or [], hole=hole, hole_emit=hole_emit, emission=1)
        mesh = rte.rte_mesh_create(n, (0, 0, 0), hi, emit_faces=emit, walls=walls, hole=hole,
                                   hole_emit=hole_emit, emission=1)
    return P, mesh, torch.tensor(kap, device=DEV, dtype=torch.float64)


def _pairs(P, rng, count):
    """Random pairs, each vertex's own column (the in-plane limit) and pairs on
    a common face (the kernel vanishes there)."""
    g, em = P.grid, P.emitting
    rows = [rng.integers(0, g.N, count), em[:40], rng.choice(em, count)]
    cols = [rng.choice(em, count), em[:40], rng.choice(em, count)]
    return np.concatenate(rows).astype(np.int64), np.concatenate(cols).astype(np.int64)


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("precision", [rte.RTE_FP64, rte.RTE_FP32])
def test_cosine_weighted_surface_entries_match_oracle(case, precision):
    P, mesh, kap = _case(**CASES[case], seed=case)
    rows, cols = _pairs(P, np.random.default_rng(300 + case), 2000)
    ref = P.surface_pairs(rows, cols)
    r, c = torch.tensor(rows, device=DEV), torch.tensor(cols, device=DEV)
    out = torch.empty(len(rows), device=DEV, dtype=torch.float64)
    rte.rte_entries(mesh, rte.RTE_SURFACE, kap, r, c, out, precision)
    got = out.cpu().numpy()
    nz = ref != 0
    assert nz.sum() > len(rows) // 2
    assert np.all(got[~nz] == 0)
    err = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
    if precision == rte.RTE_FP64:
        tol = np.full(err.shape, 1e-12)
    else:
        # the FP32 entry bound of the isotropic source: 1e-6 (1 + tau), tau the
        # larger of the direct and reflected optical depths
        pos = P.grid.positions()
        tau = P.tau(pos[rows], pos[cols])
        for w in range(len(P.walls)):
            tau = np.maximum(tau, P.tau(pos[rows], pos[cols], wall=w))
        tol = 1e-6 * (1.0 + tau[nz])
    w = np.argmax(err / tol)
    assert np.all(err < tol), (err[w], tol[w], rows[nz][w], cols[nz][w])


def test_cosine_weighted_source_differs_from_the_isotropic_one():
    """The option reaches the kernel: at the same pair the two laws give
    different entries, and the in-plane diagonal entry is halved."""
    P, mesh, kap = _case(**CASES[0])
    n = CASES[0]["n"]
    mesh_iso = rte.rte_mesh_create(n, (0, 0, 0), CASES[0]["hi"], emit_faces=CASES[0]["emit"])
    em = P.emitting
    inner = [int(P.grid.vid(np.array([i, 4, 3]))) for i in range(1, 8)] + [int(P.grid.vid(np.array([2, 2, 2])))] * 3
    rows = torch.tensor(np.r_[em[:10], inner], device=DEV)
    cols = torch.tensor(np.r_[em[:10], em[20:30]], device=DEV)
    a = torch.empty(20, device=DEV, dtype=torch.float64)
    b = torch.empty_like(a)
    rte.rte_entries(mesh, rte.RTE_SURFACE, kap, rows, cols, a, rte.RTE_FP64)
    rte.rte_entries(mesh_iso, rte.RTE_SURFACE, kap, rows, cols, b, rte.RTE_FP64)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.all(a[10:] > 0) and np.all(b[10:] > 0) and np.all(a[10:] != b[10:])
    # on the diagonal, the in-plane term is the whole entry (the kernel vanishes in the face)
    assert np.allclose(a[:10], 0.5 * b[:10], rtol=1e-15, atol=0)


def test_cosine_weighted_dense_solve_matches_oracle():
    wl = inputs.config_tiny(9)
    P, mesh, kap = _case(wl.n, (1.0, 1.0, 1.0), wl.emit_faces)
    G, S = P.dense_G(), P.dense_S()
    ref = osolve.fixed_point([G], (S @ (osolve.SIGMA * wl.T_wall[0] ** 4))[None], grey=True, tol=1e-13)
    opts = lambda kind: rte.hmat_opts(kind=kind, dense=True)
    Gh = rte.rte_hmat_assemble(mesh, kap[None, :].contiguous(), opts(rte.RTE_VOLUME))
    Sh = rte.rte_hmat_assemble(mesh, kap[None, :].contiguous(), opts(rte.RTE_SURFACE))
    Tw = torch.tensor(wl.T_wall, device=DEV)
    T = torch.empty((1, mesh.N), device=DEV, dtype=torch.float64)
    J = torch.empty((1, 1, mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, Gh, Sh, Tw, T, J, grey=True, tol=1e-13, max_iter=500)
    assert st["converged"] and st["monotone_violations"] == 0
    Jg, Tg = J.cpu().numpy()[0, 0], T.cpu().numpy()[0]
    assert np.max(np.abs(Jg - ref.J[0])) / np.max(ref.J[0]) < 1e-10
    assert np.max(np.abs(Tg - ref.T) / np.maximum(ref.T, 1e-300)) < 1e-10


@pytest.mark.parametrize("precision,gpu_tol,tol", [(rte.RTE_FP64, 1e-14, 1e-10), (rte.RTE_MIXED_BF16, 1e-9, 1e-6)])
def test_cosine_weighted_hmatrix_solve_matches_oracle(precision, gpu_tol, tol):
    """Compressed operators with the cosine-weighted source: the stored surface
    operator against the oracle's dense one within the ACA bound, and the solve
    against the oracle's fixed point of the read-back operators."""
    import readback
    g = Grid((13, 13, 13))
    kap = inputs.smooth_kappa(g.positions())
    P = Problem(g, kap, emit_faces=1 | 8, emission=1)
    mesh = rte.rte_mesh_create(g.n, emit_faces=1 | 8, emission=1)
    kt = torch.tensor(kap[None, :], device=DEV)
    opts = lambda kind: rte.hmat_opts(kind=kind, leaf_size=32, eta=2.0, aca_eps=1e-5, precision=precision)
    oG, oS = opts(rte.RTE_VOLUME), opts(rte.RTE_SURFACE)
    Gh, Sh = rte.rte_hmat_assemble(mesh, kt, oG), rte.rte_hmat_assemble(mesh, kt, oS)
    HG, HS = readback.gpu_operator(mesh, Gh, oG), readback.gpu_operator(mesh, Sh, oS)
    x = np.random.default_rng(7).uniform(0.5, 2.0, mesh.L)
    Sd = P.dense_S()
    assert np.linalg.norm(HS @ x - Sd @ x) / np.linalg.norm(Sd @ x) < 1e-4
    ref = osolve.fixed_point([HG], (HS @ np.full(mesh.L, osolve.SIGMA))[None], grey=True, tol=1e-14)
    T = torch.empty((1, mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, Gh, Sh, torch.ones((1, mesh.L), device=DEV, dtype=torch.float64), T,
                                   grey=True, tol=gpu_tol, max_iter=500, precision=precision)
    assert st["converged"]
    assert np.max(np.abs(T.cpu().numpy()[0] - ref.T) / ref.T) < tol
