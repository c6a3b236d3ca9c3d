"""GPU arithmetic against the oracle applied to the GPU's own compressed operator.

The library's assembled operator (cluster orders, dense blocks, low-rank
factors) is read back through the C ABI, widened to FP64, and applied by the
oracle's plain block-by-block product and fixed point (oracle/hmatrix.py,
pinned against the dense oracle in test_oracle_hmatrix.py).  This separates
the library's arithmetic error from the compression error of the ACA
(Section "Compression"), which is measured separately against the dense
oracle: the tolerances here are those of the arithmetic, element by element.

* matvec, FP64 storage: |y - y_ref| <= 1e-12 (|H| |x|) per element;
* matvec, FP32 storage (FP32 accumulation): <= 1e-6 (|H| |x|);
* matvec, BF16 hi + lo storage, accurate operator: <= 1e-6 (|H| |x|);
  low operator against the hi parts alone: <= 3e-5 (|H| |x|) (the vector
  and V^T x are carried as two BF16 parts, 16 significant bits each);
* fixed point (Algorithm of Section "Fixed Point Iterations") against the
  oracle's fixed point of the same operators: FP64 <= 1e-10, FP32 <= 1e-5,
  mixed precision (defect-corrected, FP64 residual) <= 1e-6, relative per
  vertex."""
import numpy as np
import pytest
import torch

import readback
from oracle import solve as osolve
from oracle.core import Grid, Problem
from paper_2306_05789_amd import inputs, rte

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _smooth(X):
    return 0.5 + 0.4 * np.sin(2 * np.pi * X[:, 0]) * np.cos(2 * np.pi * X[:, 1]) * X[:, 2]


@pytest.fixture(scope="module")
def cube15():
    """15^3 unit cube, smooth kappa, wall x = 0 emitting: the oracle's dense G, S."""
    g = Grid((15, 15, 15))
    kap = _smooth(g.positions())
    P = Problem(g, kap, emit_faces=1)
    mesh = rte.rte_mesh_create(g.n, emit_faces=1)
    return P, mesh, torch.tensor(kap[None, :], device=DEV), P.dense_G(), P.dense_S()


def _opts(kind, precision, leaf=32, **kw):
    return rte.hmat_opts(kind=kind, leaf_size=leaf, eta=2.0, aca_eps=1e-5, precision=precision, **kw)


def _matvec(H, X, n_out, band=0):
    xt = torch.tensor(np.ascontiguousarray(X), device=DEV)
    y = torch.empty((X.shape[0], n_out), device=DEV, dtype=torch.float64)
    rte.rte_hmat_matvec(H, band, xt, y)
    return y.cpu().numpy()


def _vectors(n, count, seed):
    rng = np.random.default_rng(seed)
    base = [np.ones(n), rng.uniform(0.0, 1.0, n), rng.standard_normal(n)]
    while len(base) < count:
        base.append(rng.uniform(-0.5, 2.0, n))
    return np.stack(base[:count])


def _check(got, ref, scale, tol, what):
    err = np.abs(got - ref) / scale
    assert err.max() <= tol, (what, err.max())
    return err.max()


@pytest.mark.parametrize("precision,tol", [(rte.RTE_FP64, 1e-12), (rte.RTE_FP32, 1e-6),
                                           (rte.RTE_MIXED_BF16, 1e-6)])
@pytest.mark.parametrize("kind", [rte.RTE_VOLUME, rte.RTE_SURFACE])
@pytest.mark.parametrize("nrhs", [3, 16])
def test_hmatvec_matches_oracle_on_the_same_operator(cube15, precision, tol, kind, nrhs):
    P, mesh, kap, G, S = cube15
    opts = _opts(kind, precision)
    H = rte.rte_hmat_assemble(mesh, kap, opts)
    Href = readback.gpu_operator(mesh, H, opts)
    n_src = mesh.N if kind == rte.RTE_VOLUME else mesh.L
    assert len(Href.lowrank) > 0
    X = _vectors(n_src, nrhs, 10 + nrhs)
    Y = _matvec(H, X, mesh.N)
    e = _check(Y, Href.matvec(X), Href.abs_matvec(X), tol, "matvec")
    print(f"matvec vs oracle on the same operator, precision {precision} kind {kind} nrhs {nrhs}: {e:.2e}")
    # compression error of the same operator against the dense oracle (reported bound)
    D = G if kind == rte.RTE_VOLUME else S
    comp = np.linalg.norm(Href.matvec(X[1]) - D @ X[1]) / np.linalg.norm(D @ X[1])
    assert comp < 3e-4, comp


def test_low_operator_matches_oracle_on_the_hi_parts(cube15):
    """Mixed storage, low operator (inner sweeps): BF16 hi factors with FP32
    accumulation, against the oracle applying the hi parts in FP64."""
    P, mesh, kap, G, S = cube15
    opts = _opts(rte.RTE_VOLUME, rte.RTE_MIXED_BF16)
    H = rte.rte_hmat_assemble(mesh, kap, opts)
    Hlo = readback.gpu_operator(mesh, H, opts, op=rte.RTE_OP_LOW)
    X = _vectors(mesh.N, 16, 3)
    xt = torch.tensor(X[None], device=DEV)
    y = torch.empty_like(xt)
    rte.rte_hmat_matvec_batched(H, xt, y, op=rte.RTE_OP_LOW)
    e = _check(y.cpu().numpy()[0], Hlo.matvec(X), Hlo.abs_matvec(X), 3e-5, "low operator")
    print(f"low operator vs oracle on the hi parts: {e:.2e}")


def test_dense_readback_is_the_oracle_matrix():
    """No compression (dense = 1), FP64, with a reflective wall: the read-back
    operator is the oracle's dense G entry by entry (1e-12)."""
    g = Grid((9, 8, 7), (0, 0, 0), (1.0, 0.9, 0.8))
    kap = np.random.default_rng(8).uniform(0.2, 2.0, g.N)
    P = Problem(g, kap, emit_faces=1 | 8, wall_axis=2, wall_side=0, R=0.5)
    mesh = rte.rte_mesh_create(g.n, (0, 0, 0), g.hi, reflect_axis=2, reflect_side=0, R=0.5, emit_faces=1 | 8)
    for kind, ref in ((rte.RTE_VOLUME, P.dense_G()), (rte.RTE_SURFACE, P.dense_S())):
        opts = rte.hmat_opts(kind=kind, dense=True, leaf_size=16)
        H = rte.rte_hmat_assemble(mesh, torch.tensor(kap[None, :], device=DEV), opts)
        D = readback.gpu_operator(mesh, H, opts).to_dense()
        nz = ref != 0
        assert np.all(D[~nz] == 0)
        assert np.max(np.abs(D[nz] - ref[nz]) / np.abs(ref[nz])) < 1e-12


def test_grey_hmatrix_solve_matches_oracle_fixed_point(cube15):
    """Grey FP64 H-matrix solve: T and J against the oracle's fixed point of the
    read-back operators (1e-10)."""
    P, mesh, kap, G, S = cube15
    oG, oS = _opts(rte.RTE_VOLUME, rte.RTE_FP64), _opts(rte.RTE_SURFACE, rte.RTE_FP64)
    Gh, Sh = rte.rte_hmat_assemble(mesh, kap, oG), rte.rte_hmat_assemble(mesh, kap, oS)
    HG, HS = readback.gpu_operator(mesh, Gh, oG), readback.gpu_operator(mesh, Sh, oS)
    ref = osolve.fixed_point([HG], (HS @ np.full(mesh.L, osolve.SIGMA))[None], grey=True, tol=1e-14)
    T = torch.empty((1, mesh.N), device=DEV, dtype=torch.float64)
    J = torch.empty((1, 1, mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, Gh, Sh, torch.ones((1, mesh.L), device=DEV, dtype=torch.float64), T, J,
                                   grey=True, tol=1e-14, max_iter=500)
    assert st["converged"]
    assert np.max(np.abs(T.cpu().numpy()[0] - ref.T) / ref.T) < 1e-10
    assert np.max(np.abs(J.cpu().numpy()[0, 0] - ref.J[0]) / ref.J[0]) < 1e-10


NU = np.array([0.5, 1.4, 4.0])
N3, HI = (17, 9, 9), (2.0, 1.0, 1.0)


@pytest.fixture(scope="module")
def reflect3():
    """Box [0,2]x[0,1]^2 on 17x9x9, wall z = 0 with R = 0.5, x = 0 emitting at T = 1,
    three bands with kappa_nu = kappa(x) nu^-1.5."""
    g = Grid(N3, (0, 0, 0), HI)
    kb = inputs.smooth_kappa(g.positions())[None, :] * NU[:, None] ** -1.5
    mesh = rte.rte_mesh_create(N3, (0, 0, 0), HI, reflect_axis=2, reflect_side=0, R=0.5, emit_faces=1)
    return g, kb, mesh


@pytest.mark.parametrize("precision,gpu_tol,tol", [(rte.RTE_FP64, 1e-14, 1e-10), (rte.RTE_FP32, 1e-7, 1e-5),
                                                   (rte.RTE_MIXED_BF16, 1e-9, 1e-6)])
def test_reflective_band_solve_matches_oracle_fixed_point(reflect3, precision, gpu_tol, tol):
    """Band formulation with a reflective wall: the GPU fixed point (FP64, FP32, or
    BF16 sweeps with FP64 defect correction) against the oracle's fixed point
    (per-vertex bisection) of the same compressed G and S, read back per band."""
    g, kb, mesh = reflect3
    kt = torch.tensor(kb, device=DEV)
    oG, oS = _opts(rte.RTE_VOLUME, precision), _opts(rte.RTE_SURFACE, precision)
    Gh, Sh = rte.rte_hmat_assemble(mesh, kt, oG), rte.rte_hmat_assemble(mesh, kt, oS)
    HG = [readback.gpu_operator(mesh, Gh, oG, band=b) for b in range(len(NU))]
    HS = [readback.gpu_operator(mesh, Sh, oS, band=b) for b in range(len(NU))]
    SE = np.stack([HS[b] @ osolve.planck(NU[b], np.ones(mesh.L)) for b in range(len(NU))])
    ref = osolve.fixed_point(HG, SE, grey=False, nu=NU, kappa_v=kb, tol=1e-14)
    T = torch.empty((1, mesh.N), device=DEV, dtype=torch.float64)
    J = torch.empty((1, len(NU), mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, Gh, Sh, torch.ones((1, mesh.L), device=DEV, dtype=torch.float64), T, J,
                                   grey=False, nu=NU, tol=gpu_tol, max_iter=3000, precision=precision,
                                   allow_not_converged=precision == rte.RTE_FP32)
    # FP32 sweeps stall at their rounding level; the others reach the FP64 residual
    assert st["converged"] or (precision == rte.RTE_FP32 and st["residual"] < 1e-5)
    err_T = np.max(np.abs(T.cpu().numpy()[0] - ref.T) / ref.T)
    err_J = np.max(np.abs(J.cpu().numpy()[0] - ref.J)) / np.max(np.abs(ref.J))
    print(f"solve vs oracle on the same operator, precision {precision}: T {err_T:.2e}, J {err_J:.2e}, "
          f"{st['iterations']} sweeps, residual {st['residual']:.1e}")
    assert err_T < tol and err_J < tol, (err_T, err_J)


def test_batched_multiband_matvec_matches_oracle(reflect3):
    """All bands x 16 right-hand sides in one launch per phase (mixed storage, both
    operators) against the oracle's product of each band's read-back operator."""
    g, kb, mesh = reflect3
    kt = torch.tensor(kb, device=DEV)
    opts = _opts(rte.RTE_VOLUME, rte.RTE_MIXED_BF16)
    H = rte.rte_hmat_assemble(mesh, kt, opts)
    X = np.stack([_vectors(mesh.N, 16, 40 + b) for b in range(len(NU))])
    xt = torch.tensor(X, device=DEV)
    for op, tol in ((rte.RTE_OP_ACCURATE, 1e-6), (rte.RTE_OP_LOW, 3e-5)):
        y = torch.empty_like(xt)
        rte.rte_hmat_matvec_batched(H, xt, y, op=op)
        Y = y.cpu().numpy()
        for b in range(len(NU)):
            Hb = readback.gpu_operator(mesh, H, opts, band=b, op=op)
            _check(Y[b], Hb.matvec(X[b]), Hb.abs_matvec(X[b]), tol, ("band", b, op))
