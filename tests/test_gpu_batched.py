"""GPU: all bands and many right-hand sides at once (one launch per matvec
phase over every band and right-hand side), and sweeps replayed from captured
hipGraphs, against per-band / single right-hand-side calls of the same library
and against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import solve as osolve
from oracle.core import Grid, Problem
from paper_2306_05789_amd import inputs, rte

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LEAF = 16


@pytest.fixture(scope="module")
def small():
    """Unit cube 11^3, 3 bands kappa_b = c_b kappa(x) (c_b lognormal), all faces emit,
    16 right-hand sides of wall temperatures in [0.5, 2]."""
    wl = inputs.batched(n=11, bands=3, nrhs=16)
    mesh = rte.rte_mesh_create(wl.n, emit_faces=wl.emit_faces)
    return wl, mesh


def _assemble(mesh, wl, kind, precision):
    return rte.rte_hmat_assemble(mesh, torch.tensor(wl.kappa, device=DEV),
                                 rte.hmat_opts(kind=kind, leaf_size=LEAF, precision=precision))


@pytest.mark.parametrize("precision", [rte.RTE_FP64, rte.RTE_FP32, rte.RTE_MIXED_BF16])
def test_batched_matvec_equals_single_calls(small, precision):
    """Every band and right-hand side of the batched product equals the single-band,
    single right-hand-side product.  On the matrix cores (BF16 storage) every column
    is reduced in the same fixed order whatever shares the launch: bit for bit.  FP64
    with 16 right-hand sides runs on the FP64 matrix cores and one at a time on the
    vector ALUs, FP32 in groups of 4 with kernels instantiated per group width that
    the compiler may contract differently: rounding level."""
    wl, mesh = small
    G = _assemble(mesh, wl, rte.RTE_VOLUME, precision)
    nb, nr = wl.kappa.shape[0], 16
    x = torch.tensor(np.random.default_rng(11).uniform(0.0, 2.0, (nb, nr, mesh.N)), device=DEV)
    ops = [rte.RTE_OP_ACCURATE] + ([rte.RTE_OP_LOW] if precision == rte.RTE_MIXED_BF16 else [])
    for op in ops:
        y = torch.empty_like(x)
        rte.rte_hmat_matvec_batched(G, x, y, op)
        assert torch.isfinite(y).all()
        for r in (0, 7, 15):
            x1 = x[:, r:r + 1, :].contiguous()
            y1 = torch.empty_like(x1)
            rte.rte_hmat_matvec_batched(G, x1, y1, op)
            if precision == rte.RTE_MIXED_BF16:
                assert torch.equal(y1[:, 0], y[:, r]), (op, r)
            else:
                tol = 1e-13 if precision == rte.RTE_FP64 else 2e-6
                assert torch.max(torch.abs(y1[:, 0] - y[:, r]) / torch.abs(y[:, r])).item() < tol, (op, r)
        if op == rte.RTE_OP_ACCURATE:
            for b in range(nb):
                yb = torch.empty((nr, mesh.N), device=DEV, dtype=torch.float64)
                rte.rte_hmat_matvec(G, b, x[b].contiguous(), yb)
                assert torch.equal(yb, y[b]), b
    if precision == rte.RTE_MIXED_BF16:
        # the BF16-hi operator is a perturbation of the hi + lo one at the BF16 level
        ya, yl = torch.empty_like(x), torch.empty_like(x)
        rte.rte_hmat_matvec_batched(G, x, ya, rte.RTE_OP_ACCURATE)
        rte.rte_hmat_matvec_batched(G, x, yl, rte.RTE_OP_LOW)
        rel = (torch.linalg.norm(ya - yl) / torch.linalg.norm(ya)).item()
        assert 1e-6 < rel < 1e-2, rel


def _solve(mesh, G, S, wl, Tw, precision, tol, launch=None, time_matvecs=False):
    T = torch.empty((Tw.shape[0], mesh.N), device=DEV, dtype=torch.float64)
    J = torch.empty((Tw.shape[0], wl.kappa.shape[0], mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, G, S, Tw, T, J, grey=False, nu=wl.nu, tol=tol, max_iter=3000,
                                   precision=precision, launch=launch, time_matvecs=time_matvecs)
    return T, J, st


@pytest.mark.parametrize("precision", [rte.RTE_FP64, rte.RTE_MIXED_BF16])
def test_multiband_assembly_equals_single_band_assemblies(small, precision):
    """The bands of a multi-band operator are assembled two at a time on two host
    threads and streams; each band's operator is bit for bit the one a single-band
    assembly of that band gives (ranks, stored bytes, products)."""
    wl, mesh = small
    kap = torch.tensor(wl.kappa, device=DEV)
    opts = rte.hmat_opts(kind=rte.RTE_VOLUME, leaf_size=LEAF, precision=precision)
    G = rte.rte_hmat_assemble(mesh, kap, opts)
    x = torch.tensor(np.random.default_rng(12).uniform(0.0, 2.0, (3, mesh.N)), device=DEV)
    total = 0
    for b in range(wl.kappa.shape[0]):
        Gb = rte.rte_hmat_assemble(mesh, kap[b:b + 1].contiguous(), opts)
        total += rte.rte_hmat_stats(Gb)["bytes"]
        y, yb = torch.empty_like(x), torch.empty_like(x)
        rte.rte_hmat_matvec(G, b, x, y)
        rte.rte_hmat_matvec(Gb, 0, x, yb)
        assert torch.equal(y, yb), b
    assert rte.rte_hmat_stats(G)["bytes"] == total


def test_batched_solve_equals_single_rhs_solves(small):
    """16 right-hand sides in one solve against each solved alone (FP64 storage): the
    batched solve stops on the slowest right-hand side, so the others take extra
    sweeps of a converged iteration and move by far less than the tolerance."""
    wl, mesh = small
    G = _assemble(mesh, wl, rte.RTE_VOLUME, rte.RTE_FP64)
    S = _assemble(mesh, wl, rte.RTE_SURFACE, rte.RTE_FP64)
    Tw = torch.tensor(wl.T_wall, device=DEV)
    T16, J16, st = _solve(mesh, G, S, wl, Tw, rte.RTE_FP64, 1e-12)
    # monotone up to rounding: an ACA block is not exactly nonnegative, so a vertex can
    # step down by a rounding-level amount near convergence
    assert st["converged"] and st["monotone_violations"] <= 1e-4 * st["iterations"] * Tw.shape[0] * mesh.N
    for r in (0, 5, 15):
        T1, J1, st1 = _solve(mesh, G, S, wl, Tw[r:r + 1].contiguous(), rte.RTE_FP64, 1e-12)
        assert st1["iterations"] <= st["iterations"]
        assert torch.max(torch.abs(T1[0] - T16[r]) / T16[r]).item() < 1e-9
        assert torch.max(torch.abs(J1[0] - J16[r]) / J16[r]).item() < 1e-9


@pytest.mark.parametrize("precision", [rte.RTE_FP64, rte.RTE_MIXED_BF16])
def test_graph_launch_equals_stream_launch(small, precision):
    """Sweeps replayed from captured graphs (with host reads and syncs between the
    replays) give the stream-launched results bit for bit, at every precision."""
    wl, mesh = small
    G = _assemble(mesh, wl, rte.RTE_VOLUME, precision)
    S = _assemble(mesh, wl, rte.RTE_SURFACE, precision)
    Tw = torch.tensor(wl.T_wall[:4], device=DEV)
    Ts, Js, sts = _solve(mesh, G, S, wl, Tw, precision, 1e-7, launch=rte.RTE_LAUNCH_STREAM)
    Tg, Jg, stg = _solve(mesh, G, S, wl, Tw, precision, 1e-7, launch=rte.RTE_LAUNCH_GRAPH)
    assert sts["graphs"] == 0 and stg["graphs"] >= 2
    assert stg["iterations"] == sts["iterations"] and stg["outer_steps"] == sts["outer_steps"]
    assert stg["residual"] == sts["residual"]
    assert torch.equal(Tg, Ts) and torch.equal(Jg, Js)
    # and again on the same matrices: a fresh set of graphs, the same numbers
    Tg2, _, stg2 = _solve(mesh, G, S, wl, Tw, precision, 1e-7, launch=rte.RTE_LAUNCH_GRAPH)
    assert torch.equal(Tg2, Ts) and stg2["iterations"] == sts["iterations"]
    # timed sweeps (three graphs per sweep with events between): the same numbers,
    # and every volume matvec timed
    Tt, Jt, stt = _solve(mesh, G, S, wl, Tw, precision, 1e-7, launch=rte.RTE_LAUNCH_GRAPH, time_matvecs=True)
    assert torch.equal(Tt, Ts) and torch.equal(Jt, Js) and stt["iterations"] == sts["iterations"]
    # from T0 = 0 the first sweep has a zero source and streams no operator
    assert stt["matvecs_low"] + stt["matvecs_acc"] == stt["iterations"] - 1
    assert stt["ms_matvec_acc"] > 0 and (precision != rte.RTE_MIXED_BF16 or stt["ms_matvec_low"] > 0)
    assert stg["ms_matvec_low"] == -1.0 and sts["matvecs_acc"] > 0


@pytest.mark.parametrize("precision", [rte.RTE_FP64, rte.RTE_MIXED_BF16])
def test_residual_history(small, precision):
    """The residual of every sweep: from J = 0 the first is exactly 1 (J^1 = S^E,
    all of it new), the last is the reported one, at most tol."""
    wl, mesh = small
    G = _assemble(mesh, wl, rte.RTE_VOLUME, precision)
    S = _assemble(mesh, wl, rte.RTE_SURFACE, precision)
    Tw = torch.tensor(wl.T_wall[:2], device=DEV)
    T = torch.empty((2, mesh.N), device=DEV, dtype=torch.float64)
    st = rte.rte_fixed_point_solve(mesh, G, S, Tw, T, grey=False, nu=wl.nu, tol=1e-8, max_iter=3000,
                                   precision=precision, history=True)
    h = st["residuals"]
    assert st["converged"] and len(h) == st["iterations"] > 2
    assert h[0] == 1.0 and h[-1] == st["residual"] <= 1e-8
    assert np.all(h[1:] < 1.0)


def test_mixed_batched_solve_matches_oracle(small):
    """Mixed precision (FP32 entries and ACA, BF16 factors, FP64 defect correction),
    all bands and 4 right-hand sides at once, against the dense FP64 oracle per
    right-hand side; the difference is the ACA compression (eps 1e-5)."""
    wl, mesh = small
    G = _assemble(mesh, wl, rte.RTE_VOLUME, rte.RTE_MIXED_BF16)
    S = _assemble(mesh, wl, rte.RTE_SURFACE, rte.RTE_MIXED_BF16)
    R = 4
    Tw = torch.tensor(wl.T_wall[:R], device=DEV)
    T, J, st = _solve(mesh, G, S, wl, Tw, rte.RTE_MIXED_BF16, 1e-7)
    assert st["converged"] and st["residual"] <= 1e-7 and st["outer_steps"] >= 2
    g = Grid(wl.n)
    probs = [Problem(g, wl.kappa[b], emit_faces=wl.emit_faces) for b in range(len(wl.nu))]
    Gs = [P.dense_G() for P in probs]
    Ss = [P.dense_S() for P in probs]
    Tn = T.cpu().numpy()
    for r in range(R):
        SEs = np.array([Ss[b] @ osolve.planck(wl.nu[b], wl.T_wall[r]) for b in range(len(wl.nu))])
        ref = osolve.fixed_point(Gs, SEs, grey=False, nu=wl.nu, kappa_v=wl.kappa, tol=1e-13)
        assert np.max(np.abs(Tn[r] - ref.T) / ref.T) < 3e-4, r


@pytest.mark.parametrize("precision", [rte.RTE_FP64, rte.RTE_MIXED_BF16])
def test_autotuner_picks_a_shape_and_results_hold(small, precision, tmp_path):
    """The autotuner times its candidate launch shapes on the matrix, keeps the
    fastest and caches it; every shape computes the same product to rounding."""
    from paper_2306_05789_amd import tune
    wl, mesh = small
    G = _assemble(mesh, wl, rte.RTE_VOLUME, precision)
    nb = wl.kappa.shape[0]
    x = torch.tensor(np.random.default_rng(12).uniform(0.5, 2.0, (nb, 16, mesh.N)), device=DEV)
    y0, y1 = torch.empty_like(x), torch.empty_like(x)
    rte.rte_hmat_matvec_batched(G, x, y0, rte.RTE_OP_ACCURATE)
    cache = str(tmp_path / "tune.json")
    r = tune.autotune(G, nrhs=16, cache=cache, reps=2)
    assert r["source"] == "timed" and r["trials"] >= 6 and r["ms"] > 0
    assert rte.rte_hmat_get_config(G) == r["config"]
    rte.rte_hmat_matvec_batched(G, x, y1, rte.RTE_OP_ACCURATE)
    rel = (torch.max(torch.abs(y1 - y0) / torch.abs(y0))).item()
    assert rel < 1e-12, rel
    for cfg in ({"phase_b_waves": 4, "phase_a_kib": 16, "phase_a_tiles": 4},
                {"phase_b_waves": 8, "phase_a_kib": 256, "phase_a_tiles": 2 if precision == rte.RTE_MIXED_BF16 else 4}):
        rte.rte_hmat_set_config(G, cfg)
        rte.rte_hmat_matvec_batched(G, x, y1, rte.RTE_OP_ACCURATE)
        assert (torch.max(torch.abs(y1 - y0) / torch.abs(y0))).item() < 1e-12
        if precision == rte.RTE_MIXED_BF16:
            ya, yb = torch.empty_like(x), torch.empty_like(x)
            rte.rte_hmat_matvec_batched(G, x, yb, rte.RTE_OP_LOW)
            rte.rte_hmat_set_config(G, r["config"])
            rte.rte_hmat_matvec_batched(G, x, ya, rte.RTE_OP_LOW)
            assert (torch.max(torch.abs(ya - yb) / torch.abs(ya))).item() < 1e-5
    if precision == rte.RTE_MIXED_BF16:
        # 8 tiles per phase-A task (low operator; the accurate one keeps tasks of 4):
        # every tile sums over the same steps in the same order, so both products
        # are bitwise those of 4-tile tasks
        outs = []
        for t in (4, 8):
            rte.rte_hmat_set_config(G, {"phase_b_waves": 8, "phase_a_kib": 256, "phase_a_tiles": t})
            yl, ya = torch.empty_like(x), torch.empty_like(x)
            rte.rte_hmat_matvec_batched(G, x, yl, rte.RTE_OP_LOW)
            rte.rte_hmat_matvec_batched(G, x, ya, rte.RTE_OP_ACCURATE)
            outs.append((yl, ya))
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
        rte.rte_hmat_set_config(G, r["config"])
    # a second run of the same shape takes the cached choice without timing
    G2 = _assemble(mesh, wl, rte.RTE_VOLUME, precision)
    r2 = tune.autotune(G2, nrhs=16, cache=cache, reps=2)
    assert r2["source"] == "cache" and rte.rte_hmat_get_config(G2) == r["config"]
    with pytest.raises(rte.RteError):
        rte.rte_hmat_set_config(G, {"phase_b_waves": 3, "phase_a_kib": 64, "phase_a_tiles": 4})


def test_leaf_size_search_scores_every_candidate():
    """The leaf-size search assembles at each candidate, autotunes its matvec and
    keeps the one with the smallest assembly + sweeps x matvec time."""
    from paper_2306_05789_amd import tune
    n = 17
    mesh = rte.rte_mesh_create((n, n, n), emit_faces=1)
    kap = torch.tensor(inputs.smooth_kappa(inputs.grid_positions((n, n, n), (0, 0, 0), (1, 1, 1)))[None, :],
                       device=DEV)
    best, rec = tune.tune_leaf_size(mesh, kap, {"kind": rte.RTE_VOLUME, "precision": rte.RTE_FP64},
                                    candidates=(32, 64), sweeps=20, reps=2)
    assert [r["leaf_size"] for r in rec] == [32, 64]
    assert all(r["assemble_ms"] > 0 and r["matvec_ms"] > 0 and r["bytes"] > 0 for r in rec)
    assert best == min(rec, key=lambda r: r["score_ms"])["leaf_size"]
    assert all(abs(r["score_ms"] - (r["assemble_ms"] + 20 * r["matvec_ms"])) < 1e-9 for r in rec)
