"""Host-side checks of librte.so that need no GPU: every symbol of include/rte.h
is exported, the host cluster/block trees equal the oracle's exactly (index
work is compared bit-exactly), and invalid arguments are rejected before any
device work."""
import os
import re

import numpy as np
import pytest

from oracle.core import Grid, Problem
from oracle.htree import block_tree, cluster_tree
from paper_2306_05789_amd import rte

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    header = open(os.path.join(ROOT, "include", "rte.h")).read()
    names = set(re.findall(r"\b(rte_[a-z_]+)\s*\(", header))
    assert len(names) >= 15
    lib = rte.load()
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(rte.SIGNATURES) == names


def _oracle_plan(n, lo, hi, kind, emit, leaf, eta, dense=False):
    g = Grid(n, lo, hi)
    pts = g.positions()
    tperm, troot = cluster_tree(pts, leaf)
    if kind == rte.RTE_VOLUME:
        sperm, sroot, snat = tperm, troot, tperm
    else:
        em = g.emitting_vertices(emit)
        sperm, sroot = cluster_tree(pts[em], leaf)
        snat = em[sperm]
    d, l = block_tree(troot, sroot, eta if not dense else 0.0)
    if dense:
        d, l = d + l, []
    return tperm, snat, d, l


@pytest.mark.parametrize("n,hi,kind,emit,leaf,wall", [
    ((11, 11, 11), (1, 1, 1), rte.RTE_VOLUME, 1, 64, None),
    ((21, 21, 21), (1, 1, 1), rte.RTE_VOLUME, 1, 64, None),
    ((33, 17, 17), (2, 1, 1), rte.RTE_VOLUME, 1, 64, None),
    ((17, 13, 9), (1.3, 1, 0.7), rte.RTE_VOLUME, 1, 32, None),
    ((21, 21, 21), (1, 1, 1), rte.RTE_SURFACE, 63, 64, None),
    ((33, 17, 17), (2, 1, 1), rte.RTE_SURFACE, 1, 64, None),
    ((33, 17, 17), (2, 1, 1), rte.RTE_VOLUME, 1, 64, (2, 0)),
    ((17, 13, 9), (1.3, 1, 0.7), rte.RTE_VOLUME, 1, 32, (1, 1)),
    ((33, 17, 17), (2, 1, 1), rte.RTE_SURFACE, 1, 64, (2, 0)),
])
def test_host_trees_match_oracle_exactly(n, hi, kind, emit, leaf, wall):
    kw = {} if wall is None else dict(reflect_axis=wall[0], reflect_side=wall[1], R=0.5)
    mesh = rte.rte_mesh_create(n, (0, 0, 0), hi, emit_faces=emit, **kw)
    plan = rte.rte_plan_create(mesh, rte.hmat_opts(kind=kind, leaf_size=leaf, eta=2.0))
    tp, sp, blocks = rte.rte_plan_export(plan)
    rte.rte_plan_destroy(plan)
    otp, osp, od, ol = _oracle_plan(n, (0, 0, 0), hi, kind, emit, leaf, 2.0)
    assert np.array_equal(tp, otp)
    assert np.array_equal(sp, osp)
    dense = [tuple(b[:4]) for b in blocks if b[4] == 0]
    low = [tuple(b[:4]) for b in blocks if b[4] == 1]
    assert dense == [tuple(b) for b in od]
    assert low == [tuple(b) for b in ol]


def test_dense_option_keeps_every_block_dense():
    mesh = rte.rte_mesh_create((9, 9, 9))
    plan = rte.rte_plan_create(mesh, rte.hmat_opts(dense=True, leaf_size=64))
    info = rte.rte_plan_info(plan)
    assert info.n_lowrank == 0 and info.dense_entries == 729 * 729
    rte.rte_plan_destroy(plan)


def test_mesh_sizes_and_emitting_ids():
    mesh = rte.rte_mesh_create((5, 4, 3), emit_faces=1 | 32)
    g = Grid((5, 4, 3))
    assert mesh.N == 60
    assert np.array_equal(rte.rte_mesh_emitting_ids(mesh), g.emitting_vertices(1 | 32))


@pytest.mark.parametrize("emit,hole,hole_emit", [
    (0, ((2, 2, 2), (5, 5, 5)), 63),          # a hole inside the box, every face emitting
    (1 | 32, ((0, 1, 2), (2, 4, 6)), 2 | 8),  # reaching the faces x = 0 and z = 1: covered squares
    (2 | 8 | 32, ((0, 0, 0), (2, 2, 2)), 2 | 8 | 32),   # the academic test's corner cube
])
def test_emitting_ids_with_a_hole_match_oracle(emit, hole, hole_emit):
    n = (8, 7, 7)
    mesh = rte.rte_mesh_create(n, emit_faces=emit, hole=hole, hole_emit=hole_emit)
    g = Grid(n)
    P = Problem(g, np.ones(g.N), emit_faces=emit, hole=hole, hole_emit=hole_emit)
    assert np.array_equal(rte.rte_mesh_emitting_ids(mesh), P.emitting)
    assert mesh.L == len(P.emitting)


@pytest.mark.parametrize("kw,frag", [
    (dict(n=(1, 4, 4)), "at least 2"),
    (dict(n=(6, 6, 6), hole=((1, 1, 1), (1, 3, 3))), "non-empty box"),
    (dict(n=(6, 6, 6), hole=((1, 1, 1), (3, 3, 6))), "non-empty box"),
    (dict(n=(6, 6, 6), hole=((0, 1, 1), (3, 3, 3)), hole_emit=1), "inside the box"),
    (dict(n=(6, 6, 6), hole=((1, 1, 1), (3, 3, 5)), hole_emit=32), "inside the box"),
    (dict(n=(6, 6, 6), hole_emit=2), "without a hole"),
    (dict(n=(4, 4, 4), hi=(0, 1, 1)), "lo < hi"),
    (dict(n=(4, 4, 4), reflect_axis=3), "reflect_axis"),
    (dict(n=(4, 4, 4), reflect_axis=2, R=1.5), "R must"),
    (dict(n=(4, 4, 4), reflect_axis=0, reflect_side=0, R=0.5, emit_faces=1), "cannot also emit"),
    (dict(n=(4, 4, 4), emit_faces=64), "6 bits"),
    (dict(n=(4, 4, 4), emission=2), "emission"),
    (dict(n=(1024, 1024, 256)), "2^28 vertices"),
])
def test_mesh_validation(kw, frag):
    with pytest.raises(rte.RteError) as e:
        rte.rte_mesh_create(**kw)
    assert e.value.status == rte.RTE_E_INVALID_ARG and frag in str(e.value)


@pytest.mark.parametrize("kw,frag", [
    (dict(leaf_size=0), "leaf_size"),
    (dict(eta=-1.0), "eta"),
    (dict(aca_eps=0.0), "aca_eps"),
    (dict(precision=7), "precision"),
    (dict(kind=5), "kind"),
    (dict(aca_hits=3), "aca_hits"),
    (dict(recompress=True, aca_hits=-1), "aca_hits"),
])
def test_plan_validation(kw, frag):
    mesh = rte.rte_mesh_create((4, 4, 4))
    with pytest.raises(rte.RteError) as e:
        rte.rte_plan_create(mesh, rte.hmat_opts(**kw))
    assert frag in str(e.value)


def test_surface_plan_needs_an_emitting_face():
    mesh = rte.rte_mesh_create((4, 4, 4), emit_faces=0)
    with pytest.raises(rte.RteError):
        rte.rte_plan_create(mesh, rte.hmat_opts(kind=rte.RTE_SURFACE))


def _min_levels(v, tol):
    """Brute force: the fewest groups of the sorted values, each spanning at most a
    factor (1 + tol)^2 (one level within (1 + tol) of all), over every split into runs."""
    x = np.sort(np.log(v))
    n, best = len(x), len(x)
    for mask in range(1 << (n - 1)):
        cuts = [0] + [i + 1 for i in range(n - 1) if (mask >> i) & 1] + [n]
        if all(x[b - 1] - x[a] <= 2 * np.log1p(tol) + 1e-12 for a, b in zip(cuts, cuts[1:])):
            best = min(best, len(cuts) - 1)
    return best


def test_kappa_levels_are_the_fewest_within_tolerance():
    rng = np.random.default_rng(41)
    for trial in range(40):
        n = int(rng.integers(1, 10))
        v = np.exp(rng.normal(0.0, 1.0, n))
        tol = float(rng.choice([0.05, 0.2, 0.5]))
        levels, mp = rte.rte_kappa_levels(v, tol)
        assert np.all(np.diff(levels) > 0)
        ratio = v / levels[mp]
        assert np.all(ratio <= 1 + tol + 1e-12) and np.all(1 / ratio <= 1 + tol + 1e-12)
        assert len(levels) == _min_levels(v, tol), (v, tol)
    # equal values share a level; one value is its own level times 1 / (1 + tol)
    levels, mp = rte.rte_kappa_levels([2.0, 2.0, 2.0], 0.1)
    assert len(levels) == 1 and np.all(mp == 0) and abs(levels[0] - 2.2) < 1e-15


@pytest.mark.parametrize("values,tol,mx", [([1.0, -1.0], 0.1, 8), ([1.0, 2.0], 0.0, 8), ([1.0, 100.0], 0.1, 1),
                                           ([np.nan], 0.1, 4)])
def test_kappa_levels_validation(values, tol, mx):
    with pytest.raises(rte.RteError):
        rte.rte_kappa_levels(values, tol, mx)
