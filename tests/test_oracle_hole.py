"""Pins of the oracle's non-convex domain: the box minus a box of grid cells
(the inner cube of Section "An Academic Test"), treated as Remark rem1 says,
kappa = +infinity in the removed part.  Each test checks the oracle against
something other than itself: a slab test for the blocking, the box operator
without the hole, the solid angle of the hole's faces, closure, and the
mirror-doubled domain.  No GPU is used.
"""
import numpy as np
import pytest

from oracle import solve
from oracle.core import Grid, Problem

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _problem(n, hi=(1, 1, 1), kappa=None, **kw):
    g = Grid(tuple(n), (0.0, 0.0, 0.0), tuple(float(v) for v in hi))
    if kappa is None:
        kappa = np.ones(g.N)
    elif callable(kappa):
        kappa = kappa(g.positions())
    return Problem(g, np.asarray(kappa, dtype=np.float64), **kw)


def _meets_open_box(p, q, lo, hi):
    """Slab test: does the segment p -> q run a positive length inside the open
    box (lo, hi)?  Returns (meets, margin) with margin the clipped parameter
    length, or how far a grazing segment is from entering."""
    t0, t1 = 0.0, 1.0
    for a in range(3):
        d = q[a] - p[a]
        if d == 0.0:
            if not (lo[a] < p[a] < hi[a]):
                return False, -min(abs(p[a] - lo[a]), abs(p[a] - hi[a]))
            continue
        ta, tb = (lo[a] - p[a]) / d, (hi[a] - p[a]) / d
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return t1 > t0, t1 - t0


def _hole_box(g, hole):
    """The region a segment may not cross, in coordinates: the hole's open box,
    open past every box face the hole reaches (a covered part of a box face is
    not in the closed domain either)."""
    lo = np.array(hole[0]) * np.array(g.h)
    hi = np.array(hole[1]) * np.array(g.h)
    lo = np.where(np.array(hole[0]) == 0, -np.inf, lo)
    hi = np.where(np.array(hole[1]) == np.array(g.n) - 1, np.inf, hi)
    return lo, hi


def _box(P):
    """The same problem on the whole box (no hole)."""
    return Problem(P.grid, P.kappa, emit_faces=P.emit_faces, walls=P.walls)


def _star_has_hole_cell(g, hole, v):
    lo, hi = hole
    idx = g.index(v)
    for o in range(8):
        c = idx - np.array([(o >> a) & 1 for a in range(3)])
        if np.all(c >= 0) and np.all(c <= np.array(g.n) - 2) and all(lo[a] <= c[a] < hi[a] for a in range(3)):
            return True
    return False


def test_tau_is_infinite_iff_the_segment_crosses_the_hole():
    rng = np.random.default_rng(21)
    hole = ((2, 1, 1), (4, 3, 4))
    P = _problem((7, 6, 6), hi=(1.2, 1.0, 1.0), kappa=lambda X: rng.uniform(0.2, 2.0, len(X)), hole=hole)
    g = P.grid
    lo = np.array(hole[0]) * np.array(g.h)
    hi = np.array(hole[1]) * np.array(g.h)
    p = rng.uniform(0, 1, (400, 3)) * [1.2, 1.0, 1.0]
    q = rng.uniform(0, 1, (400, 3)) * [1.2, 1.0, 1.0]
    # segments along the hole's faces and edges graze it: not blocked
    p = np.vstack([p, [[lo[0], 0.0, 0.5], [0.0, lo[1], lo[2]], [hi[0], hi[1], 0.0]]])
    q = np.vstack([q, [[lo[0], 1.0, 0.7], [1.2, lo[1], lo[2]], [hi[0], hi[1], 1.0]]])
    tau = P.tau(p, q)
    tau_box = _box(P).tau(p, q)
    n_blocked = 0
    for k in range(len(p)):
        meets, margin = _meets_open_box(p[k], q[k], lo, hi)
        if abs(margin) < 1e-9:
            continue
        if meets:
            n_blocked += 1
            assert np.isinf(tau[k]), k
        else:
            assert tau[k] == tau_box[k], k     # the same march, nothing blocked
    assert 50 < n_blocked < 350
    assert np.all(np.isfinite(tau[-3:]))


def _lattice_blocked(p, q, lo, hi):
    """Exact slab test in rationals for lattice points (grid units): does p -> q
    run a positive length inside the open box (lo, hi) (None: unbounded)?"""
    from fractions import Fraction
    t0, t1 = Fraction(0), Fraction(1)
    for a in range(3):
        d = q[a] - p[a]
        if d == 0:
            if not ((lo[a] is None or p[a] > lo[a]) and (hi[a] is None or p[a] < hi[a])):
                return False
            continue
        ends = [Fraction(b - p[a], d) for b in (lo[a], hi[a]) if b is not None]
        if d > 0:
            t0 = max(t0, ends[0]) if lo[a] is not None else t0
            t1 = min(t1, ends[-1]) if hi[a] is not None else t1
        else:
            t1 = min(t1, ends[0]) if lo[a] is not None else t1
            t0 = max(t0, ends[-1]) if hi[a] is not None else t0
    return t1 > t0


def test_tau_blocking_between_all_vertex_pairs_is_exact():
    """Every vertex pair of a small grid, grazing pairs included: tau is infinite
    exactly when the exact rational slab test finds a positive length outside
    the closed domain (the hole reaches the face y = 0, so the covered part of
    that face blocks as well)."""
    hole = ((1, 0, 1), (3, 2, 3))
    P = _problem((5, 4, 5), kappa=np.full(100, 0.7), hole=hole)
    g = P.grid
    lo = [1, None, 1]
    hi = [3, 2, 3]
    idx = g.index(np.arange(g.N))
    pi, qi = np.meshgrid(np.arange(g.N), np.arange(g.N), indexing="ij")
    pi, qi = pi.ravel(), qi.ravel()
    keep = pi < qi
    pi, qi = pi[keep], qi[keep]
    x = g.positions()
    tau = P.tau(x[pi], x[qi])
    ref = np.array([_lattice_blocked(idx[a], idx[b], lo, hi) for a, b in zip(pi, qi)])
    assert np.array_equal(np.isinf(tau), ref)
    assert 200 < ref.sum() < len(ref) - 200


def test_hole_entries_are_the_visible_entries_of_the_box():
    """Columns whose star has no hole cell: G(hole) = G(box) where the vertices see
    each other and 0 where the hole hides them; rows and columns of the vertices
    with no domain cell are zero; hole cells are in no star."""
    rng = np.random.default_rng(22)
    hole = ((1, 2, 0), (3, 4, 2))          # touches the face z = 0
    kap = rng.uniform(0.2, 1.5, 6 * 6 * 5)
    P = _problem((6, 6, 5), kappa=kap, emit_faces=2 | 8, hole=hole)
    B = _box(P)
    g = P.grid
    G, Gb = P.dense_G(), B.dense_G()
    x = g.positions()
    lo, hi = _hole_box(g, hole)
    assert lo[2] == -np.inf
    idx = g.index(np.arange(g.N))
    inactive = np.all((idx > np.array(hole[0])) & (idx < np.array(hole[1])), axis=1) | \
        (np.all((idx[:, :2] > np.array(hole[0][:2])) & (idx[:, :2] < np.array(hole[1][:2])), axis=1) & (idx[:, 2] == 0))
    assert inactive.sum() == 2                 # (2, 3, 1) inside, (2, 3, 0) on the face z = 0 under it
    assert np.all(G[inactive] == 0) and np.all(G[:, inactive] == 0)
    clean = np.array([not _star_has_hole_cell(g, hole, v) for v in range(g.N)])
    n_hidden = 0
    for i in np.nonzero(~inactive)[0]:
        for j in np.nonzero(clean)[0]:
            meets, margin = _meets_open_box(x[i], x[j], lo, hi)
            if abs(margin) < 1e-12:
                # grazing (touching the hole's boundary only): not blocked
                assert G[i, j] == Gb[i, j]
            elif meets:
                n_hidden += 1
                assert G[i, j] == 0.0
            else:
                assert G[i, j] == Gb[i, j]
    assert n_hidden > 500
    # columns next to the hole lose the hole's cells of their star
    touched = ~clean & ~inactive
    assert np.all(G[:, touched] <= Gb[:, touched] + 1e-300)
    assert np.all(G[:, touched].sum(0) < Gb[:, touched].sum(0))
    # the box faces y = 1 and x = 1 do not meet the hole: S(hole) = S(box) where visible
    S, Sb = P.dense_S(), B.dense_S()
    assert np.array_equal(P.emitting, B.emitting)
    for i in np.nonzero(~inactive)[0]:
        for k, l in enumerate(P.emitting):
            meets, margin = _meets_open_box(x[i], x[l], lo, hi)
            assert S[i, k] == (0.0 if meets and margin > 1e-12 else Sb[i, k])


def _rect_solid_angle(x, a, plane, r0, r1):
    """Solid angle of the rectangle r0 <= (y_b, y_c) <= r1 in the plane y_a = plane
    seen from x (b < c the other axes): the signed sum over its corners of
    arctan(uv / (d sqrt(u^2 + v^2 + d^2))), u, v the corner's offsets."""
    b, c = [k for k in range(3) if k != a]
    d = abs(x[a] - plane)
    tot = 0.0
    for cu, su in ((r1[0], 1), (r0[0], -1)):
        for cv, sv in ((r1[1], 1), (r0[1], -1)):
            u, v = cu - x[b], cv - x[c]
            tot += su * sv * np.arctan(u * v / (d * np.sqrt(u * u + v * v + d * d)))
    return tot


def test_hole_faces_emit_their_solid_angle_at_kappa0():
    """kappa -> 0, only the hole's faces emit: S^E = sum over the faces the point
    sees of Omega_face(x) / (4 pi) (eq. SE1 with the hole's faces as the wall)."""
    pts = np.array([[0.0, 0.5, 0.5], [0.875, 0.875, 0.125], [0.5, 0.875, 0.5], [0.125, 0.25, 0.375]])
    lo, hi = np.array([0.25] * 3), np.array([0.75] * 3)
    errs = []
    for n in (9, 17, 33):
        m = (n - 1) // 4
        P = _problem((n, n, n), kappa=np.zeros(n ** 3), emit_faces=0, hole=((m,) * 3, (3 * m,) * 3), hole_emit=63)
        ids = P.grid.vid(np.rint(pts * (n - 1)).astype(np.int64))
        SE = P.surface_block(ids, P.emitting).sum(axis=1)
        ref = np.zeros(len(pts))
        for k, x in enumerate(pts):
            for a in range(3):
                b, c = [q for q in range(3) if q != a]
                for plane, sgn in ((lo[a], -1), (hi[a], 1)):
                    if (x[a] - plane) * sgn > 0:   # in front of the face
                        ref[k] += _rect_solid_angle(x, a, plane, (lo[b], lo[c]), (hi[b], hi[c])) / (4 * np.pi)
        errs.append(np.max(np.abs(SE - ref) / ref))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 5e-3
    # a vertex inside a hole face sees half the sphere; one on an edge of the hole, pi from each face
    P = _problem((9, 9, 9), kappa=np.zeros(729), emit_faces=0, hole=((2,) * 3, (6,) * 3), hole_emit=63)
    face, edge = P.grid.vid([[6, 4, 4], [6, 6, 4]])
    S = P.surface_block([face, edge], P.emitting).sum(axis=1)
    assert abs(S[0] - 0.5) < 1e-15 and abs(S[1] - 0.5) < 1e-15


def test_closure_with_an_emitting_hole():
    """Absorbed plus transmitted fractions sum to one along every ray when the box's
    and the hole's faces all emit: sum_j G^{ij} + sum_l S^{il} -> 1 (variable kappa)."""
    devs = []
    for n in (9, 17, 33):
        m = (n - 1) // 4
        P = _problem((n, n, n), kappa=lambda X: 0.5 + 0.4 * np.sin(2 * np.pi * X[:, 0]) * X[:, 2],
                     emit_faces=63, hole=((m, m, m), (3 * m, 3 * m, 2 * m)), hole_emit=63)
        i = int(P.grid.vid(np.rint(np.array([0.125, 0.5, 0.375]) * (n - 1)).astype(np.int64)))
        tot = P.volume_block([i], np.arange(P.grid.N)).sum() + P.surface_block([i], P.emitting).sum()
        devs.append(abs(1.0 - tot))
    assert devs[0] > devs[1] > devs[2] and devs[2] < 0.02


def test_covered_box_face_squares_do_not_emit():
    """A hole touching an emitting box face covers part of it: the covered vertices
    are no surface unknowns and the rest of the face emits as before."""
    P = _problem((7, 6, 6), emit_faces=1, hole=((0, 1, 2), (2, 4, 5)))
    g = P.grid
    em = P.emitting
    idx = g.index(em)
    assert np.all(idx[:, 0] == 0)
    # the hole reaches the face z = 1 too: the vertices on that edge under it are covered
    covered = [(j, k) for j in range(6) for k in range(6) if 1 < j < 4 and 2 < k]
    assert len(em) == 36 - len(covered)
    assert not any((j, k) in covered for j, k in idx[:, 1:])


def _doubled_with_hole(P, hole, hole_emit):
    """The mirror-doubled domain (wall at x = 0) with the hole and its mirror image."""
    g = P.grid
    na = g.n[0]
    gd = Grid((2 * na - 1, g.n[1], g.n[2]), (-g.hi[0], g.lo[1], g.lo[2]), g.hi)
    idx = gd.index(np.arange(gd.N))
    src = idx.copy()
    src[:, 0] = np.abs(idx[:, 0] - (na - 1))
    (l0, l1, l2), (h0, h1, h2) = hole
    assert l0 == 0
    dh = ((na - 1 - h0, l1, l2), (na - 1 + h0, h1, h2))
    emit = hole_emit | (1 if hole_emit & 2 else 0)
    return Problem(gd, P.kappa[g.vid(src)], emit_faces=P.emit_faces, flip_axis=0, flip_cells=na - 1,
                   hole=dh, hole_emit=emit)


def test_reflective_wall_under_the_hole_equals_doubled_domain():
    """The academic test's corner: the hole touches the reflective plane.  With
    R = 1 the operators equal those of the doubled domain (hole and its mirror
    image merged) folded onto the original vertices, entry by entry."""
    rng = np.random.default_rng(23)
    hole, hole_emit = ((0, 1, 1), (2, 3, 3)), 2 | 8 | 32
    P = _problem((5, 5, 5), kappa=lambda X: rng.uniform(0.2, 1.5, len(X)), emit_faces=8 | 32,
                 walls=[(0, 0, 1.0)], hole=hole, hole_emit=hole_emit)
    Pd = _doubled_with_hole(P, hole, hole_emit)
    g, gd = P.grid, Pd.grid
    shift = np.array([g.n[0] - 1, 0, 0])
    flip = np.array([-1, 1, 1])
    idx = g.index(np.arange(g.N))
    dir_ids, mir_ids = gd.vid(idx + shift), gd.vid(idx * flip + shift)
    G = P.dense_G()
    Gd = Pd.volume_block(dir_ids, np.concatenate([dir_ids, mir_ids]))
    fold = Gd[:, :g.N] + np.where(idx[:, 0] > 0, 1.0, 0.0)[None, :] * Gd[:, g.N:]
    assert np.max(np.abs(G - fold)) < 1e-13 * np.max(np.abs(G))
    em = P.emitting
    eidx = g.index(em)
    S = P.dense_S()
    Sd = Pd.surface_block(dir_ids, np.concatenate([gd.vid(eidx + shift), gd.vid(eidx * flip + shift)]))
    foldS = Sd[:, :len(em)] + np.where(eidx[:, 0] > 0, 1.0, 0.0)[None, :] * Sd[:, len(em):]
    assert np.max(np.abs(S - foldS)) < 1e-13 * np.max(np.abs(S))
    # the hole matters (the check has teeth)
    P0 = _problem((5, 5, 5), kappa=P.kappa, emit_faces=8 | 32, walls=[(0, 0, 1.0)])
    assert np.max(np.abs(P0.dense_G() - G)) > 1e-2 * np.max(np.abs(G))


def test_fixed_point_with_a_hole_leaves_removed_vertices_cold():
    """The fixed point on a domain with a hole: the removed vertices keep J = T = 0,
    the rest is monotone and equals the direct solve (grey)."""
    n = 9
    P = _problem((n, n, n), kappa=lambda X: 0.3 + X[:, 1], emit_faces=0, hole=((2, 2, 2), (5, 6, 5)),
                 hole_emit=63)
    G = P.dense_G()
    SE = P.dense_S() @ np.full(len(P.emitting), solve.SIGMA)
    res = solve.fixed_point([G], SE[None], grey=True, tol=1e-14, keep_history=True)
    idx = P.grid.index(np.arange(P.grid.N))
    inside = np.all((idx > [2, 2, 2]) & (idx < [5, 6, 5]), axis=1)
    assert inside.sum() == 2 * 3 * 2
    assert np.all(res.T[inside] == 0) and np.all(res.J[0, inside] == 0)
    assert np.all(res.T[~inside] > 0)
    J = solve.direct_grey(G, SE)
    assert np.max(np.abs(res.J[0] - J)) < 1e-12 * np.max(J)
    for a, b in zip(res.T_history, res.T_history[1:]):
        assert np.all(b >= a - 1e-15 * np.abs(b))
