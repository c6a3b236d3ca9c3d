"""Symmetric simplex quadrature rules, derived from their moment equations.

TEST INFRASTRUCTURE: part of the FP64 CPU oracle.  Only tests, the smoke check
and the benchmark's CPU-baseline leg may import this package.

The method integrates the kernel against P1 hat functions with quadrature
points inside the elements: a degree-5 rule with 14 points when the target
vertex is close, and a degree-2 rule with 4 points otherwise (Section
"FEM discretization and Compressed H-Matrices").  The boundary (triangle)
integrals of the surface source matrix use the analogous triangle rules
(degree 2 with 3 points, degree 5 with 7 points).

No rule constant is typed in from memory: each rule is the solution of its
moment equations (exact integration of every barycentric monomial up to the
rule's degree), found by least squares from seeded random starts and then
required to be unique among the interior, positive-weight solutions.

Barycentric monomial averages over a d-simplex (Dirichlet integral):
    mean(lambda^alpha) = d! * prod(alpha_i!) / (d + |alpha|)!
"""
from __future__ import annotations

import itertools
import math
from functools import lru_cache

import numpy as np
from scipy.optimize import least_squares


def monomial_mean(alpha) -> float:
    """Average of prod(lambda_i^alpha_i) over the simplex with len(alpha) vertices."""
    d = len(alpha) - 1
    num = math.factorial(d) * math.prod(math.factorial(a) for a in alpha)
    return num / math.factorial(d + sum(alpha))


@lru_cache(maxsize=None)
def exponents(nvert: int, degree: int):
    """All exponent tuples of nvert barycentric variables with total degree <= degree."""
    out = []
    for total in range(degree + 1):
        for alpha in itertools.product(range(total + 1), repeat=nvert):
            if sum(alpha) == total:
                out.append(alpha)
    return tuple(out)


@lru_cache(maxsize=None)
def _moment_table(nvert: int, degree: int):
    alphas = exponents(nvert, degree)
    return np.array(alphas, dtype=float), np.array([monomial_mean(a) for a in alphas])


def _orbit(base):
    """Distinct permutations of a barycentric tuple, in lexicographic order."""
    return sorted(set(itertools.permutations(base)), reverse=True)


def _points_tet5(p):
    a1, w1, a2, w2, c, w3 = p
    pts, wts = [], []
    for a, w in ((a1, w1), (a2, w2)):
        b = (1.0 - a) / 3.0
        for q in _orbit((a, b, b, b)):
            pts.append(q)
            wts.append(w)
    d = 0.5 - c
    for q in _orbit((c, c, d, d)):
        pts.append(q)
        wts.append(w3)
    return np.array(pts), np.array(wts)


def _points_tri5(p):
    w0, a1, w1, a2, w2 = p
    pts = [(1 / 3, 1 / 3, 1 / 3)]
    wts = [w0]
    for a, w in ((a1, w1), (a2, w2)):
        b = (1.0 - a) / 2.0
        for q in _orbit((a, b, b)):
            pts.append(q)
            wts.append(w)
    return np.array(pts), np.array(wts)


def _points_tet2(p):
    (a,) = p
    b = (1.0 - a) / 3.0
    pts = np.array(_orbit((a, b, b, b)))
    return pts, np.full(len(pts), 0.25)


def _points_tri2(p):
    (a,) = p
    b = (1.0 - a) / 2.0
    pts = np.array(_orbit((a, b, b)))
    return pts, np.full(len(pts), 1.0 / 3.0)


def moment_residual(pts: np.ndarray, wts: np.ndarray, degree: int) -> np.ndarray:
    """Rule value minus exact mean, for every barycentric monomial up to `degree`."""
    alphas, exact = _moment_table(pts.shape[1], degree)
    vals = np.prod(pts[:, None, :] ** alphas[None, :, :], axis=2)
    return wts @ vals - exact


def _solve(builder, degree, lo, hi, canon, seed, starts):
    rng = np.random.default_rng(seed)
    found = []
    for _ in range(starts):
        x0 = rng.uniform(lo, hi)
        try:
            sol = least_squares(lambda p: moment_residual(*builder(p), degree), x0,
                                xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=400)
        except ValueError:
            continue
        pts, wts = builder(sol.x)
        if np.max(np.abs(moment_residual(pts, wts, degree))) > 1e-13:
            continue
        if np.any(wts <= 1e-12) or np.any(pts <= 1e-9):
            continue
        key = canon(sol.x)
        if not any(np.allclose(key, k, atol=1e-9) for k in found):
            found.append(key)
    if len(found) != 1:
        raise RuntimeError(f"expected one interior positive rule, found {len(found)}")
    return builder(found[0])


def _canon_two_orbits(x, first_pair, cc_dd=None):
    """Order the two single-parameter orbits by their parameter so duplicates match.

    The (c,c,d,d) orbit with d = 1/2 - c is the same point set as (d,d,c,c), so
    its parameter is taken as min(c, 1/2 - c)."""
    x = np.array(x, dtype=float)
    if cc_dd is not None:
        x[cc_dd] = min(x[cc_dd], 0.5 - x[cc_dd])
    i, j = first_pair
    if x[i] > x[j]:
        x[[i, i + 1]], x[[j, j + 1]] = x[[j, j + 1]].copy(), x[[i, i + 1]].copy()
    return x


@lru_cache(maxsize=None)
def tet_rule(degree: int):
    """(points [nq,4] barycentric, weights [nq] summing to 1) on a tetrahedron."""
    if degree == 2:
        return _solve(_points_tet2, 2, [-0.5], [1.0], lambda x: np.array(x), seed=11, starts=40)
    if degree == 5:
        return _solve(_points_tet5, 5, [0.0, 0.0, 0.0, 0.0, 0.0, 0.0],
                      [1.0, 0.2, 1.0, 0.2, 0.5, 0.2],
                      lambda x: _canon_two_orbits(x, (0, 2), cc_dd=4), seed=12, starts=60)
    raise ValueError(degree)


@lru_cache(maxsize=None)
def tri_rule(degree: int):
    """(points [nq,3] barycentric, weights [nq] summing to 1) on a triangle."""
    if degree == 2:
        return _solve(_points_tri2, 2, [-0.5], [1.0], lambda x: np.array(x), seed=13, starts=40)
    if degree == 5:
        return _solve(_points_tri5, 5, [0.0, 0.0, 0.0, 0.0, 0.0], [0.5, 1.0, 0.3, 1.0, 0.3],
                      lambda x: _canon_two_orbits(x, (1, 3)), seed=14, starts=60)
    raise ValueError(degree)
