"""Planck function, band weights and the monotone fixed point, in FP64 numpy.

TEST INFRASTRUCTURE: part of the FP64 CPU oracle (see the package docstring).

Follows the Algorithm of Section "Fixed Point Iterations": starting from T^0
and J^0 = 0,
    S_b^k     = (1 - a_b) B_{nu_b}(T^k) + a_b J_b^k          (collocated source)
    J_b^{k+1} = S^E_b + G_b S_b^k
    T^{k+1}   : root of sum_b w_b kappa_b (1 - a_b) (J_b^{k+1} - B_{nu_b}(T)) = 0
The root is found per vertex by bisection (the paper uses Newton; bisection is
the slow, obviously convergent stand-in).  In the grey case (Section "An
Academic Test", eq. grey) B(T) = sigma T^4 with sigma = pi^4/15 and the root
is T = (J/sigma)^{1/4}.  The rescaled Planck function is
B_nu(T) = nu^3 / (exp(nu/T) - 1) (Section 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SIGMA = np.pi ** 4 / 15.0


def planck(nu, T):
    """nu^3 / (exp(nu/T) - 1), with B(0) = 0."""
    nu = np.asarray(nu, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        val = nu ** 3 / np.expm1(nu / T)
    return np.where(T > 0, val, 0.0)


def band_weights(nu) -> np.ndarray:
    """Trapezoid weights on the sorted band frequencies, no tails; one band: 1."""
    nu = np.asarray(nu, dtype=np.float64)
    if len(nu) == 1:
        return np.ones(1)
    assert np.all(np.diff(nu) > 0)
    w = np.zeros(len(nu))
    w[0] = 0.5 * (nu[1] - nu[0])
    w[-1] = 0.5 * (nu[-1] - nu[-2])
    w[1:-1] = 0.5 * (nu[2:] - nu[:-2])
    return w


def temperature_bisect(Jb, coef, nu, lo=None, rel=1e-15, max_iter=400):
    """Per vertex, the root T of sum_b coef_b (J_b - B_{nu_b}(T)) = 0.

    Jb, coef: [B, N].  The left side decreases in T; T = 0 where sum coef J <= 0."""
    Jb = np.asarray(Jb, dtype=np.float64)
    coef = np.asarray(coef, dtype=np.float64)
    N = Jb.shape[1]
    nu = np.asarray(nu, dtype=np.float64)[:, None]

    def f(T):
        return np.sum(coef * (Jb - planck(nu, T[None, :])), axis=0)

    pos = np.sum(coef * Jb, axis=0) > 0
    hi = np.ones(N)
    for _ in range(200):
        bad = pos & (f(hi) > 0)
        if not bad.any():
            break
        hi[bad] *= 2.0
    lo = np.zeros(N)
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        up = f(mid) > 0
        lo = np.where(up, mid, lo)
        hi = np.where(up, hi, mid)
        if np.all(hi - lo <= rel * hi):
            break
    return np.where(pos, 0.5 * (lo + hi), 0.0)


@dataclass
class FixedPointResult:
    T: np.ndarray                 # [N]
    J: np.ndarray                 # [B, N]
    iterations: int
    residuals: list = field(default_factory=list)
    T_history: list = field(default_factory=list)
    J_history: list = field(default_factory=list)


def fixed_point(G, SE, *, grey: bool, nu=None, w=None, a=None, kappa_v=None, T0=None,
                tol=1e-13, max_iter=2000, keep_history=False) -> FixedPointResult:
    """Monotone fixed point (Algorithm, eq. algo).

    G: list of B dense [N,N] operators (kappa inside, Section "FEM discretization").
    SE: [B, N] boundary source S^E_b = S_b_hat Q_b.
    grey: single band with B(T) = sigma T^4.
    a: [B] scattering coefficients (default 0); the source is S_b = (1 - a_b) B_b(T) + a_b J_b
    (eq. eqS) in both formulations.
    kappa_v: [B, N] kappa at the vertices (weights of the temperature balance).
    Stops when max_b ||J_b^{k+1} - J_b^k|| / ||J_b^{k+1}|| <= tol.
    """
    SE = np.atleast_2d(np.asarray(SE, dtype=np.float64))
    B, N = SE.shape
    a = np.zeros(B) if a is None else np.asarray(a, dtype=np.float64)
    T = np.zeros(N) if T0 is None else np.asarray(T0, dtype=np.float64).copy()
    J = np.zeros((B, N))
    res = FixedPointResult(T, J, 0)
    if not grey:
        nu = np.asarray(nu, dtype=np.float64)
        w = band_weights(nu) if w is None else np.asarray(w, dtype=np.float64)
        coef = w[:, None] * np.asarray(kappa_v, dtype=np.float64) * (1.0 - a)[:, None]
    for k in range(max_iter):
        emission = SIGMA * T[None, :] ** 4 if grey else planck(nu[:, None], T[None, :])
        S = (1.0 - a)[:, None] * emission + a[:, None] * J
        Jn = np.stack([SE[b] + G[b] @ S[b] for b in range(B)])
        num = np.linalg.norm(Jn - J, axis=1)
        den = np.linalg.norm(Jn, axis=1)
        r = float(np.max(np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)))
        if grey:
            T = (np.maximum(Jn[0], 0.0) / SIGMA) ** 0.25
        else:
            T = temperature_bisect(Jn, coef, nu)
        J = Jn
        res.residuals.append(r)
        if keep_history:
            res.T_history.append(T.copy())
            res.J_history.append(J.copy())
        if r <= tol:
            res.iterations = k + 1
            break
    else:
        res.iterations = max_iter
    res.T, res.J = T, J
    return res


def direct_grey(G, SE) -> np.ndarray:
    """Grey, no scattering: sigma T^4 = J, so J = S^E + G J and J* = (I - G)^{-1} S^E."""
    G = np.asarray(G, dtype=np.float64)
    return np.linalg.solve(np.eye(G.shape[0]) - G, np.asarray(SE, dtype=np.float64))
