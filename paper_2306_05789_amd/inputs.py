"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws and lays out inputs (grids, absorption fields, band
frequencies, wall temperatures, request streams).  It holds none of the
method's arithmetic and imports nothing from the GPU library or the oracle.

The academic test's geometry (a box with an inner cube, three reflective
planes, a low-absorption cylinder) is written out from the paper's description
(`academic`).  The paper's other workloads (the Chamonix valley terrain, the
Gemini absorption spectra) are not available, so box-shaped grids with smooth
analytic absorption fields stand in for them, at vertex counts inside the
range of the paper's table (2.7K to 196K vertices) and optical thicknesses
from about 0.1 to 10 per unit length.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FACE_X_LO, FACE_X_HI, FACE_Y_LO, FACE_Y_HI, FACE_Z_LO, FACE_Z_HI = (1 << f for f in range(6))
ALL_FACES = 63


def grid_positions(n, lo, hi) -> np.ndarray:
    """Vertex positions in natural order v = (i*n1 + j)*n2 + k."""
    axes = [np.linspace(lo[a], hi[a], n[a]) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def smooth_kappa(pos: np.ndarray) -> np.ndarray:
    """kappa(x) = 0.5 + 0.4 sin(2 pi x) cos(2 pi y) z, values in [0.1, 0.9] on the unit cube."""
    return 0.5 + 0.4 * np.sin(2 * np.pi * pos[:, 0]) * np.cos(2 * np.pi * pos[:, 1]) * pos[:, 2]


@dataclass
class Workload:
    name: str
    n: tuple
    lo: tuple
    hi: tuple
    kappa: np.ndarray              # [B, N] absorption per band at the vertices, natural order
    emit_faces: int
    grey: bool
    nu: np.ndarray = field(default_factory=lambda: np.ones(1))
    wall_axis: int = -1
    wall_side: int = 0
    R: float = 0.0
    T_wall: np.ndarray = None      # [nrhs, L] wall temperatures on the emitting vertices
    leaf_size: int = 64
    eta: float = 2.0
    aca_eps: float = 1e-5
    tol: float = 1e-10
    dense: bool = False

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def bands(self) -> int:
        return int(self.kappa.shape[0])


@dataclass
class Academic:
    """The geometry of the paper's academic test (Section "An Academic Test",
    Test-3): the box D = (0,60) x (0,100) x (0,60) (cm) minus the cube
    C = [0,10]^3 in the corner where the three reflective planes through the
    origin (R = 1) meet; C's three faces inside D emit, D's outer faces absorb
    and do not emit; kappa = 1e-4 in the cylinder (0,10) x (10,100) x (0,10)
    that prolongs C and 0.1 elsewhere (per cm; at the vertices: 1e-4 on the
    closed cylinder, the P1 interpolant in between); grey, no scattering.
    Spacing h (cm, a divisor of 10): h = 5, 2.5, 5/3, 1.25 give 3.5K, 25.6K,
    83.5K and 194K vertices, next to the paper's 2.8K to 196K meshes."""
    h: float
    n: tuple
    lo: tuple
    hi: tuple
    kappa: np.ndarray        # [N], natural order
    hole: tuple              # ((0, 0, 0), (m, m, m)), m = 10 / h cells
    hole_emit: int           # the hole's faces x = 10, y = 10, z = 10
    walls: list              # the planes x = 0, y = 0, z = 0, R = 1
    emit_faces: int = 0
    T_hole: float = 1.0      # temperature of the emitting faces (grey source sigma T^4)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))


def academic(h: float = 2.5) -> Academic:
    m = 10.0 / h
    assert abs(m - round(m)) < 1e-9, "h must divide 10"
    m = int(round(m))
    n = (6 * m + 1, 10 * m + 1, 6 * m + 1)
    lo, hi = (0.0, 0.0, 0.0), (60.0, 100.0, 60.0)
    pos = grid_positions(n, lo, hi)
    eps = 1e-9 * h
    cyl = (pos[:, 0] <= 10.0 + eps) & (pos[:, 1] >= 10.0 - eps) & (pos[:, 2] <= 10.0 + eps)
    kappa = np.where(cyl, 1e-4, 0.1)
    return Academic(h, n, lo, hi, kappa, ((0, 0, 0), (m, m, m)), FACE_X_HI | FACE_Y_HI | FACE_Z_HI,
                    [(0, 0, 1.0), (1, 0, 1.0), (2, 0, 1.0)])


def n_emitting(n, emit_faces) -> int:
    idx = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), -1).reshape(-1, 3)
    on = np.zeros(len(idx), dtype=bool)
    for f in range(6):
        if (emit_faces >> f) & 1:
            a, side = f // 2, f % 2
            on |= idx[:, a] == (n[a] - 1 if side else 0)
    return int(on.sum())


def config_tiny(n=11) -> Workload:
    """Unit cube on an n^3 grid, grey, constant kappa = 1, wall x = 0 at T = 1, dense FP64."""
    N = n ** 3
    return Workload(f"cube{n}_grey_dense", (n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                    np.ones((1, N)), FACE_X_LO, True,
                    T_wall=np.ones((1, n * n)), dense=True, tol=1e-10)


def config_hmatrix(n=41) -> Workload:
    """Unit cube on an n^3 grid, grey, smooth kappa, wall x = 0 at T = 1, FP64 H-matrix
    (leaf 64, eta 2, ACA 1e-5)."""
    pos = grid_positions((n, n, n), (0, 0, 0), (1, 1, 1))
    return Workload(f"cube{n}_grey_hmatrix", (n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                    smooth_kappa(pos)[None, :], FACE_X_LO, True,
                    T_wall=np.ones((1, n * n)), tol=1e-10)


def reflective_bands(n=(65, 33, 33), bands=8) -> Workload:
    """Box [0,2]x[0,1]^2, reflective wall z = 0 with R = 0.5, x = 0 wall at T = 1,
    bands nu_k = 0.5 * 8^(k/(B-1)) and kappa_nu = kappa(x) nu^-1.5."""
    pos = grid_positions(n, (0, 0, 0), (2, 1, 1))
    nu = 0.5 * 8.0 ** (np.arange(bands) / max(bands - 1, 1))
    kap = smooth_kappa(pos)[None, :] * nu[:, None] ** -1.5
    L = n[1] * n[2]
    return Workload(f"box{n[0]}x{n[1]}x{n[2]}_reflect_{bands}bands", tuple(n), (0.0, 0.0, 0.0),
                    (2.0, 1.0, 1.0), kap, FACE_X_LO, False, nu=nu, wall_axis=2, wall_side=0, R=0.5,
                    T_wall=np.ones((1, L)), tol=1e-6)


def catalogue(bands=32, seed=4):
    """Band catalogue of the batched and served workloads: nu_b log-spaced in
    [0.25, 16] and the kappa factor c_b of each band, lognormal(0, 1)."""
    return np.geomspace(0.25, 16.0, bands), np.random.default_rng(seed).lognormal(0.0, 1.0, bands)


def batched(n=49, bands=32, nrhs=16, seed_bands=4, seed_rhs=5) -> Workload:
    """Unit cube on n^3, `bands` bands with kappa_b = c_b kappa(x), c_b lognormal(0,1),
    nu_b log-spaced in [0.25, 16], all faces emitting with nrhs random wall
    temperature fields in [0.5, 2]."""
    pos = grid_positions((n, n, n), (0, 0, 0), (1, 1, 1))
    nu, c = catalogue(bands, seed_bands)
    L = n_emitting((n, n, n), ALL_FACES)
    Tw = np.random.default_rng(seed_rhs).uniform(0.5, 2.0, (nrhs, L))
    return Workload(f"cube{n}_{bands}bands_{nrhs}rhs", (n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                    c[:, None] * smooth_kappa(pos)[None, :], ALL_FACES, False, nu=nu, T_wall=Tw,
                    tol=1e-6)


@dataclass
class Request:
    arrival: float          # seconds from the stream start
    mesh: int               # index into the resident mesh list
    bands: np.ndarray       # subset of the band catalogue (sorted indices)
    scale: float            # kappa scale of the request; band b's multiplier is scale * c_b
    T_wall: np.ndarray      # [L] wall temperatures on the mesh's emitting vertices


def request_stream(count=256, rate=20.0, meshes=(21, 29, 41, 49), catalogue=32, seed=6):
    """Poisson arrivals at `rate`/s; mesh uniform over the resident list; 1..catalogue
    bands; kappa scale log-uniform in [0.1, 10]; wall temperatures uniform in [0.5, 2]."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for k in range(count):
        m = int(rng.integers(len(meshes)))
        nb = int(rng.integers(1, catalogue + 1))
        bands = np.sort(rng.choice(catalogue, nb, replace=False))
        scale = float(10.0 ** rng.uniform(-1.0, 1.0))
        n = meshes[m]
        Tw = rng.uniform(0.5, 2.0, n_emitting((n, n, n), ALL_FACES))
        out.append(Request(float(t[k]), m, bands, scale, Tw))
    return out
