"""ctypes front end of the oracle's C core (kernel entries, optical depths, P1 kappa).

TEST INFRASTRUCTURE: part of the FP64 CPU oracle.  Only tests, the smoke check
and the benchmark's CPU-baseline leg may import this package; the GPU library
never calls it.

The C core (`rte_oracle.c`) evaluates, in FP64 and by brute force, the matrix
entries of the P1 collocation of the integral form (Section "FEM
discretization and Compressed H-Matrices"):

    G^{ij}   = exp(-tau(x_i,x_j)) g^{ij} + R exp(-tau_bar(x_i,x_j)) g_bar^{ij}
    S^{il}   = exp(-tau(x_i,x_l)) s^{il} + R exp(-tau_bar(x_i,x_l)) s_bar^{il}

with g, s the element quadratures of kappa w^j / (4 pi r^2) and of the
solid-angle density w~^l |(x-y).n| / (4 pi r^3), and tau, tau_bar the exact
optical depths along the direct and the reflected path (Proposition 1,
Proposition 2, Corollary).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

from . import quadrature

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rte_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FACE_BITS = {"x-": 1, "x+": 2, "y-": 4, "y+": 8, "z-": 16, "z+": 32}


def build(force: bool = False) -> str:
    """Compile the C core with gcc (FP64, no fast-math, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("h", C.c_double * 3),
        ("flip_axis", C.c_int32), ("flip_cells", C.c_int32),
        ("kappa", C.POINTER(C.c_double)),
        ("n_walls", C.c_int32), ("wall_axis", C.c_int32 * 6), ("wall_side", C.c_int32 * 6),
        ("R", C.c_double * 6),
        ("emit_faces", C.c_uint32),
        ("hole_lo", C.c_int32 * 3), ("hole_hi", C.c_int32 * 3), ("hole_emit", C.c_uint32),
        ("emission", C.c_uint32),
        ("near_cheb", C.c_int32),
        ("nq_tet_far", C.c_int32), ("nq_tet_near", C.c_int32),
        ("nq_tri_far", C.c_int32), ("nq_tri_near", C.c_int32),
        ("tet_far_p", C.POINTER(C.c_double)), ("tet_far_w", C.POINTER(C.c_double)),
        ("tet_near_p", C.POINTER(C.c_double)), ("tet_near_w", C.POINTER(C.c_double)),
        ("tri_far_p", C.POINTER(C.c_double)), ("tri_far_w", C.POINTER(C.c_double)),
        ("tri_near_p", C.POINTER(C.c_double)), ("tri_near_w", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER(_Problem)
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        for name in ("og_volume_block", "og_surface_block"):
            f = getattr(_lib, name)
            f.argtypes = [P, C.c_int64, i64p, C.c_int64, i64p, f64p]
            f.restype = None
        for name in ("og_volume_pairs", "og_surface_pairs"):
            f = getattr(_lib, name)
            f.argtypes = [P, C.c_int64, i64p, i64p, f64p]
            f.restype = None
        _lib.og_kappa_points.argtypes = [P, C.c_int64, f64p, f64p]
        _lib.og_emitting_mask.argtypes = [P, np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")]
        _lib.og_emitting_mask.restype = None
        _lib.og_tau_segments.argtypes = [P, C.c_int64, f64p, f64p, C.c_int32, f64p]
        _lib.og_volume_entry.argtypes = [P, C.c_int64, C.c_int64]
        _lib.og_volume_entry.restype = C.c_double
        _lib.og_surface_entry.argtypes = [P, C.c_int64, C.c_int64]
        _lib.og_surface_entry.restype = C.c_double
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Grid:
    """Structured box grid: n vertices per axis over [lo, hi]; natural vertex order
    v = (i*n1 + j)*n2 + k."""
    n: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)

    @property
    def h(self):
        return tuple((self.hi[a] - self.lo[a]) / (self.n[a] - 1) for a in range(3))

    @property
    def N(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def index(self, v):
        v = np.asarray(v, dtype=np.int64)
        k = v % self.n[2]
        j = (v // self.n[2]) % self.n[1]
        i = v // (self.n[1] * self.n[2])
        return np.stack([i, j, k], axis=-1)

    def vid(self, idx):
        idx = np.asarray(idx, dtype=np.int64)
        return (idx[..., 0] * self.n[1] + idx[..., 1]) * self.n[2] + idx[..., 2]

    def positions(self) -> np.ndarray:
        idx = self.index(np.arange(self.N))
        return np.asarray(self.lo) + idx * np.asarray(self.h)

    def emitting_vertices(self, emit_faces: int) -> np.ndarray:
        """Natural ids of the vertices on the emitting faces, ascending."""
        idx = self.index(np.arange(self.N))
        on = np.zeros(self.N, dtype=bool)
        for f in range(6):
            if (emit_faces >> f) & 1:
                a, side = f // 2, f % 2
                on |= idx[:, a] == (self.n[a] - 1 if side else 0)
        return np.nonzero(on)[0].astype(np.int64)


@dataclass
class Problem:
    """One kappa field on one grid, with planar reflective walls, each covering a
    whole box face and reflecting once (Hypothesis 1): either one wall given by
    wall_axis / wall_side / R, or a list `walls` of (axis, side, R).

    A non-convex domain (Remark rem1): `hole` = ((i0, j0, k0), (i1, j1, k1)), the
    grid cells [i0, i1) x [j0, j1) x [k0, k1) removed from the box (kappa =
    +infinity there); bit f of `hole_emit` makes the hole's face on side f % 2
    of axis f // 2 emit into the domain.

    `emission` = 1 takes the cosine-weighted wall source of Section "Example"
    (Q = [omega.n]_- Q0: kernel cos^2 / r^2 at the wall) instead of the
    isotropic one (eq. SE1, the default 0)."""
    grid: Grid
    kappa: np.ndarray
    emit_faces: int = 1
    wall_axis: int = -1
    wall_side: int = 0
    R: float = 0.0
    near_cheb: int = 2
    flip_axis: int = -1
    flip_cells: int = 0
    walls: list = None
    hole: tuple = None
    hole_emit: int = 0
    emission: int = 0
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        self.kappa = np.ascontiguousarray(self.kappa, dtype=np.float64)
        assert self.kappa.shape == (self.grid.N,)
        rules = []
        for deg in (2, 5):
            p, w = quadrature.tet_rule(deg)
            rules.append((np.ascontiguousarray(p), np.ascontiguousarray(w)))
        for deg in (2, 5):
            p, w = quadrature.tri_rule(deg)
            rules.append((np.ascontiguousarray(p), np.ascontiguousarray(w)))
        self._keep = [self.kappa] + [a for r in rules for a in r]
        s = _Problem()
        s.n[:] = list(self.grid.n)
        s.lo[:] = list(self.grid.lo)
        s.h[:] = list(self.grid.h)
        s.flip_axis, s.flip_cells = self.flip_axis, self.flip_cells
        s.kappa = _dptr(self.kappa)
        if self.walls is None:
            self.walls = [(self.wall_axis, self.wall_side, float(self.R))] if self.wall_axis >= 0 else []
        assert len(self.walls) <= 6 and len({(a, sd) for a, sd, _ in self.walls}) == len(self.walls)
        s.n_walls = len(self.walls)
        for w, (a, sd, r) in enumerate(self.walls):
            s.wall_axis[w], s.wall_side[w], s.R[w] = int(a), int(sd), float(r)
        s.emit_faces, s.near_cheb = self.emit_faces, self.near_cheb
        assert self.emission in (0, 1)
        s.emission = self.emission
        if self.hole is not None:
            lo, hi = self.hole
            n = self.grid.n
            assert all(0 <= lo[a] < hi[a] <= n[a] - 1 for a in range(3))
            for f in range(6):   # an emitting hole face lies inside the box
                if (self.hole_emit >> f) & 1:
                    a = f // 2
                    assert (hi[a] < n[a] - 1) if f % 2 else (lo[a] > 0)
            s.hole_lo[:], s.hole_hi[:] = [int(v) for v in lo], [int(v) for v in hi]
            s.hole_emit = self.hole_emit
        else:
            assert self.hole_emit == 0
        (tfp, tfw), (tnp, tnw), (sfp, sfw), (snp, snw) = rules
        s.nq_tet_far, s.nq_tet_near, s.nq_tri_far, s.nq_tri_near = len(tfw), len(tnw), len(sfw), len(snw)
        s.tet_far_p, s.tet_far_w = _dptr(tfp), _dptr(tfw)
        s.tet_near_p, s.tet_near_w = _dptr(tnp), _dptr(tnw)
        s.tri_far_p, s.tri_far_w = _dptr(sfp), _dptr(sfw)
        s.tri_near_p, s.tri_near_w = _dptr(snp), _dptr(snw)
        self._s = s

    @property
    def ref(self):
        return C.byref(self._s)

    @property
    def emitting(self) -> np.ndarray:
        """Natural ids of the surface unknowns (corners of emitting face squares), ascending."""
        mask = np.zeros(self.grid.N, dtype=np.uint8)
        lib().og_emitting_mask(self.ref, mask)
        return np.nonzero(mask)[0].astype(np.int64)

    # -- entries ---------------------------------------------------------
    def volume_block(self, rows, cols) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty((len(rows), len(cols)))
        lib().og_volume_block(self.ref, len(rows), rows, len(cols), cols, out)
        return out

    def surface_block(self, rows, cols) -> np.ndarray:
        """Rows: target vertex ids; cols: emitting vertex ids (natural ids)."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty((len(rows), len(cols)))
        lib().og_surface_block(self.ref, len(rows), rows, len(cols), cols, out)
        return out

    def volume_pairs(self, rows, cols) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(len(rows))
        lib().og_volume_pairs(self.ref, len(rows), rows, cols, out)
        return out

    def surface_pairs(self, rows, cols) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(len(rows))
        lib().og_surface_pairs(self.ref, len(rows), rows, cols, out)
        return out

    def dense_G(self) -> np.ndarray:
        ids = np.arange(self.grid.N, dtype=np.int64)
        return self.volume_block(ids, ids)

    def dense_S(self) -> np.ndarray:
        return self.surface_block(np.arange(self.grid.N, dtype=np.int64), self.emitting)

    # -- geometry helpers ----------------------------------------------------
    def kappa_at(self, x) -> np.ndarray:
        x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
        out = np.empty(len(x))
        lib().og_kappa_points(self.ref, len(x), x, out)
        return out

    def tau(self, p, q, mirrored: bool = False, wall: int = None) -> np.ndarray:
        """Optical depth of the segments p -> q, or of the paths reflected by wall
        `wall` (mirrored=True: the first wall)."""
        p = np.ascontiguousarray(np.atleast_2d(p), dtype=np.float64)
        q = np.ascontiguousarray(np.atleast_2d(q), dtype=np.float64)
        out = np.empty(len(p))
        w = wall if wall is not None else (0 if mirrored else -1)
        assert w < len(self.walls)
        lib().og_tau_segments(self.ref, len(p), p, q, int(w), out)
        return out
