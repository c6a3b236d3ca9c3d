"""ctypes binding of librte.so (include/rte.h), argument marshalling only.

Functions keep the C names.  Device arrays are torch tensors on the current
HIP device (float64 / int64, contiguous); the current torch stream is passed
as the HIP stream.  Every computation runs in the library's HIP kernels; if
the library is not built, `load()` raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librte.so")

RTE_OK, RTE_E_INVALID_ARG, RTE_E_OUT_OF_MEMORY, RTE_E_BUDGET, RTE_E_DEVICE, RTE_E_NOT_CONVERGED, RTE_E_INTERNAL = range(7)
RTE_FP64, RTE_FP32, RTE_MIXED_BF16 = 0, 1, 2
RTE_VOLUME, RTE_SURFACE = 0, 1
PRECISIONS = {"fp64": RTE_FP64, "fp32": RTE_FP32, "mixed": RTE_MIXED_BF16}


class RteError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("reflect_axis", C.c_int32), ("reflect_side", C.c_int32), ("R", C.c_double),
                ("emit_faces", C.c_uint32), ("reflect_faces", C.c_uint32), ("R_faces", C.c_double * 6),
                ("hole_lo", C.c_int32 * 3), ("hole_hi", C.c_int32 * 3), ("hole_emit", C.c_uint32),
                ("emission", C.c_uint32)]


class HmatOpts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dense", C.c_int32), ("leaf_size", C.c_int32),
                ("eta", C.c_double), ("aca_eps", C.c_double), ("precision", C.c_int32), ("recompress", C.c_int32),
                ("aca_hits", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("n_tgt", C.c_int64), ("n_src", C.c_int64), ("n_dense", C.c_int64),
                ("n_lowrank", C.c_int64), ("dense_entries", C.c_int64), ("lowrank_sum_mn", C.c_int64),
                ("n_tgt_leaves", C.c_int64)]


class HmatStats(C.Structure):
    _fields_ = [("n_tgt", C.c_int64), ("n_src", C.c_int64), ("n_bands", C.c_int32), ("precision", C.c_int32),
                ("n_dense", C.c_int64), ("n_lowrank", C.c_int64), ("n_fallback_dense", C.c_int64),
                ("dense_entries", C.c_int64), ("lowrank_entries", C.c_int64), ("max_rank", C.c_int32),
                ("mean_rank", C.c_double), ("compression", C.c_double), ("bytes", C.c_int64),
                ("entries_evaluated", C.c_int64), ("assemble_ms", C.c_double),
                ("aca_kernel_ms", C.c_double), ("aca_launches", C.c_int32),
                ("aca_entry_ms", C.c_double), ("aca_entry_launches", C.c_int32),
                ("fill_kernel_ms", C.c_double), ("fill_launches", C.c_int32), ("aca_entries", C.c_int64),
                ("aca_retried", C.c_int64), ("alloc_ms", C.c_double), ("free_bytes", C.c_int64),
                ("lowrank_entries_aca", C.c_int64), ("recompressed_blocks", C.c_int64), ("recompress_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveDesc(C.Structure):
    _fields_ = [("n_bands", C.c_int32), ("nu", C.POINTER(C.c_double)), ("w", C.POINTER(C.c_double)),
                ("a", C.POINTER(C.c_double)), ("grey", C.c_int32), ("nrhs", C.c_int32),
                ("T_wall", C.c_void_p), ("T0", C.c_void_p), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("launch", C.c_int32), ("time_matvecs", C.c_int32),
                ("residuals", C.POINTER(C.c_double))]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("outer_steps", C.c_int32), ("residual", C.c_double),
                ("monotone_violations", C.c_int64), ("ms_total", C.c_double), ("ms_matvec", C.c_double),
                ("graphs", C.c_int32), ("ms_matvec_low", C.c_double), ("matvecs_low", C.c_int32),
                ("ms_matvec_acc", C.c_double), ("matvecs_acc", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MatvecConfig(C.Structure):
    _fields_ = [("phase_b_waves", C.c_int32), ("phase_a_kib", C.c_int32), ("phase_a_tiles", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerDesc(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("n_catalogue", C.c_int32), ("nu", C.POINTER(C.c_double)),
                ("levels_per_decade", C.c_int32), ("leaf_size", C.c_int32), ("eta", C.c_double),
                ("aca_eps", C.c_double), ("precision", C.c_int32), ("max_active", C.c_int32),
                ("recompress", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("mesh_id", C.c_int32), ("n_bands", C.c_int32), ("bands", C.POINTER(C.c_int32)),
                ("kappa_mult", C.POINTER(C.c_double)), ("a", C.POINTER(C.c_double)), ("T_wall", C.c_void_p),
                ("tol", C.c_double), ("max_iter", C.c_int32)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("converged", C.c_int32), ("iterations", C.c_int32),
                ("outer_steps", C.c_int32), ("residual", C.c_double), ("n_bands", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("budget", C.c_int64), ("resident_bytes", C.c_int64), ("operators", C.c_int64),
                ("assembled", C.c_int64), ("evicted", C.c_int64), ("over_budget", C.c_int64),
                ("submitted", C.c_int64), ("completed", C.c_int64), ("steps", C.c_int64), ("columns", C.c_int64),
                ("assemble_ms", C.c_double), ("sweep_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); the declarations of include/rte.h
SIGNATURES = {
    "rte_mesh_create": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(C.c_void_p)]),
    "rte_mesh_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "rte_mesh_emitting_ids": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rte_mesh_destroy": (None, [C.c_void_p]),
    "rte_plan_create": (C.c_int, [C.c_void_p, C.POINTER(HmatOpts), C.POINTER(C.c_void_p)]),
    "rte_plan_info": (C.c_int, [C.c_void_p, C.POINTER(PlanInfo)]),
    "rte_plan_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rte_plan_destroy": (None, [C.c_void_p]),
    "rte_entries": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_int32, C.c_void_p]),
    "rte_hmat_assemble": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(HmatOpts), C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "rte_hmat_matvec": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rte_hmat_matvec_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rte_hmat_matvec_batched": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "rte_hmat_stats": (C.c_int, [C.c_void_p, C.POINTER(HmatStats)]),
    "rte_kappa_levels": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_int32)]),
    "rte_hmat_select_bands": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "rte_hmat_get_config": (C.c_int, [C.c_void_p, C.POINTER(MatvecConfig)]),
    "rte_hmat_set_config": (C.c_int, [C.c_void_p, C.POINTER(MatvecConfig), C.c_void_p]),
    "rte_hmat_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(MatvecConfig),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "rte_hmat_time_matvec": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                       C.POINTER(C.c_double)]),
    "rte_server_create": (C.c_int, [C.POINTER(ServerDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "rte_server_add_mesh": (C.c_int, [C.c_void_p, C.POINTER(MeshDesc), C.c_void_p, C.POINTER(C.c_int32)]),
    "rte_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_int64)]),
    "rte_server_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "rte_server_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(RequestInfo)]),
    "rte_server_levels": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]),
    "rte_server_fetch": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    "rte_server_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "rte_server_destroy": (None, [C.c_void_p]),
    "rte_hmat_block_factors": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "rte_hmat_block_factors_op": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_int32),
                                            C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "rte_hmat_dense_block": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_int64),
                                       C.c_void_p, C.c_void_p]),
    "rte_hmat_destroy": (None, [C.c_void_p]),
    "rte_fixed_point_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SolveDesc),
                                        C.c_void_p, C.c_void_p, C.POINTER(SolveStats), C.c_void_p]),
    "rte_status_string": (C.c_char_p, [C.c_int]),
    "rte_last_error": (C.c_char_p, []),
    "rte_version": (C.c_char_p, []),
}

_lib = None


def load():
    """Load librte.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_05789_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(status: int, allow=(RTE_OK,)):
    if status not in allow:
        msg = load().rte_last_error().decode()
        raise RteError(status, msg)
    return status


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _darr(values):
    if values is None:
        return None
    arr = (C.c_double * len(values))(*[float(v) for v in values])
    return arr


# ---------------------------------------------------------------- mesh
class Mesh:
    def __init__(self, handle, N, L):
        self.handle, self.N, self.L = handle, N, L

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rte_mesh_destroy(self.handle)
            self.handle = None


def mesh_desc(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), reflect_axis=-1, reflect_side=0, R=0.0,
              emit_faces=1, walls=None, hole=None, hole_emit=0, emission=0) -> MeshDesc:
    """walls: further reflective faces as (axis, side, R) triples.  hole: the removed
    box of cells ((i0, j0, k0), (i1, j1, k1)), cells [i0, i1) x [j0, j1) x [k0, k1);
    hole_emit: its emitting faces (bit 2a + side).  emission: 0 for the isotropic
    wall source, 1 for the cosine-weighted one."""
    d = MeshDesc()
    d.n[:] = [int(v) for v in n]
    d.lo[:] = [float(v) for v in lo]
    d.hi[:] = [float(v) for v in hi]
    d.reflect_axis, d.reflect_side, d.R, d.emit_faces = int(reflect_axis), int(reflect_side), float(R), int(emit_faces)
    d.reflect_faces = 0
    for axis, side, r in (walls or []):
        f = 2 * int(axis) + int(side)
        d.reflect_faces |= 1 << f
        d.R_faces[f] = float(r)
    if hole is not None:
        d.hole_lo[:] = [int(v) for v in hole[0]]
        d.hole_hi[:] = [int(v) for v in hole[1]]
    d.hole_emit = int(hole_emit)
    d.emission = int(emission)
    return d


def rte_mesh_create(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), reflect_axis=-1, reflect_side=0, R=0.0,
                    emit_faces=1, walls=None, hole=None, hole_emit=0, emission=0) -> Mesh:
    d = mesh_desc(n, lo, hi, reflect_axis, reflect_side, R, emit_faces, walls, hole, hole_emit, emission)
    h = C.c_void_p()
    _check(load().rte_mesh_create(C.byref(d), C.byref(h)))
    N, L = C.c_int64(), C.c_int64()
    _check(_lib.rte_mesh_sizes(h, C.byref(N), C.byref(L)))
    return Mesh(h, N.value, L.value)


def rte_mesh_emitting_ids(mesh: Mesh):
    import numpy as np
    out = np.empty(mesh.L, dtype=np.int64)
    _check(load().rte_mesh_emitting_ids(mesh.handle, out.ctypes.data_as(C.c_void_p)))
    return out


def hmat_opts(kind=RTE_VOLUME, dense=False, leaf_size=64, eta=2.0, aca_eps=1e-5, precision=RTE_FP64,
              recompress=False, aca_hits=1) -> HmatOpts:
    o = HmatOpts()
    o.kind, o.dense, o.leaf_size = int(kind), int(bool(dense)), int(leaf_size)
    o.eta, o.aca_eps = float(eta), float(aca_eps)
    o.recompress = int(bool(recompress))
    o.aca_hits = int(aca_hits)
    o.precision = PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision)
    return o


# ---------------------------------------------------------------- plan (host only)
def rte_plan_create(mesh: Mesh, opts: HmatOpts):
    h = C.c_void_p()
    _check(load().rte_plan_create(mesh.handle, C.byref(opts), C.byref(h)))
    return h


def rte_plan_info(plan) -> PlanInfo:
    info = PlanInfo()
    _check(load().rte_plan_info(plan, C.byref(info)))
    return info


def rte_plan_export(plan):
    import numpy as np
    info = rte_plan_info(plan)
    tp = np.empty(info.n_tgt, dtype=np.int64)
    sp = np.empty(info.n_src, dtype=np.int64)
    bl = np.empty((info.n_dense + info.n_lowrank, 5), dtype=np.int64)
    _check(_lib.rte_plan_export(plan, tp.ctypes.data_as(C.c_void_p), sp.ctypes.data_as(C.c_void_p),
                                bl.ctypes.data_as(C.c_void_p)))
    return tp, sp, bl


def rte_plan_destroy(plan):
    load().rte_plan_destroy(plan)


# ---------------------------------------------------------------- device calls
def rte_entries(mesh: Mesh, kind, kappa, rows, cols, out, precision=RTE_FP64, stream=None):
    _check(load().rte_entries(mesh.handle, int(kind), _ptr(kappa), int(rows.numel()), _ptr(rows), _ptr(cols),
                              _ptr(out), int(precision), _stream(stream)))
    return out


class HMat:
    def __init__(self, handle, mesh, parent=None):
        self.handle, self.mesh = handle, mesh   # keep the mesh alive
        self.parent = parent                    # a band view keeps its operator alive

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rte_hmat_destroy(self.handle)
            self.handle = None


def rte_hmat_assemble(mesh: Mesh, kappa, opts: HmatOpts, stream=None) -> HMat:
    """kappa: float64 device tensor [n_bands, N] (or [N])."""
    n_bands = 1 if kappa.dim() == 1 else int(kappa.shape[0])
    h = C.c_void_p()
    _check(load().rte_hmat_assemble(mesh.handle, n_bands, _ptr(kappa), C.byref(opts), _stream(stream), C.byref(h)))
    return HMat(h, mesh)


def rte_kappa_levels(values, tol: float, max_levels: int = 64):
    """Adaptive kappa levels of positive multipliers: (levels ascending, map[b] = level of value b)."""
    import numpy as np
    v = np.ascontiguousarray(values, dtype=np.float64)
    levels = np.empty(max_levels, dtype=np.float64)
    mp = np.empty(len(v), dtype=np.int32)
    nl = C.c_int32()
    _check(load().rte_kappa_levels(v.ctypes.data_as(C.c_void_p), len(v), float(tol), int(max_levels),
                                   levels.ctypes.data_as(C.c_void_p), mp.ctypes.data_as(C.c_void_p), C.byref(nl)))
    return levels[:nl.value].copy(), mp


def rte_hmat_select_bands(hmat: HMat, band_op, stream=None) -> HMat:
    """View whose band b is band band_op[b] of hmat (which the view keeps alive)."""
    import numpy as np
    bo = np.ascontiguousarray(band_op, dtype=np.int32)
    h = C.c_void_p()
    _check(load().rte_hmat_select_bands(hmat.handle, len(bo), bo.ctypes.data_as(C.c_void_p), _stream(stream),
                                        C.byref(h)))
    return HMat(h, hmat.mesh, parent=hmat)


def rte_hmat_matvec(hmat: HMat, band, x, y, stream=None):
    nrhs = 1 if x.dim() == 1 else int(x.shape[0])
    _check(load().rte_hmat_matvec(hmat.handle, int(band), nrhs, _ptr(x), _ptr(y), _stream(stream)))
    return y


def rte_hmat_matvec_noalloc(hmat: HMat, band, x, y, stream=None):
    """Same as rte_hmat_matvec, with the library's fixed device workspace (no allocation)."""
    nrhs = 1 if x.dim() == 1 else int(x.shape[0])
    _check(load().rte_hmat_matvec_noalloc(hmat.handle, int(band), nrhs, _ptr(x), _ptr(y), _stream(stream)))
    return y


RTE_OP_ACCURATE, RTE_OP_LOW = 0, 1
RTE_LAUNCH_STREAM, RTE_LAUNCH_GRAPH = 0, 1
RTE_REQ_PENDING, RTE_REQ_ACTIVE, RTE_REQ_DONE = 0, 1, 2


def rte_hmat_matvec_batched(hmat: HMat, x, y, op=RTE_OP_ACCURATE, stream=None):
    """x: float64 device [n_bands, nrhs, N_src]; y: [n_bands, nrhs, N_tgt]."""
    nrhs = int(x.shape[1])
    _check(load().rte_hmat_matvec_batched(hmat.handle, nrhs, _ptr(x), _ptr(y), int(op), _stream(stream)))
    return y


def rte_hmat_get_config(hmat: HMat) -> dict:
    c = MatvecConfig()
    _check(load().rte_hmat_get_config(hmat.handle, C.byref(c)))
    return c.as_dict()


def rte_hmat_set_config(hmat: HMat, cfg: dict, stream=None):
    c = MatvecConfig(int(cfg["phase_b_waves"]), int(cfg["phase_a_kib"]), int(cfg["phase_a_tiles"]))
    _check(load().rte_hmat_set_config(hmat.handle, C.byref(c), _stream(stream)))


def rte_hmat_autotune(hmat: HMat, nrhs=1, op=RTE_OP_ACCURATE, reps=3, stream=None) -> dict:
    c, ms, n = MatvecConfig(), C.c_double(), C.c_int32()
    _check(load().rte_hmat_autotune(hmat.handle, int(nrhs), int(op), int(reps), _stream(stream), C.byref(c),
                                    C.byref(ms), C.byref(n)))
    return {"config": c.as_dict(), "ms": ms.value, "trials": n.value}


def rte_hmat_time_matvec(hmat: HMat, nrhs=1, op=RTE_OP_ACCURATE, reps=3, stream=None) -> float:
    ms = C.c_double()
    _check(load().rte_hmat_time_matvec(hmat.handle, int(nrhs), int(op), int(reps), _stream(stream), C.byref(ms)))
    return ms.value


def rte_hmat_stats(hmat: HMat) -> dict:
    st = HmatStats()
    _check(load().rte_hmat_stats(hmat.handle, C.byref(st)))
    return st.as_dict()


def rte_hmat_block_factors(hmat: HMat, band: int, block: int, factors: bool = True):
    """(rank, U [m,rank], V [n,rank]) of an admissible block; U, V are None when
    factors is False or the block is stored dense (rank -1)."""
    import numpy as np
    k, m, n = C.c_int32(), C.c_int64(), C.c_int64()
    _check(load().rte_hmat_block_factors(hmat.handle, int(band), int(block), C.byref(k), C.byref(m), C.byref(n),
                                         None, None))
    if not factors or k.value <= 0:
        return k.value, None, None
    U = np.empty((m.value, k.value))
    V = np.empty((n.value, k.value))
    _check(_lib.rte_hmat_block_factors(hmat.handle, int(band), int(block), C.byref(k), C.byref(m), C.byref(n),
                                       U.ctypes.data_as(C.c_void_p), V.ctypes.data_as(C.c_void_p)))
    return k.value, U, V


def rte_hmat_block_factors_op(hmat: HMat, band: int, block: int, op: int):
    """(rank, U, V) of an admissible block for one operator (RTE_OP_LOW: the BF16 hi
    parts of mixed-precision storage); U, V are None when the block is stored dense."""
    import numpy as np
    k, m, n = C.c_int32(), C.c_int64(), C.c_int64()
    _check(load().rte_hmat_block_factors_op(hmat.handle, int(band), int(block), int(op), C.byref(k), C.byref(m),
                                            C.byref(n), None, None))
    if k.value <= 0:
        return k.value, None, None
    U = np.empty((m.value, k.value))
    V = np.empty((n.value, k.value))
    _check(_lib.rte_hmat_block_factors_op(hmat.handle, int(band), int(block), int(op), C.byref(k), C.byref(m),
                                          C.byref(n), U.ctypes.data_as(C.c_void_p), V.ctypes.data_as(C.c_void_p)))
    return k.value, U, V


def rte_hmat_dense_count(hmat: HMat, band: int) -> int:
    cnt = C.c_int64()
    _check(load().rte_hmat_dense_block(hmat.handle, int(band), 0, RTE_OP_ACCURATE, C.byref(cnt), None, None))
    return cnt.value


def rte_hmat_dense_block(hmat: HMat, band: int, index: int, op: int = 0):
    """((t0, t1, s0, s1), A) of dense block `index` of a band, A as stored (FP64)."""
    import numpy as np
    cnt = C.c_int64()
    rng = np.empty(4, dtype=np.int64)
    _check(load().rte_hmat_dense_block(hmat.handle, int(band), int(index), int(op), C.byref(cnt),
                                       rng.ctypes.data_as(C.c_void_p), None))
    t0, t1, s0, s1 = (int(v) for v in rng)
    A = np.empty((t1 - t0, s1 - s0))
    _check(_lib.rte_hmat_dense_block(hmat.handle, int(band), int(index), int(op), C.byref(cnt),
                                     rng.ctypes.data_as(C.c_void_p), A.ctypes.data_as(C.c_void_p)))
    return (t0, t1, s0, s1), A


def rte_fixed_point_solve(mesh: Mesh, vol: HMat, surf: HMat, T_wall, T_out, J_out=None, *, grey=True,
                          nu=None, w=None, a=None, T0=None, tol=1e-10, max_iter=1000, precision=RTE_FP64,
                          launch=None, stream=None, allow_not_converged=False, time_matvecs=False,
                          history=False) -> dict:
    """T_wall: float64 device [nrhs, L]; T_out: [nrhs, N]; J_out: [nrhs, n_bands, N] or None.
    history: also return the residual of every sweep (numpy array, key "residuals")."""
    nrhs = 1 if T_wall.dim() == 1 else int(T_wall.shape[0])
    nb = 1 if grey else len(nu)
    d = SolveDesc()
    keep = [_darr(nu), _darr(w), _darr(a)]
    d.n_bands = nb
    d.nu, d.w, d.a = [C.cast(k, C.POINTER(C.c_double)) if k is not None else None for k in keep]
    d.grey, d.nrhs = int(bool(grey)), nrhs
    d.T_wall = T_wall.data_ptr()
    d.T0 = T0.data_ptr() if T0 is not None else None
    d.tol, d.max_iter, d.precision = float(tol), int(max_iter), int(precision)
    d.launch = RTE_LAUNCH_GRAPH if launch is None else int(launch)
    d.time_matvecs = int(bool(time_matvecs))
    import numpy as np
    hist = np.zeros(max(int(max_iter), 1)) if history else None
    d.residuals = hist.ctypes.data_as(C.POINTER(C.c_double)) if history else None
    st = SolveStats()
    allow = (RTE_OK, RTE_E_NOT_CONVERGED) if allow_not_converged else (RTE_OK,)
    status = _check(load().rte_fixed_point_solve(mesh.handle, vol.handle, surf.handle, C.byref(d), _ptr(T_out),
                                                 _ptr(J_out), C.byref(st), _stream(stream)), allow)
    out = st.as_dict()
    out["converged"] = status == RTE_OK
    if history:
        out["residuals"] = hist[:out["iterations"]].copy()
    return out


def rte_version() -> str:
    return load().rte_version().decode()
