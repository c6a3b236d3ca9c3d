"""Request serving on top of the library's server (rte_server_*): resident
meshes, a band catalogue, requests admitted by an HBM budget and iterated in
continuous batches, and a driver that replays an arrival schedule and
measures latency.  Every solve runs in the library; this module marshals
arguments and keeps the clock."""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import rte


class Server:
    def __init__(self, nu, *, budget=0, levels_per_decade=8, leaf_size=64, eta=2.0, aca_eps=1e-5,
                 precision=rte.RTE_MIXED_BF16, max_active=64, recompress=False, stream=None):
        self._nu = np.ascontiguousarray(nu, dtype=np.float64)
        d = rte.ServerDesc()
        d.hbm_budget, d.n_catalogue = int(budget), len(self._nu)
        d.nu = self._nu.ctypes.data_as(C.POINTER(C.c_double))
        d.levels_per_decade, d.leaf_size, d.eta, d.aca_eps = int(levels_per_decade), int(leaf_size), eta, aca_eps
        d.precision, d.max_active, d.recompress = int(precision), int(max_active), int(recompress)
        h = C.c_void_p()
        rte._check(rte.load().rte_server_create(C.byref(d), rte._stream(stream), C.byref(h)))
        self.handle = h
        self.levels_per_decade = levels_per_decade
        self._sizes = []

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "handle", None) and rte is not None and getattr(rte, "_lib", None) is not None:
            rte._lib.rte_server_destroy(self.handle)
            self.handle = None

    def add_mesh(self, n, kappa, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), emit_faces=63, emission=0) -> int:
        """kappa: float64 device [N] base field, natural order.  emission: 0 for the
        isotropic wall source, 1 for the cosine-weighted one."""
        md = rte.mesh_desc(n, lo, hi, emit_faces=emit_faces, emission=emission)
        mid = C.c_int32()
        rte._check(rte.load().rte_server_add_mesh(self.handle, C.byref(md), rte._ptr(kappa), C.byref(mid)))
        return mid.value

    def submit(self, mesh_id, bands, kappa_mult, T_wall, tol=1e-6, max_iter=2000, a=None) -> int:
        """a: scattering coefficient per band (None: no scattering)."""
        b = np.ascontiguousarray(bands, dtype=np.int32)
        m = np.ascontiguousarray(kappa_mult, dtype=np.float64)
        sc = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        q = rte.Request()
        q.mesh_id, q.n_bands = int(mesh_id), len(b)
        q.bands = b.ctypes.data_as(C.POINTER(C.c_int32))
        q.kappa_mult = m.ctypes.data_as(C.POINTER(C.c_double))
        q.a = sc.ctypes.data_as(C.POINTER(C.c_double)) if sc is not None else None
        q.T_wall = T_wall.data_ptr()
        q.tol, q.max_iter = float(tol), int(max_iter)
        rid = C.c_int64()
        rte._check(rte.load().rte_server_submit(self.handle, C.byref(q), C.byref(rid)))
        return rid.value

    def step(self):
        a, p = C.c_int32(), C.c_int32()
        rte._check(rte.load().rte_server_step(self.handle, C.byref(a), C.byref(p)))
        return a.value, p.value

    def poll(self, rid) -> dict:
        info = rte.RequestInfo()
        rte._check(rte.load().rte_server_poll(self.handle, int(rid), C.byref(info)))
        return info.as_dict()

    def levels(self, rid, n_bands) -> np.ndarray:
        out = np.zeros(n_bands, dtype=np.int32)
        rte._check(rte.load().rte_server_levels(self.handle, int(rid), out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def fetch(self, rid, T_out):
        rte._check(rte.load().rte_server_fetch(self.handle, int(rid), rte._ptr(T_out)))
        return T_out

    def stats(self) -> dict:
        st = rte.ServerStats()
        rte._check(rte.load().rte_server_stats(self.handle, C.byref(st)))
        return st.as_dict()


def run_stream(server, requests, mesh_ids, mesh_sizes, c_band, *, tol=1e-6, keep=None, device="cuda:0",
               log=None):
    """Replays `requests` (inputs.Request, arrival times in seconds from the start)
    against `server`: each is submitted when its arrival time has passed, the
    server steps while work remains, finished requests are fetched at once.
    Latency = completion - arrival.  `keep`: request indices whose temperatures
    are returned (natural order, host)."""
    import torch
    order = sorted(range(len(requests)), key=lambda k: requests[k].arrival)
    t0 = time.perf_counter()
    nxt = 0
    live = {}          # request id -> request index
    lat = np.full(len(requests), np.nan)
    info = [None] * len(requests)
    kept = {}
    while nxt < len(order) or live:
        now = time.perf_counter() - t0
        while nxt < len(order) and requests[order[nxt]].arrival <= now:
            k = order[nxt]
            q = requests[k]
            tw = torch.tensor(q.T_wall, device=device)
            rid = server.submit(mesh_ids[q.mesh], q.bands, q.scale * c_band[q.bands], tw, tol=tol)
            live[rid] = k
            nxt += 1
        if not live:
            time.sleep(max(0.0, requests[order[nxt]].arrival - (time.perf_counter() - t0)))
            continue
        server.step()
        now = time.perf_counter() - t0
        for rid in list(live):
            st = server.poll(rid)
            if st["state"] == rte.RTE_REQ_DONE:
                k = live.pop(rid)
                lat[k] = now - requests[k].arrival
                st["levels"] = server.levels(rid, st["n_bands"]).tolist()
                info[k] = st
                out = torch.empty(mesh_sizes[requests[k].mesh], device=device, dtype=torch.float64)
                server.fetch(rid, out)
                if keep is not None and k in keep:
                    kept[k] = out.cpu().numpy()
                if log:
                    log(k, st, lat[k])
    wall = time.perf_counter() - t0
    return {"latency_s": lat, "wall_s": wall, "info": info, "kept": kept,
            "solves_per_s": len(requests) / wall,
            "p50_ms": float(np.nanpercentile(lat, 50) * 1e3), "p99_ms": float(np.nanpercentile(lat, 99) * 1e3)}
