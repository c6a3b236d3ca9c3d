"""Autotuning of the H-matvec launch shape and of the leaf size.

The library times the candidate launch shapes on the assembled matrix itself
(rte_hmat_autotune: wavefronts per phase-B workgroup, phase-A task size, ranks
per phase-A task) with HIP events and keeps the fastest.  This module keeps
the winners in a JSON cache keyed by what decides them (device, precision,
sizes, bands, right-hand sides, operator), so a later run on the same problem
shape sets the shape without timing, and searches the leaf size, which
changes the H-matrix itself, by assembling candidates."""
from __future__ import annotations

import json
import os
import time

from . import rte


def _key(hmat, nrhs, op) -> str:
    import torch
    st = rte.rte_hmat_stats(hmat)
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return "|".join(str(v) for v in (dev, st["precision"], st["n_tgt"], st["n_src"], st["n_bands"],
                                      st["n_lowrank"], st["n_dense"], nrhs, op))


def autotune(hmat, nrhs=1, op=rte.RTE_OP_ACCURATE, reps=3, cache: str | None = None) -> dict:
    """Sets the fastest launch shape on `hmat`; returns it with its time and where it came from."""
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    k = _key(hmat, nrhs, op)
    if k in table:
        rte.rte_hmat_set_config(hmat, table[k]["config"])
        return dict(table[k], source="cache")
    r = rte.rte_hmat_autotune(hmat, nrhs, op, reps)
    if cache:
        table[k] = r
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(r, source="timed")


def tune_leaf_size(mesh, kappa, opts: dict, candidates=(32, 48, 64, 96), nrhs=1, op=rte.RTE_OP_ACCURATE,
                   sweeps=20, reps=3):
    """Assembles the volume matrix at each candidate leaf size, autotunes its matvec,
    and scores assembly time + `sweeps` matvecs (the cost of one solve).  Returns
    (best leaf size, per-candidate records)."""
    import torch
    rec = []
    for leaf in candidates:
        o = dict(opts, leaf_size=leaf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = rte.rte_hmat_assemble(mesh, kappa, rte.hmat_opts(**o))
        torch.cuda.synchronize()
        t_asm = (time.perf_counter() - t0) * 1e3
        r = rte.rte_hmat_autotune(H, nrhs, op, reps)
        st = rte.rte_hmat_stats(H)
        rec.append({"leaf_size": leaf, "assemble_ms": t_asm, "matvec_ms": r["ms"], "config": r["config"],
                    "bytes": st["bytes"], "score_ms": t_asm + sweeps * r["ms"]})
        del H
    best = min(rec, key=lambda x: x["score_ms"])
    return best["leaf_size"], rec
