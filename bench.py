#!/usr/bin/env python
"""Benchmark of the integral-form radiative transfer hot path on one MI355X.

Headline (the default): the batched mixed-precision workload.  Unit cube on a
49^3 grid (117,649 vertices), 32 frequency bands with kappa_b = c_b kappa(x)
(c_b lognormal(0, 1), seed 4), all six faces emitting with 16 right-hand
sides of random wall temperatures in [0.5, 2] (seed 5); leaf 64, eta 2, ACA
1e-5; FP32 entries and ACA, BF16 hi + lo factors; every solve runs BF16 sweeps
over all 32 bands and 16 right-hand sides (one launch per phase, replayed from
captured hipGraphs) with FP64 defect correction, to an FP64 relative residual
of 1e-6.  The operators (G and S of every band) are assembled once before the
timed region and stay resident; the assembly is timed and reported under its
own key.  One step = one 16-RHS fixed-point solve; `value` is right-hand-side
solves per second.

The `roofline` object covers the kernel group with the largest share of a
step, the low-operator H-matvec of the inner sweeps, event-timed by the
library inside the timed solves: algorithmic bytes (stored BF16 hi entries,
no padding, plus x read and y written in FP64) per launch / mean launch time.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload.  Extra keys: the plain FP64 GPU method against the mixed one on 4 of
the 32 bands (one GPU's share of an 8-GPU band split), the 41^3 FP64
H-matrix solve with assembly (per-step latency), and the 11^3 dense case with
the oracle timed in full.

Other workloads (`--workload`), one JSON line each:
  cube41      the 41^3 grey FP64 H-matrix solve, assembly + solve per step
  reflective  box [0,2]x[0,1]^2 on 65x33x33, mirror wall z = 0 (R = 0.5), 8 bands,
              mixed precision against plain FP64
  batched     the headline workload with an autotuned launch shape; `--bands B` takes
              every (32/B)-th band, `--compare` adds plain FP64 on the same bands
  served      256 Poisson(20/s) requests over resident 21^3/29^3/41^3/49^3 meshes
              through the request server (mixed, continuous batching) and, with
              `--compare R`, the first R of them through plain FP64 one at a time
  matvec      the headline operator's matvecs alone after a 1 GiB calibration copy
              (for the HBM traffic counters)
  academic    Test-3 of the paper's academic test (box minus an inner cube, three
              reflective planes), `--h` cm spacing: assembly + grey solve, FP64 and
              mixed, beside the paper's CPU time on its nearest mesh
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the ACA entry launches (k_aca_rows / k_aca_cols, volume,
# FP64), from rocprofv3 FETCH_SIZE and WRITE_SIZE passes over this benchmark's step,
# calibrated on a plain 1 GiB copy (FETCH_SIZE reads half the bytes, WRITE_SIZE all):
# the summary is profiles/cube41_grey_fp64_hmatrix_hbm_traffic.md.  Set to None
# whenever those kernels change.
ACA_ENTRY_TRAFFIC_BYTES = 434.5e6
FP64_PEAK_TFLOPS = 78.6
# Algorithmic FP64 operations of one kernel entry, counted from the code of the
# march and the quadrature with an FMA as 2 and a reciprocal, square root or
# exponential as 1 (compares, min/max and index arithmetic not counted):
#   per ray-march piece: crossing update 1.5 (one family advances; an axis
#     family also moves the cell), midpoint 2, sample position 6, P1 value 9,
#     accumulation 3;
#   per far-field tetrahedron (4 points of the degree-2 rule): squared
#     distances 28, kappa weights 28, common denominator 8, refined reciprocal
#     and accumulation 15;
#   per near-field cell (degree-5 rule, tabulated): 8 products, 16;
#   per entry: segment set-up 45, optical depth and exponential 2, far-field
#     distance 8, scaling 2.
# The ACA's residual update (2 k per entry at rank step k) is not counted.
F_PIECE, F_FAR_TET, F_NEAR_CELL, F_ENTRY = 21.5, 79, 16, 57


def _phi(q: int) -> int:
    r, n, p = q, q, 2
    while p * p <= n:
        if n % p == 0:
            while n % p == 0:
                n //= p
            r -= r // p
        p += 1
    if n > 1:
        r -= r // n
    return r


def _divisors(a: int):
    out = set()
    d = 1
    while d * d <= a:
        if a % d == 0:
            out.add(d)
            out.add(a // d)
        d += 1
    return out


def pieces_between(d) -> int:
    """Pieces of the segment between two grid vertices with index difference d: one
    plus the number of distinct crossing parameters m/a_f of the six plane families."""
    d0, d1, d2 = (int(v) for v in d)
    qs = set()
    for a in (abs(d0), abs(d1), abs(d2), abs(d0 - d1), abs(d1 - d2), abs(d0 - d2)):
        if a > 1:
            qs |= _divisors(a)
    qs.discard(1)
    return 1 + sum(_phi(q) for q in qs)


def valid_cells_tets(idx, n):
    """Cells of the grid around vertex idx, and the Kuhn tetrahedra of those cells
    that have idx as a vertex."""
    cells = tets = 0
    for bits in range(8):
        o = [(bits >> a) & 1 for a in range(3)]
        if all((idx[a] >= 1) if o[a] else (idx[a] <= n[a] - 2) for a in range(3)):
            cells += 1
            # tets of cell j-o containing j: corner (0,0,0) or (1,1,1) -> 6, else 2
            tets += 6 if sum(o) in (0, 3) else 2
    return cells, tets


def entry_flops_sample(n, pairs, near_cheb=2):
    """Mean algorithmic FLOPs of a volume entry over sampled (i_idx, j_idx) pairs."""
    tot = 0.0
    for ii, jj in pairs:
        d = [jj[a] - ii[a] for a in range(3)]
        near = max(abs(v) for v in d) <= near_cheb
        cells, tets = valid_cells_tets(jj, n)
        quad = F_NEAR_CELL * cells if near else F_FAR_TET * tets
        tot += F_PIECE * pieces_between(d) + quad + F_ENTRY
    return tot / len(pairs)


def cpu_baseline(wl, budget_s=12.0):
    """The oracle as it is, on sampled rows of G and S; extrapolated to the dense
    assembly of the whole workload (fixed-point iterations not included)."""
    from oracle.core import Grid, Problem
    g = Grid(wl.n)
    P = Problem(g, wl.kappa[0], emit_faces=wl.emit_faces)
    rng = np.random.default_rng(12)
    cols = np.arange(g.N)
    rows = rng.choice(g.N, 8, replace=False)
    t0 = time.perf_counter()
    P.volume_block(rows, cols)
    t_probe = time.perf_counter() - t0
    R = int(min(512, max(8, 8 * budget_s / max(t_probe, 1e-3) * 0.8)))
    rows = rng.choice(g.N, R, replace=False)
    t0 = time.perf_counter()
    P.volume_block(rows, cols)
    tG = time.perf_counter() - t0
    t0 = time.perf_counter()
    P.surface_block(rows, P.emitting)
    tS = time.perf_counter() - t0
    full = (tG + tS) / R * g.N
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / full, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{R} random rows of G (x{g.N}) and S (x{len(P.emitting)}), FP64, "
                      f"{tG + tS:.1f} s; extrapolated to the dense assembly of all {g.N} rows "
                      f"({full:.0f} s), fixed-point iterations excluded"}


def _say(msg):
    print("# " + msg, file=sys.stderr, flush=True)


def _hstats(st, keys=("assemble_ms", "aca_kernel_ms", "aca_entry_ms", "fill_kernel_ms", "bytes", "compression",
                      "mean_rank", "max_rank", "n_lowrank", "n_fallback_dense", "lowrank_entries",
                      "lowrank_entries_aca", "recompress_ms")):
    return {k: st[k] for k in keys}


def _operator_bytes(st, op):
    """Stored bytes one matvec streams: all of them, or the BF16 high parts alone
    (half of the split storage) for the low operator."""
    from paper_2306_05789_amd import rte
    if st["precision"] == rte.RTE_MIXED_BF16 and op == rte.RTE_OP_LOW:
        return st["bytes"] // 2
    return st["bytes"]


def _matvec_entry(G, nrhs, op, reps=3):
    """Event-timed all-band matvec and its HBM rate over algorithmic bytes: the
    operator's stored bytes plus x read and y written in FP64."""
    from paper_2306_05789_amd import rte
    st = rte.rte_hmat_stats(G)
    ms = rte.rte_hmat_time_matvec(G, nrhs, op, reps)
    b = _operator_bytes(st, op) + 8 * st["n_bands"] * nrhs * (st["n_src"] + st["n_tgt"])
    gbs = b / (ms * 1e-3) / 1e9
    return {"nrhs": nrhs, "op": "low" if op == rte.RTE_OP_LOW else "accurate", "ms": ms, "bytes": b,
            "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS}


def _assemble_pair(rte, mesh, kap, optG, optS):
    """G and S assembled concurrently, each by its own host thread on its own
    stream; returns both and the wall time of the pair in ms."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(2) as pool:
        fG = pool.submit(rte.rte_hmat_assemble, mesh, kap, optG, streams[0].cuda_stream)
        fS = pool.submit(rte.rte_hmat_assemble, mesh, kap, optS, streams[1].cuda_stream)
        G, S = fG.result(), fS.result()
    torch.cuda.synchronize()
    return G, S, (time.perf_counter() - t0) * 1e3


def _solve_series(rte, mesh, G, S, Tw, T, nu, precision, tol, steps, warmup):
    for _ in range(warmup):
        rte.rte_fixed_point_solve(mesh, G, S, Tw, T, grey=False, nu=nu, tol=tol, max_iter=3000, precision=precision)
    import torch
    torch.cuda.synchronize()
    lat, st = [], None
    for _ in range(steps):
        t0 = time.perf_counter()
        st = rte.rte_fixed_point_solve(mesh, G, S, Tw, T, grey=False, nu=nu, tol=tol, max_iter=3000,
                                       precision=precision)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        _say(f"solve {lat[-1] * 1e3:.1f} ms, {st['iterations']} sweeps, residual {st['residual']:.2e}")
    return lat, st


def run_reflective(args):
    """Reflective box, 8 bands: mixed precision (FP32 entries and ACA, BF16 factors,
    FP64 defect correction) against plain FP64, both to a 1e-6 residual."""
    import torch
    from paper_2306_05789_amd import inputs, rte
    wl = inputs.reflective_bands()
    dev = torch.device("cuda:0")
    mesh = rte.rte_mesh_create(wl.n, wl.lo, wl.hi, reflect_axis=wl.wall_axis, reflect_side=wl.wall_side, R=wl.R,
                               emit_faces=wl.emit_faces)
    kap = torch.tensor(wl.kappa, device=dev)
    Tw = torch.tensor(wl.T_wall, device=dev)
    res, Ts = {}, {}
    for name in (["mixed", "fp64"] if args.precision == "both" else [args.precision]):
        p = rte.PRECISIONS[name]
        G, S, wall_ms = _assemble_pair(rte, mesh, kap, rte.hmat_opts(kind=rte.RTE_VOLUME, precision=p),
                                       rte.hmat_opts(kind=rte.RTE_SURFACE, precision=p))
        gs, ss = rte.rte_hmat_stats(G), rte.rte_hmat_stats(S)
        _say(f"{name}: G {gs['assemble_ms']:.0f} ms, S {ss['assemble_ms']:.0f} ms, concurrently {wall_ms:.0f} ms")
        T = torch.empty((1, mesh.N), device=dev, dtype=torch.float64)
        lat, st = _solve_series(rte, mesh, G, S, Tw, T, wl.nu, p, 1e-6, args.steps, args.warmup)
        ops = [rte.RTE_OP_LOW, rte.RTE_OP_ACCURATE] if p == rte.RTE_MIXED_BF16 else [rte.RTE_OP_ACCURATE]
        solve_s = float(np.mean(lat))
        res[name] = {"assemble_G": _hstats(gs), "assemble_S": _hstats(ss), "assemble_wall_ms": wall_ms,
                     "solve_ms": solve_s * 1e3, "sweeps": st["iterations"], "outer_steps": st["outer_steps"],
                     "residual": st["residual"],
                     "resident_solves_per_s": 1.0 / solve_s,
                     "solves_per_s": 1.0 / (solve_s + wall_ms * 1e-3),
                     "matvec": [_matvec_entry(G, 1, op) for op in ops]}
        Ts[name] = T.cpu().numpy()
        del G, S
        torch.cuda.empty_cache()
    head = res.get("mixed", next(iter(res.values())))
    out = {"metric": "fixed-point solves/sec (assembly + solve, 1e-6 residual), 8 bands", "value": head["solves_per_s"],
           "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 entries/ACA, bf16 factors, f64 correction" if "mixed" in res else "f64",
           "data": "synthetic",
           "config": {"workload": "box65x33x33_reflective_8band", "N": mesh.N, "bands": len(wl.nu), "R": wl.R},
           "results": res}
    if len(Ts) == 2:
        out["mixed_vs_fp64_max_rel_T"] = float(np.max(np.abs(Ts["mixed"] - Ts["fp64"]) / Ts["fp64"]))
    print(json.dumps(out))


def run_batched(args):
    """49^3 cube, 32 bands x 16 right-hand sides: all bands and right-hand sides per
    launch, autotuned launch shape, mixed precision; `--compare` adds plain FP64 on
    the same bands (32 FP64 bands do not fit one GPU: take a share with --bands)."""
    import torch
    from paper_2306_05789_amd import inputs, rte, tune
    wl = inputs.batched()
    nb_all = wl.kappa.shape[0]
    bands = list(range(0, nb_all, max(1, nb_all // args.bands))) if args.bands else list(range(nb_all))
    dev = torch.device("cuda:0")
    mesh = rte.rte_mesh_create(wl.n, emit_faces=wl.emit_faces)
    kap = torch.tensor(wl.kappa[bands], device=dev)
    nu = wl.nu[bands]
    Tw = torch.tensor(wl.T_wall, device=dev)
    nrhs = Tw.shape[0]
    names = ["mixed", "fp64"] if args.compare else ["mixed"]
    res, Ts = {}, {}
    for name in names:
        p = rte.PRECISIONS[name]
        G = rte.rte_hmat_assemble(mesh, kap, rte.hmat_opts(kind=rte.RTE_VOLUME, precision=p))
        S = rte.rte_hmat_assemble(mesh, kap, rte.hmat_opts(kind=rte.RTE_SURFACE, precision=p))
        gs, ss = rte.rte_hmat_stats(G), rte.rte_hmat_stats(S)
        _say(f"{name}: {len(bands)} bands, G {gs['assemble_ms']:.0f} ms ({gs['bytes'] / 1e9:.1f} GB), "
             f"S {ss['assemble_ms']:.0f} ms")
        hot = rte.RTE_OP_LOW if p == rte.RTE_MIXED_BF16 else rte.RTE_OP_ACCURATE
        tuned = tune.autotune(G, nrhs=nrhs, op=hot, reps=2)
        _say(f"{name}: autotuned {tuned['config']} ({tuned['ms']:.2f} ms, {tuned['trials']} shapes)")
        ops = [rte.RTE_OP_LOW, rte.RTE_OP_ACCURATE] if p == rte.RTE_MIXED_BF16 else [rte.RTE_OP_ACCURATE]
        mv = [_matvec_entry(G, r, op) for op in ops for r in (1, nrhs)]
        T = torch.empty((nrhs, mesh.N), device=dev, dtype=torch.float64)
        lat, st = _solve_series(rte, mesh, G, S, Tw, T, nu, p, 1e-6, args.steps, args.warmup)
        solve_s = float(np.mean(lat))
        res[name] = {"assemble_G": _hstats(gs), "assemble_S": _hstats(ss), "autotuned": tuned,
                     "solve_ms": solve_s * 1e3, "sweeps": st["iterations"], "outer_steps": st["outer_steps"],
                     "residual": st["residual"], "graphs": st["graphs"],
                     "rhs_solves_per_s": nrhs / solve_s, "matvec": mv}
        Ts[name] = T.cpu().numpy()
        del G, S
        torch.cuda.empty_cache()
    head = res["mixed"]
    hot = next(m for m in head["matvec"] if m["op"] == "low" and m["nrhs"] == nrhs)
    out = {"metric": f"right-hand-side solves/sec at 1e-6 residual ({len(bands)} bands x {nrhs} RHS, operators resident)",
           "value": head["rhs_solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 entries/ACA, bf16 factors, f64 correction", "data": "synthetic",
           "config": {"workload": f"cube49_{len(bands)}band_{nrhs}rhs", "N": mesh.N, "bands": bands, "nrhs": nrhs},
           "roofline": {"kernel": "k_mf_phase_a + k_mf_phase_b (low operator, all bands x 16 RHS)", "bound": "hbm",
                        "achieved": hot["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hot["frac"],
                        "traffic": None},
           "results": res}
    if len(Ts) == 2:
        out["mixed_vs_fp64_max_rel_T"] = float(np.max(np.abs(Ts["mixed"] - Ts["fp64"]) / Ts["fp64"]))
        out["speedup_mixed_over_fp64"] = res["fp64"]["solve_ms"] / res["mixed"]["solve_ms"]
    print(json.dumps(out))


def run_served(args):
    """The request stream through the server: mixed precision with continuous
    batching, and (with --compare R) the first R requests through plain FP64 one
    at a time on the same server code."""
    import torch
    from paper_2306_05789_amd import inputs, rte
    from paper_2306_05789_amd.serve import Server, run_stream
    meshes = (21, 29, 41, 49)
    nu, c = inputs.catalogue(32)
    reqs = inputs.request_stream(max(args.requests, args.compare, 1))
    legs = [("mixed", rte.RTE_MIXED_BF16, 64, reqs[:args.requests])] if args.requests else []
    if args.compare:
        legs.append(("fp64", rte.RTE_FP64, 1, reqs[:args.compare]))
    res = {}
    for name, prec, active, rq in legs:
        srv = Server(nu, budget=int(args.budget_gb * 1e9), precision=prec, max_active=active,
                     recompress=args.server_recompress)
        ids = [srv.add_mesh((n, n, n), torch.tensor(inputs.smooth_kappa(
            inputs.grid_positions((n, n, n), (0, 0, 0), (1, 1, 1))), device="cuda:0")) for n in meshes]
        t0 = time.perf_counter()

        def log(k, st, lat, name=name, t0=t0):
            q = rq[k]
            _say(f"{name} [{time.perf_counter() - t0:7.1f} s] request {k} mesh {meshes[q.mesh]}^3 "
                 f"{len(q.bands)} bands: {st['iterations']} sweeps, latency {lat * 1e3:.0f} ms")
        r = run_stream(srv, rq, ids, [n ** 3 for n in meshes], c, tol=1e-6, log=log)
        res[name] = {"requests": len(rq), "max_active": active, "wall_s": r["wall_s"],
                     "solves_per_s": r["solves_per_s"], "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                     "converged": int(sum(1 for i in r["info"] if i and i["converged"])), "server": srv.stats()}
        del srv
    head = res["mixed"] if "mixed" in res else res["fp64"]
    out = {"metric": "served fixed-point solves/sec with p50/p99 latency (1e-6 residual)",
           "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 entries/ACA, bf16 factors, f64 correction" if "mixed" in res else "f64", "data": "synthetic",
           "config": {"workload": f"served_{head['requests']}req_poisson20", "meshes": list(meshes),
                      "budget_GB": args.budget_gb, "recompress": bool(args.server_recompress)},
           "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"]}, "results": res}
    print(json.dumps(out))


# HBM bytes per launch of the low-operator matvec of the headline workload (the
# four launches k_mf_xstage, k_mf_phase_a, k_mf_tstage, k_mf_phase_b), from
# rocprofv3 FETCH_SIZE and WRITE_SIZE passes calibrated on a plain 1 GiB copy
# (FETCH_SIZE reads half the bytes moved, WRITE_SIZE all): 87.8 GB read and
# 5.1 GB written, on the recompressed operator
# (profiles/cube49_32band_16rhs_mixed_matvec_traffic.md).  Set to None
# whenever those kernels or the operator's storage change.
LOW_MATVEC_TRAFFIC_BYTES = 92.9e9


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _sample_operator(mesh, G, rng, count):
    """A random sample of `count` dense and `count` low-rank blocks of band 0 of the
    volume operator, read back through the C ABI (hi + lo, widened to FP64), as an
    oracle H-operator over those blocks only; and the stored entries it holds."""
    from oracle.hmatrix import HOperator
    from paper_2306_05789_amd import rte
    st = rte.rte_hmat_stats(G)
    optG = rte.hmat_opts(kind=rte.RTE_VOLUME, precision=st["precision"])
    plan = rte.rte_plan_create(mesh, optG)
    tp, sp, blocks = rte.rte_plan_export(plan)
    rte.rte_plan_destroy(plan)
    H = HOperator(tp, sp)
    nd = rte.rte_hmat_dense_count(G, 0)
    for d in rng.choice(nd, min(count, nd), replace=False):
        (t0, t1, s0, s1), A = rte.rte_hmat_dense_block(G, 0, int(d))
        H.dense.append((t0, t1, s0, s1, A))
    low = blocks[blocks[:, 4] == 1]
    for b in rng.choice(len(low), min(count, len(low)), replace=False):
        k, U, V = rte.rte_hmat_block_factors_op(G, 0, int(b), rte.RTE_OP_ACCURATE)
        if k > 0:
            t0, t1, s0, s1 = (int(v) for v in low[b][:4])
            H.lowrank.append((t0, t1, s0, s1, U, V))
    return H, H.stored_entries()


def cpu_baseline_headline(wl, G, mesh, gstats, sstats, sweeps, nrhs, budget_s=15.0):
    """The oracle on a bounded sample of the headline workload: its entry cost on
    sampled rows of band 0 (extrapolated to the entries the assembly evaluates), and
    its FP64 block-by-block H-matvec (oracle-on-H) timed on a sample of band 0's
    read-back blocks (extrapolated to every stored entry of the 32 bands), times
    the sweeps of a solve."""
    from oracle.core import Grid, Problem
    g = Grid(wl.n)
    P = Problem(g, wl.kappa[0], emit_faces=wl.emit_faces)
    rng = np.random.default_rng(12)
    cols = np.arange(g.N)
    t0 = time.perf_counter()
    P.volume_block(rng.choice(g.N, 2, replace=False), cols)
    t_probe = (time.perf_counter() - t0) / (2 * g.N)
    R = int(min(64, max(2, 0.4 * budget_s / max(t_probe * g.N, 1e-6))))
    rows = rng.choice(g.N, R, replace=False)
    t0 = time.perf_counter()
    P.volume_block(rows, cols)
    t_entry = (time.perf_counter() - t0) / (R * g.N)
    evaluated = gstats["entries_evaluated"] + sstats["entries_evaluated"]
    t_assembly = t_entry * evaluated
    # oracle-on-H FP64 matvec over a sample of band 0's blocks
    Hs, sampled = _sample_operator(mesh, G, rng, 400)
    X = rng.uniform(0.5, 2.0, (nrhs, g.N))
    Hs.matvec(X)
    reps, t0 = 0, time.perf_counter()
    while reps < 3 or (time.perf_counter() - t0 < 0.3 * budget_s and reps < 50):
        Hs.matvec(X)
        reps += 1
    t_mv = (time.perf_counter() - t0) / reps / max(sampled, 1)   # per stored entry, 16 RHS
    stored = gstats["dense_entries"] + gstats["lowrank_entries"]  # all bands
    t_sweep = t_mv * stored
    t_solve = sweeps * t_sweep
    return {"value": nrhs / t_solve, "unit": "solves/s", "cores": _cpu_threads(), "kind": "oracle",
            "cpu": _cpu_model(),
            "sample": f"oracle entries on {R} random rows of band 0's G ({R * g.N} entries, "
                      f"{t_entry * 1e9:.0f} ns each on {_cpu_threads()} threads) and the oracle's FP64 "
                      f"block-by-block H-matvec of {nrhs} RHS over {sampled} stored entries of band 0 read back "
                      f"from the GPU ({reps} reps); extrapolated: a sweep over all {wl.bands} bands "
                      f"({stored} stored entries) {t_sweep:.1f} s, a solve of {sweeps} sweeps {t_solve:.0f} s "
                      f"with resident operators; the assembly ({evaluated} entries) {t_assembly:.0f} s"}


def run_headline(args):
    """49^3, 32 bands x 16 RHS, mixed precision, operators resident; see the module docstring."""
    import torch
    from paper_2306_05789_amd import inputs, rte
    wl = inputs.batched()
    dev = torch.device("cuda:0")
    mesh = rte.rte_mesh_create(wl.n, emit_faces=wl.emit_faces)
    kap = torch.tensor(wl.kappa, device=dev)
    Tw = torch.tensor(wl.T_wall, device=dev)
    nrhs, nb = int(Tw.shape[0]), wl.bands
    p = rte.RTE_MIXED_BF16
    rc = not args.no_recompress
    # S serves one product per solve: only G, streamed by every sweep, is recompressed
    G, S, wall_ms = _assemble_pair(rte, mesh, kap, rte.hmat_opts(kind=rte.RTE_VOLUME, precision=p, recompress=rc),
                                   rte.hmat_opts(kind=rte.RTE_SURFACE, precision=p))
    gs, ss = rte.rte_hmat_stats(G), rte.rte_hmat_stats(S)
    _say(f"assembly: G {gs['assemble_ms']:.0f} ms ({gs['bytes'] / 1e9:.1f} GB; recompression {gs['recompress_ms']:.0f} "
         f"ms, low-rank entries {gs['lowrank_entries_aca'] / 1e9:.2f} -> {gs['lowrank_entries'] / 1e9:.2f} G), "
         f"S {ss['assemble_ms']:.0f} ms ({ss['bytes'] / 1e9:.1f} GB), concurrently {wall_ms:.0f} ms")
    T = torch.empty((nrhs, mesh.N), device=dev, dtype=torch.float64)

    def solve():
        return rte.rte_fixed_point_solve(mesh, G, S, Tw, T, grey=False, nu=wl.nu, tol=wl.tol, max_iter=3000,
                                         precision=p, time_matvecs=True, history=True)

    for _ in range(args.warmup):
        st = solve()
        _say(f"warmup solve: {st['ms_total']:.1f} ms, {st['iterations']} sweeps")
    torch.cuda.synchronize()
    lat, sts = [], []
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        st = solve()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        sts.append(st)
        _say(f"step: {lat[-1] * 1e3:.1f} ms, {st['iterations']} sweeps ({st['outer_steps']} defect steps), "
             f"residual {st['residual']:.2e}; low matvec {st['ms_matvec_low'] / max(st['matvecs_low'], 1):.2f} ms "
             f"x {st['matvecs_low']}, accurate {st['ms_matvec_acc'] / max(st['matvecs_acc'], 1):.2f} ms "
             f"x {st['matvecs_acc']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    K = args.steps
    assert all(st["converged"] for st in sts)

    # --- the kernel groups of a step: the two operators' volume matvecs (events inside the graphs)
    low_ms = sum(st["ms_matvec_low"] for st in sts)
    low_n = sum(st["matvecs_low"] for st in sts)
    acc_ms = sum(st["ms_matvec_acc"] for st in sts)
    acc_n = sum(st["matvecs_acc"] for st in sts)
    solve_ms = sum(st["ms_total"] for st in sts)
    vec = 8 * nb * nrhs * (gs["n_src"] + gs["n_tgt"])            # x read, y written (FP64)
    bytes_low = 2 * (gs["dense_entries"] + gs["lowrank_entries"]) + vec      # BF16 hi parts, no padding
    bytes_acc = 4 * (gs["dense_entries"] + gs["lowrank_entries"]) + vec      # hi + lo
    per_low = low_ms / max(low_n, 1)
    per_acc = acc_ms / max(acc_n, 1)
    gbs_low = bytes_low / (per_low * 1e-3) / 1e9
    gbs_acc = bytes_acc / (per_acc * 1e-3) / 1e9
    roof = {"kernel": "low-operator H-matvec of the inner sweeps (k_mf_xstage + k_mf_phase_a + k_mf_tstage + "
                      "k_mf_phase_b, all 32 bands x 16 RHS per launch)",
            "bound": "hbm", "achieved": gbs_low, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs_low / HBM_PEAK_GBS,
            "traffic": LOW_MATVEC_TRAFFIC_BYTES, "bytes_per_launch": bytes_low, "launch_ms": per_low,
            "launches": low_n}
    out = {
        "metric": "fixed-point solves/sec + H-matvec HBM GB/s (% peak) at 1e-6 rel err; p50/p99 latency",
        "value": nrhs * K / elapsed,
        "unit": "solves/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "dtype_detail": "FP32 entries and ACA; BF16 hi + lo factors, BF16 matrix cores with FP32 "
                                          "accumulation in the sweeps; FP64 defect correction, residual and Newton",
        "data": "synthetic",
        "config": {"workload": "cube49_32band_16rhs_mixed", "N": mesh.N, "L": mesh.L, "bands": nb, "nrhs": nrhs,
                   "leaf_size": wl.leaf_size, "eta": wl.eta, "aca_eps": wl.aca_eps, "tol": wl.tol,
                   "precision": "mixed", "recompress": rc,
                   "step": "one 16-RHS fixed-point solve on resident operators"},
        "roofline": roof,
        "hmatvec": {"low": {"ms": per_low, "bytes": bytes_low, "GB_s": gbs_low, "frac": gbs_low / HBM_PEAK_GBS},
                    "accurate": {"ms": per_acc, "bytes": bytes_acc, "GB_s": gbs_acc,
                                 "frac": gbs_acc / HBM_PEAK_GBS},
                    "device_bytes_hi_lo": gs["bytes"]},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "breakdown_ms_per_step": {"low_matvecs": low_ms / K, "accurate_matvecs": acc_ms / K,
                                  "rest_of_solve": (solve_ms - low_ms - acc_ms) / K},
        "solve": {"sweeps": sts[-1]["iterations"], "defect_steps": sts[-1]["outer_steps"],
                  "residual": sts[-1]["residual"], "graphs": sts[-1]["graphs"],
                  "residuals": [float(f"{v:.3e}") for v in sts[-1]["residuals"]]},
        "assembly": {"wall_ms": wall_ms, "G": _hstats(gs), "S": _hstats(ss),
                     "entries_evaluated": gs["entries_evaluated"] + ss["entries_evaluated"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_headline(wl, G, mesh, gs, ss, sts[-1]["iterations"], nrhs)
    T_ref = T.cpu().numpy()
    del G, S
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["kappa_levels"] = _levels_leg(rte, wl, mesh, dev, T_ref, rc)
        out["fp64_vs_mixed_4band_share"] = _share4(rte, wl, mesh, dev)
        out["cube41_fp64_step"] = _cube41_leg(args)
        out["cube11_dense"] = _cube11_leg(rte, dev)
    print(json.dumps(out))


def _levels_leg(rte, wl, mesh, dev, T_ref, rc, tol=0.25):
    """The headline's 32 bands on adaptive kappa levels (each band's multiplier
    within a factor 1 + tol of its level): the levels' operators assembled once,
    band views solved as in the headline; T against the 32-operator solution."""
    import torch
    from paper_2306_05789_amd import inputs
    nu, cb = inputs.catalogue(wl.bands, 4)
    levels, mp = rte.rte_kappa_levels(cb, tol)
    base = inputs.smooth_kappa(inputs.grid_positions(wl.n, wl.lo, wl.hi))
    kap = torch.tensor(levels[:, None] * base[None, :], device=dev)
    p = rte.RTE_MIXED_BF16
    G, S, wall_ms = _assemble_pair(rte, mesh, kap, rte.hmat_opts(kind=rte.RTE_VOLUME, precision=p, recompress=rc),
                                   rte.hmat_opts(kind=rte.RTE_SURFACE, precision=p))
    gb = rte.rte_hmat_stats(G)["bytes"]
    Gv, Sv = rte.rte_hmat_select_bands(G, mp), rte.rte_hmat_select_bands(S, mp)
    Tw = torch.tensor(wl.T_wall, device=dev)
    T = torch.empty((Tw.shape[0], mesh.N), device=dev, dtype=torch.float64)
    lat, st = _solve_series(rte, mesh, Gv, Sv, Tw, T, wl.nu, p, wl.tol, 3, 1)
    Tl = T.cpu().numpy()
    res = {"tol": tol, "levels": len(levels), "bands": wl.bands, "assemble_wall_ms": wall_ms, "G_bytes": gb,
           "solve_ms": float(np.mean(lat)) * 1e3, "sweeps": st["iterations"],
           "rhs_solves_per_s": Tw.shape[0] / float(np.mean(lat)),
           "max_rel_T_vs_32_operators": float(np.max(np.abs(Tl - T_ref) / T_ref))}
    del Gv, Sv, G, S
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def _share4(rte, wl, mesh, dev):
    """4 of the 32 bands (0, 8, 16, 24): mixed against plain FP64, 16 RHS each, 1e-6."""
    import torch
    bands = [0, 8, 16, 24]
    kap = torch.tensor(wl.kappa[bands], device=dev)
    Tw = torch.tensor(wl.T_wall, device=dev)
    nu = wl.nu[bands]
    res, Ts = {}, {}
    for name in ("mixed", "fp64"):
        p = rte.PRECISIONS[name]
        G, S, wall_ms = _assemble_pair(rte, mesh, kap, rte.hmat_opts(kind=rte.RTE_VOLUME, precision=p),
                                       rte.hmat_opts(kind=rte.RTE_SURFACE, precision=p))
        T = torch.empty((Tw.shape[0], mesh.N), device=dev, dtype=torch.float64)
        lat, st = _solve_series(rte, mesh, G, S, Tw, T, nu, p, wl.tol, 3, 1)
        res[name] = {"assemble_wall_ms": wall_ms, "solve_ms": float(np.mean(lat)) * 1e3, "sweeps": st["iterations"],
                     "rhs_solves_per_s": Tw.shape[0] / float(np.mean(lat)), "G_bytes": rte.rte_hmat_stats(G)["bytes"]}
        Ts[name] = T.cpu().numpy()
        del G, S
        torch.cuda.synchronize()
    res["speedup_mixed_over_fp64"] = res["fp64"]["solve_ms"] / res["mixed"]["solve_ms"]
    res["mixed_vs_fp64_max_rel_T"] = float(np.max(np.abs(Ts["mixed"] - Ts["fp64"]) / Ts["fp64"]))
    return res


def _cube41_leg(args):
    ns = argparse.Namespace(**vars(args))
    ns.steps, ns.warmup, ns.no_cpu_baseline, ns.n = 10, 2, True, 41
    o = run_cube41(ns, emit=False)
    return {k: o[k] for k in ("value", "unit", "ms_per_step", "latency_ms", "step_ms", "roofline", "hmatvec",
                              "breakdown_ms", "solve", "config")}


def _cube11_leg(rte, dev):
    """The 11^3 dense case timed in full: GPU (dense assembly of G and S + fixed point
    to 1e-10) and the oracle (dense G and S + its fixed point to 1e-10)."""
    import torch
    from paper_2306_05789_amd import inputs
    from oracle import solve as osolve
    from oracle.core import Grid, Problem
    wl = inputs.config_tiny(11)
    mesh = rte.rte_mesh_create(wl.n, emit_faces=wl.emit_faces)
    kap = torch.tensor(wl.kappa, device=dev)
    Tw = torch.tensor(wl.T_wall, device=dev)
    T = torch.empty((1, mesh.N), device=dev, dtype=torch.float64)
    lat = []
    for k in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G = rte.rte_hmat_assemble(mesh, kap, rte.hmat_opts(kind=rte.RTE_VOLUME, dense=True))
        S = rte.rte_hmat_assemble(mesh, kap, rte.hmat_opts(kind=rte.RTE_SURFACE, dense=True))
        st = rte.rte_fixed_point_solve(mesh, G, S, Tw, T, grey=True, tol=wl.tol, max_iter=500)
        torch.cuda.synchronize()
        if k:
            lat.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    P = Problem(Grid(wl.n), wl.kappa[0], emit_faces=wl.emit_faces)
    Gd, Sd = P.dense_G(), P.dense_S()
    ref = osolve.fixed_point([Gd], (Sd @ (osolve.SIGMA * wl.T_wall[0] ** 4))[None], grey=True, tol=wl.tol)
    t_cpu = time.perf_counter() - t0
    err = float(np.max(np.abs(T.cpu().numpy()[0] - ref.T) / ref.T))
    return {"gpu_ms": float(np.mean(lat)) * 1e3, "iterations": st["iterations"], "oracle_s": t_cpu,
            "oracle_iterations": ref.iterations, "oracle_threads": _cpu_threads(), "max_rel_T_vs_oracle": err}


def run_cube41(args, emit=True):
    """The 41^3 grey FP64 H-matrix workload: one step = assembly of G and S (two host
    threads, two streams) + the fixed point to 1e-10."""
    import torch
    from paper_2306_05789_amd import inputs, rte

    wl = inputs.config_hmatrix(args.n)
    dev = torch.device("cuda:0")
    mesh = rte.rte_mesh_create(wl.n, emit_faces=wl.emit_faces)
    kap = torch.tensor(wl.kappa, device=dev)
    Tw = torch.tensor(wl.T_wall, device=dev)
    T = torch.empty((1, mesh.N), device=dev, dtype=torch.float64)
    optG = rte.hmat_opts(kind=rte.RTE_VOLUME, leaf_size=wl.leaf_size, eta=wl.eta, aca_eps=wl.aca_eps)
    optS = rte.hmat_opts(kind=rte.RTE_SURFACE, leaf_size=wl.leaf_size, eta=wl.eta, aca_eps=wl.aca_eps)

    # G and S are independent: each is assembled by its own host thread on its
    # own stream (the library synchronises the stream before returning), so
    # the small launches of the surface ACA fill the gaps of the volume one
    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(2)
    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    torch.cuda.synchronize()

    held = []   # the previous step's operators: released at the start of the next step, inside it

    def step():
        t0 = time.perf_counter()
        held.clear()
        t_free = time.perf_counter() - t0
        fG = pool.submit(rte.rte_hmat_assemble, mesh, kap, optG, streams[0].cuda_stream)
        fS = pool.submit(rte.rte_hmat_assemble, mesh, kap, optS, streams[1].cuda_stream)
        G, S = fG.result(), fS.result()
        st = rte.rte_fixed_point_solve(mesh, G, S, Tw, T, grey=True, tol=wl.tol, max_iter=1000, time_matvecs=True)
        held.extend([G, S])
        return G, S, st, t_free

    def show(tag, ms, G, S, st, t_free):
        g, q = rte.rte_hmat_stats(G), rte.rte_hmat_stats(S)
        _say(f"{tag}: {ms:.1f} ms, {st['iterations']} iterations; release {t_free * 1e3:.1f} ms; "
             f"G {g['assemble_ms']:.1f} ms (ACA kernels {g['aca_kernel_ms']:.1f}, alloc {g['alloc_ms']:.1f}); "
             f"S {q['assemble_ms']:.1f} ms (alloc {q['alloc_ms']:.1f}); solve {st['ms_total']:.1f} ms; "
             f"free {g['free_bytes'] / 2 ** 30:.1f} GiB")

    for _ in range(args.warmup):
        t0 = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        show("warmup", (time.perf_counter() - t0) * 1e3, *out)
    torch.cuda.synchronize()
    recs, lat = [], []
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        G, S, st, t_free = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        recs.append((rte.rte_hmat_stats(G), rte.rte_hmat_stats(S), st))
        show("step", lat[-1] * 1e3, G, S, st, t_free)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    K = args.steps
    gs, ss, sts = recs[-1]

    # --- kernel shares of a step (HIP events inside the library)
    aca_ms = np.mean([g["aca_kernel_ms"] + s["aca_kernel_ms"] for g, s, _ in recs])
    fill_ms = np.mean([g["fill_kernel_ms"] + s["fill_kernel_ms"] for g, s, _ in recs])
    mv_ms = np.mean([t["ms_matvec"] for _, _, t in recs])
    iters = sts["iterations"]

    # --- ACA kernel: algorithmic FLOPs per launch from the sampled entry cost
    plan = rte.rte_plan_create(mesh, optG)
    tp, sp, blocks = rte.rte_plan_export(plan)
    rte.rte_plan_destroy(plan)
    low = blocks[blocks[:, 4] == 1]
    Gh = G
    ranks = np.array([rte.rte_hmat_block_factors(Gh, 0, b, factors=False)[0] for b in range(len(low))])
    kcap = np.minimum((low[:, 1] - low[:, 0]) * (low[:, 3] - low[:, 2]) //
                      ((low[:, 1] - low[:, 0]) + (low[:, 3] - low[:, 2])), 192)
    keff = np.where(ranks > 0, ranks, kcap)
    wts = keff * ((low[:, 1] - low[:, 0]) + (low[:, 3] - low[:, 2]))
    rng = np.random.default_rng(5)
    pick = rng.choice(len(low), 2000, p=wts / wts.sum())
    nvec = np.array(wl.n)

    def gidx(v):
        return (v // (wl.n[1] * wl.n[2]), (v // wl.n[2]) % wl.n[1], v % wl.n[2])

    pairs = []
    for b in pick:
        t0, t1, s0, s1, _ = low[b]
        i = tp[rng.integers(t0, t1)]
        j = sp[rng.integers(s0, s1)]
        pairs.append((gidx(i), gidx(j)))
    f_entry = entry_flops_sample(nvec, pairs)
    aca_entries_G = gs["aca_entries"]
    nl = max(gs["aca_entry_launches"], 1)
    aca_launch_ms_G = gs["aca_entry_ms"] / nl
    flop_per_launch = f_entry * aca_entries_G / nl
    aca_tflops = flop_per_launch / (aca_launch_ms_G * 1e-3) / 1e12

    # --- H-matvec: algorithmic bytes per matvec (stored entries without padding,
    # x read and y written in FP64)
    mv_per = mv_ms / max(iters, 1)
    mv_bytes = 8 * (gs["dense_entries"] + gs["lowrank_entries"]) + 8 * (gs["n_src"] + gs["n_tgt"])
    mv_gbs = mv_bytes / (mv_per * 1e-3) / 1e9

    shares = {"aca": aca_ms, "dense_fill": fill_ms, "hmatvec": mv_ms}
    dominant = max(shares, key=shares.get)
    if dominant == "aca":
        roof = {"kernel": "k_aca_rows + k_aca_cols (FP64 kernel entries of the ACA rank steps, volume matrix)",
                "bound": "alu", "achieved": aca_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": aca_tflops / FP64_PEAK_TFLOPS, "traffic": ACA_ENTRY_TRAFFIC_BYTES,
                "traffic_unit": "bytes per launch (HBM, rocprofv3 counters)",
                "flop_per_entry": f_entry, "entries_per_launch": aca_entries_G / nl,
                "launch_ms": aca_launch_ms_G, "launches": nl}
    else:
        roof = {"kernel": "k_phase_a + k_phase_b (H-matvec)", "bound": "hbm", "achieved": mv_gbs,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": mv_gbs / HBM_PEAK_GBS, "traffic": None}

    out = {
        "metric": "fixed-point solves/sec + H-matvec HBM GB/s (% peak) at 1e-6 rel err; p50/p99 latency",
        "value": K / elapsed,
        "unit": "solves/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "N": mesh.N, "L": mesh.L, "leaf_size": wl.leaf_size, "eta": wl.eta,
                   "aca_eps": wl.aca_eps, "tol": wl.tol, "precision": "fp64"},
        "roofline": roof,
        "hmatvec": {"bound": "hbm", "achieved": mv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": mv_gbs / HBM_PEAK_GBS, "bytes_per_matvec": mv_bytes, "ms_per_matvec": mv_per,
                    "device_bytes": gs["bytes"]},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "breakdown_ms": {"aca_kernels": aca_ms, "dense_fill_kernels": fill_ms, "matvec_kernels": mv_ms,
                         "assemble_G_wall": gs["assemble_ms"], "assemble_S_wall": ss["assemble_ms"],
                         "solve_wall": sts["ms_total"],
                         "alloc_host": float(np.mean([g["alloc_ms"] + s["alloc_ms"] for g, s, _ in recs]))},
        "step_ms": [round(v * 1e3, 1) for v in lat],
        "solve": {"iterations": iters, "residual": sts["residual"], "monotone_violations": sts["monotone_violations"],
                  "resident_solves_per_s": 1e3 / sts["ms_total"]},
        "hmatrix": {"compression": gs["compression"], "mean_rank": gs["mean_rank"], "max_rank": gs["max_rank"],
                    "n_lowrank": gs["n_lowrank"], "n_fallback_dense": gs["n_fallback_dense"],
                    "entries_evaluated": gs["entries_evaluated"] + ss["entries_evaluated"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    pool.shutdown()
    del G, S, Gh
    held.clear()
    torch.cuda.synchronize()
    if emit:
        print(json.dumps(out))
    return out




# The paper's whole-run CPU times of Test-3 (Section "An Academic Test", its CPU
# table; MacBook Pro M1, precision not stated), quoted beside the nearest grid
# as context: vertices -> seconds.
PAPER_TEST3_CPU_S = {2758: 5.3, 8003: 16.5, 26189: 79.4, 84042: 389.0, 195974: 1563.0}


def run_academic(args, emit=True):
    """Test-3 of the academic test: D = (0,60) x (0,100) x (0,60) cm minus the cube
    [0,10]^3, the three planes through the origin reflecting (R = 1), the cube's
    three faces inside D emitting, kappa 0.1 per cm and 1e-4 in the cylinder
    that prolongs the cube, grey.  One step = assembly of G and S (concurrently)
    + the fixed point to a relative change of 1e-6 (the paper's six orders of
    reduction), FP64 and mixed.  The paper's CPU time on its nearest mesh is
    quoted as context."""
    import torch
    from paper_2306_05789_amd import inputs, rte
    dev = "cuda:0"
    wl = inputs.academic(args.h)
    mesh = rte.rte_mesh_create(wl.n, wl.lo, wl.hi, emit_faces=wl.emit_faces, walls=wl.walls, hole=wl.hole,
                               hole_emit=wl.hole_emit)
    kap = torch.tensor(wl.kappa[None, :], device=dev)
    Tw = torch.full((1, mesh.L), wl.T_hole, device=dev, dtype=torch.float64)
    T = torch.empty((1, mesh.N), device=dev, dtype=torch.float64)
    res = {}
    for name in ("fp64", "mixed"):
        p = rte.PRECISIONS[name]
        steps = []
        for k in range(min(max(args.steps, 1), 5) + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            G, S, wall_ms = _assemble_pair(rte, mesh, kap, rte.hmat_opts(kind=rte.RTE_VOLUME, precision=p),
                                           rte.hmat_opts(kind=rte.RTE_SURFACE, precision=p))
            t1 = time.perf_counter()
            st = rte.rte_fixed_point_solve(mesh, G, S, Tw, T, grey=True, tol=1e-6, max_iter=3000, precision=p)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            gs, ss = rte.rte_hmat_stats(G), rte.rte_hmat_stats(S)
            if k:   # the first step is the warm-up
                steps.append(((t2 - t0) * 1e3, (t1 - t0) * 1e3, (t2 - t1) * 1e3))
            _say(f"academic {name}: step {(t2 - t0) * 1e3:.0f} ms (assembly {(t1 - t0) * 1e3:.0f}, solve "
                 f"{(t2 - t1) * 1e3:.0f}), {st['iterations']} sweeps, residual {st['residual']:.1e}")
            del G, S
        stored_G = gs["dense_entries"] + gs["lowrank_entries"]
        stored_S = ss["dense_entries"] + ss["lowrank_entries"]
        ms = np.mean(np.array(steps), axis=0)
        Tn = T.cpu().numpy()[0]
        res[name] = {"step_ms": float(ms[0]), "assembly_ms": float(ms[1]), "solve_ms": float(ms[2]),
                     "sweeps": st["iterations"], "residual": st["residual"], "converged": bool(st["converged"]),
                     "compression_level_volume": 1.0 - stored_G / float(mesh.N) ** 2,
                     "compression_level_surface": 1.0 - stored_S / float(mesh.N * mesh.L),
                     "G_bytes": gs["bytes"], "S_bytes": ss["bytes"], "T_max": float(Tn.max())}
        if name == "fp64":
            T64 = Tn.copy()
        else:
            live = T64 > 0
            res[name]["max_rel_T_vs_fp64"] = float(np.max(np.abs(Tn[live] - T64[live]) / T64[live]))
    near = min(PAPER_TEST3_CPU_S, key=lambda v: abs(np.log(v / mesh.N)))
    out = {"workload": f"academic_test3_h{args.h:g}", "N": mesh.N, "L": mesh.L, "n": list(wl.n), "results": res,
           "paper_context": {"vertices": near, "cpu_s": PAPER_TEST3_CPU_S[near], "hardware": "MacBook Pro M1",
                             "what": "whole run, precision and tolerance not stated"}}
    if emit:
        print(json.dumps(out))
    return out


def run_matvec(args):
    """The headline operator alone (49^3, 32 bands, mixed storage): a 1 GiB device
    copy first (the calibration of the HBM traffic counters), then event-timed
    all-band 16-RHS matvecs of the low and the accurate operator.  Used under
    rocprofv3 --pmc to measure the matvec's HBM traffic."""
    import torch
    from paper_2306_05789_amd import inputs, rte
    wl = inputs.batched()
    mesh = rte.rte_mesh_create(wl.n, emit_faces=wl.emit_faces)
    G = rte.rte_hmat_assemble(mesh, torch.tensor(wl.kappa, device="cuda:0"),
                              rte.hmat_opts(kind=rte.RTE_VOLUME, precision=rte.RTE_MIXED_BF16,
                                            recompress=not args.no_recompress))
    st = rte.rte_hmat_stats(G)
    _say(f"assembled in {st['assemble_ms']:.0f} ms")
    a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    nrhs = int(wl.T_wall.shape[0])
    vec = 8 * st["n_bands"] * nrhs * (st["n_src"] + st["n_tgt"])
    res = {}
    for op, name, esz in ((rte.RTE_OP_LOW, "low", 2), (rte.RTE_OP_ACCURATE, "accurate", 4)):
        ms = rte.rte_hmat_time_matvec(G, nrhs, op, max(args.steps, 1))
        byt = esz * (st["dense_entries"] + st["lowrank_entries"]) + vec
        res[name] = {"ms": ms, "bytes": byt, "GB_s": byt / (ms * 1e-3) / 1e9, "frac": byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        _say(f"{name}: {ms:.2f} ms, {res[name]['GB_s']:.0f} GB/s")
    print(json.dumps({"workload": "cube49_32band_16rhs_mixed_matvec", "calibration_copy_bytes": 2 ** 30,
                      "dense_entries": st["dense_entries"], "lowrank_entries": st["lowrank_entries"],
                      "device_bytes": st["bytes"], "matvec": res}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=41, help="cube41 workload: vertices per axis of the cube")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline: skip the FP64 share, 41^3 and 11^3 legs")
    ap.add_argument("--no-recompress", action="store_true",
                    help="headline and matvec workloads: keep the ACA factors (no SVD recompression)")
    ap.add_argument("--workload", default="headline",
                    choices=("headline", "cube41", "reflective", "batched", "served", "matvec", "academic"))
    ap.add_argument("--h", type=float, default=2.5, help="academic workload: grid spacing in cm (divides 10)")
    ap.add_argument("--precision", default="both", choices=("both", "mixed", "fp64"), help="reflective workload")
    ap.add_argument("--bands", type=int, default=0, help="batched workload: bands taken (0 = all 32)")
    ap.add_argument("--compare", type=int, default=0,
                    help="batched: add plain FP64 (1); served: requests replayed through plain FP64")
    ap.add_argument("--requests", type=int, default=256,
                    help="served workload: requests of the stream served in mixed precision (0: none)")
    ap.add_argument("--budget-gb", type=float, default=250.0, help="served workload: HBM budget of the server")
    ap.add_argument("--server-recompress", action="store_true",
                    help="served workload: recompress the volume operators' ACA factors")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the multi-GPU band sharding is a design, not a build "
              "(see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    {"headline": run_headline, "cube41": run_cube41, "reflective": run_reflective, "batched": run_batched,
     "served": run_served, "matvec": run_matvec, "academic": run_academic}[args.workload](args)


if __name__ == "__main__":
    main()
