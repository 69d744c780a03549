"""Benchmark: SSP-RK3 steps of the unstructured-mesh finite-difference Euler
residual on one MI355X.

Workload: rotated Sod data (interface through (1/2, 1/2) at 30 degrees) on
[0,1]^2, a jittered 1025 x 1025 triangulation (1,050,625 real vertices, random
diagonals, +-0.15 h interior jitter, seed 0) with a 4-deep mirror ghost layer
(reflecting walls y = 0, 1; extrapolating walls x = 0, 1), NU-WENO5 edge fluxes,
degree-5 two-level least-squares divergence, SSP-RK3, FP64 (CFL: see SOD_CFL).

One step = CFL reduction + 3 x (ghost fill, edge flux, vertex step + stage
update), all in the HIP library, applied to the initial state (see SOD_CFL for
why steps are not chained).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The scheme's least-squares divergence of the Sod jump on jittered stencils
# and at the mirrored walls drives the density negative after less than one
# cell crossing of the waves, at any CFL number, so steps are not chained: every
# timed step is one full SSP-RK3 step (CFL reduction + 3 stages) from the Sod
# initial state into separate buffers.  The work per step does not depend on
# the data; at this CFL one step from the initial state stays physical.
SOD_CFL = 0.2
METRIC = "vertex-stage updates/sec + HBM GB/s vs peak; batched & adjoint vs plain path"


def kernel_bytes(A, precision_bytes=8, blocks=None, packed=None, wn_stages=3):
    """Algorithmic bytes per launch as stored (each datum counted once), averaged
    over the three stage launches of an SSP-RK3 step.
    edge:   per flux edge 6 int32 ids + 6 geometry values + 4 flux values written,
            plus every state row read once;
    vertex: per real vertex two CSR pointers, c_O (2) and the output (4), w_n (4)
            in the stages that read it (the first stage has a_0 = 0 and does
            not: wn_stages = 2 of 3 for a whole step, 3 for the stage form alone),
            per vertex entry an int32 id + 2 weights, per edge entry an int32 id +
            1 weight, plus every state row and every flux row read once.
            LDS-staged variants (blocks given): 16-bit ids instead, plus per block
            3 int32 pointers and its int32 row lists (the row data itself still
            counted once).  Packed-id variants (packed = the number of vertex and
            edge entries past each vertex's first round): the first-round ids
            are one 12-byte record per vertex and lane (96 bytes per real
            vertex), only the entries past the first round keep 16-bit ids."""
    s = precision_bytes
    nvt, nvr, nef, nzv, nze = A["nv_total"], A["nv_real"], A["ne_flux"], A["nnz_v"], A["nnz_e"]
    edge = nef * (6 * 4 + 6 * s + 4 * 8) + nvt * 4 * s
    ids = 4 if blocks is None else 2
    vertex = (nvr * (2 * 4 + 2 * 8 + 4 * s) + nvr * 4 * s * wn_stages / 3.0 + nzv * 2 * s + nze * s + nvt * 4 * s
              + nef * 4 * 8)
    if packed is None:
        vertex += (nzv + nze) * ids
    else:
        vertex += nvr * 8 * 12 + (packed[0] + packed[1]) * 2
    if blocks is not None:
        vertex += blocks["n_blocks"] * 3 * 4 + blocks["halo_rows"] * 4
    return dict(edge=edge, vertex=vertex)


def survey_bytes_per_vertex_stage(A, precision_bytes=8, wn_stages=2):
    """Algorithmic bytes per real vertex and stage of the vertex step in the
    blueprint's unit count (int32 ids, each datum once, E = ne_flux / nv_real
    edges per vertex): state 4s + CSR pointers 16 + ids (n_v + n_e) 4 +
    weights (2 n_v + n_e) s + c_O 2s + flux rows 4 * 8 * E + w_n 4s (in
    wn_stages of the 3 stages) + output 4s, with n_v, n_e the mean stencil
    sizes of the mesh.  For 19 + 44 entries and E = 3 this is 1,132 B (w_n
    counted in every stage)."""
    s = precision_bytes
    nvr = A["nv_real"]
    nv_mean, ne_mean, E = A["nnz_v"] / nvr, A["nnz_e"] / nvr, A["ne_flux"] / nvr
    return (4 * s + 16 + (nv_mean + ne_mean) * 4 + (2 * nv_mean + ne_mean) * s + 2 * s + 4 * 8 * E
            + 4 * s * wn_stages / 3.0 + 4 * s)


def survey_edge_bytes_per_vertex_stage(A, precision_bytes=8):
    """The edge step's bytes per real vertex and stage in the blueprint's unit
    count: state 4s + E (6 int32 ids + 6 arc coordinates + 2 direction values +
    the 32-byte flux row written), E = ne_flux / nv_real."""
    s = precision_bytes
    E = A["ne_flux"] / A["nv_real"]
    return 4 * s + E * (6 * 4 + 6 * s + 2 * s + 32)


# vertex variants whose first-round ids are packed, and the entries a first round covers
PACKED_VERTEX_VARIANTS = (4, 5)
BLOCK_VERTEX_VARIANTS = (3, 4, 5)
PACKED_ROUND = (24, 48)


def entries_past_first_round(A):
    """Vertex and edge entries that a packed-id variant reads with 16-bit ids
    (those past the first 24 vertex and 48 edge entries of each real vertex)."""
    import numpy as np

    nv = np.diff(np.asarray(A["vptr"], dtype=np.int64)[: A["nv_real"] + 1])
    ne = np.diff(np.asarray(A["eptr"], dtype=np.int64)[: A["nv_real"] + 1])
    return int(np.maximum(nv - PACKED_ROUND[0], 0).sum()), int(np.maximum(ne - PACKED_ROUND[1], 0).sum())


# kernel (template instance) behind each variant number of the library
EDGE_KERNELS = {0: "k_edge_flux<double, double>", 1: "k_edge_flux_lean<double, double>"}
VERTEX_KERNELS = {0: "k_vertex<double, double, 16, false>", 1: "k_vertex<double, double, 8, false>",
                  2: "k_vertex_pipe<double, double, 8, 3, 6>", 3: "k_vertex_lds<double, double, 8, 3, 6, 1, 5>",
                  4: "k_vertex_blk<double, double, 8, 3, 6, 1, 5, true>",
                  5: "k_vertex_blk<double, double, 8, 3, 6, 2, 4, true>"}
KERNEL_SOURCES = ("csrc/kernels.hpp", "csrc/batch.hpp", "csrc/adjoint.hpp", "csrc/runtime.hip", "build.py")


def source_hash():
    """Hash of every source and build file the device code is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2102_12933_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, N, reorder, grid):
    """HBM bytes per launch of `kernel` at grid size `grid` (threads) from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    sources; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash() or d.get("N") != N or d.get("reorder") != reorder:
        return None
    k = d.get("kernels", {}).get(kernel, {}).get(str(grid))
    return None if k is None else k.get("bytes_per_launch")


def short_kernel_name(name):
    """'void fdu::k_x<a, b>(args...)' -> 'k_x<a, b>' (the template instance)."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    if n.startswith("fdu::"):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def _csv_rows(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(d, suffix):
    """The one rocprofv3 output file under directory d whose name ends with suffix."""
    hits = []
    for root, _, files in os.walk(d):
        hits += [os.path.join(root, f) for f in files if f.endswith(suffix)]
    if len(hits) != 1:
        raise SystemExit(f"expected one *{suffix} under {d}, found {len(hits)}")
    return hits[0]


def counter_medians(d):
    """{(kernel, grid size): {counter: (dispatches, median value per dispatch)}}
    from a rocprofv3 --pmc output directory (csv): the same kernel runs on
    several workloads, told apart by their grid sizes."""
    import numpy as np
    per = {}
    for r in _csv_rows(_find(d, "_counter_collection.csv")):
        k = (short_kernel_name(r["Kernel_Name"]), int(r["Grid_Size"]))
        per.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: {c: (len(v), float(np.median(v))) for c, v in cs.items()} for k, cs in per.items()}


def summarize(kind, dirs, N=1025, reorder=2):
    """Markdown summaries of rocprofv3 csv outputs for profiles/ (trace: kernel
    statistics; counters: per-kernel medians; traffic: FETCH_SIZE and
    WRITE_SIZE scaled by the same counters on the 512 MiB calibration copies,
    also written to profiles/hbm_traffic.json for the roofline's traffic)."""
    import numpy as np
    out = []
    if kind == "trace":
        # one row per (kernel, grid size): the same kernel runs on several workloads
        rows = _csv_rows(_find(dirs[0], "_kernel_trace.csv"))
        groups, total = {}, 0.0
        for r in rows:
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            total += d
            key = (short_kernel_name(r["Kernel_Name"]), int(r["Grid_Size_X"]))
            groups.setdefault(key, []).append(d)
        out += ["| kernel | grid (threads) | calls | avg (us) | median (us) | min (us) | max (us) | share of GPU time |",
                "|---|---|---|---|---|---|---|---|"]
        rest = 0.0
        for (k, g), ds in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
            share = 100.0 * sum(ds) / total
            if not k.startswith("k_") or share < 0.1:
                rest += share
                continue
            out.append(f"| `{k}` | {g} | {len(ds)} | {np.mean(ds):.1f} | {np.median(ds):.1f} | {min(ds):.1f} | "
                       f"{max(ds):.1f} | {share:.1f}% |")
        out += ["", f"Launches below 0.1% of GPU time each and non-library kernels (torch fills and copies, the HIP "
                    f"runtime's buffer copies): {rest:.1f}% of GPU time together."]
    elif kind == "counters":
        med = {}
        for d in dirs:
            for k, cs in counter_medians(d).items():
                med.setdefault(k, {}).update(cs)
        names = sorted({c for cs in med.values() for c in cs})
        out += ["| kernel | grid (threads) | dispatches | " + " | ".join(names) + " |", "|---" * (len(names) + 3) + "|"]
        for k in sorted(med):
            if not k[0].startswith("k_"):
                continue
            disp = max(n for n, _ in med[k].values())
            out.append(f"| `{k[0]}` | {k[1]} | {disp} | " + " | ".join(
                f"{med[k][c][1]:.4g}" if c in med[k] else "" for c in names) + " |")
    elif kind == "traffic":
        fetch, write = counter_medians(dirs[0]), counter_medians(dirs[1])
        copy = 512 * 1024 * 1024
        calib = {}
        for label, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
            # the calibration copies are the run's last three dispatches (bench.py --calib-copy)
            rows = _csv_rows(_find(dirs[0 if label == "fetch" else 1], "_counter_collection.csv"))
            rows = sorted((r for r in rows if r["Counter_Name"] == counter), key=lambda r: int(r["Dispatch_Id"]))[-3:]
            if len(rows) < 3 or not all("copyBuffer" in r["Kernel_Name"] for r in rows):
                raise SystemExit(f"the {label} run does not end with the calibration copies (bench.py --calib-copy)")
            calib[label] = float(np.median([float(r["Counter_Value"]) for r in rows]))
        ff, wf = copy / 1024.0 / calib["fetch"], copy / 1024.0 / calib["write"]
        kern = {}
        for k in sorted(set(fetch) & set(write)):
            if not k[0].startswith("k_"):
                continue
            n, fk = fetch[k]["FETCH_SIZE"]
            _, wk = write[k]["WRITE_SIZE"]
            kern.setdefault(k[0], {})[str(k[1])] = dict(dispatches=n, fetch_kib=fk, write_kib=wk,
                                                        bytes_per_launch=int(round((fk * ff + wk * wf) * 1024)))
        doc = dict(source_hash=source_hash(), N=N, reorder=reorder,
                   calibration=dict(copy_bytes=copy, fetch_kib_read=calib["fetch"], write_kib_read=calib["write"],
                                    fetch_factor=round(ff, 4), write_factor=round(wf, 4)),
                   kernels=kern)
        with open(os.path.join(ROOT, "profiles", "hbm_traffic.json"), "w") as fh:
            json.dump(doc, fh, indent=1)
        out += [f"Calibration: the 512 MiB copy reads FETCH_SIZE = {calib['fetch']:.0f} KiB and WRITE_SIZE = "
                f"{calib['write']:.0f} KiB, so FETCH_SIZE is scaled by {ff:.3f} and WRITE_SIZE by {wf:.3f}.", "",
                "| kernel | grid (threads) | dispatches | FETCH_SIZE (KiB, median) | WRITE_SIZE (KiB, median) | "
                "HBM MB per launch (scaled) |", "|---|---|---|---|---|---|"]
        for k, per_grid in kern.items():
            for g, v in per_grid.items():
                out.append(f"| `{k}` | {g} | {v['dispatches']} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | "
                           f"{v['bytes_per_launch'] / 1e6:.1f} |")
    else:
        raise SystemExit("summarize: trace, counters or traffic")
    return "\n".join(out)


def cpu_baseline(mesh, w_input, budget_s=15.0, patch=48):
    """Oracle stage timing on a bounded sample: a patch x patch block of real
    vertices around the domain centre (the oracle computes their residual, i.e.
    the fluxes of every edge their stencils use, and the stage update)."""
    import numpy as np
    import torch
    from oracle.solver import Oracle

    N = mesh.N
    c = N // 2
    ii, jj = np.meshgrid(np.arange(c - patch // 2, c + patch // 2), np.arange(c - patch // 2, c + patch // 2),
                         indexing="ij")
    sample = (ii * N + jj).ravel()
    o = Oracle(mesh, deg=5, vertices=sample)
    w = torch.from_numpy(w_input)
    wn = w[sample].clone()
    o.residual(w)                               # warm-up
    n, t0 = 0, time.perf_counter()
    while True:
        R = o.residual(w)
        _ = 0.75 * wn + 0.25 * (w[sample] + 1e-4 * R)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s and n >= 2:
            break
    return dict(value=len(sample) * n / el, unit="vertex-stage/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{len(sample)} real vertices ({patch}x{patch} block at the domain centre) of the same "
                       f"1025^2 workload, {n} residual+stage evaluations on the state after one GPU step, "
                       f"{el:.1f} s")


def _oracle_stage_rate(mesh, deg, sample, reps=5, vjp=False, **kw):
    """Oracle residual + stage update (or, with vjp, the residual's VJP) of the
    sampled real vertices: median time of `reps` evaluations after one warm-up
    (the oracle's set-up, stencils and weights, is not timed)."""
    import numpy as np
    import torch
    from oracle.solver import Oracle
    from paper_2102_12933_amd.inputs import vortex_state

    o = Oracle(mesh, deg=deg, vertices=None if sample is None else sample, **kw)
    w = torch.from_numpy(vortex_state(mesh, beta=5.0, mach=0.5))
    verts = np.arange(mesh.nv_real) if sample is None else sample
    wn = w[verts].clone()
    Rbar = torch.ones(len(verts), 4, dtype=torch.float64)

    def unit():
        if vjp:
            o.residual_vjp(w, Rbar)
        else:
            R = o.residual(w)
            _ = 0.75 * wn + 0.25 * (w[verts] + 1e-4 * R)

    unit()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        unit()
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    return dict(vertices=int(len(verts)), s_per_stage=round(t, 5), vertex_stage_per_s=round(len(verts) / t, 1))


def oracle_config_timings(log, max_sample=4096):
    """The oracle timed on the host for the vortex workloads (accuracy study
    sizes, batch instances, adjoint), one RK stage per timed unit; meshes above
    max_sample real vertices are timed on a max_sample-vertex block of
    consecutive lattice rows around the vortex centre."""
    import numpy as np
    import torch
    from paper_2102_12933_amd.inputs import batch_specs, make_mesh

    def sample_of(m):
        if m.nv_real <= max_sample:
            return None
        N = m.N
        rows = max(1, max_sample // N)
        i0 = N // 2 - rows // 2
        return np.arange(i0 * N, (i0 + rows) * N)

    out = dict(cores=torch.get_num_threads(), kind="oracle", unit="vertex-stage/s", configs={})
    m = make_mesh(33, L=10.0, periodic=True, seed=0)
    out["configs"]["vortex 33^2, degree 3 one-level (10 steps)"] = _oracle_stage_rate(m, 3, None)
    log(f"oracle timing: 33^2 done")
    for N in (65, 129, 257, 513):
        m = make_mesh(N, L=10.0, periodic=True, seed=0)
        for deg in (3, 5):
            out["configs"][f"vortex {N}^2, degree {deg}"] = _oracle_stage_rate(m, deg, sample_of(m))
        log(f"oracle timing: {N}^2 done")
    specs = batch_specs(n=64)
    tot_v, tot_t = 0, 0.0
    for sp in specs[:4]:
        m = make_mesh(sp["N"], L=10.0, periodic=True, seed=sp["seed"])
        r = _oracle_stage_rate(m, 5, sample_of(m))
        tot_v += r["vertices"]
        tot_t += r["s_per_stage"]
    out["configs"]["batch, instances 0-3 (degree 5)"] = dict(vertices=tot_v, s_per_stage=round(tot_t, 5),
                                                            vertex_stage_per_s=round(tot_v / tot_t, 1))
    log("oracle timing: batch instances done")
    m = make_mesh(257, L=10.0, periodic=True, seed=0)
    out["configs"]["adjoint 257^2 forward stage (eps 1e-6)"] = _oracle_stage_rate(m, 5, sample_of(m), weno_eps=1e-6)
    out["configs"]["adjoint 257^2 residual VJP (autograd, eps 1e-6)"] = _oracle_stage_rate(m, 5, sample_of(m),
                                                                                          vjp=True, weno_eps=1e-6)
    log("oracle timing: adjoint done")
    return out


def fallback_edges(prep, solver, states):
    """Edges whose flux the positivity fallback changes, per stage input of one
    step: the flux arrays of the solver and of a twin without the fallback
    (same kernel variant, same arithmetic otherwise) are compared row by row;
    a row differs only where an interpolated midpoint state was not physical."""
    import torch
    from paper_2102_12933_amd import fdu

    twin = fdu.Solver(prep, device=0, positivity=0)
    v = solver.variants()
    twin.set_variants(v["edge"], v["vertex"])
    counts = []
    for w in states:
        a = solver.edge_fluxes(w)
        b = twin.edge_fluxes(w)
        counts.append(int((~((a == b).all(1))).sum().item()))
    del twin
    return counts


def bench_chained(N, steps, cfl, log):
    """Chained SSP-RK3 steps of the rotated Sod problem with walls on the regular
    diagonalized N x N mesh (no jitter, uniform diagonals): the configuration on
    which the scheme runs a long chain (on jittered random-diagonal meshes the
    least-squares divergence has growing modes).  dt from the CFL condition on
    the device every step; the state is checked at the end."""
    import numpy as np
    import torch
    from paper_2102_12933_amd import fdu
    from paper_2102_12933_amd.inputs import make_mesh, sod_state

    m = make_mesh(N, L=1.0, periodic=False, jitter=0.0, diag="uniform", seed=0, ghost_layers=4)
    prep = fdu.Prep(m, deg=5, level=0, reorder=2)
    A = prep.arrays()
    s = fdu.Solver(prep, device=0)
    w0 = torch.from_numpy(np.ascontiguousarray(sod_state(m)[A["perm"]])).cuda()
    w = w0.clone()
    scratch = torch.empty(2 * s.nv_total, 4, dtype=torch.float64, device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    s.fill_ghosts(w)
    s.autotune(w, reps=10)
    for _ in range(5):                                   # warm-up on a copy
        s.rk_step(w, scratch, dt, cfl=cfl)
    w.copy_(w0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.rk_step(w, scratch, dt, cfl=cfl)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nbad, _ = s.check_state(w)
    log(f"chained: {steps} steps on the regular {N}^2 mesh in {el * 1e3:.1f} ms, non-physical rows {nbad}")
    return dict(workload=f"rotated Sod, regular {N}x{N} diagonalized mesh with walls, {steps} chained SSP-RK3 "
                         f"steps at CFL {cfl} (dt from the CFL condition each step)",
                nv_real=int(A["nv_real"]), nnz_v=int(A["nnz_v"]), nnz_e=int(A["nnz_e"]), steps=steps,
                ms_per_step=round(el / steps * 1e3, 4), vertex_stage_per_s=A["nv_real"] * 3 * steps / el,
                non_physical_rows=int(nbad), variants=list(s.variants().values())[:2])


def bench_batched(n_inst, steps, cfl, edge_variant, vertex_variant, log, graph=True):
    """Batched vortex workload: n_inst instances (N ~ U{65..513}, strength ~ U[2,6],
    Mach ~ U[0.3,0.8]), `steps` SSP-RK3 steps captured in one HIP graph, for each
    schedule; the plain per-instance path is schedule 2 (every instance's own
    kernels in turn) in the same kind of graph."""
    import numpy as np
    import torch
    from paper_2102_12933_amd import fdu
    from paper_2102_12933_amd.inputs import batch_specs, make_mesh, vortex_state
    from paper_2102_12933_amd.tuning import autotune_batch

    t0 = time.perf_counter()
    specs = batch_specs(n=n_inst)
    solvers, w0s = [], []
    for i, sp in enumerate(specs):
        m = make_mesh(sp["N"], L=10.0, periodic=True, seed=sp["seed"])
        prep = fdu.Prep(m, deg=5, reorder=2)
        perm = prep.arrays()["perm"]
        s = fdu.Solver(prep, device=0)
        s.set_variants(edge_variant, vertex_variant)       # used by the per-instance schedule
        solvers.append(s)
        w0s.append(torch.from_numpy(np.ascontiguousarray(vortex_state(m, beta=sp["beta"], mach=sp["mach"])[perm])).cuda())
        if (i + 1) % 16 == 0:
            log(f"batch: {i + 1}/{n_inst} instances prepared ({time.perf_counter() - t0:.0f} s)")
    nv = sum(s.nv_real for s in solvers)
    b = fdu.Batch(solvers)
    ws = [w.clone() for w in w0s]
    scr = [torch.empty(2 * s.nv_total, 4, dtype=torch.float64, device="cuda") for s in solvers]
    b.set_states(ws, scr)
    best, tune_ms = autotune_batch(b, cfl, use_cache=False)
    b.set_schedule(*best)
    log(f"batch autotune: best {best}; " + ", ".join(f"{k}: {v:.2f} ms" for k, v in tune_ms.items()))
    side = torch.cuda.Stream()
    res = {}
    def best_of(sched):
        c = {k: v for k, v in tune_ms.items() if k[0] == sched}
        return min(c, key=c.get)

    for label, cand in [("per_instance", best_of(2)), ("per_phase", best_of(1)), ("persistent", best_of(0))]:
        b.set_schedule(*cand)
        for w, w0 in zip(ws, w0s):
            w.copy_(w0)
        torch.cuda.synchronize()
        if graph:
            with torch.cuda.stream(side):
                b.capture(cfl, steps)
                b.launch()                      # warm-up replay
            side.synchronize()
        else:
            b.step(cfl)
        for w, w0 in zip(ws, w0s):
            w.copy_(w0)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        with torch.cuda.stream(side):
            if graph:
                b.launch()
            else:
                for _ in range(steps):
                    b.step(cfl)
        side.synchronize()
        el = time.perf_counter() - tt
        err, dts = b.status()
        ok = err == 0 and all(bool(torch.isfinite(w).all()) for w in ws)
        res[label] = dict(schedule=list(cand), ms_per_step=round(el / steps * 1e3, 4),
                          vertex_stage_per_s=nv * 3 * steps / el, wait_timeouts=err, finite=ok)
        log(f"batch {label} {cand}: {el / steps * 1e3:.3f} ms/step, {nv * 3 * steps / el:.3e} vertex-stage/s")
    return dict(instances=n_inst, vertices=int(nv), steps=steps, cfl=cfl, graph=graph,
                best_batched=max(("per_phase", "persistent"), key=lambda k: res[k]["vertex_stage_per_s"]),
                speedup_vs_per_instance=round(max(res["per_phase"]["vertex_stage_per_s"],
                                                  res["persistent"]["vertex_stage_per_s"]) /
                                              res["per_instance"]["vertex_stage_per_s"], 3),
                schedules=res, autotune_ms={",".join(map(str, k)): round(v, 4) for k, v in tune_ms.items()})


def bench_fp32(prep, A, w0_f64, steps, cfl, log):
    """The headline workload in FP32 storage (state, geometry and weights in
    FP32, arithmetic and edge fluxes in FP64): the same non-chained steps."""
    import torch
    from paper_2102_12933_amd import fdu

    s = fdu.Solver(prep, device=0, precision="f32")
    w0 = w0_f64.float()
    w1, w2, w3 = (torch.empty_like(w0) for _ in range(3))
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    s.fill_ghosts(w0)
    tune = s.autotune(w0, reps=10)

    def step():
        s.cfl_dt(w0, cfl, dt)
        s.rk_stage(0, w0, w0, w1, dt)
        s.rk_stage(1, w0, w1, w2, dt)
        s.rk_stage(2, w0, w2, w3, dt)

    for _ in range(5):
        step()
    torch.cuda.synchronize()
    s.kernel_timer_start(capacity=3 * steps + 8, phases=("edge", "vertex"))
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt, _ = s.kernel_timer_stop()
    ok = bool(torch.isfinite(w3[:A["nv_real"]]).all())
    log(f"fp32 storage: {el / steps * 1e3:.3f} ms/step, vertex {kt['vertex'] * 1e3:.1f} us, edge {kt['edge'] * 1e3:.1f} us")
    return dict(ms_per_step=round(el / steps * 1e3, 4), vertex_stage_per_s=A["nv_real"] * 3 * steps / el,
                vertex_ms=round(kt["vertex"], 5), edge_ms=round(kt["edge"], 5), finite=ok,
                variants=[tune["edge"], tune["vertex"]])


def bench_adjoint(N, nsteps, ckpt, log):
    """Unrolled-gradient workload: vortex on an N^2 jittered periodic mesh, nsteps
    SSP-RK3 steps at the t = 0 CFL-0.5 time step, checkpoints every ckpt steps,
    gradient of sum_v A_v (p_v / rho_v^gamma - 1) with respect to the initial
    state.  WENO eps = 1e-6 (differentiable weights)."""
    import numpy as np
    import torch
    from paper_2102_12933_amd import fdu
    from paper_2102_12933_amd.autograd import rk_unroll
    from paper_2102_12933_amd.inputs import make_mesh, vertex_areas, vortex_state

    m = make_mesh(N, L=10.0, periodic=True, seed=0)
    prep = fdu.Prep(m, deg=5, reorder=2)
    perm = prep.arrays()["perm"]
    s = fdu.Solver(prep, device=0, weno_eps=1e-6)
    s.enable_adjoint()
    w0 = torch.from_numpy(np.ascontiguousarray(vortex_state(m, beta=5.0, mach=0.5)[perm])).cuda()
    dt = float(s.cfl_dt(w0, 0.5).item())
    A = torch.from_numpy(vertex_areas(m)[perm][:m.nv_real]).cuda()

    def J(w):
        wr = w[:m.nv_real]
        rho = wr[:, 0]
        p = 0.4 * (wr[:, 3] - 0.5 * (wr[:, 1] ** 2 + wr[:, 2] ** 2) / rho)
        return torch.sum(A * (p / rho ** 1.4 - 1.0))

    def fwd():
        with torch.no_grad():
            return J(rk_unroll(s, w0, nsteps, dt, ckpt))

    def fwd_bwd():
        x = w0.clone().requires_grad_(True)
        val = J(rk_unroll(s, x, nsteps, dt, ckpt))
        (g,) = torch.autograd.grad(val, x)
        return g

    fwd(); fwd_bwd()
    torch.cuda.synchronize()
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        fwd()
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):
        g = fwd_bwd()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t) / reps
    vs = m.nv_real * 3 * nsteps
    log(f"adjoint {N}^2: forward {tf * 1e3:.1f} ms, forward+backward {tb * 1e3:.1f} ms")
    return dict(workload=f"vortex {N}x{N} jittered periodic, {nsteps} SSP-RK3 steps, checkpoints every {ckpt}",
                vertices=int(m.nv_real), forward_ms=round(tf * 1e3, 3), forward_backward_ms=round(tb * 1e3, 3),
                ratio=round(tb / tf, 3), forward_vertex_stage_per_s=vs / tf, gradient_vertex_stage_per_s=vs / tb,
                grad_finite=bool(torch.isfinite(g).all()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--N", type=int, default=1025)
    ap.add_argument("--reorder", type=int, default=2, help="0 natural, 1 RCM, 2 Hilbert (default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=30)
    ap.add_argument("--cfl", type=float, default=SOD_CFL)
    ap.add_argument("--batch-instances", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-batch-graph", action="store_true", help="batched steps eagerly, not from a HIP graph")
    ap.add_argument("--adjoint-N", type=int, default=257)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-chained", action="store_true")
    ap.add_argument("--variants", type=int, nargs=2, metavar=("EDGE", "VERTEX"), default=None,
                    help="use these kernel variants instead of autotuning (profiling runs)")
    ap.add_argument("--summarize", nargs="+", metavar=("KIND", "DIR"),
                    help="print a profiles/ summary of rocprofv3 csv output: trace DIR | counters DIR... | "
                         "traffic FETCH_DIR WRITE_DIR (also writes profiles/hbm_traffic.json); no GPU")
    ap.add_argument("--oracle-configs", action="store_true",
                    help="only time the oracle on the host for the vortex, batch and adjoint workloads (no GPU)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the run, copy a 512 MiB buffer 3 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.summarize:
        print(summarize(args.summarize[0], args.summarize[1:], args.N, args.reorder))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.oracle_configs:
        print(json.dumps(oracle_config_timings(log)), flush=True)
        return

    from paper_2102_12933_amd import fdu
    from paper_2102_12933_amd.inputs import make_mesh, sod_state

    t = time.perf_counter()
    mesh = make_mesh(args.N, L=1.0, periodic=False, jitter=0.15, seed=0, ghost_layers=4)
    log(f"mesh {args.N}^2: {mesh.nv_real} real + {mesh.ng} ghost vertices, {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    prep = fdu.Prep(mesh, deg=5, level=0, reorder=args.reorder)
    A = prep.arrays()
    log(f"prep: {A['ne_flux']} flux edges, {A['nnz_v'] / A['nv_real']:.2f}+{A['nnz_e'] / A['nv_real']:.2f} "
        f"stencil entries per vertex, {time.perf_counter() - t:.1f} s")
    solver = fdu.Solver(prep, device=0)
    perm = A["perm"]
    w0 = torch.from_numpy(np.ascontiguousarray(sod_state(mesh)[perm])).cuda()
    w1, w2, w3 = (torch.empty_like(w0) for _ in range(3))
    dt = torch.empty(1, dtype=torch.float64, device="cuda")

    solver.fill_ghosts(w0)
    if args.variants is None:
        tune = solver.autotune(w0, reps=args.kernel_reps)
        log(f"autotune: edge variants {['%.1f us' % (t * 1e3) for t in tune['edge_ms']]} -> {tune['edge']}, "
            f"vertex variants {['%.1f us' % (t * 1e3) for t in tune['vertex_ms']]} -> {tune['vertex']}")
    else:
        solver.set_variants(*args.variants)
        tune = dict(edge=args.variants[0], vertex=args.variants[1], edge_ms=[], vertex_ms=[])
        log(f"variants given: edge {tune['edge']}, vertex {tune['vertex']}")

    # the small kernels (ghost fill, CFL reduction) are timed back to back here, outside the timed region
    small = solver.kernel_times(w0, reps=args.kernel_reps)

    def step():
        solver.cfl_dt(w0, args.cfl, dt)
        solver.rk_stage(0, w0, w0, w1, dt)
        solver.rk_stage(1, w0, w1, w2, dt)
        solver.rk_stage(2, w0, w2, w3, dt)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # Every launch of the dominant kernel (the longer of the edge flux and the vertex step in the
    # back-to-back times above; the roofline's kernel) in the timed region is bracketed by
    # timing-only HIP events on its stream.  The other one is timed the same way in a separate,
    # untimed run of the same steps: its events would add about 1% to the timed region.
    dom = "vertex" if small["vertex"] >= small["edge"] else "edge"
    other = "edge" if dom == "vertex" else "vertex"
    solver.kernel_timer_start(capacity=3 * args.steps + 8, phases=(dom,))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt, kcount = solver.kernel_timer_stop()
    n_other = min(args.steps, 50)
    solver.kernel_timer_start(capacity=3 * n_other + 8, phases=(other,))
    for _ in range(n_other):
        step()
    torch.cuda.synchronize()
    kt_o, kcount_o = solver.kernel_timer_stop()
    kt[other], kcount[other] = kt_o[other], kcount_o[other]
    wr = w3[:A["nv_real"]]
    rho = wr[:, 0]
    p = 0.4 * (wr[:, 3] - 0.5 * (wr[:, 1] ** 2 + wr[:, 2] ** 2) / rho)
    state_ok = bool(torch.isfinite(wr).all()) and float(rho.min()) > 0 and float(p.min()) > 0
    log(f"state after one step: rho [{float(rho.min()):.4f}, {float(rho.max()):.4f}], "
        f"p [{float(p.min()):.4f}, {float(p.max()):.4f}], dt {float(dt.item()):.3e}")
    if not state_ok:
        raise RuntimeError("non-physical state after a step")
    log(f"timed {args.steps} steps: {el * 1e3:.2f} ms; live kernel means (ms) {kt}, launches {kcount}")
    # does the positivity fallback (not in the paper) fire in the timed step?  (untimed check)
    fallback = None
    if solver.params["positivity"]:
        fallback = fallback_edges(prep, solver, (w0, w1, w2))
        log(f"positivity fallback: edges changed per stage input {fallback}")

    # the same steps captured in one HIP graph (launch gaps removed); reported beside the headline
    graph = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(args.steps):
                step()
        g.replay()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        elg = time.perf_counter() - tg
        graph = dict(ms_per_step=round(elg / args.steps * 1e3, 4),
                     vertex_stage_per_s=A["nv_real"] * 3 * args.steps / elg)
        log(f"graph replay of {args.steps} steps: {elg * 1e3:.2f} ms")
        del g

    blocks = solver.vertex_block_info() if tune["vertex"] in BLOCK_VERTEX_VARIANTS else None
    packed = entries_past_first_round(A) if tune["vertex"] in PACKED_VERTEX_VARIANTS else None
    nb = kernel_bytes(A, blocks=blocks, packed=packed, wn_stages=2)
    # the roofline's algorithmic bytes: the blueprint's per-vertex-stage figure
    # (int32 ids, every datum once) times the real vertices one launch updates
    per_unit = dict(vertex=survey_bytes_per_vertex_stage(A, 8, wn_stages=2),
                    edge=survey_edge_bytes_per_vertex_stage(A, 8))
    kern = {}
    for k in ("edge", "vertex"):
        ms = kt[k]
        kern[k] = dict(avg_ms=ms, launches=kcount[k], bytes=nb[k], gbs=nb[k] / (ms * 1e-3) / 1e9)
    names = dict(edge=EDGE_KERNELS[tune["edge"]], vertex=VERTEX_KERNELS[tune["vertex"]])
    grids = dict(edge=-(-A["ne_flux"] // 256) * 256,
                 vertex=(blocks["n_blocks"] * 256 if blocks is not None
                         else -(-A["nv_real"] * {0: 16, 1: 8, 2: 8}.get(tune["vertex"], 8) // 256) * 256))
    traffic = traffic_from_profiles(names[dom], args.N, args.reorder, grids[dom])
    alg_bytes = per_unit[dom] * A["nv_real"]
    achieved = alg_bytes / (kt[dom] * 1e-3) / 1e9
    # context for the roof: what a plain 1 GiB device-to-device copy reaches on this GPU
    # (skipped in counter-calibration runs, whose only large copies must be the 512 MiB ones)
    copy_gbs = read_gbs = None
    if not args.calib_copy:
        src = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        e1.synchronize()
        copy_gbs = round(2 * src.numel() * 8 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        # and a read-only stream over the same 1 GiB (torch's sum): the vertex step is 97% reads
        acc = src.sum()
        e0.record()
        for _ in range(5):
            acc = src.sum()
        e1.record()
        e1.synchronize()
        read_gbs = round(src.numel() * 8 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        del src, dst, acc
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel=names[dom], variant=tune[dom], avg_ms=round(kt[dom], 5), launches=kcount[dom],
                    algorithmic_bytes=round(alg_bytes), bytes_per_vertex_stage=round(per_unit[dom], 1),
                    units_per_launch=int(A["nv_real"]),
                    stored_bytes=round(nb[dom]), stored_gbs=round(kern[dom]["gbs"], 1),
                    stored_frac=round(kern[dom]["gbs"] / HBM_PEAK_GBS, 4),
                    timing=f"timing-only HIP events around every {dom} launch in the timed region",
                    other_kernel_timing=f"{other}: the same events in a separate run of {n_other} of the same steps",
                    copy_gbs=copy_gbs, read_gbs=read_gbs,
                    traffic_gbs=(round(traffic / (kt[dom] * 1e-3) / 1e9, 1) if traffic else None))
    nv_real = A["nv_real"]
    value = nv_real * 3 * args.steps / el
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "vertex-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"rotated Sod, jittered {args.N}x{args.N} triangulation of [0,1]^2 with 4-deep mirror "
                               f"ghosts, NU-WENO5 + degree-5 two-level LS, one SSP-RK3 step (CFL {args.cfl}) from "
                               f"the initial state per timed step",
                   "nv_real": int(nv_real), "ne_flux": int(A["ne_flux"]), "nnz_v": int(A["nnz_v"]),
                   "nnz_e": int(A["nnz_e"]), "reorder": ["natural", "rcm", "hilbert"][args.reorder]},
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in d.items()}
                    for k, d in kern.items()} | {"ghost_ms": round(small["ghost"], 5), "cfl_ms": round(small["cfl"], 5)},
        "vertex_blocks": blocks,
        "positivity_fallback_edges": fallback,
        "graph_replay": graph,
        "autotune": {"edge_variant": tune["edge"], "vertex_variant": tune["vertex"],
                     "edge_ms": [round(t, 5) for t in tune["edge_ms"]],
                     "vertex_ms": [round(t, 5) for t in tune["vertex_ms"]]},
    }
    if not args.no_fp32:
        out["fp32_storage"] = bench_fp32(prep, A, w0, min(args.steps, 100), args.cfl, log)
    if not args.no_chained:
        out["chained_regular"] = bench_chained(args.N, args.steps, args.cfl, log)
    if not args.no_batch:
        out["batched"] = bench_batched(args.batch_instances, args.batch_steps, 0.2, tune["edge"], tune["vertex"], log,
                                       graph=not args.no_batch_graph)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(args.adjoint_N, 20, 5, log)
    if not args.no_cpu_baseline:
        w_in = np.empty((mesh.nv, 4))
        w_in[perm] = w3.cpu().numpy()
        log("cpu baseline (oracle on a bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline(mesh, w_in)
    print(json.dumps(out), flush=True)
    if args.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
