"""Benchmark of the r1-sparse hot path on one MI355X.

A step is one application of the operator pair the metric names, float64,
on the 512 x 256 mesh with L = 200 levels (m = 203), the largest of the
single-GPU configurations (the mixed-precision case and the top of the level
sweep):

    y = J x        (structured matvec kernel)
    z = M y        (SMW block-Jacobi apply kernel)

`value` is the algorithmic HBM bytes of the pair (stored structural values
plus input and output vectors, section-3 counts) per second over the timed
steps.  Per-kernel times come from HIP events on the launch stream.  The
same JSON line carries, at the same size, the float32-preconditioner pair,
the adjoint pair (J^T x, M^T y), float64 and mixed-precision GMRES solves
and the dense-block BSR baseline (on the 512 x 128 half mesh: the full one
needs 216 GB of blocks); then the 256 x 128, L = 61 workload (the pair, the
fused kernel, eight right-hand sides, the paper's pair counts, the wide
diagonal block, the physics-shaped Jacobian, a general mesh, solves), a
device copy ceiling, and the CPU oracle timed on a bounded sample of the
headline workload, which also checks the GPU solves on sampled rows.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "J*x + SMW precond apply GB/s (%HBM peak); FP32-precond & adjoint vs FP64 plain"
HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "mesh512x256_L200"
KERNEL_SOURCES = ("k_matvec.hip", "k_matvec_impl.hpp", "k_packed.hip", "k_packed_impl.hpp",
                  "k_smw.hip", "r1s_device.hpp")



def kernel_source_hash():
    """sha256 over the sources of the matvec and SMW apply kernels."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2403_09198_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counters_path(workload):
    return os.path.join(ROOT, "profiles", f"counters_pair_fp64_{workload}.json")


def counter_kind(name):
    """'matvec' / 'apply' for the structured matvec and SMW apply kernels."""
    if name.startswith("void r1s::k_matvec") and "k_matvec_prec" not in name:
        return "matvec"
    if name.startswith("void r1s::k_smw_apply"):
        return "apply"
    return None


def counter_traffic(workload, kind):
    """HBM bytes per launch of the matvec or apply kernel from the committed
    counter summary of `workload`, or None when it was taken on other kernel
    sources."""
    try:
        with open(counters_path(workload)) as f:
            c = json.load(f)
    except OSError:
        return None
    if c.get("kernel_source_sha256") != kernel_source_hash():
        return None
    for name, k in c["kernels"].items():
        if counter_kind(name) == kind:
            return {"kernel": name, "traffic_bytes": k["traffic_bytes"]}
    return None


def summarize_counters(workload, fetch_csv, write_csv):
    """Write the counter summary from the FETCH_SIZE and WRITE_SIZE runs of
    --profile-pass.  Each counter is scaled by what it reads for the 256 MiB
    device copy in the same run (268435456 bytes read and written)."""
    import csv
    import collections

    def per_kernel(path):
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            agg[r["Kernel_Name"].split("(")[0]].append(float(r["Counter_Value"]))
        return agg

    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    copy_bytes = 1 << 28
    cp = [k for k in fetch if "copyBuffer" in k or "copy" in k.lower()][0]
    ff = copy_bytes / (max(fetch[cp]) * 1024)
    wf = copy_bytes / (max(write[cp]) * 1024)
    out = {"workload": workload, "kernel_source_sha256": kernel_source_hash(),
           "fetch_factor": round(ff, 4), "write_factor": round(wf, 4), "calibration_kernel": cp,
           "commands": [
               "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv "
               f"-d <out>/pmc_fetch -o fetch -- python3 <repo>/bench.py --workload {workload} "
               "--profile-pass",
               "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv "
               f"-d <out>/pmc_write -o write -- python3 <repo>/bench.py --workload {workload} "
               "--profile-pass",
               f"python bench.py --workload {workload} --summarize-counters <fetch csv> "
               "<write csv>"],
           "kernels": {}}
    for name in fetch:
        if counter_kind(name) is None:
            continue
        fk = sum(fetch[name]) / len(fetch[name])
        wk = sum(write[name]) / len(write[name])
        out["kernels"][name] = {"fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                                "dispatches": len(fetch[name]),
                                "traffic_bytes": int(fk * 1024 * ff + wk * 1024 * wf)}
    with open(counters_path(workload), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pair_bytes(N, B, m, nrhs=1, value_bytes=8):
    """Algorithmic bytes of one matvec and one SMW apply (values + vectors)."""
    struct_vals = N * (3 * m - 2) + (B - N) * m + 2 * B * m
    mv = value_bytes * struct_vals + 8 * 2 * nrhs * N * m
    ap = value_bytes * N * (5 * m - 1) + 8 * 2 * nrhs * N * m
    return mv, ap


def bsr_pair_bytes(N, B, m):
    return 8 * B * m * m + 8 * 2 * N * m, 8 * N * m * m + 8 * 2 * N * m


def time_pair(torch, f1, f2, steps, warmup, flush=None):
    """Run f1; f2 `steps` times after `warmup`; returns (wall s, ev1 ms list, ev2 ms list)."""
    for _ in range(warmup):
        f1()
        f2()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1, e2 in evs:
        if flush is not None:
            flush()
        e0.record()
        f1()
        e1.record()
        f2()
        e2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t1 = [a.elapsed_time(b) for a, b, _ in evs]
    t2 = [b.elapsed_time(c) for _, b, c in evs]
    return wall, t1, t2


def ceilings(torch, A, M, x, y, z, mv_b, ap_b, reps=20):
    """Context for the roofline: a device-to-device copy of 1 GiB (torch's
    copy kernel; read + written bytes per second) and the matvec / SMW apply
    timed cold, a 512 MiB buffer written before every pair so that neither
    the L2s nor the 256 MiB Infinity Cache hold any of their inputs."""
    src = torch.empty(1 << 27, dtype=torch.float64, device=x.device)
    src.fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    scratch = torch.empty(1 << 26, dtype=torch.float64, device=x.device)
    _, t1, t2 = time_pair(torch, lambda: A.matvec(x, out=y), lambda: M.apply(y, out=z), reps, 3,
                          flush=lambda: scratch.fill_(0.0))
    del scratch
    mv_ms, ap_ms = float(np.median(t1)), float(np.median(t2))
    return {"stream_copy_gbs": round(copy_gbs, 1),
            "cold": {"matvec_us": round(mv_ms * 1e3, 2), "smw_apply_us": round(ap_ms * 1e3, 2),
                     "matvec_gbs": round(mv_b / (mv_ms / 1e3) / 1e9, 1),
                     "smw_apply_gbs": round(ap_b / (ap_ms / 1e3) / 1e9, 1),
                     "note": "median of %d, a 512 MiB buffer written before each pair" % reps}}


def capture(torch, fn):
    """Capture fn's launches (on torch's current stream) into a HIP graph."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


SOLVE_REPS = 5  # GMRES solves averaged per reported solve time (after a warm one)

# Steps per captured graph: consecutive steps replayed from one graph avoid
# the launch gap between graph replays (every step still launches its
# kernels and re-reads all of its data from HBM).
STEPS_PER_GRAPH = 10


def step_graphs(torch, step):
    """HIP graphs of STEPS_PER_GRAPH steps and of one step."""
    def many():
        for _ in range(STEPS_PER_GRAPH):
            step()
    return capture(torch, many), capture(torch, step)


def replay(graphs, steps):
    """Run exactly `steps` steps from the graphs of step_graphs."""
    many, one = graphs
    for _ in range(steps // STEPS_PER_GRAPH):
        many.replay()
    for _ in range(steps % STEPS_PER_GRAPH):
        one.replay()


def kernel_ms(torch, fn, reps=100):
    """Average duration of fn's single kernel: HIP events around `reps`
    back-to-back launches on the current stream."""
    for _ in range(5):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def measure_pair(torch, f1, f2, steps, warmup):
    """Graph-replayed (f1; f2) steps: wall seconds for `steps` replays, and
    the per-kernel average durations of f1 and f2 in ms (events around each
    launch of the alternating sequence)."""
    graphs = step_graphs(torch, lambda: (f1(), f2()))
    replay(graphs, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    replay(graphs, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, t1, t2 = time_pair(torch, f1, f2, steps, warmup)
    return wall, float(np.mean(t1)), float(np.mean(t2))


def measure_one(torch, f, steps, warmup):
    """Graph-replayed single-kernel steps: wall seconds for `steps` replays
    and the kernel's average duration in ms (events around each launch)."""
    graphs = step_graphs(torch, f)
    replay(graphs, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    replay(graphs, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for e0, e1 in evs:
        e0.record()
        f()
        e1.record()
    torch.cuda.synchronize()
    return wall, float(np.mean([a.elapsed_time(b) for a, b in evs]))


def profile_pass(torch, A, M, x, y, z):
    """Kernels for a counter run: 20 matvecs, 20 applies, and 5 copies of a
    256 MiB buffer (the calibration kernel of known size)."""
    for _ in range(20):
        A.matvec(x, out=y)
    for _ in range(20):
        M.apply(y, out=z)
    src = torch.ones(1 << 25, dtype=torch.float64, device=x.device)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("profile pass done: copy kernel moves %d bytes read + %d written" % (src.numel() * 8,
                                                                          src.numel() * 8))


def ranks_pair(torch, nx, ny, L, ranks, steps, warm, seed=0, band=1, arrow=False,
               physics_values=False, dra=False, explicit=False, solve=None):
    """The float64 pair with several rank-one pairs per block (the paper's
    9 / 2 structure) and optionally the wide diagonal-block pattern;
    algorithmic bytes from the library's storage counts.  physics_values:
    the HLL finite-volume Jacobian of a multi-species gas (8 / 6 pairs,
    level/flow coupling; with dra also the DRa source, arrow = 2) in place of
    random values; explicit: the same Jacobian given as a general pattern of
    the diagonal block (the layout written out entry by entry); solve =
    (restart, rtol) adds GMRES solves of it."""
    from paper_2403_09198_amd import gen, physics, r1s

    dev = "cuda:0"
    if physics_values:
        ranks, band, arrow = (physics.R_DIAG, physics.R_OFF), 1, 2 if dra else 1
    log(f"ranks pair: mesh {nx}x{ny} L={L} ranks {ranks} band {band} arrow {arrow}"
        + (" (HLL Jacobian)" if physics_values else "") + (" as a general pattern" if explicit else ""))
    if physics_values:
        p = physics.make_problem(nx, ny, L, seed=seed, dra=dra)
    elif not explicit:
        p = gen.make_problem(nx, ny, L, seed=seed, r_diag=ranks[0], r_off=ranks[1], band=band,
                             arrow=arrow)
    if explicit:
        # the layout's pattern written out entry by entry, values drawn for it
        ip, ix = gen.layout_pattern(L, band, arrow)
        p = gen.make_pattern_problem(nx, ny, L, ip, ix, seed=seed, r_diag=ranks[0],
                                     r_off=ranks[1])
        vals = {k: torch.from_numpy(p[k]).to(dev) for k in gen.PATTERN_PROBLEM_FIELDS}
        del p
        A = r1s.R1PatternMatrix(nx, ny, L, (ip, ix), vals, keep_f32=True, ranks=ranks)
    else:
        keys = gen.FIELDS + tuple(k for k in gen.PATTERN_FIELDS if k in p)
        vals = {k: torch.from_numpy(p[k]).to(dev) for k in keys}
        del p
        A = r1s.R1Matrix(nx, ny, L, vals, keep_f32=True, ranks=ranks, band=band, arrow=arrow)
    del vals
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    t_setup = time.perf_counter() - t0
    # again, as a Newton step would (the first includes loading the setup
    # kernels and growing the allocator's pool)
    t0 = time.perf_counter()
    M2 = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    t_setup2 = time.perf_counter() - t0
    del M2
    st = A.storage()
    mv, ap = st["matvec_bytes"], st["smw_apply_bytes"]
    x = torch.from_numpy(gen.make_vector(nx, ny, L, seed=0)).to(dev)
    y, z = torch.empty_like(x), torch.empty_like(x)
    N = nx * ny
    row = {"r_diag": ranks[0], "r_off": ranks[1], "band": band, "arrow": int(arrow),
           "explicit_pattern": bool(explicit),
           "stored_values": st["structured_values"],
           "smw_setup_ms": round(t_setup * 1e3, 2),
           "smw_setup_repeat_ms": round(t_setup2 * 1e3, 2)}
    for tag, f1, f2, vb in (
            ("f64", lambda: A.matvec(x, out=y), lambda: M.apply(y, out=z), 8),
            ("f32", lambda: A.matvec(x, out=y, precision="f32"),
             lambda: M.apply(y, out=z, precision="f32"), 4),
            ("adjoint", lambda: A.matvec(x, out=y, trans=True),
             lambda: M.apply(y, out=z, trans=True), 8)):
        # float32 values halve the matrix-side bytes; vectors stay float64
        vec_b = 8 * 2 * N * (L + 3)
        nbytes = (mv - vec_b) * vb // 8 + vec_b + (ap - vec_b) * vb // 8 + vec_b
        wall, k1, k2 = measure_pair(torch, f1, f2, steps, warm)
        row[tag] = {"gbs": round(nbytes / (wall / steps) / 1e9, 1),
                    "us_per_step": round(wall / steps * 1e6, 2),
                    "matvec_us": round(k1 * 1e3, 2), "apply_us": round(k2 * 1e3, 2),
                    "matvec_gbs": round(((mv - vec_b) * vb // 8 + vec_b) / (k1 / 1e3) / 1e9, 1),
                    "apply_gbs": round(((ap - vec_b) * vb // 8 + vec_b) / (k2 / 1e3) / 1e9, 1)}
    if solve is not None:
        b = torch.from_numpy(gen.make_rhs(nx, ny, L, seed=seed)).to(dev)
        for mode in ("f64", "mixed"):
            r1s.gmres(A, M, b, restart=solve[0], rtol=solve[1], mode=mode)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(SOLVE_REPS):
                res = r1s.gmres(A, M, b, restart=solve[0], rtol=solve[1], mode=mode)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / SOLVE_REPS
            row[f"solve_{mode}"] = {"ms": round(el * 1e3, 2), "iters": res.stats[0]["iters"],
                                    "outer": res.stats[0]["outer"],
                                    "rel_residual": res.stats[0]["rel_residual"]}
        del b
    del A, M, x, y, z
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return row


def mesh_pair(torch, n_points, L, ranks, steps, warm, shuffle=True, seed=0):
    """The float64 pair on a general mesh: a Delaunay triangulation of
    n_points random points (every triangle a cell, at most 3 neighbours),
    cell numbering shuffled unless shuffle is False."""
    from paper_2403_09198_amd import gen, r1s

    dev = "cuda:0"
    ip, ix = gen.delaunay_graph(n_points, seed=seed, shuffle=shuffle)
    N = len(ip) - 1
    log(f"mesh pair: delaunay {N} cells L={L} ranks {ranks} shuffle={shuffle}")
    p = gen.make_graph_problem(ip, ix, L, seed=seed, r_diag=ranks[0], r_off=ranks[1])
    vals = {k: torch.from_numpy(p[k]).to(dev) for k in gen.GRAPH_FIELDS}
    del p
    A = r1s.R1GraphMatrix(ip, ix, L, vals, keep_f32=True, ranks=ranks)
    del vals
    M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    st = A.storage()
    mv, ap = st["matvec_bytes"], st["smw_apply_bytes"]
    x = torch.from_numpy(np.random.default_rng(0).standard_normal((1, N, L + 3))).to(dev)
    y, z = torch.empty_like(x), torch.empty_like(x)
    row = {"cells": N, "blocks": int(st["n_blocks"]), "L": L, "r_diag": ranks[0],
           "r_off": ranks[1], "shuffled": shuffle, "index_bytes": int(st["index_bytes"])}
    for tag, f1, f2 in (("f64", lambda: A.matvec(x, out=y), lambda: M.apply(y, out=z)),
                        ("adjoint", lambda: A.matvec(x, out=y, trans=True),
                         lambda: M.apply(y, out=z, trans=True))):
        wall, k1, k2 = measure_pair(torch, f1, f2, steps, warm)
        row[tag] = {"gbs": round((mv + ap) / (wall / steps) / 1e9, 1),
                    "us_per_step": round(wall / steps * 1e6, 2),
                    "matvec_us": round(k1 * 1e3, 2), "apply_us": round(k2 * 1e3, 2),
                    "matvec_gbs": round(mv / (k1 / 1e3) / 1e9, 1)}
    del A, M, x, y, z
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return row


def sweep(torch, levels=(32, 61, 120, 200), steps=50, warm=5):
    """Level sweep on the 512 x 256 mesh: structured pairs (float64, float32,
    adjoint) against the dense-block BSR pair.  BSR storage grows as m^2, so
    for L = 200 the BSR pair runs on the 512 x 128 half mesh (130 GB) and the
    structured pair is measured there as well."""
    from paper_2403_09198_amd import gen, r1s

    dev = "cuda:0"
    rows = []
    for L in levels:
        for nx, ny, with_bsr in ((512, 256, L <= 120), (512, 128, L > 120)):
            if (nx, ny) == (512, 128) and L <= 120:
                continue
            m, N = L + 3, nx * ny
            B = 5 * N - 2 * nx - 2 * ny
            log(f"sweep: mesh {nx}x{ny} L={L}")
            p = gen.make_problem(nx, ny, L, seed=0)
            vals = {k: torch.from_numpy(p[k]).to(dev) for k in gen.FIELDS}
            del p
            A = r1s.R1Matrix(nx, ny, L, vals, keep_f32=True)
            del vals
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
            t_setup = time.perf_counter() - t0
            x = torch.from_numpy(gen.make_vector(nx, ny, L, seed=0)).to(dev)
            y, z = torch.empty_like(x), torch.empty_like(x)
            mv, ap = pair_bytes(N, B, m)
            mv32, ap32 = pair_bytes(N, B, m, value_bytes=4)
            row = {"nx": nx, "ny": ny, "L": L, "m": m, "cells": N,
                   "structured_bytes": 8 * (N * (3 * m - 2) + (B - N) * m + 2 * B * m),
                   "bsr_bytes": 8 * B * m * m, "smw_setup_ms": round(t_setup * 1e3, 2)}
            for tag, f1, f2, nbytes in (
                    ("f64", lambda: A.matvec(x, out=y), lambda: M.apply(y, out=z), mv + ap),
                    ("f32", lambda: A.matvec(x, out=y, precision="f32"),
                     lambda: M.apply(y, out=z, precision="f32"), mv32 + ap32),
                    ("adjoint", lambda: A.matvec(x, out=y, trans=True),
                     lambda: M.apply(y, out=z, trans=True), mv + ap)):
                wall, k1, k2 = measure_pair(torch, f1, f2, steps, warm)
                row[tag] = {"us_per_step": round(wall / steps * 1e6, 2),
                            "gbs": round(nbytes / (wall / steps) / 1e9, 1),
                            "matvec_us": round(k1 * 1e3, 2), "apply_us": round(k2 * 1e3, 2),
                            "cell_updates_per_s": round(N / (wall / steps), 1)}
            if with_bsr:
                try:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    Bm = r1s.BSRMatrix(A)
                    t_asm = time.perf_counter() - t0
                    t0 = time.perf_counter()
                    P = r1s.DenseLUPreconditioner(Bm)
                    t_lu = time.perf_counter() - t0
                    bmv, bap = bsr_pair_bytes(N, B, m)
                    nb = 5
                    wall, k1, k2 = measure_pair(torch, lambda: Bm.matvec(x, out=y),
                                                lambda: P.apply(y, out=z), nb, 1)
                    row["bsr"] = {"us_per_step": round(wall / nb * 1e6, 2),
                                  "gbs": round((bmv + bap) / (wall / nb) / 1e9, 1),
                                  "matvec_us": round(k1 * 1e3, 2), "lu_apply_us": round(k2 * 1e3, 2),
                                  "assemble_ms": round(t_asm * 1e3, 1),
                                  "lu_setup_ms": round(t_lu * 1e3, 1)}
                    row["speedup_structured_vs_bsr"] = round(
                        row["bsr"]["us_per_step"] / row["f64"]["us_per_step"], 2)
                    row["matvec_speedup"] = round(k1 * 1e3 / row["f64"]["matvec_us"], 2)
                    row["apply_speedup"] = round(k2 * 1e3 / row["f64"]["apply_us"], 2)
                    del Bm, P
                except Exception as e:  # report, never hide
                    row["bsr"] = {"error": str(e)}
            print(json.dumps(row), flush=True)
            rows.append(row)
            del A, M, x, y, z
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    return rows


def solvers(torch):
    """Time-to-solution of the mixed-precision and adjoint workloads."""
    from paper_2403_09198_amd import autograd, gen, r1s

    dev = "cuda:0"
    # mixed precision: 512 x 256, L = 200, GMRES(50) to 1e-10
    w = gen.WORKLOADS["mesh512x256_L200"]
    log(f"solvers: {w.name}")
    p = gen.make_problem(w.nx, w.ny, w.L, seed=w.seed)
    vals = {k: torch.from_numpy(p[k]).to(dev) for k in gen.FIELDS}
    del p
    A = r1s.R1Matrix(w.nx, w.ny, w.L, vals, keep_f32=True)
    del vals
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = r1s.SMWPreconditioner(A, keep_f32=True)
    t_setup = time.perf_counter() - t0
    b = torch.from_numpy(gen.make_rhs(w.nx, w.ny, w.L, seed=w.seed)).to(dev)
    row = {"workload": w.name, "smw_setup_ms": round(t_setup * 1e3, 2)}
    xs = {}
    for tag, kw in (("f64", dict(mode="f64")),
                    ("mixed_ir_1e-4", dict(mode="mixed", inner_rtol=1e-4, max_outer=10)),
                    ("mixed_ir_1e-5", dict(mode="mixed", inner_rtol=1e-5, max_outer=10)),
                    ("mixed_ir", dict(mode="mixed", inner_rtol=1e-6, max_outer=10)),
                    ("f32_inner_only", dict(mode="mixed", inner_rtol=1e-6, max_outer=1))):
        r1s.gmres(A, M, b, restart=50, rtol=1e-10, raise_on_noconv=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = r1s.gmres(A, M, b, restart=50, rtol=1e-10, raise_on_noconv=False, **kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        xs[tag] = res.x
        st = res.stats[0]
        row[tag] = {"ms": round(el * 1e3, 2), "iters": st["iters"], "outer": st["outer"],
                    "rel_residual_f64": st["rel_residual"], "converged": bool(st["converged"])}
    ref = xs["f64"]
    for tag in xs:
        if tag != "f64":
            row[tag]["rel_diff_vs_f64_solve"] = float(torch.linalg.norm(xs[tag] - ref) /
                                                      torch.linalg.norm(ref))
    best = min((t for t in xs if t.startswith("mixed_ir")), key=lambda t: row[t]["ms"])
    row["best_mixed"] = best
    row["mixed_speedup"] = round(row["f64"]["ms"] / row[best]["ms"], 3)
    print(json.dumps(row), flush=True)
    del A, M, b, xs, ref
    torch.cuda.empty_cache()

    # adjoint: 256 x 128, L = 61, batch of 8, loss = sum w . x
    w = gen.WORKLOADS["adjoint256x128_L61_b8"]
    log(f"solvers: {w.name}")
    p = gen.make_problem(w.nx, w.ny, w.L, seed=w.seed)
    params = {k: torch.from_numpy(p[k]).to(dev).requires_grad_(True) for k in gen.FIELDS}
    b = torch.from_numpy(gen.make_rhs(w.nx, w.ny, w.L, nrhs=w.nrhs, seed=w.seed)).to(dev)
    wt = torch.from_numpy(gen.make_loss_weights(w.nx, w.ny, w.L, nrhs=w.nrhs, seed=w.seed)).to(dev)
    b.requires_grad_(True)
    row = {"workload": w.name, "nrhs": w.nrhs}
    for rep in range(2):  # the second repetition is timed
        for t in list(params.values()) + [b]:
            t.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = autograd.solve(b, params, w.nx, w.ny, w.L, restart=50, rtol=1e-10)
        loss = (x * wt).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    row["forward_ms"] = round((t1 - t0) * 1e3, 2)
    row["backward_ms"] = round((t2 - t1) * 1e3, 2)
    print(json.dumps(row), flush=True)


def cpu_model():
    """The host CPU's model name (Linux), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_cores():
    """Worker processes for the all-cores legs: the CPU share the process may
    use (OMP_NUM_THREADS where the job sets it), at most 16."""
    n = os.environ.get("OMP_NUM_THREADS")
    n = int(n) if n and n.isdigit() else (os.cpu_count() or 1)
    return max(1, min(16, n))


# The CPU legs run the oracle on a sub-mesh of the headline workload's
# generator (same L and m, same value distributions): every block row of it
# has the full workload's structure.
CPU_SUBMESH = (16, 16)


def _cpu_leg(args):
    """One worker of a CPU leg: the oracle's float64 pair on its share of the
    sub-mesh's block rows, repeated for `budget` seconds.  path 'dense': the
    dense-block matvec + dense-LU block-Jacobi (blocks assembled and factored
    beforehand); 'structured': the CSR + BR1 product of section 5.2 and the
    SMW solve of section 6 (formats and index arrays built beforehand).
    Returns (passes, cells, seconds)."""
    path, L, seed, part, nparts, budget = args
    from threadpoolctl import threadpool_limits

    from oracle import assemble, blockjacobi, formats, ops
    from paper_2403_09198_amd import gen

    nx, ny = CPU_SUBMESH
    N, m = nx * ny, L + 3
    p = gen.make_problem(nx, ny, L, seed=seed)
    cells = list(range(part, N, nparts))
    x = np.random.default_rng(5).standard_normal((N, m))
    with threadpool_limits(limits=1):
        if path == "dense":
            indptr, indices, data, rows = assemble.assemble_bsr(p, nx, ny, L, cells)
            LU, piv = blockjacobi.lu_factor(assemble.diagonal_blocks(p, nx, ny, L, cells))

            def once():
                y = ops.bsr_matvec(indptr, indices, data, rows, x, N)
                blockjacobi.lu_solve(LU, piv, y[0])
        else:
            csr = formats.structured_csr(p, nx, ny, L)
            br1 = formats.structured_br1(p, nx, ny)
            # the rows of this worker's cells: CSR rows and BR1 block rows
            ind, ptr = csr[1], csr[2]
            sub_rows = [c * m + k for c in cells for k in range(m)]
            sub_ptr = np.concatenate([[0], np.cumsum([ptr[r + 1] - ptr[r] for r in sub_rows])])
            sel = np.concatenate([np.arange(ptr[r], ptr[r + 1]) for r in sub_rows])
            sub_csr = (csr[0][sel], ind[sel], sub_ptr)
            # the worker's block rows, renumbered 0..len(cells)-1
            blocks = []
            for i, c in enumerate(cells):
                for b in range(br1["block_indptr"][c], br1["block_indptr"][c + 1]):
                    q0, q1 = br1["pair_indptr"][b], br1["pair_indptr"][b + 1]
                    blocks.append((i, int(br1["block_indices"][b]),
                                   [(br1["column_data"][q], br1["row_data"][q])
                                    for q in range(q0, q1)]))
            sub_br1 = formats.br1_bsr(blocks, len(cells))
            xf = np.ravel(x)

            def once():
                y = formats.csr_matvec(*sub_csr, xf)
                y, _ = formats.br1_matvec(sub_br1, xf, m, m, y=y)
                yc = y.reshape(len(cells), m)
                for i, c in enumerate(cells):
                    blockjacobi.smw_solve(p, c, L, yc[i])
        once()
        reps, t0 = 0, time.perf_counter()
        while True:
            once()
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget:
                break
    return reps, len(cells), el


def cpu_baseline(L, seed=0, budget_s=4.0):
    """The oracle's float64 pair (dense path and structured path) on the
    sub-mesh, one process and one per host core.  Rates are in GB/s of the
    same algorithmic bytes as the GPU line (the structured pair's per-cell
    bytes times the cells processed), so the figures compare work done."""
    import concurrent.futures as cf

    nx, ny = CPU_SUBMESH
    N, m = nx * ny, L + 3
    B = 5 * N - 2 * nx - 2 * ny
    mv, ap = pair_bytes(N, B, m)
    per_cell = (mv + ap) / N
    cores = host_cores()
    legs = {}
    for path in ("dense", "structured"):
        for nproc in (1, cores):
            jobs = [(path, L, seed, i, nproc, budget_s) for i in range(nproc)]
            if nproc == 1:
                res = [_cpu_leg(jobs[0])]
            else:
                with cf.ProcessPoolExecutor(max_workers=nproc) as ex:
                    res = list(ex.map(_cpu_leg, jobs))
            gbs = sum(r * c * per_cell / el for r, c, el in res) / 1e9
            legs[f"{path}_{'1core' if nproc == 1 else f'{nproc}cores'}"] = {
                "gbs": round(gbs, 4), "processes": nproc,
                "passes": [r for r, _, _ in res], "seconds": round(max(el for _, _, el in res), 2)}
            log(f"cpu baseline {path} x{nproc}: {gbs:.4f} GB/s")
    best = max(legs, key=lambda k: legs[k]["gbs"])
    return {
        "value": legs[best]["gbs"], "unit": "GB/s", "cores": legs[best]["processes"],
        "kind": "oracle",
        "sample": (f"{nx}x{ny} sub-mesh of the same generator at L={L} (m={m}, {N} block rows); "
                   f"float64 pair y = J x, z = M y by the oracle: 'dense' = dense-block matvec + "
                   f"dense-LU block-Jacobi, 'structured' = CSR + BR1 product (sec. 5.2) + SMW "
                   f"solve (sec. 6), each for {budget_s:.0f} s on 1 process and on one process "
                   f"per core (block rows split between them, 1 BLAS thread each); GB/s of the "
                   f"structured pair's algorithmic bytes per cell; value = the best leg ({best})"),
        "legs": legs,
        "host": cpu_model() or platform.processor() or platform.machine(),
        "host_cpus": os.cpu_count(), "cores_used": cores,
    }


def oracle_solve_checks(p, nx, ny, L, b, xs, k=24):
    """The float64 residual b - J x of each GPU solve on sampled block rows,
    by the oracle's dense-block rows: componentwise against (|J||x| + |b|)
    and normwise over the rows, for each solution in `xs` (host arrays)."""
    from oracle import ops

    rng = np.random.default_rng(11)
    N = nx * ny
    cells = sorted(set(rng.choice(N, size=min(k, N), replace=False).tolist()) |
                   {0, nx - 1, N - nx, N - 1})
    pa = {key: np.abs(v) for key, v in p.items() if isinstance(v, np.ndarray)}
    bs = b[:, cells]
    out = {}
    for tag, x in xs.items():
        r = bs - ops.matvec_rows(p, nx, ny, L, x, cells)
        scale = ops.matvec_rows(pa, nx, ny, L, np.abs(x), cells) + np.abs(bs)
        out[tag] = {"cells": len(cells),
                    "max_componentwise": float(np.max(np.abs(r) / scale)),
                    "sampled_rel_residual": float(np.linalg.norm(r) / np.linalg.norm(bs))}
    return out


def pair_line(torch, A, M, x, y, z, steps, warm, mv_b, ap_b):
    """Graph-replayed float64 pair steps and per-kernel event durations."""
    graphs = step_graphs(torch, lambda: (A.matvec(x, out=y), M.apply(y, out=z)))
    replay(graphs, warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    replay(graphs, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-kernel durations: HIP events around every launch of the same
    # alternating sequence, on the stream the library launches on (timing a
    # kernel back-to-back with itself would let the 256 MB Infinity Cache
    # hold part of its working set)
    _, t_mv, t_ap = time_pair(torch, lambda: A.matvec(x, out=y), lambda: M.apply(y, out=z),
                              steps, warm)
    return wall, t_mv, t_ap


def solve_rows(torch, A, M, b, restart, rtol, modes=("f64", "mixed")):
    from paper_2403_09198_amd import r1s
    out, xs = {}, {}
    for mode in modes:
        r1s.gmres(A, M, b, restart=restart, rtol=rtol, mode=mode)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(SOLVE_REPS):
            res = r1s.gmres(A, M, b, restart=restart, rtol=rtol, mode=mode)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / SOLVE_REPS
        out[f"solve_{mode}"] = {"ms": round(el * 1e3, 2), "iters": res.stats[0]["iters"],
                                "outer": res.stats[0]["outer"],
                                "rel_residual": res.stats[0]["rel_residual"]}
        xs[mode] = res.x
    if "f64" in xs and "mixed" in xs:
        out["solve_mixed"]["rel_diff_vs_f64_solve"] = float(
            torch.linalg.norm(xs["mixed"] - xs["f64"]) / torch.linalg.norm(xs["f64"]))
    return out, xs


def c2_block(torch, steps, warm):
    """The 256 x 128, L = 61 workload (m = 64): the pair, the pair as one
    kernel, eight right-hand sides, the paper's pair counts, the wide
    diagonal block, the physics-shaped Jacobian, a general mesh, solves."""
    from paper_2403_09198_amd import gen, r1s

    dev = "cuda:0"
    w = gen.WORKLOADS["mesh256x128_L61"]
    nx, ny, L, m, N = w.nx, w.ny, w.L, w.m, w.N
    B = 5 * N - 2 * nx - 2 * ny
    log(f"c2 block: {w.name}")
    p = gen.make_problem(nx, ny, L, seed=w.seed)
    A = r1s.R1Matrix(nx, ny, L, {k: torch.from_numpy(p[k]).to(dev) for k in gen.FIELDS},
                     keep_f32=True)
    M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    del p
    x = torch.from_numpy(gen.make_vector(nx, ny, L, seed=0)).to(dev)
    y, z = torch.empty_like(x), torch.empty_like(x)
    mv_b, ap_b = pair_bytes(N, B, m)
    wall, t_mv, t_ap = pair_line(torch, A, M, x, y, z, steps, warm, mv_b, ap_b)
    mv_ms, ap_ms = float(np.mean(t_mv)), float(np.mean(t_ap))
    out = {"workload": w.name, "bytes_per_step": mv_b + ap_b,
           "gbs": round((mv_b + ap_b) / (wall / steps) / 1e9, 1),
           "us_per_step": round(wall / steps * 1e6, 2),
           "pct_hbm_peak": round(100 * (mv_b + ap_b) / (wall / steps) / 1e9 / HBM_PEAK_GBS, 2),
           "matvec_us": round(mv_ms * 1e3, 2), "apply_us": round(ap_ms * 1e3, 2),
           "matvec_gbs": round(mv_b / (mv_ms / 1e3) / 1e9, 1),
           "apply_gbs": round(ap_b / (ap_ms / 1e3) / 1e9, 1),
           "matvec_traffic": counter_traffic(w.name, "matvec"),
           "apply_traffic": counter_traffic(w.name, "apply")}
    # the pair as one kernel (r1s_matvec_prec: y = J x is written and goes
    # straight into the SMW solve, so it is not read back)
    for key, prec, vb in (("fused_pair", "f64", mv_b + ap_b),
                          ("fused_fp32_pair", "f32", sum(pair_bytes(N, B, m, value_bytes=4)))):
        fb = vb - 8 * N * m
        wallF, kF = measure_one(
            torch, lambda prec=prec: M.apply_after_matvec(x, precision=prec, out_y=y, out_z=z),
            steps, warm)
        out[key] = {"gbs": round(fb / (wallF / steps) / 1e9, 1),
                    "us_per_step": round(wallF / steps * 1e6, 2),
                    "kernel_us": round(kF * 1e3, 2), "bytes_per_step": fb}
    # eight right-hand sides per call: the matrix and factors are read once
    # per batch (the adjoint workload's batch size)
    nb8 = 8
    x8 = torch.from_numpy(gen.make_vector(nx, ny, L, nrhs=nb8, seed=1)).to(dev)
    y8, z8 = torch.empty_like(x8), torch.empty_like(x8)
    mv8, ap8 = pair_bytes(N, B, m, nrhs=nb8)
    n8 = max(20, steps // 4)
    wall8, k1, k2 = measure_pair(torch, lambda: A.matvec(x8, out=y8),
                                 lambda: M.apply(y8, out=z8), n8, 10)
    out["batched_pair_nrhs8"] = {
        "gbs": round((mv8 + ap8) / (wall8 / n8) / 1e9, 1),
        "us_per_step": round(wall8 / n8 * 1e6, 2),
        "us_per_rhs": round(wall8 / n8 / nb8 * 1e6, 2),
        "matvec_us": round(k1 * 1e3, 2), "apply_us": round(k2 * 1e3, 2),
        "speedup_per_rhs_vs_single": round((wall / steps) / (wall8 / n8 / nb8), 2)}
    del x8, y8, z8
    b = torch.from_numpy(gen.make_rhs(nx, ny, L, seed=w.seed)).to(dev)
    rows, _ = solve_rows(torch, A, M, b, w.restart, w.rtol)
    out.update(rows)
    del A, M, x, y, z, b
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # the paper's rank structure (9 pairs per diagonal block, 2 per
    # neighbour block) on the same mesh
    out["paper_ranks_pair"] = ranks_pair(torch, nx, ny, L, gen.PAPER_RANKS, steps, warm)
    # and a wider diagonal block: level band of half-width 4 with
    # level/flow coupling (banded-LU block-Jacobi)
    out["wide_pattern_pair"] = ranks_pair(torch, nx, ny, L, gen.PAPER_RANKS, steps, warm,
                                          band=4, arrow=True)
    # the same pattern given as a general (explicit) pattern of the diagonal
    # block: host symbolic LU, one lane per cell numeric LU and solves
    out["explicit_pattern_pair"] = ranks_pair(torch, nx, ny, L, gen.PAPER_RANKS, steps, warm,
                                              band=4, arrow=True, explicit=True)
    # the atom density coupled to every level (arrow = 2)
    out["atom_pattern_pair"] = ranks_pair(torch, nx, ny, L, gen.PAPER_RANKS, steps, warm,
                                          band=1, arrow=2)
    # physics-shaped values: the HLL finite-volume Jacobian of a multi-species
    # gas (8 / 6 pairs, level/flow coupling), with GMRES solves of it; and
    # with the DRa source (atom coupling)
    for key, dra in (("physics_pair", False), ("physics_dra_pair", True)):
        try:
            out[key] = ranks_pair(torch, nx, ny, L, None, steps, warm, physics_values=True,
                                  dra=dra, solve=(w.restart, w.rtol))
        except Exception as e:  # report, never hide
            out[key] = {"error": str(e)}
    # general mesh: about 32 800 triangle cells (Delaunay of 16 400 random
    # points), the same L, one pair per block; shuffled and mesh-ordered
    out["general_mesh_pair"] = mesh_pair(torch, 16400, L, (1, 1), steps, warm)
    out["general_mesh_pair_ordered"] = mesh_pair(torch, 16400, L, (1, 1), steps, warm,
                                                 shuffle=False)
    return out


def solve_timeline(torch, reps=3):
    """GMRES(50) solves of the 256 x 128, L = 61 system to 1e-10, each
    between two torch marker kernels (an add before, a multiply after) so
    that a kernel trace separates them; prints each solve's host wall time."""
    from paper_2403_09198_amd import gen, r1s

    dev = "cuda:0"
    w = gen.WORKLOADS["mesh256x128_L61"]
    p = gen.make_problem(w.nx, w.ny, w.L, seed=w.seed)
    A = r1s.R1Matrix(w.nx, w.ny, w.L, {k: torch.from_numpy(p[k]).to(dev) for k in gen.FIELDS})
    M = r1s.SMWPreconditioner(A)
    b = torch.from_numpy(gen.make_rhs(w.nx, w.ny, w.L, seed=w.seed)).to(dev)
    for _ in range(3):
        r1s.gmres(A, M, b, restart=w.restart, rtol=w.rtol)
    mark = torch.zeros(1, device=dev)
    torch.cuda.synchronize()
    for rep in range(reps):
        mark.add_(1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = r1s.gmres(A, M, b, restart=w.restart, rtol=w.rtol)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mark.mul_(2.0)
        torch.cuda.synchronize()
        print(json.dumps({"solve": rep, "wall_ms": round((t1 - t0) * 1e3, 3),
                          "iters": res.stats[0]["iters"]}), flush=True)


def summarize_timeline(csv_path):
    """Per solve of a --solve-timeline trace: the span from its first kernel's
    start to its last kernel's end, the sum of its kernel durations, and the
    device idle time in between (host round trips and launch gaps)."""
    import csv
    rows = sorted(csv.DictReader(open(csv_path)), key=lambda r: int(r["Start_Timestamp"]))
    seg, segs = None, []
    for r in rows:
        name = r["Kernel_Name"]
        if "vectorized_elementwise" in name and "add" in name.lower() and seg is None:
            seg = []
        elif "vectorized_elementwise" in name and "Mul" in name and seg is not None:
            segs.append(seg)
            seg = None
        elif seg is not None:
            seg.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    for i, sg in enumerate(segs):
        span = (sg[-1][1] - sg[0][0]) / 1e3
        busy = sum(e - b for b, e in sg) / 1e3
        print(json.dumps({"solve": i, "kernels": len(sg), "span_us": round(span, 1),
                          "kernel_us": round(busy, 1), "idle_us": round(span - busy, 1),
                          "idle_pct": round(100 * (span - busy) / span, 2)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--ranks", default="1,1",
                    help="rank-one pairs per diagonal,neighbour block of the timed step "
                         "(the workload's own layout is 1,1)")
    ap.add_argument("--band", type=int, default=1,
                    help="level-band half-width of the diagonal block for the timed step")
    ap.add_argument("--arrow", action="store_true",
                    help="level/flow coupling in the diagonal block for the timed step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the FP64 pair (for profiling runs)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the counter summary of --workload from two --pmc runs of "
                         "--profile-pass")
    ap.add_argument("--solvers", action="store_true",
                    help="mixed-precision and adjoint time-to-solution (one JSON line each)")
    ap.add_argument("--sweep", action="store_true",
                    help="512x256 level sweep against the BSR baseline (one JSON line per case)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="run the fixed kernel sequence used for hardware-counter runs")
    ap.add_argument("--nrhs", type=int, default=1,
                    help="right-hand sides of the --profile-pass vectors (8: the batched "
                         "operator of the adjoint workload)")
    ap.add_argument("--solve-timeline", action="store_true",
                    help="three 256x128, L=61 GMRES solves between marker kernels (for a "
                         "kernel trace) and their unprofiled wall times")
    ap.add_argument("--summarize-timeline", metavar="KERNEL_TRACE_CSV",
                    help="device idle time between the kernels of each solve of a "
                         "--solve-timeline kernel trace")
    args = ap.parse_args()
    if args.summarize_timeline:
        summarize_timeline(args.summarize_timeline)
        return
    if args.solve_timeline:
        import torch
        solve_timeline(torch)
        return
    if args.summarize_counters:
        summarize_counters(args.workload, *args.summarize_counters)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2403_09198_amd import gen, r1s

    if args.sweep:
        sweep(torch)
        return
    if args.solvers:
        solvers(torch)
        return
    w = gen.WORKLOADS[args.workload]
    nx, ny, L, m, N = w.nx, w.ny, w.L, w.m, w.N
    B = 5 * N - 2 * nx - 2 * ny
    dev = "cuda:0"
    log(f"workload {w.name}: mesh {nx}x{ny}, L={L}, m={m}, blocks={B}")
    ranks = tuple(int(v) for v in args.ranks.split(","))
    plain = ranks == (1, 1) and args.band == 1 and not args.arrow
    p = gen.make_problem(nx, ny, L, seed=w.seed, inv_dt=w.inv_dt, r_diag=ranks[0],
                         r_off=ranks[1], band=args.band, arrow=args.arrow)
    keys = gen.FIELDS + tuple(k for k in gen.PATTERN_FIELDS if k in p)
    vals = {k: torch.from_numpy(p[k]).to(dev) for k in keys}
    A = r1s.R1Matrix(nx, ny, L, vals, keep_f32=True, ranks=ranks, band=args.band,
                     arrow=args.arrow)
    M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    del vals
    x = torch.from_numpy(gen.make_vector(nx, ny, L, seed=0)).to(dev)
    y = torch.empty_like(x)
    z = torch.empty_like(x)

    mv_b, ap_b = pair_bytes(N, B, m)
    if not plain:
        st = A.storage()
        mv_b, ap_b = st["matvec_bytes"], st["smw_apply_bytes"]
    steps, warm = args.steps, args.warmup
    if args.profile_pass:
        if args.nrhs > 1:
            x = torch.from_numpy(gen.make_vector(nx, ny, L, nrhs=args.nrhs, seed=1)).to(dev)
            y, z = torch.empty_like(x), torch.empty_like(x)
        profile_pass(torch, A, M, x, y, z)
        return

    # one step = matvec + apply, captured as HIP graphs (STEPS_PER_GRAPH steps
    # per graph) and replayed
    wall, t_mv, t_ap = pair_line(torch, A, M, x, y, z, steps, warm, mv_b, ap_b)
    ms_step = wall / steps * 1e3
    value = (mv_b + ap_b) / (wall / steps) / 1e9
    mv_ms, ap_ms = float(np.mean(t_mv)), float(np.mean(t_ap))
    log(f"fp64 pair: {ms_step * 1e3:.1f} us/step, matvec {mv_ms * 1e3:.1f} us, "
        f"apply {ap_ms * 1e3:.1f} us, {value:.0f} GB/s")
    ach = mv_b / (mv_ms / 1e3) / 1e9
    tr = counter_traffic(w.name, "matvec") if plain else None
    tra = counter_traffic(w.name, "apply") if plain else None
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": steps, "warmup": warm, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": nx, "ny": ny, "L": L, "m": m, "nrhs": 1,
                   "pairs_per_block": {"diagonal": ranks[0], "neighbour": ranks[1]},
                   "diag_block_band": args.band, "level_flow_coupling": bool(args.arrow),
                   "step": "y = J x then z = M y (SMW block-Jacobi), float64, replayed from "
                           "HIP graphs of %d steps" % STEPS_PER_GRAPH,
                   "bytes_per_step": mv_b + ap_b},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "cell_updates_per_s": round(N / (wall / steps), 1),
        "roofline": {"bound": "hbm",
                     "kernel": (tr["kernel"] if tr else "structured matvec (J x)"),
                     "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": tr["traffic_bytes"] if tr else None,
                     "avg_launch_us": round(mv_ms * 1e3, 2),
                     "algorithmic_bytes_per_launch": mv_b},
        "kernels_us": {"matvec_f64": round(mv_ms * 1e3, 2), "smw_apply_f64": round(ap_ms * 1e3, 2)},
        "kernels_us_median_min": {
            "matvec_f64": [round(float(np.median(t_mv)) * 1e3, 2), round(float(np.min(t_mv)) * 1e3, 2)],
            "smw_apply_f64": [round(float(np.median(t_ap)) * 1e3, 2), round(float(np.min(t_ap)) * 1e3, 2)]},
        "kernel_gbs": {"matvec_f64": round(ach, 1),
                       "smw_apply_f64": round(ap_b / (ap_ms / 1e3) / 1e9, 1)},
        "smw_apply_roofline": {"achieved": round(ap_b / (ap_ms / 1e3) / 1e9, 1),
                               "frac": round(ap_b / (ap_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                               "traffic": tra["traffic_bytes"] if tra else None,
                               "kernel": tra["kernel"] if tra else None,
                               "algorithmic_bytes_per_launch": ap_b},
    }
    # counted bytes per second (the FETCH_SIZE + WRITE_SIZE traffic of one
    # launch over its average duration) beside the algorithmic rate
    if tr:
        out["roofline"]["traffic_gbs"] = round(tr["traffic_bytes"] / (mv_ms / 1e3) / 1e9, 1)
    if tra:
        out["smw_apply_roofline"]["traffic_gbs"] = round(tra["traffic_bytes"] / (ap_ms / 1e3) / 1e9, 1)
    if not args.no_extras:  # (kept out of profiled runs: the cold pairs would enter the averages)
        ce = ceilings(torch, A, M, x, y, z, mv_b, ap_b)
        out["ceilings"] = ce
        out["roofline"]["frac_of_copy"] = round(ach / ce["stream_copy_gbs"], 4)
        log(f"copy {ce['stream_copy_gbs']:.0f} GB/s; cold matvec {ce['cold']['matvec_us']} us, "
            f"apply {ce['cold']['smw_apply_us']} us")

    xs = {}
    b = None
    if not args.no_extras:
        # float32 values + accumulation (vectors stay float64)
        mv32, ap32 = pair_bytes(N, B, m, value_bytes=4)
        wall32, k1, k2 = measure_pair(torch, lambda: A.matvec(x, out=y, precision="f32"),
                                      lambda: M.apply(y, out=z, precision="f32"), steps, warm)
        out["fp32_pair"] = {
            "gbs": round((mv32 + ap32) / (wall32 / steps) / 1e9, 1),
            "us_per_step": round(wall32 / steps * 1e6, 2),
            "matvec_us": round(k1 * 1e3, 2), "apply_us": round(k2 * 1e3, 2),
            "speedup_vs_fp64": round(wall / wall32, 3)}
        # adjoint pair J^T x, M^T y (same bytes as forward)
        wallT, k1, k2 = measure_pair(torch, lambda: A.matvec(x, out=y, trans=True),
                                     lambda: M.apply(y, out=z, trans=True), steps, warm)
        out["adjoint_pair"] = {
            "gbs": round((mv_b + ap_b) / (wallT / steps) / 1e9, 1),
            "us_per_step": round(wallT / steps * 1e6, 2),
            "matvec_T_us": round(k1 * 1e3, 2), "apply_T_us": round(k2 * 1e3, 2),
            "ratio_vs_fp64": round(wallT / wall, 3)}
        # GMRES(50) to 1e-10 in float64 and in mixed-precision refinement
        b = torch.from_numpy(gen.make_rhs(nx, ny, L, seed=w.seed)).to(dev)
        rows, xsd = solve_rows(torch, A, M, b, w.restart, w.rtol)
        out.update(rows)
        xs = {k: v.cpu().numpy() for k, v in xsd.items()}
        # device copy ceiling (torch copy kernel, read + write bytes)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        cp_ms = kernel_ms(torch, lambda: dst.copy_(src), reps=10)
        out["torch_copy_gbs"] = round(2 * src.numel() * 8 / (cp_ms / 1e3) / 1e9, 1)
        del src, dst, xsd
    del A, M, x, y, z
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_extras and plain:
        # dense-block BSR baseline: quadratic in m, so at m > 128 on the half
        # mesh (512 x 128 at L = 200: 107.6 GB of blocks + 21.6 GB of LU)
        hx, hy = (nx, ny // 2) if m > 128 else (nx, ny)
        try:
            out["bsr_pair"] = bsr_compare(torch, hx, hy, L, w.seed, steps)
        except Exception as e:  # report, never hide
            out["bsr_pair"] = {"error": str(e)}
        out["c2"] = c2_block(torch, steps, warm)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(L, seed=w.seed)
        if xs:
            log("oracle checks of the solves on sampled rows ...")
            chk = oracle_solve_checks(p, nx, ny, L, b.cpu().numpy(), xs)
            for mode, c in chk.items():
                out[f"solve_{mode}"]["oracle_rows"] = c
    print(json.dumps(out), flush=True)


def bsr_compare(torch, nx, ny, L, seed, steps):
    """The structured float64 pair against the dense-block BSR pair (BSR
    matvec + dense-LU block-Jacobi apply) on the same matrix."""
    from paper_2403_09198_amd import gen, r1s

    dev = "cuda:0"
    m, N = L + 3, nx * ny
    B = 5 * N - 2 * nx - 2 * ny
    log(f"bsr comparison: mesh {nx}x{ny} L={L}")
    p = gen.make_problem(nx, ny, L, seed=seed)
    A = r1s.R1Matrix(nx, ny, L, {k: torch.from_numpy(p[k]).to(dev) for k in gen.FIELDS})
    del p
    M = r1s.SMWPreconditioner(A)
    x = torch.from_numpy(gen.make_vector(nx, ny, L, seed=0)).to(dev)
    y, z = torch.empty_like(x), torch.empty_like(x)
    mv, ap = pair_bytes(N, B, m)
    ws, _, _ = measure_pair(torch, lambda: A.matvec(x, out=y), lambda: M.apply(y, out=z),
                            steps, 10)
    Bm = r1s.BSRMatrix(A)
    P = r1s.DenseLUPreconditioner(Bm)
    bmv, bap = bsr_pair_bytes(N, B, m)
    nb = 5 if m > 128 else max(10, steps // 10)
    wallB, k1, k2 = measure_pair(torch, lambda: Bm.matvec(x, out=y), lambda: P.apply(y, out=z),
                                 nb, 2)
    res = {"mesh": f"{nx}x{ny}", "L": L, "stored_values": B * m * m,
           "gbs": round((bmv + bap) / (wallB / nb) / 1e9, 1),
           "us_per_step": round(wallB / nb * 1e6, 2),
           "matvec_us": round(k1 * 1e3, 2), "lu_apply_us": round(k2 * 1e3, 2),
           "structured_us_per_step": round(ws / steps * 1e6, 2),
           "speedup_structured_vs_bsr": round((wallB / nb) / (ws / steps), 2)}
    del A, M, Bm, P, x, y, z
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
