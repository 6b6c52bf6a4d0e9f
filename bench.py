"""Benchmark of the r1-sparse hot path on one MI355X.

A step is one application of the operator pair the metric names, on the
256 x 128 mesh with L = 61 levels (m = 64), float64:

    y = J x        (structured matvec kernel)
    z = M y        (SMW block-Jacobi apply kernel)

`value` is the algorithmic HBM bytes of the pair (stored structural values
plus input and output vectors, section-3 counts) per second over the timed
steps.  Per-kernel times come from HIP events on the launch stream.  The
same JSON line carries the float32-preconditioner pair, the adjoint pair
(J^T x, M^T y), the dense-block BSR baseline pair on the same matrix, a
cold-cache variant, a full GMRES solve, a device copy ceiling and the CPU
oracle timed on a bounded sample of the same workload.

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
COUNTERS = os.path.join(ROOT, "profiles", "counters_pair_fp64_mesh256x128_L61.json")
KERNEL_SOURCES = ("k_matvec.hip", "k_matvec_impl.hpp", "k_smw.hip", "r1s_device.hpp")


def kernel_source_hash():
    """sha256 over the sources of the matvec and SMW apply kernels."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2403_09198_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel_prefix):
    """HBM bytes per launch from the committed counter summary, or None when
    it was taken on other kernel sources."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except OSError:
        return None
    if c.get("kernel_source_sha256") != kernel_source_hash():
        return None
    k = c["kernels"].get(kernel_prefix)
    return None if k is None else k["traffic_bytes"]


def summarize_counters(fetch_csv, write_csv):
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
    out = {"kernel_source_sha256": kernel_source_hash(), "fetch_factor": round(ff, 4),
           "write_factor": round(wf, 4), "calibration_kernel": cp,
           "commands": [
               "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv "
               "-d <out>/pmc_fetch -o fetch -- python3 <repo>/bench.py --profile-pass",
               "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv "
               "-d <out>/pmc_write -o write -- python3 <repo>/bench.py --profile-pass",
               "python bench.py --summarize-counters <fetch csv> <write csv>"],
           "kernels": {}}
    for name in fetch:
        if not name.startswith(("void r1s::k_matvec", "void r1s::k_smw_apply")):
            continue
        fk = sum(fetch[name]) / len(fetch[name])
        wk = sum(write[name]) / len(write[name])
        out["kernels"][name] = {"fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                                "dispatches": len(fetch[name]),
                                "traffic_bytes": int(fk * 1024 * ff + wk * 1024 * wf)}
    with open(COUNTERS, "w") as f:
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
               physics_values=False, solve=None):
    """The float64 pair with several rank-one pairs per block (the paper's
    9 / 2 structure) and optionally the wide diagonal-block pattern;
    algorithmic bytes from the library's storage counts.  physics_values:
    the HLL finite-volume Jacobian of a multi-species gas (8 / 6 pairs,
    level/flow coupling) in place of random values; solve = (restart, rtol)
    adds GMRES solves of it."""
    from paper_2403_09198_amd import gen, physics, r1s

    dev = "cuda:0"
    if physics_values:
        ranks, band, arrow = (physics.R_DIAG, physics.R_OFF), 1, True
    log(f"ranks pair: mesh {nx}x{ny} L={L} ranks {ranks} band {band} arrow {arrow}"
        + (" (HLL Jacobian)" if physics_values else ""))
    if physics_values:
        p = physics.make_problem(nx, ny, L, seed=seed)
    else:
        p = gen.make_problem(nx, ny, L, seed=seed, r_diag=ranks[0], r_off=ranks[1], band=band,
                             arrow=arrow)
    keys = gen.FIELDS + tuple(k for k in gen.PATTERN_FIELDS if k in p)
    vals = {k: torch.from_numpy(p[k]).to(dev) for k in keys}
    del p
    A = r1s.R1Matrix(nx, ny, L, vals, keep_f32=True, ranks=ranks, band=band, arrow=arrow)
    del vals
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    t_setup = time.perf_counter() - t0
    st = A.storage()
    mv, ap = st["matvec_bytes"], st["smw_apply_bytes"]
    x = torch.from_numpy(gen.make_vector(nx, ny, L, seed=0)).to(dev)
    y, z = torch.empty_like(x), torch.empty_like(x)
    N = nx * ny
    row = {"r_diag": ranks[0], "r_off": ranks[1], "band": band, "arrow": bool(arrow),
           "stored_values": st["structured_values"],
           "smw_setup_ms": round(t_setup * 1e3, 2)}
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


def cpu_baseline(p, nx, ny, L, budget_s=12.0):
    """The oracle's dense-block matvec + dense-LU block-Jacobi apply on a
    sample of block rows (blocks assembled and factored beforehand), repeated
    for about `budget_s` seconds; GB/s of the same algorithmic bytes."""
    from threadpoolctl import threadpool_limits

    from oracle import assemble, blockjacobi, ops

    N, m = nx * ny, L + 3
    ncell = min(N, 1024)
    cells = list(range(ncell))
    x = np.random.default_rng(5).standard_normal((1, N, m))
    indptr, indices, data, rows = assemble.assemble_bsr(p, nx, ny, L, cells)
    D = assemble.diagonal_blocks(p, nx, ny, L, cells)
    LU, piv = blockjacobi.lu_factor(D)
    B_s = len(indices)
    mv, ap = pair_bytes(ncell, B_s, m)
    reps = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            y = ops.bsr_matvec(indptr, indices, data, rows, x, N)
            blockjacobi.lu_solve(LU, piv, y[0])
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    return {
        "value": round((mv + ap) * reps / el / 1e9, 4), "unit": "GB/s", "cores": 1,
        "kind": "oracle",
        "sample": (f"{ncell} of {N} block rows ({B_s} dense blocks, m={m}) of the same "
                   f"workload, dense-block matvec + dense-LU block-Jacobi apply, blocks "
                   f"assembled and factored beforehand, {reps} passes in {el:.1f} s, "
                   f"1 BLAS thread"),
        "seconds": round(el, 2),
        "host": cpu_model() or platform.processor() or platform.machine(),
        "host_cpus": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="mesh256x128_L61")
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
                    help="write the counter summary from two --pmc runs of --profile-pass")
    ap.add_argument("--solvers", action="store_true",
                    help="mixed-precision and adjoint time-to-solution (one JSON line each)")
    ap.add_argument("--sweep", action="store_true",
                    help="512x256 level sweep against the BSR baseline (one JSON line per case)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="run the fixed kernel sequence used for hardware-counter runs")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
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
    if ranks != (1, 1) or args.band != 1 or args.arrow:
        st = A.storage()
        mv_b, ap_b = st["matvec_bytes"], st["smw_apply_bytes"]
    steps, warm = args.steps, args.warmup
    if args.profile_pass:
        profile_pass(torch, A, M, x, y, z)
        return

    # one step = matvec + apply, captured as HIP graphs (STEPS_PER_GRAPH steps
    # per graph) and replayed
    graphs = step_graphs(torch, lambda: (A.matvec(x, out=y), M.apply(y, out=z)))
    replay(graphs, warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    replay(graphs, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / steps * 1e3
    value = (mv_b + ap_b) / (wall / steps) / 1e9
    # per-kernel durations: HIP events around every launch of the same
    # alternating sequence, on the stream the library launches on (timing a
    # kernel back-to-back with itself would let the 256 MB Infinity Cache
    # hold most of its working set)
    _, t_mv, t_ap = time_pair(torch, lambda: A.matvec(x, out=y), lambda: M.apply(y, out=z),
                              steps, warm)
    mv_ms, ap_ms = float(np.mean(t_mv)), float(np.mean(t_ap))
    log(f"fp64 pair: {ms_step * 1e3:.1f} us/step, matvec {mv_ms * 1e3:.1f} us, "
        f"apply {ap_ms * 1e3:.1f} us, {value:.0f} GB/s")
    ach = mv_b / (mv_ms / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": steps, "warmup": warm, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": nx, "ny": ny, "L": L, "m": m, "nrhs": 1,
                   "pairs_per_block": {"diagonal": ranks[0], "neighbour": ranks[1]},
                   "diag_block_band": args.band, "level_flow_coupling": bool(args.arrow),
                   "step": "y = J x then z = M y (SMW block-Jacobi), float64, replayed from HIP graphs of %d steps" % STEPS_PER_GRAPH,
                   "bytes_per_step": mv_b + ap_b},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "cell_updates_per_s": round(N / (wall / steps), 1),
        "roofline": {"bound": "hbm", "kernel": "k_matvec<double,1,1,false,false,1,1,false> (J x)",
                     "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(
                         "void r1s::k_matvec<double, 1, 1, false, false, 1, 1, false>"),
                     "avg_launch_us": round(mv_ms * 1e3, 2),
                     "algorithmic_bytes_per_launch": mv_b},
        "kernels_us": {"matvec_f64": round(mv_ms * 1e3, 2), "smw_apply_f64": round(ap_ms * 1e3, 2)},
        "kernels_us_median_min": {
            "matvec_f64": [round(float(np.median(t_mv)) * 1e3, 2), round(float(np.min(t_mv)) * 1e3, 2)],
            "smw_apply_f64": [round(float(np.median(t_ap)) * 1e3, 2), round(float(np.min(t_ap)) * 1e3, 2)]},
        "kernel_gbs": {"matvec_f64": round(ach, 1),
                       "smw_apply_f64": round(ap_b / (ap_ms / 1e3) / 1e9, 1)},
    }

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
        # the same pair as one kernel (r1s_matvec_prec: y = J x is written and
        # goes straight into the SMW solve, so it is not read back); bytes are
        # the pair's less that read of y
        if ranks == (1, 1) and args.band == 1 and not args.arrow:
            for key, prec, vb in (("fused_pair", "f64", mv_b + ap_b),
                                  ("fused_fp32_pair", "f32", sum(pair_bytes(N, B, m, value_bytes=4)))):
                fb = vb - 8 * N * m
                wallF, kF = measure_one(
                    torch, lambda prec=prec: M.apply_after_matvec(x, precision=prec, out_y=y, out_z=z),
                    steps, warm)
                two = wall if prec == "f64" else wall32
                out[key] = {"gbs": round(fb / (wallF / steps) / 1e9, 1),
                            "us_per_step": round(wallF / steps * 1e6, 2),
                            "kernel_us": round(kF * 1e3, 2), "bytes_per_step": fb,
                            "speedup_vs_two_kernels": round(two / wallF, 3)}
                log(f"{key}: {wallF / steps * 1e6:.1f} us/step ({two / wallF:.3f}x the two kernels)")
        # eight right-hand sides per call: the matrix and factors are read
        # once per batch (the adjoint workload's batch size)
        if ranks == (1, 1) and args.band == 1 and not args.arrow:
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
        # cold: a 1 GiB buffer is read before every step (a read leaves clean
        # lines, so no write-back of the flush competes with the timed kernels)
        scratch = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        sink = torch.empty((), dtype=torch.float64, device=dev)
        _, t1, t2 = time_pair(torch, lambda: A.matvec(x, out=y), lambda: M.apply(y, out=z),
                              min(steps, 50), 5, flush=lambda: torch.sum(scratch, dim=0, out=sink))
        cold = (float(np.mean(t1)) + float(np.mean(t2))) / 1e3
        out["cold_fp64_pair"] = {"gbs": round((mv_b + ap_b) / cold / 1e9, 1),
                                 "matvec_us": round(float(np.mean(t1)) * 1e3, 2),
                                 "apply_us": round(float(np.mean(t2)) * 1e3, 2)}
        # device copy ceiling (torch copy kernel, read + write bytes)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        cp_ms = kernel_ms(torch, lambda: dst.copy_(src), reps=10)
        out["torch_copy_gbs"] = round(2 * src.numel() * 8 / (cp_ms / 1e3) / 1e9, 1)
        del scratch, src, dst
        # dense-block BSR baseline on the same matrix
        try:
            Bm = r1s.BSRMatrix(A)
            P = r1s.DenseLUPreconditioner(Bm)
            bmv, bap = bsr_pair_bytes(N, B, m)
            nb = max(10, steps // 10)
            wallB, k1, k2 = measure_pair(torch, lambda: Bm.matvec(x, out=y),
                                         lambda: P.apply(y, out=z), nb, 3)
            out["bsr_pair"] = {
                "gbs": round((bmv + bap) / (wallB / nb) / 1e9, 1),
                "us_per_step": round(wallB / nb * 1e6, 2),
                "matvec_us": round(k1 * 1e3, 2), "lu_apply_us": round(k2 * 1e3, 2),
                "stored_values": B * m * m,
                "speedup_structured_vs_bsr": round((wallB / nb) / (wall / steps), 2)}
            del Bm, P
        except Exception as e:  # report, never hide
            out["bsr_pair"] = {"error": str(e)}
        # the paper's rank structure (9 pairs per diagonal block, 2 per
        # neighbour block) on the same mesh
        out["paper_ranks_pair"] = ranks_pair(torch, nx, ny, L, gen.PAPER_RANKS, steps, warm)
        # and a wider diagonal block: level band of half-width 4 with
        # level/flow coupling (banded-LU block-Jacobi, one lane per cell)
        out["wide_pattern_pair"] = ranks_pair(torch, nx, ny, L, gen.PAPER_RANKS, steps, warm,
                                              band=4, arrow=True)
        # the same mesh with physics-shaped values: the HLL finite-volume
        # Jacobian of a multi-species gas (8 / 6 pairs, level/flow coupling),
        # with GMRES solves of it
        try:
            out["physics_pair"] = ranks_pair(torch, nx, ny, L, None, steps, warm,
                                             physics_values=True, solve=(w.restart, w.rtol))
        except Exception as e:  # report, never hide
            out["physics_pair"] = {"error": str(e)}
        # general mesh: about 32 800 triangle cells (Delaunay of 16 400 random
        # points), the same L, one pair per block; shuffled and mesh-ordered
        # cell numbering
        out["general_mesh_pair"] = mesh_pair(torch, 16400, L, (1, 1), steps, warm)
        out["general_mesh_pair_ordered"] = mesh_pair(torch, 16400, L, (1, 1), steps, warm,
                                                     shuffle=False)
        # full GMRES(50) solve to 1e-10 (float64) and the mixed-precision solve
        b = torch.from_numpy(gen.make_rhs(nx, ny, L, seed=w.seed)).to(dev)
        for mode in ("f64", "mixed"):
            r1s.gmres(A, M, b, restart=w.restart, rtol=w.rtol, mode=mode)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(SOLVE_REPS):
                res = r1s.gmres(A, M, b, restart=w.restart, rtol=w.rtol, mode=mode)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / SOLVE_REPS
            out[f"solve_{mode}"] = {"ms": round(el * 1e3, 2), "iters": res.stats[0]["iters"],
                                    "outer": res.stats[0]["outer"],
                                    "rel_residual": res.stats[0]["rel_residual"]}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(p, nx, ny, L)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
