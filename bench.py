#!/usr/bin/env python3
"""Benchmark: iteration-batched hipGraph replay vs one launch per kernel.

Headline workload: the FDTD Maxwell solver of a PEC cavity, 256^3 cells,
10,000 steps per job (per step an H update, an E update and the soft
source; the fused H + E step by default, so two kernels per step), the
largest single-GPU configuration of the study (FDTD solver, Sec. III-C;
results in Sec. IV-B).  Fields start at zero and a Gaussian pulse (width 20
steps, delay 80) is added to Ez at a seeded node; the state is resident on
the device before timing starts.

Procedure (Sec. III-C):
  1. the autotuner picks the kernel variant and the iteration batch b for
     the 10,000-step job (graph creation included in its objective, Eq. 1);
  2. warm up, then time `--steps` whole jobs at that b, each job paying its
     own graph creation (T = T_C + T_E, Eq. 1), and the same jobs launching
     every kernel separately (the baseline);
  3. roofline: the step time from the HIP events around the timed replays
     (on the problem's stream) against the per-cell-step bytes, next to the
     attainable DRAM rate of the kernel's stream mix (six read and six
     write streams) measured live with the streaming probe;
  4. CPU baseline: the oracle on a bounded sample of the same cavity, on
     one core and on all cores; the same sample on the GPU gives the error
     against the float64 oracle;
  5. the skeleton chain (the paper's characterisation vehicle, Sec. IV-A):
     b sweep with 10 repeats per b, fits of Eqs. 2 and 6 with standard
     errors, graph vs per-launch, graph memory, the two builders;
  6. the other workloads and the Table I structure over vector sizes.
One JSON line is printed.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SEED = 20250116
HBM_PEAK_GBS = 8000.0
# the headline cavity
N_FDTD = 256
FDTD_STEPS = 10000
FDTD_B_CANDIDATES = [10, 20, 50, 100, 200, 500, 1000, 2000]   # divisors of 10,000
FDTD_BYTES_PER_CELL_STEP = 72.0     # three field reads + three read-modify-writes per half step
FDTD_KERNEL_BYTES_PER_NODE = 48.0   # the fused step: six fields read, six written
# the skeleton chain
N_ELEM = 1 << 16
K = 4
ITERS = 10000
SKEL_COUNTERS = os.path.join(ROOT, "profiles", "skeleton_2p16_hbm_counters.json")
SKEL_TRACE = os.path.join(ROOT, "profiles", "skeleton_2p16_trace_gaps.json")
FDTD_COUNTERS = os.path.join(ROOT, "profiles", "fdtd_256_fused_hbm_counters.json")
FDTD_TB2_COUNTERS = os.path.join(ROOT, "profiles", "fdtd_256_tb2_hbm_counters.json")
FDTD_ROWS_COUNTERS = os.path.join(ROOT, "profiles", "fdtd_256_tb2_rows_hbm_counters.json")
FDTD_TB3_COUNTERS = os.path.join(ROOT, "profiles", "fdtd_256_tb3_rows_hbm_counters.json")
MISC_SOURCE = os.path.join(ROOT, "paper_2501_09398_amd", "csrc", "kernels_misc.hip")
FDTD_SOURCE = os.path.join(ROOT, "paper_2501_09398_amd", "csrc", "fdtd.hip")


def note(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed jobs per arm (each 10,000 cavity steps)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--b", type=int, default=0, help="fix the cavity's batch size (skips the autotuner)")
    ap.add_argument("--fdtd-variant", type=int, default=8, help="cavity kernel variant with --b")
    ap.add_argument("--fdtd-depth", type=int, default=2, help="steps per launch of that variant with --b")
    ap.add_argument("--only", choices=("all", "fdtd", "skeleton"), default="all",
                    help="'fdtd': the headline cavity alone; 'skeleton': the skeleton chain alone")
    ap.add_argument("--arm", choices=("both", "graph", "per_launch"), default="both",
                    help="time both arms, or one alone (for tracing one arm)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other workloads and the Table I sizes")
    ap.add_argument("--skeleton-b", type=int, default=0, help="fix the skeleton's batch size")
    ap.add_argument("--no-sweep", action="store_true", help="skip the skeleton's b sweep (needs --skeleton-b)")
    ap.add_argument("--sweep-reps", type=int, default=10, help="repeats per b in the skeleton sweep")
    ap.add_argument("--kernel-only-b", type=int, default=0,
                    help="with --kernel-only: run the steps twice in graph batches of this b (the first run "
                         "builds the graphs; traces then show warm replays)")
    ap.add_argument("--kernel-only", choices=sorted(KERNEL_RUNS),
                    help="run only one workload's kernels per launch for a few steps (counter runs)")
    ap.add_argument("--stream-calibration", action="store_true",
                    help="only time the streaming probe for the read / write stream mixes of the "
                         "stencil and FDTD kernels (attainable DRAM throughput per mix)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy of known size (2^26 floats read and written by the "
                         "element-wise kernel with a=1, b=0), to scale hardware byte counters")
    return ap.parse_args()


KERNEL_RUNS = {
    # name: (problem, shape, coeffs-attr, variant, steps per launch loop[, temporal depth])
    "skeleton_2p16": ("SKELETON", (N_ELEM,), None, 1, 100),
    "heat2d_16384": ("HEAT2D", (16384, 16384), "HEAT_COEFFS", 13, 5),
    "heat3d_8x4096": ("HEAT3D", (8, 4096, 4096), "HEAT_COEFFS", 9, 5),
    "fdtd_256": ("FDTD3D", (256, 64), "FDTD_COEFFS", 2, 5),
    "fdtd_256_fused": ("FDTD3D", (256, 64), "FDTD_COEFFS", 7, 10),
    "fdtd_256_tb2": ("FDTD3D", (256, 64), "FDTD_COEFFS", 8, 10, 2),     # 5 launches of 2 steps
    "fdtd_256_tb2_rows16": ("FDTD3D", (256, 64), "FDTD_COEFFS", 9, 10, 2),
    "fdtd_256_tb2_rows12": ("FDTD3D", (256, 64), "FDTD_COEFFS", 10, 10, 2),
    "fdtd_256_tb3_rows": ("FDTD3D", (256, 64), "FDTD_COEFFS", 10, 9, 3),      # 3 launches of 3 steps
    "surrogate_512": ("HEAT2D_SURROGATE", (512, 512), "HEAT_COEFFS", 1, 160),
    "surrogate_512_layered": ("HEAT2D_SURROGATE", (512, 512), "HEAT_COEFFS", 2, 160),
    # 64 square grids of side round(64 * 16^u) (shape filled in from the seed)
    "multigrid_64": ("HEAT2D_MULTI", None, "HEAT_COEFFS", 2, 10),
    "multigrid_64_cell": ("HEAT2D_MULTI", None, "HEAT_COEFFS", 1, 10),
    "multigrid_64_tb": ("HEAT2D_MULTI", None, "HEAT_COEFFS", 3, 60, 6),    # 10 launches of 6 steps
    "heat2d_16384_region": ("HEAT2D", (16384, 16384), "HEAT_COEFFS", 21, 40, 8),   # 5 launches of 8 steps
    "heat3d_8x4096_strip_tb": ("HEAT3D", (8, 4096, 4096), "HEAT_COEFFS", 11, 20, 4),   # 5 launches of 4
    # the launch-bound configurations, for traces of graph replays
    "heat2d_256": ("HEAT2D", (256, 256), "HEAT_COEFFS", 16, 1000, 8),        # register strips, 8 steps
    "heat3d_8x512": ("HEAT3D", (8, 512, 512), "HEAT_COEFFS", 11, 2000, 5),   # register strips, 5 steps
    "fdtd_128": ("FDTD3D", (128, 64), "FDTD_COEFFS", 0, 1000),
}


def kernel_only(name, b=0):
    """Run one workload's kernels per launch for a few steps and nothing else
    (for hardware-counter runs, which serialise every dispatch); with b > 0
    run the steps twice in graph batches of b (for kernel traces of warm
    replays: the second run replays the graphs the first one built)."""
    import torch
    import paper_2501_09398_amd as kb
    prob, shape, co, var, steps = KERNEL_RUNS[name][:5]
    depth = KERNEL_RUNS[name][5] if len(KERNEL_RUNS[name]) > 5 else 1
    coeffs = (K,) if co is None else getattr(kb, co)
    if prob == "HEAT2D_MULTI":
        import synth
        sides = synth.multigrid_sides(SEED, 64)
        shape = [64] + [v for sd in sides for v in (sd, sd)]
    if prob == "HEAT2D_SURROGATE":
        import numpy as np
        import synth
        coeffs = tuple(coeffs) + (0.8, 1e30, 16)          # check never falls back
    with kb.Problem(getattr(kb, prob), shape, coeffs, SEED, device=0) as p:
        p.set_option(kb.OPT_TILE, var)
        p.set_option(kb.OPT_TDEPTH, depth)
        if prob == "HEAT2D_SURROGATE":                    # a network with every layer active
            w = synth.surrogate_init(SEED)
            w[19104:19393] = synth.uniform_f32(SEED, 9, 289, -0.06, 0.06)
            p.write(kb.F_W, w.astype(np.float32))
        for _ in range(2 if b > 0 else 1):
            p.run(steps, b)
            p.last_timing()
    torch.cuda.synchronize()
    print(json.dumps({"kernel_only": name, "steps": steps, "b": b}), flush=True)


# (reads, writes) of the kernels whose HBM fraction the benchmark reports:
# copy; heat2d (T, P -> T); FDTD H or E kernel (6 -> 3); fused FDTD step
# (6 -> 6); a wider read-heavy mix
STREAM_MIXES = ((1, 1), (2, 1), (3, 1), (2, 2), (3, 3), (6, 3), (6, 6), (8, 1), (8, 8))


def stream_calibration():
    """Attainable DRAM throughput per stream mix: 2^28 floats per array
    (1 GiB each, four times the 256 MB last-level cache, so repeated
    launches cannot be served from it), 10 timed launches."""
    import torch
    import paper_2501_09398_amd as kb
    n = 1 << 28
    rows = []
    for nin, nout in STREAM_MIXES:
        sec = kb.stream_probe(nin, nout, n, reps=10)
        gbs = (nin + nout) * n * 4 / sec / 1e9
        rows.append({"reads": nin, "writes": nout, "us": sec * 1e6, "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS})
    torch.cuda.synchronize()
    print(json.dumps({"stream_calibration": rows, "elements_per_array": n}), flush=True)


def copy_calibration():
    """Three launches of the element-wise kernel as a plain copy: 256 MiB
    read and 256 MiB written per launch."""
    import torch
    import paper_2501_09398_amd as kb
    n = 1 << 26
    with kb.Problem(kb.SKELETON, (n,), (1, 1.0, 0.0), 0, device=0) as p:
        p.run(3, 0)
        p.last_timing()
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"elements": n, "bytes_read": 4 * n, "bytes_written": 4 * n,
                                           "launches": 3}}), flush=True)


def source_hash(path, start, end):
    """Hash of one kernel's source text, to tell whether stored hardware
    counters still describe the current kernel."""
    import hashlib
    src = open(path).read()
    a = src.index(start)
    b = src.index(end, a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def skeleton_kernel_hash():
    return source_hash(MISC_SOURCE, "template <int VEC>", "void make_skeleton")


def fdtd_fused_kernel_hash():
    return source_hash(FDTD_SOURCE, "void fdtd_fused_kernel(", "bool make_fdtd_fused")


def fdtd_tb2_kernel_hash():
    return source_hash(FDTD_SOURCE, "void fdtd_tb2_kernel(", "bool make_fdtd_tb2")


def fdtd_tb2_rows_kernel_hash():
    # the kernel and the access helpers above it
    return source_hash(FDTD_SOURCE, "struct Q4 {", "bool make_fdtd_tb2_rows")


def fdtd_tb3_rows_kernel_hash():
    # the kernel and its access helpers (it also uses those of the two-step one)
    return source_hash(FDTD_SOURCE, "struct Q4 {", "bool make_fdtd_tb3_rows")


def stored_traffic(path, current_hash):
    """Measured HBM bytes per launch from a committed counter summary, or
    None when it is missing or was taken on another version of the kernel."""
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != current_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def stored_json(path):
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return None


def host_info():
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(avail, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else avail
    return {"cpu_model": model, "cores_available": avail, "threads_used": threads}


def graph_memory(kb, np, torch, steps=8, graphs_per_step=4, b=2000):
    """Device memory held by instantiated, uploaded batch graphs vs their
    node count (the paper's Fig. 2 bars).  Graphs are added cumulatively --
    `graphs_per_step` more graphs of K*b nodes per point, all kept alive
    (one per problem handle, every workspace allocated before the first
    reading) -- so each point moves the free-memory reading (which changes
    in 2 MiB steps) by several MiB; bytes per node is the least-squares
    slope over the points."""
    probs = [kb.Problem(kb.SKELETON, (N_ELEM,), (K,), SEED, device=0) for _ in range(steps * graphs_per_step)]
    torch.cuda.synchronize()
    f0 = torch.cuda.mem_get_info()[0]
    pts = []
    for s in range(steps):
        for p in probs[s * graphs_per_step:(s + 1) * graphs_per_step]:
            p.run(b, b)
            p.last_timing()
        torch.cuda.synchronize()
        pts.append(((s + 1) * graphs_per_step * K * b, f0 - torch.cuda.mem_get_info()[0]))
    for p in probs:
        p.destroy()
    x = np.array([q[0] for q in pts], float)
    y = np.array([q[1] for q in pts], float)
    slope, icpt = np.polyfit(x, y, 1)
    return {"bytes_per_node": float(slope), "bytes_fixed": float(icpt), "graphs_per_point": graphs_per_step,
            "nodes_per_graph": K * b, "points_nodes_bytes": [[int(a), int(c)] for a, c in pts],
            "monotone": bool(np.all(np.diff(y) >= 0))}


def table1_sweep(kb, pm, np, sizes=tuple(1 << e for e in range(10, 23, 2)), reps=2):
    """The structure of the paper's Table I on MI355X: for each vector size
    of the K = 4 skeleton chain (2^10 .. 2^22), 10,000 iterations per launch
    and in graph batches over the 22 divisors of 10^4 up to 2000, Eq. 2 and
    Eq. 6 fitted by least squares (MAE as in the table), the model's b*
    against the measured best, and the speed-up at b*."""
    cands = pm.divisors(ITERS, 1, 2000)
    rows = []
    for n in sizes:
        with kb.Problem(kb.SKELETON, (n,), (K,), SEED) as p:
            p.set_option(kb.OPT_GRAPH_CACHE, 0)         # every run pays its own T_C
            p.run(ITERS, 0)
            p.last_timing()
            per_launch = float(np.median([_run_exec(p, 0) for _ in range(reps)]))
            sweep = []
            for b in cands:
                ts = [_run_both(p, b) for _ in range(reps)]
                sweep.append((b, float(np.median([t[0] for t in ts])), float(np.median([t[1] for t in ts]))))
        S = np.array([q[0] for q in sweep], float)
        model = pm.Model(pm.fit_creation(K * S, [q[1] for q in sweep]),
                         pm.fit_execution(S, [q[2] for q in sweep]), K=K)
        b_model, t_model = model.best(cands)
        total = {q[0]: q[1] + q[2] for q in sweep}
        b_meas = min(total, key=total.get)
        rows.append({"n": n, "per_launch_ms": per_launch * 1e3,
                     "k_c_us_per_node": model.creation.k_c * 1e6, "b_c_ms": model.creation.b_c * 1e3,
                     "mae_c_ms": model.creation.mae * 1e3,
                     "a_ms": model.execution.a * 1e3, "b_ms": model.execution.b * 1e3,
                     "mae_e_ms": model.execution.mae * 1e3,
                     "b_model": b_model, "b_closed_form": model.s_closed_form(), "b_measured_best": b_meas,
                     "total_at_b_model_ms": total[b_model] * 1e3, "total_at_b_measured_ms": total[b_meas] * 1e3,
                     "speedup_at_b_model": per_launch / total[b_model]})
    return rows


def _run_exec(p, b):
    p.run(ITERS, b)
    return p.last_timing()["t_exec_s"]


def _run_both(p, b):
    p.run(ITERS, b)
    t = p.last_timing()
    return t["t_create_s"], t["t_exec_s"]


def builders_and_update(kb, np, batches=(100, 1000, 2500), reps=3):
    """T_C of the two builders (explicit kernel nodes, stream capture of the
    per-launch loop) vs batch size, and what a change of node arguments
    costs: refitting the cached graphs in place (hipGraphExecUpdate) vs
    dropping them and paying T_C again on the next run."""
    out = {"t_create_ms": {}, "update": {}}
    a_new = np.array([0.95, 0.97, 0.99, 0.93], np.float32)
    for builder, name in ((0, "explicit"), (1, "capture")):
        with kb.Problem(kb.SKELETON, (N_ELEM,), (K,), SEED, device=0) as p:
            p.set_option(kb.OPT_BUILDER, builder)
            p.set_option(kb.OPT_GRAPH_CACHE, 0)
            row = {}
            for b in batches:
                tc = []
                for _ in range(reps):
                    p.run(b, b)
                    tc.append(p.last_timing()["t_create_s"])
                row[str(b)] = float(np.median(tc)) * 1e3
            out["t_create_ms"][name] = row
    for b in batches:
        row = {}
        for mode, name in ((0, "drop_and_rebuild"), (1, "refit_in_place")):
            with kb.Problem(kb.SKELETON, (N_ELEM,), (K,), SEED, device=0) as p:
                p.set_option(kb.OPT_GRAPH_UPDATE, mode)
                p.run(b, b)
                p.last_timing()
                upd, tc = [], []
                for r in range(reps):
                    p.write(kb.F_A, a_new if r % 2 == 0 else a_new * np.float32(0.999))
                    p.run(b, b)
                    t = p.last_timing()
                    upd.append(t["t_update_s"])
                    tc.append(t["t_create_s"])
                row[name] = {"write_ms": float(np.median(upd)) * 1e3, "next_run_t_create_ms": float(np.median(tc)) * 1e3}
        out["update"][str(b)] = row
    return out


def workloads(kb, pm, autotune, np):
    """The other workloads of the study, each per launch vs graph batches,
    plus the large grids against the HBM roofline.  Seeded synthetic inputs
    of each workload's shape; every run starts from the device-resident state."""
    import torch
    out = {}

    def torch_sync():
        torch.cuda.synchronize()

    def arm(p, n, b, reps=3):
        p.run(n, b)
        p.last_timing()                      # warm-up (builds the graph if any)
        te = []
        for _ in range(reps):
            p.run(n, b)
            te.append(p.last_timing()["t_exec_s"])
        return float(np.median(te))

    def cold(p, n, b):
        p.set_option(kb.OPT_GRAPH_CACHE, 0)
        p.run(n, b)
        t = p.last_timing()
        p.set_option(kb.OPT_GRAPH_CACHE, 1)
        return t["t_create_s"] + t["t_exec_s"]

    # 2D thermal stencil, 256x256, 1000 steps (launch-bound)
    note("workloads: heat2d 256^2")
    n = 1000
    d = {"steps": n, "cells": 256 * 256}
    with kb.Problem(kb.HEAT2D, (256, 256), kb.HEAT_COEFFS, SEED) as p:
        p.set_option(kb.OPT_TILE, 1)
        d["per_launch_us_step"] = arm(p, n, 0) / n * 1e6
        for b in (1, 10, 100, 1000):
            d[f"graph_b{b}_us_step"] = arm(p, n, b) / n * 1e6
            d[f"graph_b{b}_cold_us_step"] = cold(p, n, b) / n * 1e6
    tr = autotune.tune(kb, kb.HEAT2D, (256, 256), kb.HEAT_COEFFS, n, seed=SEED, reps=2)
    d["autotuned"] = {"variant": tr.variant, "depth": tr.depth, "b": tr.b,
                      "us_step": tr.us_per_step_warm, "cold_us_step": tr.us_per_step_cold,
                      "t_create_ms": tr.t_create_s * 1e3, "b_measured_best": tr.b_measured}
    d["speedup_graph_b100_vs_per_launch"] = d["per_launch_us_step"] / d["graph_b100_us_step"]
    d["speedup_autotuned_vs_per_launch"] = d["per_launch_us_step"] / tr.us_per_step_warm
    d["gcell_upd_s_autotuned"] = 256 * 256 / tr.us_per_step_warm / 1e3
    out["heat2d_256x256_1000"] = d

    # 3D stencil 8x512x512, 2000 steps
    note("workloads: heat3d 8x512^2")
    n = 2000
    d = {"steps": n, "cells": 8 * 512 * 512}
    with kb.Problem(kb.HEAT3D, (8, 512, 512), kb.HEAT_COEFFS, SEED) as p:
        for v in (1, 4):
            p.set_option(kb.OPT_TILE, v)
            d[f"v{v}_per_launch_us_step"] = arm(p, n, 0, 2) / n * 1e6
            d[f"v{v}_graph_b100_us_step"] = arm(p, n, 100, 2) / n * 1e6
        # temporal blocking: 4 steps per launch, graph batches of 100 launches
        p.set_option(kb.OPT_TILE, 5)
        p.set_option(kb.OPT_TDEPTH, 4)
        d["v5_t4_per_launch_us_step"] = arm(p, n, 0, 2) / n * 1e6
        d["v5_t4_graph_b100_us_step"] = arm(p, n, 100, 2) / n * 1e6
    # variant, depth and b from the autotuner
    tr = autotune.tune(kb, kb.HEAT3D, (8, 512, 512), kb.HEAT_COEFFS, n, seed=SEED, reps=2)
    d["autotuned"] = {"variant": tr.variant, "depth": tr.depth, "b": tr.b,
                      "us_step": tr.us_per_step_warm, "cold_us_step": tr.us_per_step_cold,
                      "t_create_ms": tr.t_create_s * 1e3, "b_measured_best": tr.b_measured}
    d["autotuned_graph_us_step"] = tr.us_per_step_warm
    best = min(d[k] for k in d if "graph" in k and k.endswith("us_step"))
    d["gcell_upd_s"] = 8 * 512 * 512 / best / 1e3
    out["heat3d_8x512x512_2000"] = d

    # many uneven grids, one kernel per step over all of them
    note("workloads: 64 uneven grids")
    import synth
    sides = synth.multigrid_sides(SEED, 64)
    shape = [64] + [v for s in sides for v in (s, s)]
    n = 2000
    cells = sum(s * s for s in sides)
    d = {"steps": n, "grids": 64, "cells": cells}
    with kb.Problem(kb.HEAT2D_MULTI, shape, kb.HEAT_COEFFS, SEED) as p:
        for v, name in ((2, "strip"), (1, "cell"), (3, "tb_t1")):
            p.set_option(kb.OPT_TILE, v)
            d[f"{name}_per_launch_us_step"] = arm(p, n, 0, 2) / n * 1e6
            d[f"{name}_graph_b100_us_step"] = arm(p, n, 100, 2) / n * 1e6
    # temporal blocking: variant, depth and b from the autotuner
    tr = autotune.tune(kb, kb.HEAT2D_MULTI, shape, kb.HEAT_COEFFS, n, seed=SEED, reps=2)
    d["autotuned"] = {"variant": tr.variant, "depth": tr.depth, "b": tr.b,
                      "us_step": tr.us_per_step_warm, "cold_us_step": tr.us_per_step_cold,
                      "t_create_ms": tr.t_create_s * 1e3, "b_measured_best": tr.b_measured,
                      "kernel_table": [(v, t, round(us, 3)) for v, t, us in tr.kernel_table]}
    with kb.Problem(kb.HEAT2D_MULTI, shape, kb.HEAT_COEFFS, SEED) as p:
        p.set_option(kb.OPT_TILE, tr.variant)
        p.set_option(kb.OPT_TDEPTH, tr.depth)
        d["autotuned_per_launch_us_step"] = arm(p, n, 0, 2) / n * 1e6
        d["autotuned_graph_us_step"] = arm(p, n, tr.b, 2) / n * 1e6
        # the persistent arm: one cooperative launch for all 2000 steps,
        # super-steps of t steps separated by grid-wide barriers
        p.set_option(kb.OPT_PERSISTENT, 1)
        for t in (1, tr.depth, 8):
            p.set_option(kb.OPT_TDEPTH, t)
            d[f"persistent_t{t}_us_step"] = arm(p, n, 0, 2) / n * 1e6
    # the alternative the grouped kernel replaces: 64 separate problems, each
    # advanced on its own (one launch per grid per step, or one graph each)
    probs = [kb.Problem(kb.HEAT2D, (sd, sd), kb.HEAT_COEFFS, SEED + g) for g, sd in enumerate(sides)]
    ns = 200
    for b, name in ((0, "separate_per_launch_us_step"), (100, "separate_graph_b100_us_step")):
        for q in probs:
            q.run(ns, b)
        torch_sync()
        t0 = time.perf_counter()
        for q in probs:
            q.run(ns, b)
        torch_sync()
        d[name] = (time.perf_counter() - t0) / ns * 1e6
    for q in probs:
        q.destroy()
    one_step = min(d["strip_graph_b100_us_step"], d["cell_graph_b100_us_step"], d["tb_t1_graph_b100_us_step"])
    best = min(one_step, d["autotuned_graph_us_step"])
    d["gcell_upd_s"] = cells / best / 1e3
    # one step per launch: 12 B per cell-step must cross HBM
    d["hbm_frac_one_step_per_launch"] = 12.0 * cells / (one_step * 1e-6) / (HBM_PEAK_GBS * 1e9)
    d["speedup_best_vs_separate_per_launch"] = d["separate_per_launch_us_step"] / best
    out["multigrid_64_2000"] = d

    # FDTD cavities
    note("workloads: FDTD cavities")
    # (separate H and E kernels: 72 B per node-step; the fused step: 48 B)
    for N, n in ((128, 10000), (256, 2000)):
        d = {"steps": n, "cells": N ** 3}
        with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, SEED) as p:
            for v, name in ((2, "separate"), (0, "fused")):     # 0: the default fused variant for N
                p.set_option(kb.OPT_TILE, v)
                d[f"{name}_per_launch_us_step"] = arm(p, n, 0, 1) / n * 1e6
                d[f"{name}_graph_b100_us_step"] = arm(p, n, 100, 1) / n * 1e6
        d["graph_b100_us_step"] = min(d["separate_graph_b100_us_step"], d["fused_graph_b100_us_step"])
        d["gcell_upd_s"] = N ** 3 / d["graph_b100_us_step"] / 1e3
        for name, B in (("separate", 72.0), ("fused", 48.0)):
            d[f"{name}_hbm_frac"] = B * (N + 1) ** 3 / (d[f"{name}_graph_b100_us_step"] * 1e-6) / (HBM_PEAK_GBS * 1e9)
        d["speedup_fused_vs_separate"] = d["separate_graph_b100_us_step"] / d["fused_graph_b100_us_step"]
        if N == 128:
            tr = autotune.tune(kb, kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, n, seed=SEED, reps=2,
                               b_candidates=[10, 20, 50, 100, 200, 500, 1000, 2000])
            d["autotuned"] = {"variant": tr.variant, "depth": tr.depth, "b": tr.b, "us_step": tr.us_per_step_warm,
                              "t_create_ms": tr.t_create_s * 1e3, "b_measured_best": tr.b_measured}
        out[f"fdtd_{N}^3_{n}"] = d

    note("workloads: surrogate")
    # learned 16-step surrogate at 512^2 (network, residual check and the
    # predicated fallback in every block) vs the plain stencil
    from paper_2501_09398_amd import sg_train
    if os.path.exists(sg_train.WEIGHTS_FILE):
        w = sg_train.load_weights()
        N, k, n = 512, 16, 160
        T0, _ = synth.heat2d_init(SEED, N, N)
        P = synth.hot_spot_power(SEED, N, N)
        d = {"steps": n, "cells": N * N, "k": k, "blocks": n // k}
        for var, name in ((1, "fused"), (2, "per_layer")):
            with kb.Problem(kb.HEAT2D_SURROGATE, (N, N), kb.HEAT_COEFFS + (0.8, 1e-3, k), SEED) as p:
                p.set_option(kb.OPT_TILE, var)
                p.write(kb.F_T, T0)
                p.write(kb.F_P, P)
                p.write(kb.F_W, w)
                d[f"{name}_per_launch_us_block"] = arm(p, n, 0, 2) / (n // k) * 1e6
                d[f"{name}_graph_b10_us_block"] = arm(p, n, 10, 2) / (n // k) * 1e6
                st = p.read(kb.F_SGSTATS)
                d[f"{name}_fallback_rate"] = float(st[1]) / max(1.0, float(st[0]))
        tr = autotune.tune(kb, kb.HEAT2D, (N, N), kb.HEAT_COEFFS, n, seed=SEED, reps=2)
        d["plain_autotuned"] = {"variant": tr.variant, "depth": tr.depth, "b": tr.b,
                                "us_block": tr.us_per_step_warm * k}
        d["speed_vs_plain"] = tr.us_per_step_warm * k / d["fused_graph_b10_us_block"]
        # algorithmic MFMA work: 2 * (9*2*32 + 2 * 9*32*32 + 9*32) = 38,592 FLOP
        # per pixel and application (10.12 GFLOP at 512^2), against the
        # 2.5 PFLOP/s dense bf16 peak; the block time includes the check and
        # the (predicated) fallback node
        gflop = 38592.0 * N * N / 1e9
        d["network_gflop"] = gflop
        d["fused_block_tflops"] = gflop / (d["fused_graph_b10_us_block"] * 1e-6) / 1e3
        d["fused_block_mfma_frac"] = d["fused_block_tflops"] / 2500.0
        ev = sg_train.evaluate(w, [SEED + 1, SEED + 2])
        d["accuracy_vs_plain_gpu"] = {key: max(r[key] for r in ev) for key in ev[0] if key != "seed"}
        out["surrogate_512_k16"] = d

    # large grids against the HBM roofline (working sets >> 256 MB cache)
    note("workloads: large grids")
    big = {}
    for name, prob, shp, var, bytes_per_cell in (
            ("heat2d_16384^2", kb.HEAT2D, (16384, 16384), 13, 12.0),
            ("heat2d_8192^2", kb.HEAT2D, (8192, 8192), 13, 12.0),
            ("heat3d_8x4096^2", kb.HEAT3D, (8, 4096, 4096), 9, 8.5)):
        with kb.Problem(prob, shp, kb.HEAT_COEFFS, SEED) as p:
            p.set_option(kb.OPT_TILE, var)
            t = arm(p, 20, 0, 2) / 20
        cells = int(np.prod(shp))
        gbs = bytes_per_cell * cells / t / 1e9
        big[name] = {"us_step": t * 1e6, "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS, "gcell_upd_s": cells / t / 1e9}
    # the same grids with temporal blocking: t steps per launch from one read
    # of T and P and one write of T, so the one-step roofline above no longer
    # bounds the step; frac is the kernel's own bytes per launch over its
    # duration, effective_frac the one-step bytes per step over the step time
    for name, prob, shp, cands, bytes_per_cell in (
            ("heat2d_16384^2", kb.HEAT2D, (16384, 16384), [(19, 6), (19, 8), (20, 6), (20, 8), (21, 6), (21, 8)], 12.0),
            ("heat2d_8192^2", kb.HEAT2D, (8192, 8192), [(19, 6), (19, 8), (20, 6), (20, 8), (21, 6), (21, 8)], 12.0),
            ("heat3d_8x4096^2", kb.HEAT3D, (8, 4096, 4096), [(11, 2), (11, 3), (11, 4), (11, 6)], 8.5)):
        cells = int(np.prod(shp))
        rows = []
        with kb.Problem(prob, shp, kb.HEAT_COEFFS, SEED) as p:
            for v, t in cands:
                p.set_option(kb.OPT_TILE, v)
                p.set_option(kb.OPT_TDEPTH, t)
                rows.append((arm(p, 24, 0, 2) / 24, v, t))
        ts, v, t = min(rows)
        gbs = bytes_per_cell * cells / (ts * t) / 1e9
        big[f"{name}_temporal"] = {"variant": v, "depth": t, "us_step": ts * 1e6, "gcell_upd_s": cells / ts / 1e9,
                                   "speedup_vs_one_step": big[name]["us_step"] / (ts * 1e6),
                                   "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS,
                                   "effective_frac": bytes_per_cell * cells / ts / 1e9 / HBM_PEAK_GBS,
                                   "tried": [{"variant": vv, "depth": tt, "us_step": x * 1e6} for x, vv, tt in rows]}
    d = out["fdtd_256^3_2000"]
    for name in ("separate", "fused"):
        big[f"fdtd_256^3_{name}"] = {"us_step": d[f"{name}_graph_b100_us_step"], "frac": d[f"{name}_hbm_frac"],
                                     "GB_s": d[f"{name}_hbm_frac"] * HBM_PEAK_GBS,
                                     "gcell_upd_s": 256 ** 3 / d[f"{name}_graph_b100_us_step"] / 1e3}
    out["large_grids_hbm"] = big
    return out


def workloads_cpu_baseline(kb, np, out):
    """CPU-baseline leg of the other workloads: the oracle timed on this
    host's cores (one thread, then every thread this process may use) on a
    stated sample of each workload, and the GPU's result on that same
    sample (the configuration the autotuner chose) against the float32
    oracle (0.0 = the same bits) and the float64 oracle (relative max-norm;
    for the surrogate also on the increment T - T0)."""
    import oracle
    import synth
    info = host_info()
    nt = info["threads_used"]
    res = {"host": info}

    def rel(a, b):
        a = np.asarray(a, np.float64)
        return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))

    def timed(fn, threads):
        with oracle.threads(threads):
            t0 = time.perf_counter()
            r = fn()
            return r, time.perf_counter() - t0

    def gpu_run(prob, shape, coeffs, seed, tuned, steps, writes=()):
        with kb.Problem(prob, shape, coeffs, seed) as p:
            for fid, v in writes:
                p.write(fid, v)
            if tuned:
                p.set_option(kb.OPT_TILE, tuned["variant"])
                p.set_option(kb.OPT_TDEPTH, tuned.get("depth", 1))
                p.run(steps, tuned["b"])
            else:
                p.run(steps, 100)
            return p.read(kb.F_T)

    def entry(cell_steps_1, t1, cell_steps_n, tn, sample, got, r32, r64, **extra):
        d = {"cpu_value_gcell_upd_s": cell_steps_n / tn / 1e9, "cores": nt, "seconds": tn,
             "single_thread_gcell_upd_s": cell_steps_1 / t1 / 1e9, "single_thread_seconds": t1,
             "sample": sample, "kind": "oracle",
             "gpu_rel_maxnorm_vs_float32_oracle": rel(got, r32),
             "gpu_bit_exact_vs_float32_oracle": bool(np.array_equal(got, r32)),
             "gpu_rel_maxnorm_vs_float64_oracle": rel(got, r64),
             "float32_oracle_rel_maxnorm_vs_float64": rel(r32, r64)}
        d.update(extra)
        return d

    # 2D thermal stencil 256^2, the whole 1000-step job
    note("cpu baseline: heat2d 256^2")
    n = 1000
    T0, P = synth.heat2d_init(SEED, 256, 256)
    got = gpu_run(kb.HEAT2D, (256, 256), kb.HEAT_COEFFS, SEED, out["heat2d_256x256_1000"]["autotuned"], n)
    r32, t1 = timed(lambda: oracle.heat2d(T0, P, n, dtype=np.float32), 1)
    _, tn = timed(lambda: oracle.heat2d(T0, P, n, dtype=np.float32), nt)
    r64, _ = timed(lambda: oracle.heat2d(T0, P, n, dtype=np.float64), nt)
    cs = 256 * 256 * n
    res["heat2d_256x256_1000"] = entry(cs, t1, cs, tn, "the whole job: 256^2, 1000 steps from the seeded state",
                                       got, r32, r64)

    # 3D stencil 8 x 512^2, the whole 2000-step job (one thread: 200 steps)
    note("cpu baseline: heat3d 8x512^2")
    n, n1 = 2000, 200
    T0, P = synth.heat3d_init(SEED, 8, 512, 512)
    got = gpu_run(kb.HEAT3D, (8, 512, 512), kb.HEAT_COEFFS, SEED, out["heat3d_8x512x512_2000"]["autotuned"], n)
    _, t1 = timed(lambda: oracle.heat3d(T0, P, n1, dtype=np.float32), 1)
    r32, tn = timed(lambda: oracle.heat3d(T0, P, n, dtype=np.float32), nt)
    r64, _ = timed(lambda: oracle.heat3d(T0, P, n, dtype=np.float64), nt)
    c = 8 * 512 * 512
    res["heat3d_8x512x512_2000"] = entry(c * n1, t1, c * n, tn,
                                         "the whole job: 8x512^2, 2000 steps (single thread: the first 200)",
                                         got, r32, r64)

    # 64 uneven grids: the first 200 steps of the job (one thread: 20)
    note("cpu baseline: 64 uneven grids")
    sides = synth.multigrid_sides(SEED, 64)
    shape = [64] + [v for sd in sides for v in (sd, sd)]
    n, n1 = 200, 20
    T0s, Ps = synth.multigrid_init(SEED, sides)
    got = gpu_run(kb.HEAT2D_MULTI, shape, kb.HEAT_COEFFS, SEED, out["multigrid_64_2000"]["autotuned"], n)
    _, t1 = timed(lambda: [oracle.heat2d(a, b, n1, dtype=np.float32) for a, b in zip(T0s, Ps)], 1)
    r32, tn = timed(lambda: [oracle.heat2d(a, b, n, dtype=np.float32) for a, b in zip(T0s, Ps)], nt)
    r64, _ = timed(lambda: [oracle.heat2d(a, b, n, dtype=np.float64) for a, b in zip(T0s, Ps)], nt)
    cells = sum(sd * sd for sd in sides)
    r32 = np.concatenate([r.ravel() for r in r32])
    r64 = np.concatenate([r.ravel() for r in r64])
    res["multigrid_64_2000"] = entry(cells * n1, t1, cells * n, tn,
                                     f"the first {n} steps of the job ({cells} cells in 64 grids; single thread: "
                                     f"{n1} steps)", got, r32, r64)

    # FDTD cavity 128^3: the first 100 steps of the job, source on
    note("cpu baseline: FDTD 128^3")
    N, n, n1 = 128, 100, 20
    src = synth.fdtd_source_cell(SEED, N)
    g64, g32 = oracle.fdtd_pulse(n + 1)
    tuned = out["fdtd_128^3_10000"].get("autotuned")
    with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, SEED) as p:
        if tuned:
            p.set_option(kb.OPT_TILE, tuned["variant"])
            p.set_option(kb.OPT_TDEPTH, tuned.get("depth", 1))
        p.run(n, 20)
        gotf = {k: p.read(fid) for k, fid in kb.FDTD_FIELDS.items()}
    z32, z64 = oracle.fdtd_zero_fields(N, np.float32), oracle.fdtd_zero_fields(N, np.float64)
    _, t1 = timed(lambda: oracle.fdtd(z32, N, n1, src=src, g=g32, dtype=np.float32), 1)
    (f32, _), tn = timed(lambda: oracle.fdtd(z32, N, n, src=src, g=g32, dtype=np.float32), nt)
    (f64, _), _ = timed(lambda: oracle.fdtd(z64, N, n, src=src, g=g64, dtype=np.float64), nt)
    keys = list(oracle.FDTD_FIELDS)
    got = np.concatenate([gotf[k].ravel() for k in keys])
    r32 = np.concatenate([f32[k].ravel() for k in keys])
    r64 = np.concatenate([f64[k].ravel() for k in keys])
    res["fdtd_128^3_10000"] = entry(N ** 3 * n1, t1, N ** 3 * n, tn,
                                    f"the first {n} steps of the job (all six fields; single thread: {n1})",
                                    got, r32, r64)

    # learned surrogate 512^2: ten blocks of 16 steps against the plain
    # stencil in float64; the CPU leg is the float64 network oracle (one
    # application) and the plain float64 stencil
    from paper_2501_09398_amd import sg_train
    if os.path.exists(sg_train.WEIGHTS_FILE):
        note("cpu baseline: surrogate 512^2")
        w = sg_train.load_weights()
        N, k, n = 512, 16, 160
        T0, _ = synth.heat2d_init(SEED, N, N)
        P = synth.hot_spot_power(SEED, N, N)
        with kb.Problem(kb.HEAT2D_SURROGATE, (N, N), kb.HEAT_COEFFS + (0.8, 1e-3, k), SEED) as p:
            p.set_option(kb.OPT_TILE, 1)
            p.write(kb.F_T, T0)
            p.write(kb.F_P, P)
            p.write(kb.F_W, w)
            p.run(n, 10)
            got = p.read(kb.F_T).astype(np.float64)
            st = p.read(kb.F_SGSTATS)
        plain = gpu_run(kb.HEAT2D, (N, N), kb.HEAT_COEFFS, SEED, None, n, writes=((kb.F_T, T0), (kb.F_P, P)))
        r64, tp = timed(lambda: oracle.heat2d(T0, P, n, dtype=np.float64), nt)
        _, tnet = timed(lambda: oracle.sg_forward(w.astype(np.float64), T0, P), nt)
        inc = r64 - T0
        e_inc = lambda a: float(np.max(np.abs((np.asarray(a, np.float64) - T0) - inc)) / np.max(np.abs(inc)))
        # one explicit step of 16c per block: the method's cheapest stand-in
        eul = T0.astype(np.float64)
        for _ in range(n // k):
            eul = oracle.heat2d(eul, P, 1, c=k * 1e-3, dtype=np.float64)
        res["surrogate_512_k16"] = {
            "sample": f"{n // k} blocks of {k} steps at 512^2 from the seeded state with hot spots",
            "surrogate_rel_maxnorm_vs_float64": rel(got, r64), "surrogate_inc_rel_maxnorm_vs_float64": e_inc(got),
            "plain_gpu_rel_maxnorm_vs_float64": rel(plain, r64), "plain_gpu_inc_rel_maxnorm_vs_float64": e_inc(plain),
            "euler16c_rel_maxnorm_vs_float64": rel(eul, r64), "euler16c_inc_rel_maxnorm_vs_float64": e_inc(eul),
            "persistence_rel_maxnorm_vs_float64": rel(T0, r64),
            "fallbacks": int(st[1]), "blocks": int(st[0]),
            "cpu_plain_float64_gcell_upd_s": N * N * n / tp / 1e9,
            "cpu_network_float64_s_per_application": tnet, "cores": nt, "kind": "oracle"}
    return res


def fdtd_headline(args, kb, autotune, np, torch):
    """The cavity job: autotuned variant and b, graph arm (each job pays
    its own T_C) and per-launch arm, roofline from the replay events."""
    from paper_2501_09398_amd import perfmodel as pm
    N, n = N_FDTD, FDTD_STEPS
    cells, nodes = N ** 3, (N + 1) ** 3
    tuned = None
    if args.b > 0:
        variant, depth, b = args.fdtd_variant, args.fdtd_depth, args.b
    else:
        note("cavity: autotuning the kernel variant and b")
        tr = autotune.tune(kb, kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, n, seed=SEED, reps=1, probe_steps=200,
                           b_candidates=FDTD_B_CANDIDATES,
                           kernel_candidates_override=[(2, 1), (5, 1), (7, 1), (8, 2), (9, 2), (10, 2), (10, 3)])
        variant, depth, b = tr.variant, tr.depth, tr.b
        tuned = {"variant": tr.variant, "depth": tr.depth, "b": tr.b, "b_measured_best": tr.b_measured,
                 "kernel_table_us_step": [(v, t, round(us, 2)) for v, t, us in tr.kernel_table],
                 "batch_table_ms": [[bb, round(tc * 1e3, 3), round(te * 1e3, 3)] for bb, tc, te in tr.batch_table],
                 "model": tr.model}
    p = kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, SEED, device=0)
    p.set_option(kb.OPT_TILE, variant)
    p.set_option(kb.OPT_TDEPTH, depth)
    p.set_option(kb.OPT_GRAPH_CACHE, 0)          # every job pays its own T_C (Eq. 1)
    Kf = p.kernels_per_iter()

    def job(bb):
        p.run(n, bb)
        return p.last_timing()                   # synchronises

    def arm(bb):
        for _ in range(args.warmup):
            job(bb)
        torch.cuda.synchronize()
        T, TC, TE = [], [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s0 = time.perf_counter()
            t = job(bb)
            T.append(time.perf_counter() - s0)
            TC.append(t["t_create_s"])
            TE.append(t["t_exec_s"])
        torch.cuda.synchronize()
        return T, TC, TE, time.perf_counter() - t0

    out = {"variant": variant, "depth": depth, "b": b, "kernels_per_iter": Kf, "autotune": tuned}
    g_T = g_TC = g_TE = None
    wall = None
    if args.arm in ("both", "graph"):
        note(f"cavity: graph arm, variant {variant} depth {depth} b {b}")
        g_T, g_TC, g_TE, wall = arm(b)
        out["graph"] = {"b": b, "us_per_iter": float(np.mean(g_T)) / n * 1e6,
                        "us_per_iter_warm": float(np.mean(g_TE)) / n * 1e6,
                        "us_per_iter_warm_std": float(np.std(g_TE)) / n * 1e6,
                        "t_create_ms": float(np.mean(g_TC)) * 1e3,
                        "gcell_upd_s": cells * n / float(np.mean(g_T)) / 1e9}
    if args.arm in ("both", "per_launch"):
        note("cavity: per-launch arm")
        b_T, _, b_TE, b_wall = arm(0)
        out["per_launch"] = {"us_per_iter": float(np.mean(b_T)) / n * 1e6,
                             "us_per_iter_device": float(np.mean(b_TE)) / n * 1e6,
                             "us_per_iter_device_std": float(np.std(b_TE)) / n * 1e6,
                             "gcell_upd_s": cells * n / float(np.mean(b_T)) / 1e9}
        if wall is None:
            wall, g_TE = b_wall, b_TE
    if g_T is not None and args.arm == "both":
        sp, sp_err = pm.speedup(b_T, g_T)
        out["speedup"], out["speedup_err"] = sp, sp_err
        out["speedup_device"] = float(np.mean(b_TE)) / float(np.mean(g_TE))
    out["wall_s"] = wall
    out["value"] = cells * n * args.steps / wall / 1e9
    # roofline of the dominant kernel.  Its own algorithmic bytes per launch:
    # the six fields of every node read once and written once (48 B per
    # node), whether the launch advances one step (the fused step) or two
    # (the two-step kernels).  Its duration is bounded above by the launch's
    # share of the step time from the events around the timed replays (the
    # share also holds the iteration's second kernel, if any -- the source or
    # the step counter's advance -- and the node-to-node gaps); the committed
    # kernel trace gives the kernel's own duration.  The one-step figure of
    # the method (72 B per cell-step with separate H and E kernels) over the
    # step time is reported beside it as the effective rate.
    step_s = float(np.mean(g_TE)) / n
    p.destroy()
    eff = variant or (7 if N >= 176 else 5)          # the default fused variant for the size
    blocked = eff >= 8 and depth in (2, 3)            # two or three steps per launch
    if blocked and depth == 3:
        name = "fdtd_tb3_rows_kernel<true,true,4>"
    elif blocked:
        name = {8: "fdtd_tb2_kernel<true>", 9: "fdtd_tb2_rows_kernel<true,16,false,true>",
                10: "fdtd_tb2_rows_kernel<true,12,true,true>"}[eff]
    else:
        name = {7: "fdtd_fused_kernel<1,true>", 5: "fdtd_fused_kernel<1,false>", 6: "fdtd_fused_kernel<8,false>",
                8: "fdtd_fused_kernel<1,true>", 9: "fdtd_fused_kernel<1,true>",
                10: "fdtd_fused_kernel<1,true>"}.get(eff, "fdtd_h_vec_kernel + fdtd_e_vec_kernel")
    steps_per_launch = depth if blocked else 1
    probe_s = kb.stream_probe(6, 6, 1 << 28, reps=10)
    mix_gbs = 12 * (1 << 28) * 4 / probe_s / 1e9
    launch_s = step_s * steps_per_launch
    kern_bytes = FDTD_KERNEL_BYTES_PER_NODE * nodes
    kern = kern_bytes / launch_s / 1e9
    effective = FDTD_BYTES_PER_CELL_STEP * cells / step_s / 1e9
    if name.startswith("fdtd_tb3_rows"):
        traffic = stored_traffic(FDTD_TB3_COUNTERS, fdtd_tb3_rows_kernel_hash())
    elif name.startswith("fdtd_tb2_rows"):
        traffic = stored_traffic(FDTD_ROWS_COUNTERS, fdtd_tb2_rows_kernel_hash())
    elif name.startswith("fdtd_tb2"):
        traffic = stored_traffic(FDTD_TB2_COUNTERS, fdtd_tb2_kernel_hash())
    else:
        traffic = stored_traffic(FDTD_COUNTERS, fdtd_fused_kernel_hash())
    out["roofline"] = {
        "bound": "hbm", "achieved": kern, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kern / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": name, "bytes_per_launch": kern_bytes, "bytes_per_node_launch": FDTD_KERNEL_BYTES_PER_NODE,
        "nodes_per_launch": nodes, "steps_per_launch": steps_per_launch,
        "launch_us_upper": launch_s * 1e6, "step_us": step_s * 1e6,
        "stream_mix_6r6w_GB_s": mix_gbs, "frac_of_stream_mix": kern / mix_gbs,
        # the method's one-step bytes (separate H and E kernels) per step time
        "effective_GB_s": effective, "effective_bytes_per_cell_step": FDTD_BYTES_PER_CELL_STEP,
        "effective_frac": effective / HBM_PEAK_GBS,
        "trace": stored_json(os.path.join(ROOT, "profiles", "fdtd_256_graph_trace.json"))}
    # the three-step kernel also spends half its launch issuing vector
    # instructions: the committed instruction counters (same kernel source)
    # give the issue time per SIMD, set here against the live launch time
    if name.startswith("fdtd_tb3_rows"):
        sq = stored_json(os.path.join(ROOT, "profiles", "fdtd_256_tb3_rows_sq_counters.json"))
        if sq and sq.get("kernel_source_sha") == fdtd_tb3_rows_kernel_hash():
            out["roofline"]["valu_issue_us_per_simd"] = sq["valu_issue_us_per_simd"]
            out["roofline"]["valu_issue_frac"] = sq["valu_issue_us_per_simd"] / (launch_s * 1e6)
    return out


def fdtd_cpu_baseline(kb, np, torch, steps_single=100, steps_all=1000):
    """The float32 oracle on a bounded sample of the cavity -- 256^3 from
    seeded random fields (no denormals in the timed loops) with the source
    on -- on one core and on all the cores this process may use; the GPU
    runs the same sample, which gives its error against the float64 oracle
    (and bit-equality with the float32 oracle)."""
    import oracle
    import synth
    info = host_info()
    N = N_FDTD
    M = N + 1
    rng = np.random.default_rng(SEED)
    f0 = {k: rng.uniform(-1.0, 1.0, (M, M, M)).astype(np.float32) for k in oracle.FDTD_FIELDS}
    src = synth.fdtd_source_cell(SEED, N)
    g64, g32 = oracle.fdtd_pulse(steps_all + 1)
    with oracle.threads(1):
        t0 = time.perf_counter()
        oracle.fdtd(f0, N, steps_single, src=src, g=g32, dtype=np.float32)
        t1 = time.perf_counter() - t0
    with oracle.threads(info["threads_used"]):
        t0 = time.perf_counter()
        ref32, _ = oracle.fdtd(f0, N, steps_all, src=src, g=g32, dtype=np.float32)
        tn = time.perf_counter() - t0
        ref64, _ = oracle.fdtd(f0, N, steps_all, src=src, g=g64, dtype=np.float64)
    with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, SEED, device=0) as p:
        for k, fid in kb.FDTD_FIELDS.items():
            p.write(fid, f0[k])
        p.run(steps_all, 20)
        got = {k: p.read(fid) for k, fid in kb.FDTD_FIELDS.items()}
    scale = max(float(np.max(np.abs(ref64[k]))) for k in oracle.FDTD_FIELDS)
    err64 = max(float(np.max(np.abs(got[k].astype(np.float64) - ref64[k]))) for k in oracle.FDTD_FIELDS) / scale
    exact = all(np.array_equal(got[k], ref32[k]) for k in oracle.FDTD_FIELDS)
    cells = N ** 3
    cpu = {"value": cells * steps_all / tn / 1e9, "unit": "Gcell-upd/s", "cores": info["threads_used"],
           "kind": "oracle",
           "sample": f"{steps_all} steps of the 256^3 cavity (float32 oracle, {info['threads_used']} threads, "
                     f"{tn:.1f} s) from seeded random fields with the source on; single thread: "
                     f"{steps_single} steps in {t1:.1f} s; {info['cpu_model']}",
           "single_thread": {"value": cells * steps_single / t1 / 1e9, "cores": 1, "steps": steps_single,
                             "seconds": t1},
           "cpu_model": info["cpu_model"], "cores_available": info["cores_available"]}
    fp64 = {"rel_maxnorm_vs_float64": err64, "bit_exact_vs_float32_oracle": exact, "steps": steps_all,
            "sample": "the CPU-baseline sample (256^3, random fields, source on), all six fields"}
    return cpu, fp64


def skeleton_section(args, kb, pm, np, torch, workloads_on):
    """The skeleton chain (2^16 float32, K = 4, 10,000 iterations per job):
    the b sweep (each b `sweep_reps` times, mean and standard deviation),
    Eq. 2 and Eq. 6 fitted with standard errors, graph jobs at the model's
    b against per-launch jobs, the per-node rate against the node floor."""
    prob = kb.Problem(kb.SKELETON, (N_ELEM,), (K,), SEED, device=0)
    prob.set_option(kb.OPT_GRAPH_CACHE, 0)       # every job pays its own T_C
    elem_updates = N_ELEM * K * ITERS

    def job(b):
        prob.run(ITERS, b)
        return prob.last_timing()

    cands = pm.divisors(ITERS, 1, 2000)
    sweep, model = [], None
    if not args.no_sweep and args.arm != "per_launch":
        job(100)
        for b in cands:
            reps = [job(b) for _ in range(args.sweep_reps)]
            tc = [t["t_create_s"] for t in reps]
            te = [t["t_exec_s"] for t in reps]
            sweep.append((b, float(np.mean(tc)), float(np.std(tc)), float(np.mean(te)), float(np.std(te))))
        S = np.array([s[0] for s in sweep], float)
        model = pm.Model(pm.fit_creation(K * S, [s[1] for s in sweep]),
                         pm.fit_execution(S, [s[3] for s in sweep]), K=K)
        b_model, _ = model.best(cands)
        measured_total = {s[0]: s[1] + s[3] for s in sweep}
        b_measured = min(measured_total, key=measured_total.get)
    b_star = args.skeleton_b if args.skeleton_b > 0 else (b_model if model else 100)
    steps = max(args.steps, 1)
    res = {"workload": "skeleton chain: K=4 element-wise kernels x<-a_k*x+b_k on 2^16 float32, 10000 "
                       "iterations per job", "b": b_star}
    g_T = g_TE = g_TC = None
    if args.arm in ("both", "graph"):
        for _ in range(max(1, args.warmup)):
            job(b_star)
        torch.cuda.synchronize()
        g_T, g_TC, g_TE = [], [], []
        for _ in range(steps):
            s0 = time.perf_counter()
            t = job(b_star)
            g_T.append(time.perf_counter() - s0)
            g_TC.append(t["t_create_s"])
            g_TE.append(t["t_exec_s"])
        res["graph"] = {"b": b_star, "us_per_iter": float(np.mean(g_T)) / ITERS * 1e6,
                        "us_per_iter_warm": float(np.mean(g_TE)) / ITERS * 1e6,
                        "t_create_ms": float(np.mean(g_TC)) * 1e3,
                        "gcell_upd_s": elem_updates / float(np.mean(g_T)) / 1e9}
    if args.arm in ("both", "per_launch"):
        for _ in range(max(1, args.warmup)):
            job(0)
        torch.cuda.synchronize()
        b_T, b_TE = [], []
        for _ in range(steps):
            s0 = time.perf_counter()
            t = job(0)
            b_T.append(time.perf_counter() - s0)
            b_TE.append(t["t_exec_s"])
        res["per_launch"] = {"us_per_iter": float(np.mean(b_T)) / ITERS * 1e6,
                             "us_per_iter_device": float(np.mean(b_TE)) / ITERS * 1e6,
                             "gcell_upd_s": elem_updates / float(np.mean(b_T)) / 1e9}
        if g_T is not None:
            sp, sp_err = pm.speedup(b_T, g_T)
            res["speedup"], res["speedup_err"] = sp, sp_err
            # crossover: graph launches after which T_C has paid for itself
            save = (float(np.mean(b_TE)) - float(np.mean(g_TE))) / ITERS
            res["crossover_batches"] = float(np.mean(g_TC)) / (b_star * save) if b_star > 0 and save > 0 else None
    prob.destroy()
    if g_TE is not None:
        # per graph node: the replay time divided by the nodes (kernel plus
        # the gap to the next node), against the node time of the same
        # chain on 2^10 elements (no work to speak of)
        n_launch = K * ITERS
        node_s = float(np.mean(g_TE)) / n_launch
        with kb.Problem(kb.SKELETON, (1 << 10,), (K,), SEED, device=0) as q:
            q.run(ITERS, b_star)
            q.last_timing()
            te = []
            for _ in range(3):
                q.run(ITERS, b_star)
                te.append(q.last_timing()["t_exec_s"])
        floor_s = float(np.median(te)) / n_launch
        bytes_per_launch = N_ELEM * 8
        trace = stored_json(SKEL_TRACE)
        res["per_node"] = {"node_us": node_s * 1e6, "node_floor_us": floor_s * 1e6,
                           "frac_of_node_floor": floor_s / node_s,
                           "per_node_effective_GB_s": bytes_per_launch / node_s / 1e9,
                           "bytes_per_launch": bytes_per_launch,
                           "traffic": stored_traffic(SKEL_COUNTERS, skeleton_kernel_hash())}
        if trace:
            kus = trace.get("graph_kernel_median_us")
            res["per_node"]["trace"] = trace
            if kus:
                res["per_node"]["trace_kernel_frac"] = bytes_per_launch / (kus * 1e-6) / 1e9 / HBM_PEAK_GBS
    if model is not None:
        c, e = model.creation, model.execution
        res["model"] = {"k_c_s_per_node": c.k_c, "k_c_se": c.k_c_se, "b_c_s": c.b_c, "b_c_se": c.b_c_se,
                        "mae_c_s": c.mae, "a_s": e.a, "a_se": e.a_se, "b_s": e.b, "b_se": e.b_se, "mae_e_s": e.mae,
                        "b_model": b_model, "b_closed_form": model.s_closed_form(), "b_measured_best": b_measured,
                        # a = (iterations) * (T_a - T_i): the extra gap of a
                        # graph launch over a node-to-node gap
                        "T_a_minus_T_i_us": e.a / ITERS * 1e6, "T_a_minus_T_i_se_us": e.a_se / ITERS * 1e6,
                        "repeats_per_b": args.sweep_reps}
        res["sweep_b_tc_ms_mean_std_te_ms_mean_std"] = [
            [s[0], round(s[1] * 1e3, 4), round(s[2] * 1e3, 4), round(s[3] * 1e3, 4), round(s[4] * 1e3, 4)]
            for s in sweep]
        gm = graph_memory(kb, np, torch)
        mm = pm.MemoryModel(gm["bytes_per_node"], max(gm["bytes_fixed"], 0.0))
        gm["b_model_under_budget"] = {}
        for budget in (1 << 20, 4 << 20):
            ok = [bb for bb in cands if bb * K <= mm.max_nodes(budget)] or [1]
            gm["b_model_under_budget"][f"{budget >> 20}MiB"] = model.best(ok)[0]
        res["graph_memory"] = gm
        res["graph_builders"] = builders_and_update(kb, np)
        if workloads_on:
            res["table1_sizes"] = table1_sweep(kb, pm, np)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              f"(a decomposition over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.stream_calibration:
        stream_calibration()
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.kernel_only:
        kernel_only(args.kernel_only, args.kernel_only_b)
        return

    import numpy as np
    import torch

    import paper_2501_09398_amd as kb
    from paper_2501_09398_amd import autotune
    from paper_2501_09398_amd import perfmodel as pm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    kb.lib()
    torch.cuda.set_device(torch.device("cuda", 0))
    workloads_on = not args.no_workloads and args.arm == "both" and args.only == "all"

    line = {"metric": "µs/iter & Gcell-upd/s: hipGraph batch-b vs per-launch; % HBM peak"}
    if args.only in ("all", "fdtd"):
        h = fdtd_headline(args, kb, autotune, np, torch)
        line.update({
            "value": h["value"], "unit": "Gcell-upd/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": h["wall_s"] / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32",
            "data": "synthetic: PEC cavity, fields zero, Gaussian soft source (width 20, delay 80 steps) on Ez "
                    "at the seeded node",
            "config": {"workload": "FDTD Yee PEC cavity 256^3, Courant 0.5, 10000 steps per job (H update, E update "
                                   "and soft source per step), graph batch b with loop peeling",
                       "N": N_FDTD, "steps_per_job": FDTD_STEPS, "b": h["b"], "variant": h["variant"],
                       "steps_per_iter": h["depth"],
                       "kernels_per_iter": h["kernels_per_iter"], "parallelism": "single GPU"},
            "arms": {k: h.get(k) for k in ("graph", "per_launch", "speedup", "speedup_err", "speedup_device")},
            "roofline": h["roofline"], "autotune": h["autotune"]})
        if not args.no_cpu_baseline:
            note("cavity: CPU oracle baseline and the float64 error")
            cpu, fp64 = fdtd_cpu_baseline(kb, np, torch)
            line["cpu_baseline"] = cpu
            line["fp64_error"] = fp64
        else:
            line["cpu_baseline"] = None
    line["host"] = host_info()
    if args.only in ("all", "skeleton"):
        note("skeleton chain: b sweep, fits, arms")
        sk = skeleton_section(args, kb, pm, np, torch, workloads_on)
        if args.only == "skeleton":
            line.update({"value": sk.get("graph", sk.get("per_launch", {})).get("gcell_upd_s"),
                         "unit": "Gcell-upd/s", "n_gpus": 1, "steps": max(args.steps, 1), "warmup": args.warmup,
                         "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                         "config": {"workload": sk["workload"], "b": sk["b"]}})
        line["skeleton"] = sk
    if workloads_on:
        note("other workloads")
        line["workloads"] = workloads(kb, pm, autotune, np)
        if not args.no_cpu_baseline:
            line["workloads_cpu_baseline"] = workloads_cpu_baseline(kb, np, line["workloads"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
