"""Performance model of iteration-batch unrolling (Sec. III-B, Eqs. 1-6).

Notation of the paper: S iterations are unrolled into one graph (the
iteration batch size), I_k is the total number of kernel executions and
I = I_k / S the number of graph launches (Eq. 4).

  Eq. 1   T   = T_C + T_E
  Eq. 2   T_C = k_c S + b_c                      graph creation (incl. upload)
  Eq. 3   T_E = T_l + (T_k S + T_i (S-1)) I + T_a (I-1)
  Eq. 5   T_E = I_k (T_a - T_i) / S + I_k (T_k + T_i) - T_a + T_l
  Eq. 6   T_E = a / S + b,  a = I_k (T_a - T_i),  b = I_k (T_k + T_i) - T_a + T_l

For an iteration of K kernels the graph has K*S nodes, so the creation
model is fitted against node counts and the execution model against S.
The coefficients are fitted by ordinary least squares and scored by the
mean absolute error, as in Table I.  The optimum minimises Eq. 1 over the
admissible batch sizes; with T_C and T_E as above the continuous optimum is
S* = sqrt(a / (K k_c)).
"""
from __future__ import annotations

import math
import os
from dataclasses import asdict, dataclass

import numpy as np


@dataclass
class CreationFit:
    k_c: float        # seconds per node (Eq. 2 slope)
    b_c: float        # seconds (Eq. 2 intercept)
    mae: float
    k_c_se: float = 0.0   # standard errors of the least-squares coefficients
    b_c_se: float = 0.0

    def __call__(self, nodes):
        return self.k_c * np.asarray(nodes, dtype=np.float64) + self.b_c


@dataclass
class ExecutionFit:
    a: float          # seconds * iterations (Eq. 6)
    b: float          # seconds (Eq. 6)
    mae: float
    a_se: float = 0.0
    b_se: float = 0.0

    def __call__(self, S):
        return self.a / np.asarray(S, dtype=np.float64) + self.b


def _lstsq2(A, y):
    """Ordinary least squares with two coefficients: (coef, MAE, standard
    errors from the residual variance RSS/(n-2) and (A^T A)^-1)."""
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    r = A @ coef - y
    n = len(y)
    se = np.zeros(2)
    if n > 2:
        cov = (r @ r) / (n - 2) * np.linalg.inv(A.T @ A)
        se = np.sqrt(np.maximum(np.diag(cov), 0.0))
    return coef, float(np.mean(np.abs(r))), se


def fit_creation(nodes, t_create) -> CreationFit:
    """Least-squares fit of Eq. 2, T_C = k_c * nodes + b_c."""
    x = np.asarray(nodes, dtype=np.float64)
    y = np.asarray(t_create, dtype=np.float64)
    A = np.stack([x, np.ones_like(x)], axis=1)
    (k, c), mae, se = _lstsq2(A, y)
    return CreationFit(float(k), float(c), mae, float(se[0]), float(se[1]))


def fit_execution(S, t_exec) -> ExecutionFit:
    """Least-squares fit of Eq. 6, T_E = a / S + b (linear in 1/S)."""
    s = np.asarray(S, dtype=np.float64)
    y = np.asarray(t_exec, dtype=np.float64)
    A = np.stack([1.0 / s, np.ones_like(s)], axis=1)
    (a, b), mae, se = _lstsq2(A, y)
    return ExecutionFit(float(a), float(b), mae, float(se[0]), float(se[1]))


def exec_time_eq3(T_l, T_k, T_i, T_a, S, I):
    """Eq. 3: first launch, I graphs of S kernels with gaps T_i, I-1 gaps T_a."""
    return T_l + (T_k * S + T_i * (S - 1)) * I + T_a * (I - 1)


def exec_time_eq5(T_l, T_k, T_i, T_a, S, I_k):
    """Eq. 5: Eq. 3 with I = I_k / S."""
    return I_k * (T_a - T_i) / S + I_k * (T_k + T_i) - T_a + T_l


def eq6_coefficients(T_l, T_k, T_i, T_a, I_k):
    """(a, b) of Eq. 6 from the timing components."""
    return I_k * (T_a - T_i), I_k * (T_k + T_i) - T_a + T_l


def divisors(n, lo=1, hi=None):
    hi = n if hi is None else hi
    out = []
    for d in range(1, int(math.isqrt(n)) + 1):
        if n % d == 0:
            out += [d, n // d]
    return sorted(x for x in set(out) if lo <= x <= hi)


@dataclass
class Model:
    creation: CreationFit
    execution: ExecutionFit
    K: int = 1        # kernels per iteration (nodes = K * S)
    # graphs a run builds per batch size S (default one).  A problem whose
    # iterations alternate between two buffers needs, for odd S and at least
    # two batches, one graph per start buffer, and pays T_C twice.
    graphs: dict | None = None

    def n_graphs(self, S):
        S = np.atleast_1d(np.asarray(S))
        if not self.graphs:
            return np.ones(S.shape, np.float64)
        return np.array([float(self.graphs.get(int(s), 1)) for s in S.ravel()]).reshape(S.shape)

    def total(self, S):
        """Eq. 1 with the fitted Eq. 2 (per graph, times the graphs the run
        builds) and Eq. 6."""
        scalar = np.ndim(S) == 0
        S = np.atleast_1d(np.asarray(S, dtype=np.float64))
        t = self.n_graphs(S) * self.creation(self.K * S) + self.execution(S)
        return t[0] if scalar else t

    def s_closed_form(self):
        """Continuous minimiser of k_c K S + a / S."""
        if self.execution.a <= 0 or self.creation.k_c <= 0:
            return math.inf
        return math.sqrt(self.execution.a / (self.K * self.creation.k_c))

    def best(self, candidates):
        """Admissible S with the smallest modelled total time."""
        c = np.asarray(list(candidates))
        t = self.total(c)
        i = int(np.argmin(t))
        return int(c[i]), float(t[i])

    def as_dict(self):
        return {"creation": asdict(self.creation), "execution": asdict(self.execution), "K": self.K,
                "S_closed_form": self.s_closed_form(),
                "graphs": {str(k): v for k, v in self.graphs.items()} if self.graphs else None}


@dataclass
class MemoryModel:
    """Device memory an instantiated, uploaded graph holds: linear in its
    kernel nodes (the footprint the paper's Fig. 2 bars grow with).  The
    defaults are the MI355X fit of the benchmark (skeleton chain, ROCm
    7.2, eight cumulative points of four 8000-node graphs each): 262 bytes
    per node and no fixed part -- each such graph took exactly one 2 MiB
    allocation unit, so this is an upper bound for graphs of that size."""
    bytes_per_node: float = 262.144
    bytes_fixed: float = 0.0

    def __call__(self, nodes):
        return self.bytes_fixed + self.bytes_per_node * np.asarray(nodes, dtype=np.float64)

    def max_nodes(self, budget):
        """Largest node count whose graph fits `budget` bytes (0 if none)."""
        if budget <= self.bytes_fixed:
            return 0
        return int((budget - self.bytes_fixed) // self.bytes_per_node)


def fit_memory(nodes, mem_bytes) -> MemoryModel:
    """Least-squares fit of graph bytes = fixed + per_node * nodes."""
    x = np.asarray(nodes, dtype=np.float64)
    y = np.asarray(mem_bytes, dtype=np.float64)
    A = np.stack([x, np.ones_like(x)], axis=1)
    (k, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    return MemoryModel(float(k), float(c))


def speedup(base_times, graph_times):
    """Speed-up as the ratio of mean times, with the error of Sec. III-C:
    the relative standard deviations of the two arms added in quadrature
    (the square root of the summed squares of std/mean), times the ratio."""
    b = np.asarray(base_times, dtype=np.float64)
    g = np.asarray(graph_times, dtype=np.float64)
    s = b.mean() / g.mean()
    rel = math.sqrt((b.std() / b.mean()) ** 2 + (g.std() / g.mean()) ** 2)
    return float(s), float(s * rel)


# ---------------------------------------------------------------------------
# Inter-kernel gaps from a kernel trace (the T_i and T_a of Eq. 3 / Fig. 1)
# ---------------------------------------------------------------------------
def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(f"none of {names} in the trace's columns {sorted(row)}")


def read_kernel_trace(path, name_filter=None):
    """Dispatches of a rocprofv3 kernel-trace CSV, sorted by start time:
    list of (name, start_ns, end_ns, grid_x)."""
    import csv
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            name = _col(r, "Kernel_Name", "KernelName", "Name")
            if name_filter and not any(s in name for s in name_filter):
                continue
            rows.append((name, int(_col(r, "Start_Timestamp", "BeginNs", "Start")),
                         int(_col(r, "End_Timestamp", "EndNs", "End")),
                         int(_col(r, "Grid_Size_X", "Grid_Size", "grid_size_x", "Grid_X"))))
    rows.sort(key=lambda t: t[1])
    return rows


def trace_gaps(rows, K, b, iters, graph_jobs, launch_jobs):
    """Gaps (next start - this end) and durations of a trace made of
    `graph_jobs` jobs in graph batches of b iterations followed by
    `launch_jobs` jobs launched per kernel, each job `iters` iterations of
    K dispatches (rows from read_kernel_trace, only the job's kernels).
    Inside a graph job a gap after dispatch j (counted from the job's
    start) is a node-to-node gap T_i unless j+1 is a multiple of K*b, where
    one graph launch ends and the next begins (T_a between graphs, Eq. 3).
    In a per-launch job every gap is a launch-to-launch gap (the T_a of the
    baseline loop, Fig. 1).  Gaps between jobs (host work, graph creation)
    are left out.  Returns medians, means and 10th / 90th percentiles in
    microseconds."""
    per_job = K * iters
    need = (graph_jobs + launch_jobs) * per_job
    if len(rows) < need:
        raise ValueError(f"trace has {len(rows)} dispatches, the run needs {need}")
    rows = rows[:need]
    g_in, g_between, l_gap, g_dur, l_dur, names = [], [], [], [], [], {}
    for job in range(graph_jobs + launch_jobs):
        seg = rows[job * per_job:(job + 1) * per_job]
        graph = job < graph_jobs
        for j, (name, s, e, _) in enumerate(seg):
            d = (e - s) / 1e3
            (g_dur if graph else l_dur).append(d)
            names.setdefault(name, []).append(d)
            if j + 1 == len(seg):
                continue
            gap = (seg[j + 1][1] - e) / 1e3
            if not graph:
                l_gap.append(gap)
            elif (j + 1) % (K * b) == 0:
                g_between.append(gap)
            else:
                g_in.append(gap)

    def stats(v):
        if not v:
            return None
        a = np.asarray(v, float)
        return {"n": int(a.size), "median_us": float(np.median(a)), "mean_us": float(a.mean()),
                "p10_us": float(np.percentile(a, 10)), "p90_us": float(np.percentile(a, 90))}
    out = {"K": K, "b": b, "iters": iters, "graph_jobs": graph_jobs, "launch_jobs": launch_jobs,
           "T_i_in_graph_gap": stats(g_in), "T_a_between_graphs_gap": stats(g_between),
           "T_a_per_launch_gap": stats(l_gap), "graph_kernel_duration": stats(g_dur),
           "per_launch_kernel_duration": stats(l_dur),
           "kernels": {n: stats(v) for n, v in names.items()}}
    if g_dur:
        out["graph_kernel_median_us"] = out["graph_kernel_duration"]["median_us"]
    return out


def _main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Inter-kernel gaps of a rocprofv3 kernel trace (T_i, T_a of Eq. 3).")
    ap.add_argument("csv", help="the *_kernel_trace.csv of rocprofv3 --kernel-trace --output-format csv")
    ap.add_argument("--kernel", action="append", required=True, help="substring of the job's kernel names")
    ap.add_argument("--K", type=int, required=True, help="dispatches per iteration")
    ap.add_argument("--b", type=int, required=True, help="iterations per graph batch")
    ap.add_argument("--iters", type=int, required=True, help="iterations per job")
    ap.add_argument("--graph-jobs", type=int, required=True)
    ap.add_argument("--launch-jobs", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0, help="keep only dispatches of this grid size (x)")
    ap.add_argument("--out", help="write the summary as JSON here")
    a = ap.parse_args(argv)
    rows = read_kernel_trace(a.csv, a.kernel)
    if a.grid:
        rows = [r for r in rows if r[3] == a.grid]
    res = trace_gaps(rows, a.K, a.b, a.iters, a.graph_jobs, a.launch_jobs)
    res["source"] = os.path.basename(a.csv)
    txt = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(txt)


if __name__ == "__main__":
    _main()
