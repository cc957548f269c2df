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
from dataclasses import asdict, dataclass

import numpy as np


@dataclass
class CreationFit:
    k_c: float        # seconds per node (Eq. 2 slope)
    b_c: float        # seconds (Eq. 2 intercept)
    mae: float

    def __call__(self, nodes):
        return self.k_c * np.asarray(nodes, dtype=np.float64) + self.b_c


@dataclass
class ExecutionFit:
    a: float          # seconds * iterations (Eq. 6)
    b: float          # seconds (Eq. 6)
    mae: float

    def __call__(self, S):
        return self.a / np.asarray(S, dtype=np.float64) + self.b


def fit_creation(nodes, t_create) -> CreationFit:
    """Least-squares fit of Eq. 2, T_C = k_c * nodes + b_c."""
    x = np.asarray(nodes, dtype=np.float64)
    y = np.asarray(t_create, dtype=np.float64)
    A = np.stack([x, np.ones_like(x)], axis=1)
    (k, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    return CreationFit(float(k), float(c), float(np.mean(np.abs(A @ np.array([k, c]) - y))))


def fit_execution(S, t_exec) -> ExecutionFit:
    """Least-squares fit of Eq. 6, T_E = a / S + b (linear in 1/S)."""
    s = np.asarray(S, dtype=np.float64)
    y = np.asarray(t_exec, dtype=np.float64)
    A = np.stack([1.0 / s, np.ones_like(s)], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    return ExecutionFit(float(a), float(b), float(np.mean(np.abs(A @ np.array([a, b]) - y))))


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
    7.2): about 206 bytes per node plus about 150 KB per graph."""
    bytes_per_node: float = 206.0
    bytes_fixed: float = 150e3

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
