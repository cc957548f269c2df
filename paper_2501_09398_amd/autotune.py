"""Autotuner: kernel variant, temporal-blocking depth and iteration batch b.

Sec. VI of the paper names automatic characterisation and choice of the
iteration batch size as the missing piece of the method.  Here it is done
per problem and shape, in two stages, through the C ABI only:

1. kernel stage -- for every kernel variant (and, for the temporal-blocking
   variants of the 2D, 3D and many-grid stencils, every temporal depth t)
   time the warm execution of a fixed number of steps with a moderate batch
   (graph already built), and keep the fastest (warm microseconds per step; all variants give the same
   bits, so only time decides);
2. batch stage -- for the chosen kernel, sweep b over the admissible batch
   sizes (divisors of the iteration count, Eq. 4), measure T_C and T_E with
   repeats, fit Eq. 2 and Eq. 6 (perfmodel) and take the b that minimises
   the modelled T = T_C + T_E (Eq. 1); the measured best b is reported too.
   Eq. 2 is fitted per graph: a run of an alternating (ping-pong) problem
   with odd b builds one graph per start buffer, so its T_C is divided by
   the graphs it built, and the model charges each b the graphs its run
   builds.

The objective of the batch stage is the paper's (creation included); the
warm per-step time at that b is reported beside it.
"""
from __future__ import annotations

from dataclasses import asdict, dataclass, field

import numpy as np

from . import perfmodel as pm

# Kernel variants worth trying per problem (KB_OPT_TILE values) and the
# temporal depths tried for the LDS-tile variants of the 2D stencil.
HEAT2D_DIRECT = [1]
HEAT2D_TILE = [2, 3, 4, 5, 6, 7]
HEAT2D_VEC = [8, 9, 10, 11, 13, 14]
HEAT2D_DEPTHS = [1, 2, 4, 8, 16]
HEAT2D_REGION_DEPTHS = [2, 4, 6, 8]      # variants 18 to 21
HEAT2D_WIDE_STRIP_DEPTHS = [8, 12, 16]   # variants 22 and 23
HEAT3D_DEPTHS = [1, 2, 3, 4, 6]          # variant 5 (layer stacks of <= 8)
HEAT3D_STRIP_DEPTHS = [2, 3, 4, 5, 6, 8]  # variant 11 (layer stacks of <= 8)
MULTI_DEPTHS = [1, 2, 3, 4, 5, 6, 7, 8]  # many-grid variants 3 to 6


def kernel_candidates(kb, problem, shape):
    """(variant, depth) pairs valid for the problem and shape."""
    if problem == kb.HEAT2D:
        c = [(v, 1) for v in HEAT2D_DIRECT]
        c += [(v, t) for v in HEAT2D_TILE for t in HEAT2D_DEPTHS]
        c += [(v, t) for v in (15, 16, 17) for t in HEAT2D_DEPTHS if t <= 8]
        c += [(v, t) for v in (18, 19, 20, 21) for t in HEAT2D_REGION_DEPTHS]
        c += [(v, t) for v in (22, 23) for t in HEAT2D_WIDE_STRIP_DEPTHS]
        if shape[1] % 4 == 0:
            c += [(v, 1) for v in HEAT2D_VEC]
        return c
    if problem == kb.HEAT3D:
        c = [(1, 1)] + ([(2, 1), (3, 1), (4, 1), (6, 1), (7, 1), (8, 1), (9, 1), (10, 1)] if shape[2] % 4 == 0 else [])
        if shape[0] <= 8:
            c += [(5, t) for t in HEAT3D_DEPTHS] + [(11, t) for t in HEAT3D_STRIP_DEPTHS]
        return c
    if problem == kb.SKELETON:
        return [(1, 1), (2, 1), (3, 1)]
    if problem == kb.FDTD3D:
        # one step per launch; two steps per launch (60-node tiles, and the
        # whole-row kernels up to N = 256, which also take three)
        two = [(8, 2)] + ([(9, 2), (10, 2), (10, 3)] if shape[0] <= 256 else [])
        return [(1, 1), (2, 1), (3, 1), (4, 1), (5, 1), (6, 1), (7, 1)] + two
    if problem == kb.HEAT2D_MULTI:
        return [(1, 1), (2, 1)] + [(v, t) for v in (3, 4, 5, 6) for t in MULTI_DEPTHS]
    return [(0, 1)]


@dataclass
class TuneResult:
    variant: int
    depth: int
    b: int
    us_per_step_warm: float
    t_create_s: float
    us_per_step_cold: float
    kernel_table: list = field(default_factory=list)     # (variant, depth, warm us/step)
    batch_table: list = field(default_factory=list)      # (b, T_C s, T_E s)
    model: dict | None = None
    b_measured: int = 0

    def as_dict(self):
        return asdict(self)


def _warm_time(p, n, b, reps):
    p.run(n, b)
    p.last_timing()
    ts = []
    for _ in range(reps):
        p.run(n, b)
        ts.append(p.last_timing()["t_exec_s"])
    return float(np.median(ts))


def tune(kb, problem, shape, coeffs, n_steps, seed=0, probe_steps=None, b_probe=None,
         b_candidates=None, reps=3, kernel_candidates_override=None, max_nodes=4096,
         graph_mem_budget=None, mem_model=None):
    """Tune (variant, depth, b) for running n_steps of the problem.

    kb: the binding module.  probe_steps: steps timed per kernel candidate
    (default min(n_steps, 200), rounded to a multiple of 16).
    graph_mem_budget: bytes of device memory the batch graph may hold; b
    is then limited to graphs that fit by the linear memory model
    (`mem_model`, a perfmodel.MemoryModel; the MI355X fit by default).
    Returns a TuneResult; the problem objects it creates are destroyed
    again.
    """
    if graph_mem_budget is not None:
        mm = mem_model or pm.MemoryModel()
        max_nodes = min(max_nodes, mm.max_nodes(graph_mem_budget))
    if probe_steps is None:
        probe_steps = max(16, min(n_steps, 200) // 16 * 16)
    cands = kernel_candidates_override or kernel_candidates(kb, problem, shape)
    table = []
    with kb.Problem(problem, shape, coeffs, seed) as p:
        K = p.kernels_per_iter()
        for v, t in cands:
            p.set_option(kb.OPT_TILE, v)
            p.set_option(kb.OPT_TDEPTH, t)          # depth 1 is accepted by every problem
            iters = probe_steps // t
            bp = b_probe or max(1, min(iters, 400 // (K * 1)))
            sec = _warm_time(p, iters * t, bp, reps)
            table.append((v, t, sec / (iters * t) * 1e6))
    best_v, best_t, _ = min(table, key=lambda r: r[2])

    n_iter = n_steps // best_t
    if b_candidates is None:
        b_candidates = [d for d in pm.divisors(n_iter) if d * K <= max_nodes] or [1]
    else:
        b_candidates = [b for b in b_candidates if b * K <= max_nodes] or [1]
    sweep = []
    with kb.Problem(problem, shape, coeffs, seed) as p:
        p.set_option(kb.OPT_TILE, best_v)
        p.set_option(kb.OPT_TDEPTH, best_t)
        p.set_option(kb.OPT_GRAPH_CACHE, 0)
        graphs = {}
        for b in b_candidates:
            tc, te = [], []
            for _ in range(reps):
                p.run(n_iter * best_t, b)
                tm = p.last_timing()
                tc.append(tm["t_create_s"])
                te.append(tm["t_exec_s"])
                graphs[b] = int(tm["n_graphs_built"])
            sweep.append((b, float(np.median(tc)), float(np.median(te))))
    S = np.array([s[0] for s in sweep], float)
    model = None
    if len(sweep) >= 3:
        per_graph = [s[1] / max(1, graphs[s[0]]) for s in sweep]
        model = pm.Model(pm.fit_creation(K * S, per_graph),
                         pm.fit_execution(S, [s[2] for s in sweep]), K=K,
                         graphs={b: max(1, g) for b, g in graphs.items()})
        b_star, _ = model.best(b_candidates)
    measured = {s[0]: s[1] + s[2] for s in sweep}
    b_meas = min(measured, key=measured.get)
    if model is None:
        b_star = b_meas
    row = next(s for s in sweep if s[0] == b_star)
    return TuneResult(variant=best_v, depth=best_t, b=b_star,
                      us_per_step_warm=row[2] / (n_iter * best_t) * 1e6,
                      t_create_s=row[1],
                      us_per_step_cold=(row[1] + row[2]) / (n_iter * best_t) * 1e6,
                      kernel_table=table, batch_table=sweep,
                      model=model.as_dict() if model else None, b_measured=b_meas)
