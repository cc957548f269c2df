"""Autotuner logic against a synthetic timing model (no GPU), and on the GPU
against the real library."""
import math

import numpy as np
import pytest

from paper_2501_09398_amd import autotune, perfmodel as pm


class FakeKB:
    """Stands in for the binding: timings follow Eqs. 2 and 3 exactly.
    Temporal depth counts only for the temporal-blocking variants of the
    problem the fake was created for."""
    HEAT2D, HEAT3D, SKELETON, FDTD3D, HEAT2D_MULTI = 1, 2, 3, 4, 5
    TB = {1: {2, 3, 4, 5, 6, 7, 15, 16, 17, 18, 19, 20, 21, 22, 23}, 2: {5, 11}, 5: {3, 4, 5, 6}}
    OPT_BUILDER, OPT_TILE, OPT_TDEPTH, OPT_GRAPH_CACHE, OPT_MAX_NODES = 1, 2, 3, 4, 5
    # per-launch kernel time (s) per variant; variant 6 with depth 8 is best
    T_K = {1: 3e-6, 2: 4e-6, 3: 3.5e-6, 4: 3.6e-6, 5: 3.4e-6, 6: 3.2e-6, 7: 3.9e-6,
           8: 2.9e-6, 9: 2.95e-6, 10: 3.1e-6, 11: 3.3e-6, 12: 3.5e-6, 13: 2.8e-6, 14: 2.85e-6,
           15: 3.3e-6, 16: 3.25e-6, 17: 3.35e-6, 18: 3.3e-6, 19: 3.4e-6, 20: 3.3e-6, 21: 3.4e-6, 22: 3.3e-6, 23: 3.35e-6}
    T_I, T_A, K_C, B_C = 0.5e-6, 8e-6, 3e-6, 2e-4

    @staticmethod
    def graphs(problem, b, nb):
        """Graphs a run builds: the stencils alternate between two buffers,
        so odd b with two or more batches needs one graph per start buffer."""
        if nb == 0:
            return 0
        return 2 if problem != FakeKB.SKELETON and b % 2 == 1 and nb >= 2 else 1

    class Problem:
        def __init__(self, kbm, problem, shape, coeffs, seed):
            self.kbm, self.problem, self.v, self.t, self.last = kbm, problem, 1, 1, None

        def __enter__(self):
            return self

        def __exit__(self, *a):
            pass

        def kernels_per_iter(self):
            return 1

        def set_option(self, opt, val):
            if opt == FakeKB.OPT_TILE:
                self.v = val
            elif opt == FakeKB.OPT_TDEPTH:
                self.t = val

        def run(self, n, b):
            t = self.t if self.v in FakeKB.TB.get(self.problem, ()) else 1
            iters = n // t
            tk = FakeKB.T_K[self.v] * (1 + 0.1 * t) / t * t    # deeper steps cost a little more each
            nb = iters // b
            te = iters * (tk + FakeKB.T_I) + nb * (FakeKB.T_A - FakeKB.T_I)
            g = FakeKB.graphs(self.problem, b, nb)
            self.last = {"t_create_s": g * (FakeKB.K_C * b + FakeKB.B_C), "t_exec_s": te, "n_graphs_built": g}

        def last_timing(self):
            return self.last


def fake_kb():
    kb = FakeKB()
    kb.Problem = lambda *a: FakeKB.Problem(kb, *a)
    return kb


def test_tuner_picks_fastest_kernel_and_model_batch():
    kb = fake_kb()
    res = autotune.tune(kb, kb.HEAT2D, (256, 256), (), 1000, reps=1)
    # per step: variant v with depth t costs T_K[v]*(1+0.1t) + T_I/t + ...;
    # the cheapest per step is the one with the largest depth
    per_step = {(v, t): (FakeKB.T_K[v] * (1 + 0.1 * t) + FakeKB.T_I) / t
                for v, t in autotune.kernel_candidates(kb, kb.HEAT2D, (256, 256))}
    assert (res.variant, res.depth) == min(per_step, key=per_step.get)
    n_iter = 1000 // res.depth
    assert n_iter % res.b == 0
    # exact data: the fitted model recovers a = n_iter (T_a - T_i) and k_c,
    # and b is the admissible minimiser of k_c b + a / b
    a = n_iter * (FakeKB.T_A - FakeKB.T_I)
    assert math.isclose(res.model["execution"]["a"], a, rel_tol=1e-9)
    assert math.isclose(res.model["creation"]["k_c"], FakeKB.K_C, rel_tol=1e-9)
    cands = [d for d in pm.divisors(n_iter) if d <= 4096]
    g = lambda b: FakeKB.graphs(kb.HEAT2D, b, n_iter // b)
    expect = min(cands, key=lambda b: g(b) * (FakeKB.K_C * b + FakeKB.B_C) + a / b)
    assert res.b == expect


def test_tuner_charges_both_parity_graphs_for_odd_b():
    """An alternating problem with odd b builds two graphs: the fit of
    Eq. 2 divides T_C by the graphs built (so k_c, b_c stay per graph), and
    the model's total charges odd b twice.  250 steps with candidates 10,
    25 (odd: two graphs) and 50: 25 would win with one graph, and the
    optimum moves to 50."""
    kb = fake_kb()
    n, cands = 250, [10, 25, 50]
    a = n * (FakeKB.T_A - FakeKB.T_I)
    one = {b: FakeKB.K_C * b + FakeKB.B_C + a / b for b in cands}
    assert min(one, key=one.get) == 25
    res = autotune.tune(kb, kb.HEAT2D, (256, 256), (), n, reps=1, b_candidates=cands,
                        kernel_candidates_override=[(1, 1)])
    assert math.isclose(res.model["creation"]["k_c"], FakeKB.K_C, rel_tol=1e-9)
    assert math.isclose(res.model["creation"]["b_c"], FakeKB.B_C, rel_tol=1e-9)
    assert res.model["graphs"] == {"10": 1, "25": 2, "50": 1}
    two = {b: (2 if b % 2 else 1) * (FakeKB.K_C * b + FakeKB.B_C) + a / b for b in cands}
    assert res.b == min(two, key=two.get) == 50


@pytest.mark.parametrize("problem,shape", [(3, (8, 64, 64)), (5, (3, 100, 100, 70, 70, 64, 64))])
def test_tuner_applies_depth_for_3d_and_many_grids(problem, shape):
    """The winning depth of a temporal-blocking variant is the one timed:
    the tuner sets the depth option for every problem, not only the 2D one."""
    kb = fake_kb()
    prob = {3: kb.HEAT3D, 5: kb.HEAT2D_MULTI}[problem]
    res = autotune.tune(kb, prob, shape, (), 1200, reps=1)
    assert res.variant in FakeKB.TB[prob] and res.depth > 1
    per_step = {(v, t): (FakeKB.T_K[v] * (1 + 0.1 * t) + FakeKB.T_I) / (t if v in FakeKB.TB[prob] else 1)
                for v, t in autotune.kernel_candidates(kb, prob, shape)}
    assert (res.variant, res.depth) == min(per_step, key=per_step.get)


def test_graph_memory_budget_limits_b():
    """With a device-memory budget for the batch graph, b stays within the
    node count the linear memory model allows (fixed + per-node bytes), and
    the unconstrained optimum is kept when it fits."""
    kb = fake_kb()
    free = autotune.tune(kb, kb.SKELETON, (1024,), (), 1000, reps=1)
    mm = pm.MemoryModel(bytes_per_node=200.0, bytes_fixed=1e5)
    budget = 1e5 + 200.0 * 20                         # 20 nodes
    res = autotune.tune(kb, kb.SKELETON, (1024,), (), 1000, reps=1, graph_mem_budget=budget, mem_model=mm)
    assert res.b * 1 <= 20 and 1000 % res.b == 0
    assert free.b > 20                                # the budget did bind
    roomy = autotune.tune(kb, kb.SKELETON, (1024,), (), 1000, reps=1, graph_mem_budget=1e9)
    assert roomy.b == free.b
    assert mm.max_nodes(1e5) == 0 and mm.max_nodes(1e5 + 401) == 2
    fit = pm.fit_memory([100, 1000, 5000], [1e5 + 2e4, 1e5 + 2e5, 1e5 + 1e6])
    assert math.isclose(fit.bytes_per_node, 200.0) and math.isclose(fit.bytes_fixed, 1e5)


def test_kernel_candidates_respect_alignment():
    kb = FakeKB()
    c_aligned = autotune.kernel_candidates(kb, kb.HEAT2D, (64, 256))
    c_ragged = autotune.kernel_candidates(kb, kb.HEAT2D, (64, 250))
    assert any(8 <= v <= 14 for v, _ in c_aligned)          # float4 rows need nx % 4 == 0
    assert not any(8 <= v <= 14 for v, _ in c_ragged)
    assert any(v == 15 for v, _ in c_ragged)                 # register strips do not
    assert autotune.kernel_candidates(kb, kb.HEAT3D, (8, 64, 66)) == (
        [(1, 1)] + [(5, t) for t in autotune.HEAT3D_DEPTHS] + [(11, t) for t in autotune.HEAT3D_STRIP_DEPTHS])
    assert autotune.kernel_candidates(kb, kb.HEAT3D, (9, 64, 66)) == [(1, 1)]


@pytest.mark.gpu
def test_autotuned_heat2d_is_bitwise_and_not_slower():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_09398_amd as kb
    kb.lib()
    shape, n = (256, 256), 1000
    res = autotune.tune(kb, kb.HEAT2D, shape, kb.HEAT_COEFFS, n, seed=3, reps=2)
    print("tuned:", res.variant, res.depth, res.b, res.us_per_step_warm)
    with kb.Problem(kb.HEAT2D, shape, kb.HEAT_COEFFS, 3) as p:
        p.run(n, 0)
        base = p.read(kb.F_T)
        per_launch = p.last_timing()["t_exec_s"] / n * 1e6
    with kb.Problem(kb.HEAT2D, shape, kb.HEAT_COEFFS, 3) as p:
        p.set_option(kb.OPT_TILE, res.variant)
        p.set_option(kb.OPT_TDEPTH, res.depth)
        p.run(n, res.b)
        assert np.array_equal(p.read(kb.F_T), base)
    assert res.us_per_step_warm <= per_launch
