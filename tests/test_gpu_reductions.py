"""GPU parity of the in-chain reductions (KB_OPT_REDUCE_EVERY) through the
C ABI.

Every m steps two extra kernels reduce the state inside the iteration chain
(graph nodes of the batch graphs).  The log must be (i) bitwise the same for
per-launch runs, every batch size b (dividing m, a multiple of m, or
neither) and both builders, also when a run is split over several calls,
and (ii) equal to float64 sums of the states at steps m, 2m, ... (the sums
differ only in order: within n * 2^-50 * sum|x|).  The skeleton and FDTD
states are those of the float32 oracle (bit-identical to the GPU's); the
heat states are the GPU's own plain path read back every m steps (the
float32 heat oracle evaluates the literal formula, so it differs from the
GPU's fixed fused order in an occasional last bit; the heat parity tests
pin that path to the oracle within 1e-5).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu

HEAT = (1e-3, 1.0, 1.0, 10.0, 300.0)


@pytest.fixture(scope="module")
def kb():
    need_gpu()
    import paper_2501_09398_amd as kb
    kb.lib()
    return kb


def fsum(*arrays, square=False):
    return math.fsum(v for a in arrays for v in (a.astype(np.float64).ravel() ** 2 if square
                                                 else a.astype(np.float64).ravel()))


def close(got, ref, n):
    return abs(got - ref) <= n * 2.0 ** -50 * abs(ref) + 1e-300


def heat2d_log(kb, b, builder, runs, m=10, shape=(40, 56), seed=3):
    with kb.Problem(kb.HEAT2D, shape, HEAT, seed) as p:
        p.set_option(kb.OPT_TILE, 1)
        p.set_option(kb.OPT_BUILDER, builder)
        p.set_option(kb.OPT_REDUCE_EVERY, m)
        for n in runs:
            p.run(n, b)
        return p.reduction_log(), p.read(kb.F_T)


def gpu_states(kb, problem, shape, seed, m, count, field):
    """States after m, 2m, ... steps of the plain GPU path (per launch)."""
    out = []
    with kb.Problem(problem, shape, HEAT, seed) as p:
        if problem != kb.HEAT2D_MULTI:
            p.set_option(kb.OPT_TILE, 1)
        for _ in range(count):
            p.run(m, 0)
            out.append(p.read(field))
    return out


def test_heat2d_reduction_log_vs_states(kb):
    announce("heat2d reductions vs states")
    m, n, shape = 10, 100, (40, 56)
    log, _ = heat2d_log(kb, 0, 0, [n], m, shape)
    assert log.shape == (n // m, 4)
    states = gpu_states(kb, kb.HEAT2D, shape, 3, m, n // m, kb.F_T)
    T0, P = synth.heat2d_init(3, *shape)
    for e, T in enumerate(states):
        assert log[e, 0] == (e + 1) * m
        assert close(log[e, 1], fsum(T), T.size)
        assert log[e, 2] == 0.0 and log[e, 3] == 0.0
    # and the states are the oracle's within the heat parity bar
    ref = oracle.heat2d(T0, P, n, dtype=np.float32)
    assert np.max(np.abs(states[-1] - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("b,builder,runs", [
    (5, 0, [100]), (7, 0, [100]), (20, 0, [100]), (30, 0, [100]),
    (7, 1, [100]), (20, 1, [100]), (5, 0, [13, 37, 50]), (7, 1, [3, 97])])
def test_heat2d_reduction_log_bitwise_across_batches(kb, b, builder, runs):
    announce(f"heat2d reductions b={b} builder={builder} runs={runs}")
    ref_log, ref_T = heat2d_log(kb, 0, 0, [100])
    log, T = heat2d_log(kb, b, builder, runs)
    assert np.array_equal(log, ref_log)
    assert np.array_equal(T, ref_T)


def test_reduction_option_resets_and_switches_off(kb):
    announce("reduction option reset")
    with kb.Problem(kb.HEAT2D, (32, 32), HEAT, 4) as p:
        p.set_option(kb.OPT_TILE, 1)
        p.set_option(kb.OPT_REDUCE_EVERY, 4)
        p.run(12, 3)
        assert p.reduction_log().shape[0] == 3
        p.set_option(kb.OPT_REDUCE_EVERY, 5)      # restart: count and phase
        p.run(11, 0)
        log = p.reduction_log()
        assert log.shape[0] == 2 and list(log[:, 0]) == [5.0, 10.0]
        p.set_option(kb.OPT_REDUCE_EVERY, 0)
        p.run(20, 4)
        assert p.reduction_log().shape[0] == 0


@pytest.mark.parametrize("problem,shape,tile,t,b", [
    ("HEAT2D", (64, 72), 6, 4, 0), ("HEAT2D", (64, 72), 16, 4, 3), ("HEAT3D", (8, 40, 70), 11, 2, 5),
    ("HEAT2D_MULTI", [3, 100, 90, 64, 64, 17, 150], 3, 4, 2)])
def test_reduction_log_with_temporal_blocking(kb, problem, shape, tile, t, b):
    """With t steps per iteration and m a multiple of t, every reduction
    point ends an iteration: the log equals the one-step kernels' bit for
    bit (same states, same fixed-order sums), per launch and in graphs."""
    announce(f"reductions with temporal blocking {problem} variant {tile} t={t} b={b}")
    prob = getattr(kb, problem)
    m, n = 8, 96
    logs = []
    for v, d, bb in ((1 if problem != "HEAT2D_MULTI" else 2, 1, 0), (tile, t, b)):
        with kb.Problem(prob, shape, HEAT, 5) as p:
            p.set_option(kb.OPT_TILE, v)
            p.set_option(kb.OPT_TDEPTH, d)
            p.set_option(kb.OPT_REDUCE_EVERY, m)
            p.run(40, bb)
            p.run(56, bb)
            logs.append(p.reduction_log())
    assert logs[0].shape == (n // m, 4)
    assert np.array_equal(logs[0], logs[1])


def test_reduction_rejects_misaligned_temporal_blocking_and_surrogate(kb):
    with kb.Problem(kb.HEAT2D, (64, 64), HEAT, 5) as p:
        p.set_option(kb.OPT_TILE, 6)
        p.set_option(kb.OPT_TDEPTH, 4)
        p.set_option(kb.OPT_REDUCE_EVERY, 6)          # not a multiple of t
        with pytest.raises(kb.KBError):
            p.run(16, 0)
        p.set_option(kb.OPT_REDUCE_EVERY, 8)
        with pytest.raises(kb.KBError):
            p.run(18, 0)                                # leaves single steps
        p.run(16, 0)
        p.set_option(kb.OPT_TDEPTH, 1)
        p.run(2, 0)                                     # 18 steps so far
        p.set_option(kb.OPT_TDEPTH, 4)
        with pytest.raises(kb.KBError):
            p.run(8, 0)                                 # iterations off the grid of t
    with kb.Problem(kb.HEAT2D_SURROGATE, (64, 64), HEAT, 5) as p:
        with pytest.raises(kb.KBError):
            p.set_option(kb.OPT_REDUCE_EVERY, 8)


@pytest.mark.parametrize("b", [0, 6])
def test_heat3d_reduction_log(kb, b):
    announce(f"heat3d reductions b={b}")
    shape, m, n = (3, 20, 24), 4, 40
    with kb.Problem(kb.HEAT3D, shape, HEAT, 6) as p:
        p.set_option(kb.OPT_TILE, 1)
        p.set_option(kb.OPT_REDUCE_EVERY, m)
        p.run(n, b)
        log = p.reduction_log()
    states = gpu_states(kb, kb.HEAT3D, shape, 6, m, n // m, kb.F_T)
    assert log.shape[0] == n // m
    for e, T in enumerate(states):
        assert close(log[e, 1], fsum(T), T.size)


@pytest.mark.parametrize("b", [0, 4, 9])
def test_skeleton_reduction_log(kb, b):
    announce(f"skeleton reductions b={b}")
    n, m, iters = 5000, 3, 60
    with kb.Problem(kb.SKELETON, (n,), (4,), 7) as p:
        p.set_option(kb.OPT_REDUCE_EVERY, m)
        p.run(iters, b)
        log = p.reduction_log()
    x0, a, bb = synth.skeleton_init(7, n, 4)
    assert log.shape[0] == iters // m
    x = x0
    for e in range(iters // m):
        x = oracle.skeleton(x, a, bb, m, dtype=np.float32)
        assert close(log[e, 1], fsum(x), n)


@pytest.mark.parametrize("b", [0, 6, 7])
@pytest.mark.parametrize("variant", [2, 5])
def test_fdtd_energy_log(kb, b, variant):
    announce(f"fdtd energy reductions b={b} variant={variant}")
    N, m, steps, seed = 12, 5, 40, 8
    with kb.Problem(kb.FDTD3D, (N, 64), kb.FDTD_COEFFS, seed) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.set_option(kb.OPT_REDUCE_EVERY, m)
        p.run(steps, b)
        log = p.reduction_log()
    src = synth.fdtd_source_cell(seed, N)
    _, g32 = oracle.fdtd_pulse(steps + 1)
    f = oracle.fdtd_zero_fields(N, np.float32)
    assert log.shape[0] == steps // m
    for e in range(steps // m):
        f, _ = oracle.fdtd(f, N, m, src=src, g=g32, n_start=e * m, dtype=np.float32)
        ee = fsum(f["Ex"], f["Ey"], f["Ez"], square=True)
        hh = fsum(f["Hx"], f["Hy"], f["Hz"], square=True)
        n = 3 * (N + 1) ** 3
        assert close(log[e, 1], ee, n) and close(log[e, 2], hh, n), e


def test_multigrid_reduction_log(kb):
    announce("many-grid reductions")
    sides = [16, 33, 9]
    shape = [len(sides)] + [v for s in sides for v in (s, s)]
    m, n = 5, 30
    with kb.Problem(kb.HEAT2D_MULTI, shape, HEAT, 9) as p:
        p.set_option(kb.OPT_REDUCE_EVERY, m)
        p.run(n, 4)
        log = p.reduction_log()
    states = gpu_states(kb, kb.HEAT2D_MULTI, shape, 9, m, n // m, kb.F_T)
    assert log.shape[0] == n // m
    for e, T in enumerate(states):
        assert close(log[e, 1], fsum(T), T.size)
