"""GPU parity of the thermal stencils through the C ABI.

Bars: the seeded initial state is bit-identical to the generator; the float32
GPU result is within 1e-5 relative max-norm of the float32 oracle; every
graph-batched run (any b, either builder, with peeling) and every kernel
variant (direct, LDS tile, temporal depth t) is bit-identical to the direct
per-launch run; the error against the float64 oracle is reported.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu, rel_maxnorm

pytestmark = pytest.mark.gpu

HEAT = dict(c=1e-3, Rx=1.0, Ry=1.0, Rz=10.0, Tamb=300.0)
HEAT_ANISO = dict(c=1e-3, Rx=1.0, Ry=2.0, Rz=10.0, Tamb=300.0)


def coeffs(d):
    return (d["c"], d["Rx"], d["Ry"], d["Rz"], d["Tamb"])


@pytest.fixture(scope="module")
def kb():
    need_gpu()
    import paper_2501_09398_amd as kb
    kb.lib()
    return kb


def run_heat2d(kb, shape, steps, b=0, seed=0, c=HEAT, tile=0, tdepth=1, builder=0):
    with kb.Problem(kb.HEAT2D, shape, coeffs(c), seed) as p:
        if tile:
            p.set_option(kb.OPT_TILE, tile)
            p.set_option(kb.OPT_TDEPTH, tdepth)
        p.set_option(kb.OPT_BUILDER, builder)
        rc = p.run(steps, b)
        assert rc == 0
        return p.read(kb.F_T)


def test_heat2d_initial_state_matches_generator(kb):
    announce("heat2d init 37x70 seed 3")
    with kb.Problem(kb.HEAT2D, (37, 70), coeffs(HEAT), 3) as p:
        T0, P = synth.heat2d_init(3, 37, 70)
        assert np.array_equal(p.read(kb.F_T), T0)
        assert np.array_equal(p.read(kb.F_P), P)


@pytest.mark.parametrize("shape,steps,c", [((64, 80), 50, HEAT), ((37, 130), 33, HEAT_ANISO),
                                           ((256, 256), 200, HEAT), ((1, 5), 20, HEAT), ((7, 1), 20, HEAT)])
def test_heat2d_vs_oracle(kb, shape, steps, c):
    announce(f"heat2d oracle {shape} steps {steps}")
    T0, P = synth.heat2d_init(1, *shape)
    got = run_heat2d(kb, shape, steps, seed=1, c=c)
    ref32 = oracle.heat2d(T0, P, steps, dtype=np.float32, **c)
    ref64 = oracle.heat2d(T0, P, steps, **c)
    assert rel_maxnorm(got, ref32) < 1e-5
    err64 = rel_maxnorm(got, ref64)
    print(f"heat2d {shape} x{steps}: rel err vs float64 oracle {err64:.3e}, vs float32 {rel_maxnorm(got, ref32):.3e}")


def test_heat2d_full_size_workload(kb):
    # 256x256, 1000 steps, graph batches of 100 (the configuration the
    # benchmark times) against the float32 and float64 oracles.
    announce("heat2d 256x256 1000 steps b=100")
    T0, P = synth.heat2d_init(20250116, 256, 256)
    got = run_heat2d(kb, (256, 256), 1000, b=100, seed=20250116)
    ref32 = oracle.heat2d(T0, P, 1000, dtype=np.float32)
    ref64 = oracle.heat2d(T0, P, 1000)
    assert rel_maxnorm(got, ref32) < 1e-5
    print(f"heat2d 256^2 x1000: vs f32 {rel_maxnorm(got, ref32):.3e} vs f64 {rel_maxnorm(got, ref64):.3e}")


@pytest.mark.parametrize("b", [1, 2, 3, 7, 10, 100])
@pytest.mark.parametrize("builder", [0, 1])
def test_heat2d_graph_bitwise_equals_per_launch(kb, b, builder):
    announce(f"heat2d graph b={b} builder={builder}")
    shape, steps = (61, 150), 101
    base = run_heat2d(kb, shape, steps, b=0, seed=2)
    got = run_heat2d(kb, shape, steps, b=b, seed=2, builder=builder)
    assert np.array_equal(base, got)


def test_heat2d_split_runs_and_cache(kb):
    announce("heat2d split runs")
    shape = (50, 70)
    whole = run_heat2d(kb, shape, 90, b=0, seed=4)
    with kb.Problem(kb.HEAT2D, shape, coeffs(HEAT), 4) as p:
        for n, b in [(13, 5), (30, 5), (7, 0), (40, 3)]:
            p.run(n, b)
        t = p.last_timing()
        assert t["n_graphs_built"] == 0 or t["n_graphs_built"] <= 2
        assert np.array_equal(p.read(kb.F_T), whole)


def test_heat2d_write_resume(kb):
    announce("heat2d write/resume")
    shape = (40, 40)
    whole = run_heat2d(kb, shape, 60, b=6, seed=5)
    with kb.Problem(kb.HEAT2D, shape, coeffs(HEAT), 5) as p:
        p.run(25, 5)
        state = p.read(kb.F_T)
    with kb.Problem(kb.HEAT2D, shape, coeffs(HEAT), 999) as q:
        q.write(kb.F_T, state)
        q.write(kb.F_P, synth.heat2d_init(5, *shape)[1])
        q.run(35, 7)
        assert np.array_equal(q.read(kb.F_T), whole)


@pytest.mark.parametrize("tile", [2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("tdepth", [1, 2, 5, 16])
def test_heat2d_tile_variants_bitwise(kb, tile, tdepth):
    announce(f"heat2d tile {tile} t={tdepth}")
    shape, steps = (70, 133), 37
    base = run_heat2d(kb, shape, steps, seed=6)
    got = run_heat2d(kb, shape, steps, seed=6, tile=tile, tdepth=tdepth)
    assert np.array_equal(base, got)
    got_g = run_heat2d(kb, shape, steps, b=2, seed=6, tile=tile, tdepth=tdepth)
    assert np.array_equal(base, got_g)


@pytest.mark.parametrize("shape", [(70, 133), (256, 256), (16, 16), (17, 33), (1, 40), (40, 1), (3, 5), (100, 9)])
@pytest.mark.parametrize("tdepth", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("tile", [15, 16, 17])
def test_heat2d_strip_temporal_variant_bitwise(kb, shape, tdepth, tile):
    """Variants 15-17 (16x16 tiles, region columns' rows in registers -- 4,
    2 or 1 per thread -- strip ends in LDS): same bits as the one-cell
    kernel for every depth, with a step count that leaves a remainder, per
    launch and in graph batches; tiles at every edge, grids smaller than a
    tile, single rows and columns."""
    announce(f"heat2d strip {shape} variant {tile} t={tdepth}")
    steps = 37
    base = run_heat2d(kb, shape, steps, seed=8)
    assert np.array_equal(base, run_heat2d(kb, shape, steps, seed=8, tile=tile, tdepth=tdepth))
    assert np.array_equal(base, run_heat2d(kb, shape, steps, b=3, seed=8, tile=tile, tdepth=tdepth))


@pytest.mark.parametrize("shape", [(70, 133), (256, 256), (33, 65), (1, 40), (40, 1), (3, 5), (100, 9), (130, 200)])
@pytest.mark.parametrize("tdepth", [1, 3, 8, 12, 16])
@pytest.mark.parametrize("tile", [22, 23])
def test_heat2d_wide_strip_temporal_variant_bitwise(kb, shape, tdepth, tile):
    """Variants 22 and 23 (32x32 tiles in regions of up to 64 x 64 cells, 4
    or 8 rows per thread, a wave per row group, up to 16 steps per launch):
    same bits as the one-cell kernel per launch and in graph batches (37
    steps leave a remainder), and within 1e-5 of the float32 oracle."""
    announce(f"heat2d wide strip {shape} variant {tile} t={tdepth}")
    steps = 37
    base = run_heat2d(kb, shape, steps, seed=11)
    assert np.array_equal(base, run_heat2d(kb, shape, steps, seed=11, tile=tile, tdepth=tdepth))
    assert np.array_equal(base, run_heat2d(kb, shape, steps, b=3, seed=11, tile=tile, tdepth=tdepth))
    T0, P = synth.heat2d_init(11, *shape)
    assert rel_maxnorm(base, oracle.heat2d(T0, P, steps, dtype=np.float32)) < 1e-5


@pytest.mark.parametrize("tile", [15, 16, 17])
def test_heat2d_strip_depth_limit(kb, tile):
    with kb.Problem(kb.HEAT2D, (64, 64), coeffs(HEAT), 0) as p:
        p.set_option(kb.OPT_TILE, tile)
        p.set_option(kb.OPT_TDEPTH, 16)
        with pytest.raises(kb.KBError):
            p.run(32, 0)


@pytest.mark.parametrize("shape", [(70, 133), (256, 256), (130, 300), (64, 64), (1, 40), (40, 1), (3, 5), (257, 49)])
@pytest.mark.parametrize("tdepth", [1, 2, 3, 6, 8])
@pytest.mark.parametrize("tile", [18, 19, 20, 21])
def test_heat2d_region_temporal_variant_bitwise(kb, shape, tdepth, tile):
    """Variants 18-21 (regions of 64 or 128 columns x 64 or 128 rows, 16
    rows of one or two columns per lane in registers, strip ends in LDS):
    same bits as the
    one-cell kernel for every depth, with a step count that leaves a
    remainder, per launch and in graph batches; regions cut at every edge,
    grids smaller than a region, single rows and columns; within 1e-5 of
    the float32 oracle."""
    announce(f"heat2d region {shape} variant {tile} t={tdepth}")
    steps = 37
    base = run_heat2d(kb, shape, steps, seed=9)
    assert np.array_equal(base, run_heat2d(kb, shape, steps, seed=9, tile=tile, tdepth=tdepth))
    assert np.array_equal(base, run_heat2d(kb, shape, steps, b=3, seed=9, tile=tile, tdepth=tdepth))
    T0, P = synth.heat2d_init(9, *shape)
    assert rel_maxnorm(base, oracle.heat2d(T0, P, steps, dtype=np.float32)) < 1e-5


@pytest.mark.parametrize("tile,tdepth", [(18, 8), (19, 6), (21, 6)])
def test_heat2d_region_large_grid(kb, tile, tdepth):
    """A large-grid case (8192^2, 256 MiB per field) in the launch shape the
    large-grid benchmark times: 13 steps as full-depth launches of the
    region kernel plus the remainder, bit-identical to the streaming
    one-step kernel, and sampled rows within 1e-5 of the float32 oracle
    (13 steps only reach 13 rows, so the first 20 rows of the grid are an
    exact sub-problem of the full one)."""
    announce(f"heat2d region 8192^2 variant {tile} t={tdepth}")
    shape, steps = (8192, 8192), 13
    base = run_heat2d(kb, shape, steps, seed=10, tile=13)
    got = run_heat2d(kb, shape, steps, seed=10, tile=tile, tdepth=tdepth)
    assert np.array_equal(base, got)
    T0, P = synth.heat2d_init(10, *shape)
    ref = oracle.heat2d(np.ascontiguousarray(T0[:40]), np.ascontiguousarray(P[:40]), steps, dtype=np.float32)
    assert rel_maxnorm(got[:20], ref[:20]) < 1e-5


@pytest.mark.parametrize("tile", [18, 19, 20, 21])
def test_heat2d_region_depth_limit(kb, tile):
    with kb.Problem(kb.HEAT2D, (64, 64), coeffs(HEAT), 0) as p:
        p.set_option(kb.OPT_TILE, tile)
        p.set_option(kb.OPT_TDEPTH, 9)
        with pytest.raises(kb.KBError):
            p.run(18, 0)


@pytest.mark.parametrize("shape", [(70, 132), (33, 260), (5, 4), (1, 4), (4, 8), (130, 1024), (9, 516)])
@pytest.mark.parametrize("tile", [8, 9, 10, 11, 12, 13, 14])
def test_heat2d_vector_variants_bitwise(kb, shape, tile):
    announce(f"heat2d vec tile {tile} {shape}")
    steps = 23
    base = run_heat2d(kb, shape, steps, seed=16, tile=1)
    assert np.array_equal(base, run_heat2d(kb, shape, steps, seed=16, tile=tile))
    assert np.array_equal(base, run_heat2d(kb, shape, steps, b=5, seed=16, tile=tile))
    T0, P = synth.heat2d_init(16, *shape)
    assert rel_maxnorm(base, oracle.heat2d(T0, P, steps, dtype=np.float32)) < 1e-5


def test_heat2d_vector_variant_needs_aligned_rows(kb):
    with kb.Problem(kb.HEAT2D, (8, 10), coeffs(HEAT), 0) as p:
        with pytest.raises(kb.KBError):
            p.set_option(kb.OPT_TILE, 11)


def test_heat2d_tiny_grids_temporal(kb):
    for shape in [(1, 1), (2, 3), (5, 1), (3, 200)]:
        announce(f"heat2d tiny {shape}")
        base = run_heat2d(kb, shape, 20, seed=7)
        got = run_heat2d(kb, shape, 20, seed=7, tile=3, tdepth=8)
        assert np.array_equal(base, got)
        T0, P = synth.heat2d_init(7, *shape)
        assert rel_maxnorm(got, oracle.heat2d(T0, P, 20, dtype=np.float32)) < 1e-5


def test_heat2d_zero_steps_and_errors(kb):
    with kb.Problem(kb.HEAT2D, (16, 16), coeffs(HEAT), 8) as p:
        T0 = p.read(kb.F_T)
        p.run(0, 0)
        p.run(0, 5)
        assert np.array_equal(p.read(kb.F_T), T0)
        with pytest.raises(kb.KBError):
            p.run(-1, 0)
        with pytest.raises(kb.KBError):
            p.run(10, -2)
        p.set_option(kb.OPT_MAX_NODES, 10)
        with pytest.raises(kb.KBError):
            p.run(100, 11)
        with pytest.raises(kb.KBError):
            p.set_option(kb.OPT_TDEPTH, 17)
        with pytest.raises(kb.KBError):
            p.set_option(kb.OPT_TILE, 99)
    with pytest.raises(kb.KBError):
        kb.Problem(kb.HEAT2D, (16, 16), (0.3, 1.0, 1.0, 10.0, 300.0), 0)   # c*(2+2+0.1) >= 1


def test_heat2d_reduce_mean(kb):
    announce("heat2d reduce")
    with kb.Problem(kb.HEAT2D, (300, 200), coeffs(HEAT), 9) as p:
        p.run(100, 10)
        T = p.read(kb.F_T).astype(np.float64)
        s1 = p.reduce()[0]
        s2 = p.reduce()[0]
        assert s1 == s2
        exact = float(np.sum(T))
        assert abs(s1 - exact) <= T.size * 2.0 ** -50 * np.sum(np.abs(T))


# ---- 3D ----------------------------------------------------------------------

def run_heat3d(kb, shape, steps, b=0, seed=0, builder=0, tile=0, tdepth=1):
    with kb.Problem(kb.HEAT3D, shape, coeffs(HEAT), seed) as p:
        p.set_option(kb.OPT_BUILDER, builder)
        p.set_option(kb.OPT_TILE, tile)
        p.set_option(kb.OPT_TDEPTH, tdepth)
        p.run(steps, b)
        return p.read(kb.F_T)


def test_heat3d_initial_state(kb):
    with kb.Problem(kb.HEAT3D, (3, 20, 70), coeffs(HEAT), 11) as p:
        T0, P = synth.heat3d_init(11, 3, 20, 70)
        assert np.array_equal(p.read(kb.F_T), T0)
        assert np.array_equal(p.read(kb.F_P), P)


@pytest.mark.parametrize("shape,steps", [((3, 20, 70), 40), ((8, 64, 64), 100), ((1, 9, 9), 10), ((2, 1, 1), 5)])
def test_heat3d_vs_oracle(kb, shape, steps):
    announce(f"heat3d oracle {shape} x{steps}")
    T0, P = synth.heat3d_init(12, *shape)
    got = run_heat3d(kb, shape, steps, seed=12)
    ref32 = oracle.heat3d(T0, P, steps, dtype=np.float32)
    ref64 = oracle.heat3d(T0, P, steps)
    assert rel_maxnorm(got, ref32) < 1e-5
    print(f"heat3d {shape}: vs f64 {rel_maxnorm(got, ref64):.3e}")


@pytest.mark.parametrize("shape", [(3, 20, 72), (8, 64, 64), (2, 5, 4), (1, 3, 260), (5, 33, 516)])
@pytest.mark.parametrize("tile", [2, 3, 4, 6, 7, 8, 9, 10])
def test_heat3d_vector_variant_bitwise(kb, shape, tile):
    announce(f"heat3d vec {tile} {shape}")
    base = run_heat3d(kb, shape, 17, seed=17, tile=1)
    assert np.array_equal(base, run_heat3d(kb, shape, 17, seed=17, tile=tile))
    assert np.array_equal(base, run_heat3d(kb, shape, 17, b=4, seed=17, tile=tile))
    T0, P = synth.heat3d_init(17, *shape)
    assert rel_maxnorm(base, oracle.heat3d(T0, P, 17, dtype=np.float32)) < 1e-5


@pytest.mark.parametrize("shape", [(8, 64, 64), (8, 70, 95), (3, 20, 72), (1, 3, 260), (5, 33, 33),
                                   (2, 5, 4), (7, 100, 1), (8, 1, 1), (6, 45, 46), (8, 130, 200)])
@pytest.mark.parametrize("tile,tdepth", [(5, 1), (5, 2), (5, 3), (5, 6), (11, 1), (11, 2), (11, 5), (11, 8)])
def test_heat3d_temporal_blocking_bitwise(kb, shape, tile, tdepth):
    """Variant 5 (t steps per launch over 32x32 column tiles, columns in
    registers, planes in LDS) and variant 11 (64-column regions, every
    layer of a column's rows in registers, edge clamps specialised) against
    the one-step kernel: same bits for every depth, with a step count that
    leaves a remainder (run per step), per launch and in graph batches;
    tiles smaller than the halo, single rows and columns, interior regions,
    every layer count up to 8."""
    announce(f"heat3d temporal {shape} variant {tile} t={tdepth}")
    steps = 17
    base = run_heat3d(kb, shape, steps, seed=19, tile=1)
    assert np.array_equal(base, run_heat3d(kb, shape, steps, seed=19, tile=tile, tdepth=tdepth))
    assert np.array_equal(base, run_heat3d(kb, shape, steps, b=2, seed=19, tile=tile, tdepth=tdepth))


@pytest.mark.parametrize("shape", [(8, 1100, 1000), (5, 700, 903)])
@pytest.mark.parametrize("tdepth", [1, 2, 4, 7])
def test_heat3d_strip_many_blocks_bitwise(kb, shape, tdepth):
    """Variant 11 on grids of more than one region per compute unit, where
    the kernel updates the rows with one register set (smaller grids use
    two): the same bits as the one-step kernel per launch and in graph
    batches, and the first rows within 1e-5 of the float32 oracle (17
    steps reach 17 rows, so the first 20 rows of a 40-row cut are exact)."""
    announce(f"heat3d strip many blocks {shape} t={tdepth}")
    steps = 17
    base = run_heat3d(kb, shape, steps, seed=21, tile=1)
    assert np.array_equal(base, run_heat3d(kb, shape, steps, seed=21, tile=11, tdepth=tdepth))
    assert np.array_equal(base, run_heat3d(kb, shape, steps, b=2, seed=21, tile=11, tdepth=tdepth))
    T0, P = synth.heat3d_init(21, *shape)
    ref = oracle.heat3d(np.ascontiguousarray(T0[:, :40]), np.ascontiguousarray(P[:40]), steps, dtype=np.float32)
    assert rel_maxnorm(base[:, :20], ref[:, :20]) < 1e-5


@pytest.mark.parametrize("tile,tdepth,b", [(5, 4, 50), (11, 5, 40)])
def test_heat3d_temporal_blocking_full_size(kb, tile, tdepth, b):
    """8x512x512 for 2000 steps in graph batches: the same bits as the
    one-step kernel."""
    announce(f"heat3d temporal 8x512x512 2000 steps variant {tile} t={tdepth}")
    shape = (8, 512, 512)
    base = run_heat3d(kb, shape, 2000, b=100, seed=20250116, tile=1)
    assert np.array_equal(base, run_heat3d(kb, shape, 2000, b=b, seed=20250116, tile=tile, tdepth=tdepth))


def test_heat3d_temporal_blocking_limits(kb):
    with kb.Problem(kb.HEAT3D, (9, 16, 16), coeffs(HEAT), 0) as p:
        for v in (5, 11):
            with pytest.raises(kb.KBError):
                p.set_option(kb.OPT_TILE, v)          # more than 8 layers
    with kb.Problem(kb.HEAT3D, (8, 16, 16), coeffs(HEAT), 0) as p:
        with pytest.raises(kb.KBError):
            p.set_option(kb.OPT_TDEPTH, 9)
        p.set_option(kb.OPT_TILE, 5)
        p.set_option(kb.OPT_TDEPTH, 7)                # variant 5 stops at 6
        with pytest.raises(kb.KBError):
            p.run(14, 0)
        p.set_option(kb.OPT_TILE, 11)
        p.run(16, 0)


@pytest.mark.parametrize("b", [1, 4, 9])
def test_heat3d_graph_bitwise(kb, b):
    announce(f"heat3d graph b={b}")
    base = run_heat3d(kb, (4, 33, 90), 50, seed=13)
    for builder in (0, 1):
        assert np.array_equal(base, run_heat3d(kb, (4, 33, 90), 50, b=b, seed=13, builder=builder))


def test_heat3d_full_size_sampled(kb):
    # 512x512x8 at the benchmark's launch configuration: 200 steps against
    # the float32 oracle on the whole field, then the mean closed form after
    # 2000 steps (the clamped Laplacian sums to zero).
    announce("heat3d 8x512x512")
    shape = (8, 512, 512)
    T0, P = synth.heat3d_init(20250116, *shape)
    got = run_heat3d(kb, shape, 200, b=100, seed=20250116)
    ref32 = oracle.heat3d(T0, P, 200, dtype=np.float32)
    assert rel_maxnorm(got, ref32) < 1e-5
    with kb.Problem(kb.HEAT3D, shape, coeffs(HEAT), 20250116) as p:
        p.run(2000, 100)
        mean = p.reduce()[0] / T0.size
    m0 = np.mean(T0.astype(np.float64))
    pbar = np.sum(P.astype(np.float64)) / T0.size
    ref = 300 + pbar * 10 + (m0 - 300 - pbar * 10) * (1 - 1e-4) ** 2000
    assert abs(mean - ref) / ref < 1e-5


# ---- many grids ------------------------------------------------------------

@pytest.mark.parametrize("variant,depth", [(1, 1), (2, 1), (3, 1), (3, 3), (3, 8), (4, 2), (4, 8),
                                           (5, 1), (5, 3), (5, 8), (6, 2), (6, 7), (6, 8)])
def test_multigrid_matches_single_grids(kb, variant, depth):
    """variant 1: one cell per thread; 2: 64 x 8 strips per wave; 3:
    temporal blocking over (64 - 2t)-square tiles, 4: over 64 x 128
    regions, 5 and 6: over 128-column regions two columns per lane (30
    steps = whole iterations of t steps plus single steps).  Grids narrower
    and wider than a wave and than a tile, single rows and a single cell."""
    announce(f"multigrid 8 grids variant {variant} depth {depth}")
    sides = [(17, 70), (64, 64), (5, 130), (100, 33), (1, 1), (40, 250), (33, 1), (9, 65), (130, 127), (300, 290)]
    shape = [len(sides)] + [v for s in sides for v in s]
    with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), 14) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.set_option(kb.OPT_TDEPTH, depth)
        p.run(30, 7)
        allT = p.read(kb.F_T)
    T0 = synth.uniform_f32(14, synth.TAG_T0, allT.size, *synth.T0_RANGE)
    P = synth.uniform_f32(14, synth.TAG_P, allT.size, *synth.P_RANGE)
    off = 0
    for ny, nx in sides:
        n = ny * nx
        ref = oracle.heat2d(T0[off:off + n].reshape(ny, nx), P[off:off + n].reshape(ny, nx), 30, dtype=np.float32)
        got = allT[off:off + n].reshape(ny, nx)
        assert rel_maxnorm(got, ref) < 1e-5
        # bit-identical to a single-grid run of the same data
        with kb.Problem(kb.HEAT2D, (ny, nx), coeffs(HEAT), 0) as q:
            q.write(kb.F_T, T0[off:off + n])
            q.write(kb.F_P, P[off:off + n])
            q.run(30, 0)
            assert np.array_equal(q.read(kb.F_T), got)
        off += n


def test_multigrid_graph_bitwise(kb):
    sides = synth.multigrid_sides(3, 8, 16, 200)
    shape = [len(sides)] + [v for s in sides for v in (s, s)]
    outs = []
    for v, t, b in ((2, 1, 0), (2, 1, 1), (2, 1, 5), (1, 1, 0), (1, 1, 5), (3, 4, 0), (3, 4, 2), (3, 5, 3),
                    (4, 3, 2)):
        with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), 15) as p:
            p.set_option(kb.OPT_TILE, v)
            p.set_option(kb.OPT_TDEPTH, t)
            p.run(23, b)
            outs.append(p.read(kb.F_T))
            if v >= 3:
                with pytest.raises(kb.KBError):
                    p.set_option(kb.OPT_TDEPTH, 9)
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_multigrid_full_size_workload_all_variants(kb):
    """64 grids of side round(64 * 16^u) (about 12.9 M cells): every
    variant (temporal blocking at depths 4 and 8 included) gives the same
    bits after 24 steps."""
    announce("multigrid 64 grids full size")
    sides = synth.multigrid_sides(20250116, 64)
    shape = [64] + [v for s in sides for v in (s, s)]
    outs = []
    for v, t in ((1, 1), (2, 1), (3, 4), (3, 8), (4, 6), (5, 6), (6, 8)):
        with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), 20250116) as p:
            p.set_option(kb.OPT_TILE, v)
            p.set_option(kb.OPT_TDEPTH, t)
            p.run(24, 3 if t == 1 else 1)
            outs.append(p.read(kb.F_T))
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


@pytest.mark.parametrize("variant,depth,b", [(2, 1, 100), (3, 6, 37), (6, 8, 25)])
def test_multigrid_full_size_2000_steps_vs_oracle(kb, variant, depth, b):
    """The 64-grid workload for 2000 steps as the benchmark runs it: the
    strip kernel in graph batches of 100, and temporal blocking at depths
    and batches the autotuner picks on MI355X (333 launches of 6 steps in 9
    graphs of 37, then 2 single steps; 250 launches of 8 steps over
    two-column regions in 10 graphs of 25).  The three smallest grids against
    the float32 oracle, and every grid's mean against its closed form (the
    clamped Laplacian sums to zero on each grid)."""
    announce(f"multigrid 64 grids 2000 steps variant {variant} depth {depth} b={b}")
    seed = 20250116
    sides = synth.multigrid_sides(seed, 64)
    shape = [64] + [v for s in sides for v in (s, s)]
    with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), seed) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.set_option(kb.OPT_TDEPTH, depth)
        p.run(2000, b)
        allT = p.read(kb.F_T)
    T0s, Ps = synth.multigrid_init(seed, sides)
    off = 0
    grids = []
    for s, T0, P in zip(sides, T0s, Ps):
        grids.append((s, T0, P, allT[off:off + s * s].reshape(s, s)))
        off += s * s
    for s, T0, P, got in sorted(grids, key=lambda g: g[0])[:3]:
        ref32 = oracle.heat2d(T0, P, 2000, dtype=np.float32)
        assert rel_maxnorm(got, ref32) < 1e-5, s
    for s, T0, P, got in grids:
        m0 = np.mean(T0.astype(np.float64))
        pbar = np.mean(P.astype(np.float64))
        ref = 300 + pbar * 10 + (m0 - 300 - pbar * 10) * (1 - 1e-4) ** 2000
        assert abs(np.mean(got.astype(np.float64)) - ref) / ref < 1e-5, s


@pytest.mark.parametrize("depth", [1, 4, 6])
def test_multigrid_persistent_matches_per_launch(kb, depth):
    """One cooperative launch for all steps (super-steps of t steps with a
    grid barrier between them, then n mod t steps) gives the bits of the
    per-launch strip kernel, over two consecutive runs (the buffer parity
    carries over) and a run of zero steps."""
    announce(f"multigrid persistent depth {depth}")
    sides = [(17, 70), (64, 64), (5, 130), (100, 33), (1, 1), (40, 250), (33, 1), (9, 65), (130, 127), (300, 290)]
    shape = [len(sides)] + [v for s in sides for v in s]
    with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), 21) as p:
        p.set_option(kb.OPT_TILE, 2)
        p.run(23, 0)
        ref1 = p.read(kb.F_T)
        p.run(14, 0)
        ref2 = p.read(kb.F_T)
    with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), 21) as p:
        p.set_option(kb.OPT_PERSISTENT, 1)
        p.set_option(kb.OPT_TDEPTH, depth)
        p.run(23, 5)                              # batch_b is ignored
        assert p.last_timing()["n_kernel_launches"] == 1
        assert np.array_equal(p.read(kb.F_T), ref1)
        p.run(0, 0)
        p.run(14, 0)
        assert np.array_equal(p.read(kb.F_T), ref2)


def test_multigrid_persistent_full_size(kb):
    """The 64-grid workload: 100 steps in one persistent launch at depth 6
    equal 100 steps of the strip kernel in graph batches."""
    announce("multigrid persistent full size")
    seed = 20250116
    sides = synth.multigrid_sides(seed, 64)
    shape = [64] + [v for s in sides for v in (s, s)]
    outs = []
    for persistent in (0, 1):
        with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), seed) as p:
            if persistent:
                p.set_option(kb.OPT_PERSISTENT, 1)
                p.set_option(kb.OPT_TDEPTH, 6)
            else:
                p.set_option(kb.OPT_TILE, 2)
            p.run(100, 10)
            outs.append(p.read(kb.F_T))
    assert np.array_equal(outs[0], outs[1])


def test_persistent_option_rejections(kb):
    with kb.Problem(kb.HEAT2D, (64, 64), coeffs(HEAT), 1) as p:
        with pytest.raises(kb.KBError):
            p.set_option(kb.OPT_PERSISTENT, 1)
    with kb.Problem(kb.HEAT2D_MULTI, [2, 64, 64, 70, 70], coeffs(HEAT), 1) as p:
        with pytest.raises(kb.KBError):
            p.set_option(kb.OPT_PERSISTENT, 2)
        p.set_option(kb.OPT_PERSISTENT, 1)
        p.set_option(kb.OPT_REDUCE_EVERY, 10)
        with pytest.raises(kb.KBError):
            p.run(20, 0)


def test_persistent_barrier_timeout_is_reported(kb):
    """The bounded barrier wait: with a spin limit of one poll, a block that
    reaches a barrier before the others gives up at once, raises the error
    flag, and every block runs to its end; kb_run reports the failure.  The
    next run with the automatic limit is correct again (from a rewritten
    state)."""
    announce("multigrid persistent barrier time-out")
    sides = synth.multigrid_sides(20250116, 64)
    shape = [64] + [v for s in sides for v in (s, s)]
    with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), 5) as p:
        T0 = p.read(kb.F_T)
        p.set_option(kb.OPT_PERSISTENT, 1)
        p.set_option(kb.OPT_TDEPTH, 4)
        p.set_option(kb.OPT_SPIN_LIMIT, 1)
        with pytest.raises(kb.KBError):
            p.run(40, 0)
        p.set_option(kb.OPT_SPIN_LIMIT, 0)
        p.write(kb.F_T, T0)
        p.run(40, 0)
        got = p.read(kb.F_T)
    with kb.Problem(kb.HEAT2D_MULTI, shape, coeffs(HEAT), 5) as q:
        q.set_option(kb.OPT_TILE, 2)
        q.run(40, 0)
        assert np.array_equal(q.read(kb.F_T), got)
