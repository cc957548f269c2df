"""Parity at the sizes the benchmark times on the large grids.

The default kernels for large grids (heat2d variant 13 at 16384^2, heat3d
variant 9 at 8 x 4096^2, the fused FDTD step with streaming stores,
variant 7, at 256^3) and the temporal-blocking kernels timed beside them
run here at those sizes, in the launch configurations the benchmark uses:

* every variant is bit-identical, over the whole grid, to the one-cell
  reference kernel (heat) or to the float32 oracle (FDTD, every node);
* heat: row bands at the top edge, in the middle and at the bottom edge
  against the float32 oracle run on the band plus a halo of one row per
  step (a step moves information by one row, so the band's rows are an
  exact sub-problem), within the 1e-5 relative max-norm bar.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu, rel_maxnorm

gpu = pytest.mark.gpu

HEAT = (1e-3, 1.0, 1.0, 10.0, 300.0)


@pytest.fixture(scope="module")
def kb():
    need_gpu()
    import paper_2501_09398_amd as kb
    kb.lib()
    return kb


def run(kb, prob, shape, steps, seed, variant, depth=1, b=0):
    with kb.Problem(prob, shape, HEAT, seed) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.set_option(kb.OPT_TDEPTH, depth)
        p.run(steps, b)
        return p.read(kb.F_T)


def band_rows(ny, steps):
    return [(0, 40), (ny // 2 - 20, ny // 2 + 20), (ny - 40, ny)]


def band_inputs_2d(seed, ny, nx, lo, hi):
    """Rows lo..hi of the seeded T0 and P (the same draws as the whole grid)."""
    n = (hi - lo) * nx
    T0 = synth.uniform_f32(seed, synth.TAG_T0, n, *synth.T0_RANGE, offset=lo * nx).reshape(hi - lo, nx)
    P = synth.uniform_f32(seed, synth.TAG_P, n, *synth.P_RANGE, offset=lo * nx).reshape(hi - lo, nx)
    return T0, P


def band_inputs_3d(seed, nz, ny, nx, lo, hi):
    T0 = np.stack([synth.uniform_f32(seed, synth.TAG_T0, (hi - lo) * nx, *synth.T0_RANGE,
                                     offset=(z * ny + lo) * nx).reshape(hi - lo, nx) for z in range(nz)])
    P = synth.uniform_f32(seed, synth.TAG_P, (hi - lo) * nx, *synth.P_RANGE, offset=lo * nx).reshape(hi - lo, nx)
    return T0, P


def check_bands_2d(got, seed, steps):
    ny, nx = got.shape
    for a, b in band_rows(ny, steps):
        lo, hi = max(0, a - steps - 1), min(ny, b + steps + 1)
        T0, P = band_inputs_2d(seed, ny, nx, lo, hi)
        ref = oracle.heat2d(T0, P, steps, dtype=np.float32)
        e = rel_maxnorm(got[a:b], ref[a - lo:b - lo])
        e64 = rel_maxnorm(got[a:b], oracle.heat2d(T0, P, steps)[a - lo:b - lo])
        print(f"rows {a}..{b}: vs float32 oracle {e:.2e}, vs float64 {e64:.2e}")
        assert e < 1e-5, (a, b)


def check_bands_3d(got, seed, steps):
    nz, ny, nx = got.shape
    for a, b in band_rows(ny, steps):
        lo, hi = max(0, a - steps - 1), min(ny, b + steps + 1)
        T0, P = band_inputs_3d(seed, nz, ny, nx, lo, hi)
        ref = oracle.heat3d(T0, P, steps, dtype=np.float32)
        e = rel_maxnorm(got[:, a:b], ref[:, a - lo:b - lo])
        e64 = rel_maxnorm(got[:, a:b], oracle.heat3d(T0, P, steps)[:, a - lo:b - lo])
        print(f"rows {a}..{b}: vs float32 oracle {e:.2e}, vs float64 {e64:.2e}")
        assert e < 1e-5, (a, b)


def test_band_inputs_are_the_grid_rows():
    """The band generators draw exactly the rows of the whole grid's inputs."""
    T0, P = synth.heat2d_init(3, 50, 70)
    t, p = band_inputs_2d(3, 50, 70, 20, 31)
    assert np.array_equal(t, T0[20:31]) and np.array_equal(p, P[20:31])
    T0, P = synth.heat3d_init(4, 3, 50, 70)
    t, p = band_inputs_3d(4, 3, 50, 70, 7, 19)
    assert np.array_equal(t, T0[:, 7:19]) and np.array_equal(p, P[7:19])


@gpu
def test_heat2d_16384_default_and_temporal(kb):
    """16384^2 (1 GiB per field): the streaming one-step kernel (variant 13,
    the default at this size) per launch and in graph batches of 10, and
    the 128 x 128-region temporal kernel (variant 21, t = 8), 24 steps
    each; against the one-cell kernel and the oracle bands."""
    shape, seed = (16384, 16384), 11
    announce("heat2d 16384^2 variant 1 (reference), 24 steps")
    ref24 = run(kb, kb.HEAT2D, shape, 24, seed, 1)
    announce("heat2d 16384^2 variant 13, 24 steps per launch")
    got = run(kb, kb.HEAT2D, shape, 24, seed, 13)
    assert np.array_equal(got, ref24)
    announce("heat2d 16384^2 variant 13, 24 steps in graph batches of 10")
    assert np.array_equal(run(kb, kb.HEAT2D, shape, 24, seed, 13, b=10), ref24)
    announce("heat2d 16384^2 variant 21 t=8, 24 steps")
    assert np.array_equal(run(kb, kb.HEAT2D, shape, 24, seed, 21, depth=8), ref24)
    check_bands_2d(got, seed, 24)


@gpu
def test_heat3d_8x4096_default_and_temporal(kb):
    """8 x 4096^2: the register-blocked rows kernel with the layer after
    next loaded ahead (variant 9, the default at this size) per launch and
    in graph batches of 10, and the 3D register strips (variant 11, t = 4),
    24 steps each; against the one-column kernel and the oracle bands (all
    eight layers)."""
    shape, seed = (8, 4096, 4096), 12
    announce("heat3d 8x4096^2 variant 1 (reference), 24 steps")
    ref24 = run(kb, kb.HEAT3D, shape, 24, seed, 1)
    announce("heat3d 8x4096^2 variant 9, 24 steps per launch")
    got = run(kb, kb.HEAT3D, shape, 24, seed, 9)
    assert np.array_equal(got, ref24)
    announce("heat3d 8x4096^2 variant 9, 24 steps in graph batches of 10")
    assert np.array_equal(run(kb, kb.HEAT3D, shape, 24, seed, 9, b=10), ref24)
    announce("heat3d 8x4096^2 variant 11 t=4, 24 steps")
    assert np.array_equal(run(kb, kb.HEAT3D, shape, 24, seed, 11, depth=4), ref24)
    check_bands_3d(got, seed, 24)


@pytest.fixture(scope="module")
def fdtd256():
    """The float32 oracle at 256^3: 100 steps from zero fields with the
    seeded source (the benchmark's workload) and 100 steps from random
    fields (every node, walls included, starts non-zero)."""
    N, steps, seed = 256, 100, 20250116
    src = synth.fdtd_source_cell(seed, N)
    _, g32 = oracle.fdtd_pulse(steps + 1)
    zero, probe = oracle.fdtd(oracle.fdtd_zero_fields(N, np.float32), N, steps, src=src, g=g32, dtype=np.float32)
    rng = np.random.default_rng(256)
    M = N + 1
    f0 = {k: rng.uniform(-1.0, 1.0, (M, M, M)).astype(np.float32) for k in oracle.FDTD_FIELDS}
    rand, rprobe = oracle.fdtd(f0, N, steps, src=src, g=g32, dtype=np.float32)
    return dict(N=N, steps=steps, seed=seed, zero=zero, probe=probe, f0=f0, rand=rand, rprobe=rprobe)


@gpu
@pytest.mark.parametrize("variant,depth", [(10, 3), (10, 2), (9, 2), (8, 2)])
def test_fdtd_256_two_step_vs_oracle(kb, fdtd256, variant, depth):
    """The temporal-blocking kernels (streaming stores at this size) at
    256^3 -- whole rows of four nodes per lane, lane 63 also writing the
    i = N column's Hx (9: 16 rows per block; 10: 12 rows, operands loaded a
    plane ahead; depth 3: three steps per launch), 60-node tiles (8) -- 100
    steps in graph batches of 11 iterations (the leftover steps as fused
    steps), bit for bit with the float32 oracle on every node, and the
    probe."""
    d = fdtd256
    N, steps = d["N"], d["steps"]
    for start in ("zero", "rand"):
        announce(f"fdtd 256^3 {start} fields, 100 steps, kernel {variant} depth {depth}, b=11")
        with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, d["seed"]) as p:
            p.set_option(kb.OPT_TILE, variant)
            p.set_option(kb.OPT_TDEPTH, depth)
            if start == "rand":
                for k, fid in kb.FDTD_FIELDS.items():
                    p.write(fid, d["f0"][k])
            p.run(steps, 11)
            probe = p.read(kb.F_PROBE)
            for k, fid in kb.FDTD_FIELDS.items():
                assert np.array_equal(p.read(fid), d[start][k]), (start, k)
        assert np.array_equal(probe[:steps], d["probe"] if start == "zero" else d["rprobe"])


@gpu
def test_fdtd_256_headline_job_vs_oracle(kb, fdtd256):
    """The benchmark's job itself: the 256^3 cavity from zero fields with
    the seeded Gaussian source, 10,000 steps with the whole-row kernel of
    three steps per launch (variant 10, depth 3; 3333 iterations in graph
    batches of b = 101, the last step fused) -- every node of the six
    fields and all 10,000 probe values bit for bit with the float32 oracle
    (about a minute of oracle time on 16 threads)."""
    d = fdtd256
    N, seed, steps = d["N"], d["seed"], 10000
    src = synth.fdtd_source_cell(seed, N)
    _, g32 = oracle.fdtd_pulse(steps + 1)
    announce("fdtd 256^3 headline job: float32 oracle, 10,000 steps")
    ref, probe_ref = oracle.fdtd(oracle.fdtd_zero_fields(N, np.float32), N, steps, src=src, g=g32,
                                 dtype=np.float32)
    announce("fdtd 256^3 headline job: GPU, variant 10 depth 3, b = 101")
    with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, seed) as p:
        p.set_option(kb.OPT_TILE, 10)
        p.set_option(kb.OPT_TDEPTH, 3)
        p.run(steps, 101)
        assert p.read(kb.F_STEP)[0] == steps
        probe = p.read(kb.F_PROBE)
        for k, fid in kb.FDTD_FIELDS.items():
            assert np.array_equal(p.read(fid), ref[k]), k
    assert np.array_equal(probe[:steps], probe_ref)


@gpu
def test_fdtd_256_variant_switching(kb, fdtd256):
    """100 steps at 256^3 from random fields, switching kernels on the way:
    the whole-row kernels of two and three steps per launch (one launch per
    iteration, the step counter advanced by the grid's last block, the
    i = N column's Hx in lane 63) per launch and in graph batches with an
    odd b, the fused step in between (which copies the column's unchanging
    values) -- bit for bit with the float32 oracle, probe and step counter
    included."""
    d = fdtd256
    N, steps = d["N"], d["steps"]
    plan = ((10, 2, 31, 5), (7, 1, 20, 0), (10, 3, 14, 3), (9, 2, 24, 0), (10, 3, 11, 0))   # variant, depth, steps, b
    assert sum(n for _, _, n, _ in plan) == steps
    announce("fdtd 256^3 rand fields, 100 steps switching 10 / 7 / 10 depth 3 / 9 / 10 depth 3")
    with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, d["seed"]) as p:
        for k, fid in kb.FDTD_FIELDS.items():
            p.write(fid, d["f0"][k])
        done = 0
        for v, t, n, b in plan:
            p.set_option(kb.OPT_TILE, v)
            p.set_option(kb.OPT_TDEPTH, t)
            assert p.kernels_per_iter() == (1 if v >= 9 and t >= 2 else 2)
            p.run(n, b)
            done += n
            assert p.read(kb.F_STEP)[0] == done
        probe = p.read(kb.F_PROBE)
        for k, fid in kb.FDTD_FIELDS.items():
            assert np.array_equal(p.read(fid), d["rand"][k]), k
    assert np.array_equal(probe[:steps], d["rprobe"])


@gpu
@pytest.mark.parametrize("variant", [7, 5, 2])
def test_fdtd_256_vs_oracle(kb, fdtd256, variant):
    """256^3 (two field sets of 0.8 GB): 100 steps in graph batches of 100
    (the benchmark's graph arm), fused step with streaming stores (7, the
    default at this size), fused with plain stores (5) and the separate H
    and E kernels (2); bit for bit with the float32 oracle on every node,
    and the probe history."""
    d = fdtd256
    N, steps = d["N"], d["steps"]
    for start in ("zero", "rand"):
        announce(f"fdtd 256^3 {start} fields, 100 steps, b=100, variant {variant}")
        with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, d["seed"]) as p:
            p.set_option(kb.OPT_TILE, variant)
            if start == "rand":
                for k, fid in kb.FDTD_FIELDS.items():
                    p.write(fid, d["f0"][k])
            p.run(steps, 100)
            probe = p.read(kb.F_PROBE)
            for k, fid in kb.FDTD_FIELDS.items():
                assert np.array_equal(p.read(fid), d[start][k]), (start, k)
        assert np.array_equal(probe[:steps], d["probe"] if start == "zero" else d["rprobe"])



@gpu
def test_largest_grids(kb):
    """The largest grids the library accepts (at most 2^31 - 1 cells): heat2d
    32767 x 65536 and heat3d 2 x 32767 x 32768 (8 GiB per field; the
    default one-step kernels, variants 13 and 9), 3 steps, row bands at the
    top, middle and bottom edges against the float32 oracle on the band plus
    a halo; the skeleton vector of 2^31 - 1 elements (four per thread and a
    tail of three), 3 iterations, its first and last 4096 elements bit for
    bit with the oracle's chain.  Fields come back through a device tensor,
    the compared rows alone to the host."""
    import torch
    steps = 3
    ny, nx, seed = 32767, 65536, 5
    announce("heat2d 32767 x 65536, variant 13, 3 steps")
    with kb.Problem(kb.HEAT2D, (ny, nx), HEAT, seed) as p:
        p.set_option(kb.OPT_TILE, 13)
        p.run(steps, 0)
        buf = torch.empty((ny, nx), dtype=torch.float32, device=p.device)
        p.read_device(kb.F_T, buf)
        bands = {ab: buf[ab[0]:ab[1]].cpu().numpy() for ab in band_rows(ny, steps)}
        del buf
    for (a, b), got in bands.items():
        lo, hi = max(0, a - steps - 1), min(ny, b + steps + 1)
        T0, P = band_inputs_2d(seed, ny, nx, lo, hi)
        e = rel_maxnorm(got, oracle.heat2d(T0, P, steps, dtype=np.float32)[a - lo:b - lo])
        print(f"heat2d rows {a}..{b}: vs float32 oracle {e:.2e}")
        assert e < 1e-5, (a, b)
    nz, ny, nx, seed = 2, 32767, 32768, 6
    announce("heat3d 2 x 32767 x 32768, variant 9, 3 steps")
    with kb.Problem(kb.HEAT3D, (nz, ny, nx), HEAT, seed) as p:
        p.set_option(kb.OPT_TILE, 9)
        p.run(steps, 0)
        buf = torch.empty((nz, ny, nx), dtype=torch.float32, device=p.device)
        p.read_device(kb.F_T, buf)
        bands = {ab: buf[:, ab[0]:ab[1]].cpu().numpy() for ab in band_rows(ny, steps)}
        del buf
    for (a, b), got in bands.items():
        lo, hi = max(0, a - steps - 1), min(ny, b + steps + 1)
        T0, P = band_inputs_3d(seed, nz, ny, nx, lo, hi)
        e = rel_maxnorm(got, oracle.heat3d(T0, P, steps, dtype=np.float32)[:, a - lo:b - lo])
        print(f"heat3d rows {a}..{b}: vs float32 oracle {e:.2e}")
        assert e < 1e-5, (a, b)
    n, seed, m = (1 << 31) - 1, 7, 4096
    announce("skeleton 2^31 - 1 elements, K = 4, 3 iterations")
    with kb.Problem(kb.SKELETON, (n,), (4,), seed) as p:
        p.run(steps, 0)
        a_k, b_k = p.read(kb.F_A), p.read(kb.F_B)
        buf = torch.empty(n, dtype=torch.float32, device=p.device)
        p.read_device(kb.F_X, buf)
        head, tail = buf[:m].cpu().numpy(), buf[n - m:].cpu().numpy()
        del buf
    for got, off in ((head, 0), (tail, n - m)):
        x0 = synth.uniform_f32(seed, synth.TAG_X0, m, *synth.X0_RANGE, offset=off)
        assert np.array_equal(got, oracle.skeleton(x0, a_k, b_k, steps, dtype=np.float32)), off

@gpu
@pytest.mark.parametrize("variant,depth", [(7, 1), (5, 1), (2, 1), (8, 2)])
def test_fdtd_largest_cavity_corners(kb, variant, depth):
    """N = 1024, the largest cavity the library accepts (two field sets of
    52 GB): seeded random fields on every node (drawn on the device), 6
    steps, no source.  A node after s steps depends only on nodes within s
    of it, so the two corner cubes of 25^3 nodes (one holding the walls at
    0, the other the walls at N and the i = N column) are exact cavities of
    N = 24 for the oracle away from their cut faces: every node farther
    than s + 1 from a cut face is compared, bit for bit, with the float32
    oracle run on the cube."""
    import torch
    N, steps, n = 1024, 6, 24
    M = N + 1
    announce(f"fdtd N=1024 corners, variant {variant} depth {depth}, {steps} steps")
    gen = torch.Generator(device="cuda").manual_seed(1000 + variant)
    lo, hi = {}, {}
    with kb.Problem(kb.FDTD3D, (N, 16), (0.5, 0.0, 80.0), 0) as p:   # width 0: no source
        p.set_option(kb.OPT_TILE, variant)
        p.set_option(kb.OPT_TDEPTH, depth)
        buf = torch.empty((M, M, M), dtype=torch.float32, device=p.device)
        for k, fid in kb.FDTD_FIELDS.items():
            buf.uniform_(-1.0, 1.0, generator=gen)
            p.write_device(fid, buf)
            lo[k] = buf[:n + 1, :n + 1, :n + 1].cpu().numpy()
            hi[k] = buf[N - n:, N - n:, N - n:].cpu().numpy()
        p.run(steps, 0)
        assert p.read(kb.F_STEP)[0] == steps
        got_lo, got_hi = {}, {}
        for k, fid in kb.FDTD_FIELDS.items():
            p.read_device(fid, buf)
            got_lo[k] = buf[:n + 1, :n + 1, :n + 1].cpu().numpy()
            got_hi[k] = buf[N - n:, N - n:, N - n:].cpu().numpy()
        del buf
    ref_lo, _ = oracle.fdtd(lo, n, steps, dtype=np.float32)
    ref_hi, _ = oracle.fdtd(hi, n, steps, dtype=np.float32)
    a, b = n - steps - 1, steps + 2          # exact: index < a (low cube), >= b (high cube)
    for k in oracle.FDTD_FIELDS:
        assert np.array_equal(got_lo[k][:a, :a, :a], ref_lo[k][:a, :a, :a]), ("low corner", k)
        assert np.array_equal(got_hi[k][b:, b:, b:], ref_hi[k][b:, b:, b:]), ("high corner", k)
        assert not np.array_equal(got_lo[k], lo[k]) and not np.array_equal(got_hi[k], hi[k]), k   # they moved
