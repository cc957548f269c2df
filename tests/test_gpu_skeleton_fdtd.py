"""GPU parity of the skeleton chain and the Yee FDTD solver through the C ABI.

Both are bit-identical to the float32 oracle: the skeleton update is one
fused multiply-add per kernel on both sides, and every FDTD coefficient is
0.5, so product and difference round the same way with or without fusion.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu, rel_maxnorm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kb():
    need_gpu()
    import paper_2501_09398_amd as kb
    kb.lib()
    return kb


# ---- skeleton -------------------------------------------------------------

def test_skeleton_initial_state(kb):
    with kb.Problem(kb.SKELETON, (1000,), (4,), 21) as p:
        x0, a, b = synth.skeleton_init(21, 1000, 4)
        assert np.array_equal(p.read(kb.F_X), x0)
        assert np.array_equal(p.read(kb.F_A), a)
        assert np.array_equal(p.read(kb.F_B), b)


@pytest.mark.parametrize("n", [1, 3, 1000, 4099, 1 << 16])
@pytest.mark.parametrize("variant", [1, 2, 3])
def test_skeleton_bitwise_vs_oracle(kb, n, variant):
    announce(f"skeleton n={n} variant={variant}")
    iters = 300
    x0, a, b = synth.skeleton_init(22, n, 4)
    with kb.Problem(kb.SKELETON, (n,), (4,), 22) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.run(iters, 0)
        got = p.read(kb.F_X)
    ref = oracle.skeleton(x0, a, b, iters, dtype=np.float32)
    assert np.array_equal(got, ref)
    print(f"skeleton n={n}: vs f64 {rel_maxnorm(got, oracle.skeleton(x0, a, b, iters)):.3e}")


@pytest.mark.parametrize("b", [1, 3, 50, 2000])
@pytest.mark.parametrize("builder", [0, 1])
def test_skeleton_graph_bitwise(kb, b, builder):
    announce(f"skeleton graph b={b} builder={builder}")
    n, iters = 4096, 2503
    outs = []
    for bb in (0, b):
        with kb.Problem(kb.SKELETON, (n,), (4,), 23) as p:
            p.set_option(kb.OPT_BUILDER, builder)
            p.run(iters, bb)
            outs.append(p.read(kb.F_X))
    assert np.array_equal(outs[0], outs[1])


def test_skeleton_full_size_workload(kb):
    # 2^16 elements, K = 4, 10,000 iterations, graph batches of 100.
    announce("skeleton 2^16 x 10000 b=100")
    n, iters = 1 << 16, 10000
    x0, a, b = synth.skeleton_init(20250116, n, 4)
    with kb.Problem(kb.SKELETON, (n,), (4,), 20250116) as p:
        p.run(iters, 100)
        got = p.read(kb.F_X)
        t = p.last_timing()
        assert t["n_graph_launches"] == 100 and t["n_nodes"] == 400
    assert np.array_equal(got, oracle.skeleton(x0, a, b, iters, dtype=np.float32))


def test_skeleton_explicit_coefficients_and_write(kb):
    with kb.Problem(kb.SKELETON, (64,), (2, 0.5, 0.5, 0.0, 0.0), 24) as p:
        x0 = p.read(kb.F_X)
        p.run(3, 2)
        assert np.array_equal(p.read(kb.F_X), x0 * np.float32(2.0 ** -6))
        p.write(kb.F_A, np.array([1.0, 1.0], np.float32))
        p.write(kb.F_B, np.array([0.25, -0.25], np.float32))
        before = p.read(kb.F_X)
        p.run(10, 4)           # graph cache was invalidated by the write
        ref = oracle.skeleton(before, np.array([1, 1], np.float32), np.array([0.25, -0.25], np.float32), 10,
                              dtype=np.float32)
        assert np.array_equal(p.read(kb.F_X), ref)


def test_skeleton_reduce(kb):
    with kb.Problem(kb.SKELETON, (100003,), (4,), 25) as p:
        p.run(10, 5)
        x = p.read(kb.F_X).astype(np.float64)
        s = p.reduce()[0]
        assert abs(s - np.sum(x)) <= x.size * 2.0 ** -50 * np.sum(np.abs(x))


# ---- FDTD -----------------------------------------------------------------

def gpu_fields(kb, p):
    return {k: p.read(f) for k, f in kb.FDTD_FIELDS.items()}


def test_fdtd_source_cell_from_seed(kb):
    for N in (8, 33):
        src = synth.fdtd_source_cell(31, N)
        with kb.Problem(kb.FDTD3D, (N, 64), kb.FDTD_COEFFS, 31) as p:
            p.run(1, 0)
            ez = p.read(kb.F_EZ)
            _, g32 = oracle.fdtd_pulse(1)
            i, j, k = src
            assert ez[k, j, i] == g32[0]
            assert np.count_nonzero(ez) == 1


@pytest.mark.parametrize("N,steps", [(8, 150), (17, 120), (32, 300), (4, 60), (5, 60), (6, 60)])
@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7])
def test_fdtd_bitwise_vs_oracle(kb, N, steps, variant):
    announce(f"fdtd N={N} steps={steps} variant={variant}")
    seed = 32
    src = synth.fdtd_source_cell(seed, N)
    _, g32 = oracle.fdtd_pulse(steps + 1)
    ref, probe_ref = oracle.fdtd(oracle.fdtd_zero_fields(N, np.float32), N, steps, src=src, g=g32,
                                 dtype=np.float32)
    with kb.Problem(kb.FDTD3D, (N, 512), kb.FDTD_COEFFS, seed) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.run(steps, 0)
        got = gpu_fields(kb, p)
        probe = p.read(kb.F_PROBE)
        assert p.read(kb.F_STEP)[0] == steps
    for k in oracle.FDTD_FIELDS:
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(probe[:steps], probe_ref)
    assert np.all(probe[steps:] == 0)


@pytest.mark.parametrize("variant,depth", [(8, 2), (9, 2), (10, 2), (10, 3)])
@pytest.mark.parametrize("N,steps", [(4, 61), (5, 60), (8, 150), (17, 121), (33, 40), (70, 23), (75, 100),
                                     (127, 9), (128, 13), (129, 12), (253, 6), (255, 7)])
def test_fdtd_two_step_kernel_vs_oracle(kb, N, steps, variant, depth):
    """Variants 8, 9 and 10 with depth 2 (two steps per launch, temporal
    blocking), and the whole rows with depth 3 (three steps per launch):
    from zero fields with the source on and from random fields on every
    node, per launch and in graph batches (a step count that is not a
    multiple of the depth ends with fused steps), bit for bit with the
    float32 oracle, probe included.  Variant 8: N = 70 and 75 span several
    tiles along i (60 nodes), j (13 rows) and k (plane segments).  Variants
    9, 10 (whole rows, four nodes per lane): N = 253 and 255 end the row
    inside and at the end of lane 63 (row padding in the last vector,
    none), N = 129 at element 1 of lane 32.  The three-step kernel keeps two
    nodes per lane up to N = 128: N = 128 fills the wave exactly (the i = N
    column in lane 63), N = 127 ends inside lane 63, the smaller sizes in
    earlier lanes."""
    announce(f"fdtd temporal blocking variant {variant} depth {depth} N={N} steps={steps}")
    seed = 36
    src = synth.fdtd_source_cell(seed, N)
    _, g32 = oracle.fdtd_pulse(steps + 1)
    M = N + 1
    rng = np.random.default_rng(N)
    f0 = {k: rng.uniform(-1.0, 1.0, (M, M, M)).astype(np.float32) for k in oracle.FDTD_FIELDS}
    for start in ("zero", "rand"):
        init = oracle.fdtd_zero_fields(N, np.float32) if start == "zero" else f0
        ref, probe_ref = oracle.fdtd(init, N, steps, src=src, g=g32, dtype=np.float32)
        for b in (0, 3):
            with kb.Problem(kb.FDTD3D, (N, 512), kb.FDTD_COEFFS, seed) as p:
                p.set_option(kb.OPT_TILE, variant)
                p.set_option(kb.OPT_TDEPTH, depth)
                if start == "rand":
                    for k, fid in kb.FDTD_FIELDS.items():
                        p.write(fid, f0[k])
                p.run(steps, b)
                got = gpu_fields(kb, p)
                probe = p.read(kb.F_PROBE)
                assert p.read(kb.F_STEP)[0] == steps
            for k in oracle.FDTD_FIELDS:
                assert np.array_equal(got[k], ref[k]), (start, b, k)
            assert np.array_equal(probe[:steps], probe_ref), (start, b)


@pytest.mark.parametrize("variant,depth", [(8, 2), (9, 2), (10, 2), (10, 3), (7, 1)])
def test_fdtd_source_on_block_edges(kb, variant, depth):
    """The source placed (coefficients i, j, k) on the rows and planes that
    two blocks of the blocked kernels compute -- one as output, the other as
    recomputed halo -- and at both ends of a row: the amplitude must enter
    every copy and the probe be recorded once.  N = 33: the three-step
    kernel's blocks output rows 7t..7t+6 and planes 9s..9s+8 (halo rows
    7t-3..7t-1 and 7t+7, 7t+8, halo planes 9s-3..9s-1); the two-step
    kernels' edges lie elsewhere among the same positions.  A short pulse
    (width 5, delay 10) makes the source large over the 40 steps; bit for
    bit with the float32 oracle, fields and probe, per launch and in graph
    batches."""
    N, steps = 33, 40
    _, g32 = oracle.fdtd_pulse(steps + 1, width=5.0, delay=10.0)
    cells = [(1, 6, 8), (32, 7, 9), (2, 8, 0), (16, 13, 17), (31, 14, 18), (5, 4, 26), (17, 32, 27), (32, 1, 32),
             (9, 9, 6), (24, 20, 11)]
    for src in cells:
        announce(f"fdtd source on block edges variant {variant} depth {depth} src={src}")
        ref, probe_ref = oracle.fdtd(oracle.fdtd_zero_fields(N, np.float32), N, steps, src=src, g=g32,
                                     dtype=np.float32)
        for b in (0, 3):
            with kb.Problem(kb.FDTD3D, (N, 64), (0.5, 5.0, 10.0) + tuple(float(c) for c in src), 0) as p:
                p.set_option(kb.OPT_TILE, variant)
                p.set_option(kb.OPT_TDEPTH, depth)
                p.run(steps, b)
                got = gpu_fields(kb, p)
                probe = p.read(kb.F_PROBE)
            for k in oracle.FDTD_FIELDS:
                assert np.array_equal(got[k], ref[k]), (src, b, k)
            assert np.array_equal(probe[:steps], probe_ref), (src, b)
            assert np.all(probe[steps:] == 0), (src, b)


def test_fdtd_two_step_depth_limits(kb):
    """Depth 1..3 for the cavity; depth 1 of variant 8 is the fused step;
    three steps per launch need the whole-row kernels (variant 8 refuses
    to run them)."""
    with kb.Problem(kb.FDTD3D, (8, 64), kb.FDTD_COEFFS, 0) as p:
        p.set_option(kb.OPT_TILE, 8)
        for bad in (0, 4):
            with pytest.raises(kb.KBError):
                p.set_option(kb.OPT_TDEPTH, bad)
        p.set_option(kb.OPT_TDEPTH, 3)
        with pytest.raises(kb.KBError):
            p.run(6, 0)
        p.set_option(kb.OPT_TDEPTH, 1)
        p.run(6, 0)
        assert p.read(kb.F_STEP)[0] == 6
        p.set_option(kb.OPT_TILE, 10)
        p.set_option(kb.OPT_TDEPTH, 3)
        assert p.kernels_per_iter() == 1
        p.run(6, 0)
        assert p.read(kb.F_STEP)[0] == 12


@pytest.mark.parametrize("b", [1, 7, 40])
@pytest.mark.parametrize("builder", [0, 1])
@pytest.mark.parametrize("variant", [2, 5])
def test_fdtd_graph_bitwise(kb, b, builder, variant):
    """Graph batches equal the per-launch loop; with the fused step (two
    buffer sets) an odd b needs the graph of each start parity."""
    announce(f"fdtd graph b={b} builder={builder} variant={variant}")
    N, steps = 20, 203
    outs = []
    for bb in (0, b):
        with kb.Problem(kb.FDTD3D, (N, 256), kb.FDTD_COEFFS, 33) as p:
            p.set_option(kb.OPT_BUILDER, builder)
            p.set_option(kb.OPT_TILE, variant)
            p.run(steps, bb)
            outs.append((gpu_fields(kb, p), p.read(kb.F_PROBE), p.read(kb.F_STEP)))
    for k in oracle.FDTD_FIELDS:
        assert np.array_equal(outs[0][0][k], outs[1][0][k])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2][0] == outs[1][2][0] == steps


def test_fdtd_fused_variant_switching(kb):
    """The fused step leaves the state in the other buffer set after an odd
    number of steps; switching to the in-place kernels and back continues
    from the current set, bit for bit with the oracle."""
    announce("fdtd fused / in-place switching")
    N, seed = 18, 35
    src = synth.fdtd_source_cell(seed, N)
    _, g32 = oracle.fdtd_pulse(200)
    ref, probe_ref = oracle.fdtd(oracle.fdtd_zero_fields(N, np.float32), N, 63, src=src, g=g32,
                                 dtype=np.float32)
    with kb.Problem(kb.FDTD3D, (N, 256), kb.FDTD_COEFFS, seed) as p:
        assert p.kernels_per_iter() == 2                   # fused by default
        for v, n, b in ((5, 33, 4), (2, 20, 3), (6, 7, 0), (3, 3, 0)):
            p.set_option(kb.OPT_TILE, v)
            assert p.kernels_per_iter() == (2 if v >= 5 else 3)
            p.run(n, b)
        got = gpu_fields(kb, p)
        probe = p.read(kb.F_PROBE)
    for k in oracle.FDTD_FIELDS:
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(probe[:63], probe_ref)


def test_fdtd_explicit_source_and_cavity_mode(kb):
    # No source (width 0); Ez initialised to the lowest TM mode with H = 0:
    # the amplitude obeys e_{n+1} + e_{n-1} = (2 - dt^2 lam) e_n.
    announce("fdtd cavity mode N=24")
    N, dt = 24, 0.5
    M = N + 1
    i = np.arange(M)
    phi = np.sin(np.pi * i[None, :] / N) * np.sin(np.pi * i[:, None] / N)
    ez = np.zeros((M, M, M), np.float32)
    ez[:N] = phi[None]
    with kb.Problem(kb.FDTD3D, (N, 16), (0.5, 0.0, 80.0), 0) as p:
        p.write(kb.F_EZ, ez)
        amps = [1.0]
        for _ in range(60):
            p.run(1, 0)
            e = p.read(kb.F_EZ)
            amps.append(float(e[N // 2, N // 2, N // 2] / phi[N // 2, N // 2]))
    e = np.array(amps)
    lam = 8 * np.sin(np.pi / (2 * N)) ** 2
    assert np.max(np.abs(e[2:] + e[:-2] - (2 - dt * dt * lam) * e[1:-1])) < 1e-5


@pytest.mark.parametrize("variant,steps", [(2, 120), (5, 121)])
def test_fdtd_energy_reduce(kb, variant, steps):
    N = 16
    with kb.Problem(kb.FDTD3D, (N, 64), kb.FDTD_COEFFS, 34) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.run(steps, 10)
        f = gpu_fields(kb, p)
        e2, h2 = p.reduce()
    ref_e = sum(np.sum(f[k].astype(np.float64) ** 2) for k in ("Ex", "Ey", "Ez"))
    ref_h = sum(np.sum(f[k].astype(np.float64) ** 2) for k in ("Hx", "Hy", "Hz"))
    assert abs(e2 - ref_e) <= 1e-12 * ref_e and abs(h2 - ref_h) <= 1e-12 * ref_h


@pytest.mark.parametrize("variant", [2, 5, 7])
def test_fdtd_full_size_sampled(kb, variant):
    # 128^3 at the benchmark's launch configuration: 100 steps (source on)
    # against the float32 oracle, bit for bit.
    announce(f"fdtd 128^3 100 steps b=50 variant {variant}")
    N, steps, seed = 128, 100, 20250116
    src = synth.fdtd_source_cell(seed, N)
    _, g32 = oracle.fdtd_pulse(steps + 1)
    ref, probe_ref = oracle.fdtd(oracle.fdtd_zero_fields(N, np.float32), N, steps, src=src, g=g32,
                                 dtype=np.float32)
    with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, seed) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.run(steps, 50)
        got = gpu_fields(kb, p)
        probe = p.read(kb.F_PROBE)
    for k in oracle.FDTD_FIELDS:
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(probe[:steps], probe_ref)


@pytest.mark.parametrize("N", [7, 12, 33])
def test_fdtd_random_fields_both_variants(kb, N):
    # Arbitrary (non-PEC) fields written through kb_write: both kernel
    # variants match the float32 oracle bit for bit, including nodes that
    # the update leaves alone.
    announce(f"fdtd random fields N={N}")
    rng = np.random.default_rng(N)
    M = N + 1
    f0 = {k: rng.standard_normal((M, M, M)).astype(np.float32) for k in oracle.FDTD_FIELDS}
    ref, _ = oracle.fdtd(f0, N, 9, dtype=np.float32)
    for variant in (1, 2, 3, 4, 5, 6, 7):
        with kb.Problem(kb.FDTD3D, (N, 16), (0.5, 0.0, 80.0), 0) as p:
            p.set_option(kb.OPT_TILE, variant)
            for k, fid in kb.FDTD_FIELDS.items():
                p.write(fid, f0[k])
            p.run(9, 4)
            for k, fid in kb.FDTD_FIELDS.items():
                assert np.array_equal(p.read(fid), ref[k]), (variant, k)


@pytest.mark.parametrize("builder", [0, 1])
@pytest.mark.parametrize("update", [0, 1])
def test_skeleton_coefficient_write_updates_or_drops_graphs(kb, builder, update):
    """New a_k, b_k after graphs are cached: with KB_OPT_GRAPH_UPDATE=1 the
    cached graphs are refitted in place (no rebuild on the next run), with 0
    they are dropped and rebuilt; both give the per-launch bits."""
    announce(f"skeleton graph update builder={builder} update={update}")
    n, b = 3000, 10
    a2 = np.array([0.95, 0.97, 0.99, 0.93], np.float32)
    b2 = np.array([0.001, -0.002, 0.003, -0.004], np.float32)
    with kb.Problem(kb.SKELETON, (n,), (4,), 41) as p:
        p.set_option(kb.OPT_BUILDER, builder)
        p.set_option(kb.OPT_GRAPH_UPDATE, update)
        p.run(100, b)
        assert p.last_timing()["n_graphs_built"] == 1
        x_mid = p.read(kb.F_X)
        p.write(kb.F_A, a2)
        p.write(kb.F_B, b2)
        p.run(100, b)
        t = p.last_timing()
        got = p.read(kb.F_X)
    if update:
        assert t["n_graphs_updated"] == 1 and t["n_graphs_built"] == 0
    else:
        assert t["n_graphs_updated"] == 0 and t["n_graphs_built"] == 1
    print(f"refit/drop {t['t_update_s'] * 1e6:.1f} us, next T_C {t['t_create_s'] * 1e6:.1f} us")
    with kb.Problem(kb.SKELETON, (n,), (4,), 41) as q:
        q.write(kb.F_X, x_mid)
        q.write(kb.F_A, a2)
        q.write(kb.F_B, b2)
        q.run(100, 0)
        assert np.array_equal(got, q.read(kb.F_X))
    assert np.array_equal(got, oracle.skeleton(x_mid, a2, b2, 100, dtype=np.float32))


def yee_energy(E, Hm, Hp):
    """Discrete energy conserved by the Yee update: 1/2 |E^n|^2 + 1/2 <H^(n-1/2), H^(n+1/2)>."""
    e = sum(math.fsum(E[k].astype(np.float64).ravel() ** 2) for k in ("Ex", "Ey", "Ez"))
    h = sum(math.fsum((Hm[k].astype(np.float64) * Hp[k].astype(np.float64)).ravel()) for k in ("Hx", "Hy", "Hz"))
    return 0.5 * e + 0.5 * h


def cavity_omega(N, dt, m, n, p):
    """Phase per step of mode (m, n, p) of the Yee PEC cavity: the discrete
    dispersion relation sin(w/2) = (dt/2) sqrt(4 (sin^2(m pi/2N) + ...))."""
    lam = 4 * sum(np.sin(q * np.pi / (2 * N)) ** 2 for q in (m, n, p))
    return 2 * np.arcsin(dt / 2 * np.sqrt(lam))


def spectral_peaks(x, d, lo, hi, rel=0.05):
    """Frequencies (rad per step) of the local maxima of |FFT| (Hann window,
    linear trend removed, zero-padded) in (lo, hi) above rel of the largest."""
    t = np.arange(x.size)
    x = x - np.polyval(np.polyfit(t, x, 1), t)
    nfft = 1 << 20
    spec = np.abs(np.fft.rfft(x * np.hanning(x.size), nfft))
    w = 2 * np.pi * np.fft.rfftfreq(nfft, d=d)
    idx = np.where((w > lo) & (w < hi))[0]
    s = spec[idx]
    loc = [idx[i] for i in range(1, len(idx) - 1) if s[i] > s[i - 1] and s[i] > s[i + 1]]
    big = max(spec[i] for i in loc)
    return [w[i] for i in loc if spec[i] > rel * big]


def test_fdtd_128_10000_steps_energy_and_lowest_mode(kb):
    """The 128^3 cavity for 10,000 steps in graph batches of 100 (the
    benchmark's launch configuration) with the in-chain reduction every 4
    steps.  (1) Once the pulse has passed (g < 1e-30 after step 300) the
    discrete energy is conserved: W at steps 300 and 9,998 agree to float32
    round-off.  (2) The lowest cavity modes: H.H(t) = sum_m |h_m|^2
    sin^2(w_m t + phi_m) (the modes are orthogonal), so the spectrum of the
    logged H.H has lines at 2 w_m only; the probe (Ez at the source) has
    lines at w_m.  The lowest three lines of each sit at the closed-form
    frequencies of modes (1,1,0), (1,1,1), (2,1,0)."""
    announce("fdtd 128^3 10000 steps b=100")
    N, dt, seed = 128, 0.5, 20250116
    with kb.Problem(kb.FDTD3D, (N, 16384), kb.FDTD_COEFFS, seed) as p:
        p.set_option(kb.OPT_REDUCE_EVERY, 4)
        p.run(300, 100)                      # fields E^300, H^(299.5)
        E300 = {k: p.read(kb.FDTD_FIELDS[k]) for k in ("Ex", "Ey", "Ez")}
        Hm300 = {k: p.read(kb.FDTD_FIELDS[k]) for k in ("Hx", "Hy", "Hz")}
        p.run(1, 0)                          # H^(300.5)
        Hp300 = {k: p.read(kb.FDTD_FIELDS[k]) for k in ("Hx", "Hy", "Hz")}
        p.run(9998 - 301, 100)               # E^9998, H^(9997.5)
        E2 = {k: p.read(kb.FDTD_FIELDS[k]) for k in ("Ex", "Ey", "Ez")}
        Hm2 = {k: p.read(kb.FDTD_FIELDS[k]) for k in ("Hx", "Hy", "Hz")}
        p.run(1, 0)                          # H^(9998.5)
        Hp2 = {k: p.read(kb.FDTD_FIELDS[k]) for k in ("Hx", "Hy", "Hz")}
        p.run(1, 0)
        log = p.reduction_log()
        probe = p.read(kb.F_PROBE)[:10000].astype(np.float64)
        assert p.read(kb.F_STEP)[0] == 10000
    W1, W2 = yee_energy(E300, Hm300, Hp300), yee_energy(E2, Hm2, Hp2)
    print(f"energy W(300) {W1:.9e} W(9998) {W2:.9e} rel change {abs(W2 - W1) / W1:.2e}")
    assert W1 > 0 and abs(W2 - W1) <= 1e-4 * W1
    assert log.shape[0] == 2500 and log[-1, 0] == 10000
    modes = [cavity_omega(N, dt, *m) for m in ((1, 1, 0), (1, 1, 1), (2, 1, 0))]
    w110 = modes[0]
    hh = log[log[:, 0] >= 300, 2]
    pk_h = [w / 2 for w in spectral_peaks(hh, 4.0, 2 * 0.3 * w110, 2 * 1.7 * w110)]
    pk_p = spectral_peaks(probe[300:], 1.0, 0.3 * w110, 1.7 * w110)
    print("closed form", [f"{w:.6f}" for w in modes])
    print("H.H lines / 2", [f"{w:.6f}" for w in pk_h[:4]], "probe lines", [f"{w:.6f}" for w in pk_p[:4]])
    for pk in (pk_h, pk_p):
        assert len(pk) >= 3
        for got, want in zip(pk[:3], modes):
            assert abs(got - want) <= 1e-3 * want, (got, want)
