"""Pins of the seeded input generator (no solver arithmetic here)."""
import os

import numpy as np

import synth


def test_splitmix64_reference_vector(golden_dir):
    # Output idx of stream (seed, tag=0) is the (idx+1)-th SplitMix64 output.
    vals = [int(l) for l in open(os.path.join(golden_dir, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    got = [int(v) for v in synth.raw64(1234567, 0, range(len(vals)))]
    assert got == vals


def test_counter_mode_is_random_access():
    # Drawing a slice directly equals slicing a longer draw.
    full = synth.raw64(7, synth.TAG_T0, np.arange(1000))
    part = synth.raw64(7, synth.TAG_T0, np.arange(400, 600))
    assert np.array_equal(full[400:600], part)


def test_tags_give_distinct_streams():
    a = synth.raw64(3, synth.TAG_T0, np.arange(64))
    b = synth.raw64(3, synth.TAG_P, np.arange(64))
    assert not np.any(a == b)


def test_uniform_ranges_and_moments():
    n = 1 << 20
    u = synth.uniform01(11, 1, np.arange(n))
    assert u.min() >= 0.0 and u.max() < 1.0
    # mean 1/2, variance 1/12 within ~5 standard errors
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
    T0, P = synth.heat2d_init(0, 256, 256)
    assert T0.dtype == np.float32 and T0.min() >= 323 and T0.max() < 343
    assert P.min() >= 0 and P.max() < 1
    x0, a, b = synth.skeleton_init(0, 4096)
    assert x0.min() >= -1 and x0.max() < 1
    assert np.all((a >= 0.9) & (a < 1.0)) and np.all((b >= -0.01) & (b < 0.01))


def test_value_is_single_rounding_of_float64_affine():
    # 24-bit uniforms times 20 are exact in float64, so T0 = fl32(323 + 20u).
    idx = np.arange(16)
    u = synth.uniform01(5, synth.TAG_T0, idx)
    T0 = synth.uniform_f32(5, synth.TAG_T0, 16, 323.0, 343.0)
    assert np.array_equal(T0, (323.0 + 20.0 * u).astype(np.float32))


def test_source_cell_in_interior():
    for seed in range(50):
        for N in (8, 128, 256):
            i, j, k = synth.fdtd_source_cell(seed, N)
            assert 2 <= i <= N - 2 and 2 <= j <= N - 2 and 1 <= k <= N - 2


def test_multigrid_sides_log_uniform():
    s = synth.multigrid_sides(20250116, 64)
    assert len(s) == 64 and min(s) >= 64 and max(s) <= 1024
    # log-uniform: median of log2(side) near 8 (= log2 of 256)
    assert 7.0 < np.median(np.log2(s)) < 9.0
