"""Pins of the oracle's skeleton chain against the closed-form affine recurrence.

One iteration applies x <- a_k x + b_k for k = 1..K, i.e. the affine map
x <- A x + B with A = a_K...a_1 and B = sum_k b_k prod_{m>k} a_m, so after n
iterations x_n = A^n x_0 + B (1 - A^n) / (1 - A).
"""
from fractions import Fraction

import numpy as np

import oracle
import synth


def affine_coeffs(a, b):
    A, B = Fraction(1), Fraction(0)
    for ak, bk in zip(a, b):
        A, B = Fraction(float(ak)) * A, Fraction(float(ak)) * B + Fraction(float(bk))
    return A, B


def test_skeleton_exact_rational_short_run():
    x0, a, b = synth.skeleton_init(0, 16, K=4)
    A, B = affine_coeffs(a, b)
    n = 12
    got = oracle.skeleton(x0, a, b, n)
    for e in range(16):
        ref = A ** n * Fraction(float(x0[e])) + B * (1 - A ** n) / (1 - A)
        assert abs(got[e] - float(ref)) <= 1e-14 * max(1.0, abs(float(ref)))


def test_skeleton_closed_form_long_run():
    x0, a, b = synth.skeleton_init(1, 4096, K=4)
    A = np.prod(a.astype(np.float64))
    B = 0.0
    for ak, bk in zip(a.astype(np.float64), b.astype(np.float64)):
        B = ak * B + bk
    n = 10000
    ref = A ** n * x0.astype(np.float64) + B * (1 - A ** n) / (1 - A)
    got = oracle.skeleton(x0, a, b, n)
    assert np.max(np.abs(got - ref)) < 1e-12
    # float32 instantiation: each kernel rounds once, and the map is a
    # contraction, so the error stays below K*u*max|x|/(1-A) (u = 2^-24).
    got32 = oracle.skeleton(x0, a, b, n, dtype=np.float32)
    bound = 4 * 2.0 ** -24 * max(1.0, np.max(np.abs(ref))) / (1 - A)
    assert np.max(np.abs(got32 - ref)) <= bound


def test_skeleton_identity_and_exact_halving():
    x0, _, _ = synth.skeleton_init(2, 1000, K=4)
    one, zero = np.ones(4, np.float32), np.zeros(4, np.float32)
    assert np.array_equal(oracle.skeleton(x0, one, zero, 50, dtype=np.float32), x0)
    half = np.full(4, 0.5, np.float32)
    got = oracle.skeleton(x0, half, zero, 3, dtype=np.float32)  # 12 halvings, exact
    assert np.array_equal(got, x0 * np.float32(2.0 ** -12))


def test_skeleton_kernel_order_matters():
    # With b_k != 0 the chain is not commutative; the oracle applies k = 1..K
    # in order: one iteration of (a=[2,1], b=[0,1]) maps x to 2x + 1.
    x0 = np.array([1.0, -3.0])
    got = oracle.skeleton(x0, np.array([2.0, 1.0]), np.array([0.0, 1.0]), 1)
    assert np.array_equal(got, 2 * x0 + 1)


def test_skeleton_float32_is_fused():
    # One rounding per kernel: a*x + b with the product kept exact.
    # (1 + 2^-12)^2 - 1 = 2^-11 + 2^-24 is a float32; rounding the product
    # first would give 2^-11.
    x0 = np.array([1.0 + 2.0 ** -12], np.float32)
    a = np.array([1.0 + 2.0 ** -12], np.float32)
    b = np.array([-1.0], np.float32)
    got = oracle.skeleton(x0, a, b, 1, dtype=np.float32)
    assert got[0] == np.float32(2.0 ** -11 + 2.0 ** -24)
