"""Pins of the surrogate's CPU oracle (conv net forward/backward, bf16
rounding, Adam) against library routines, closed forms and finite
differences -- none of which reuses the oracle's own loops."""
import math

import numpy as np
import pytest

import oracle
import synth

NW = oracle.SG_NW
OFF = {}
_o = 0
for _l, (_ci, _co) in enumerate([(2, 32), (32, 32), (32, 32), (32, 1)]):
    OFF[f"W{_l + 1}"] = (_o, (_co, _ci, 3, 3))
    _o += _co * _ci * 9
    OFF[f"b{_l + 1}"] = (_o, (_co,))
    _o += _co
assert _o == NW


def put(w, name, value):
    o, shape = OFF[name]
    w[o:o + int(np.prod(shape))] = np.asarray(value, dtype=np.float64).reshape(-1)


def random_weights(seed):
    w = synth.surrogate_init(seed).astype(np.float64)
    o, shape = OFF["W4"]
    w[o:o + 288] = synth.uniform_f32(seed + 1, 9, 288, -0.06, 0.06)
    w[o + 288] = 0.01
    return w


def test_bf16_rounding_matches_torch_and_ties_to_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(2000), rng.uniform(-1e5, 1e5, 200), [1e-30, -3e-20]]).astype(np.float32)
    ref = torch.tensor(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = oracle.bf16_round(v.astype(np.float64))
    assert np.array_equal(got, ref)
    assert oracle.bf16_round(1.0 + 2.0 ** -8) == 1.0                   # tie -> even
    assert oracle.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6   # tie -> even
    assert oracle.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7


def test_single_conv_equals_one_heat_step():
    # One 3x3 convolution with replicate padding and the heat stencil as
    # weights (T channel) plus c on P and c*Tamb/Rz as bias is exactly one
    # explicit thermal step with clamped neighbours.
    c, Rx, Ry, Rz, Tamb = 1e-3, 1.0, 2.0, 10.0, 300.0
    cx, cy, cz = c / Rx, c / Ry, c / Rz
    W = np.zeros((1, 2, 3, 3))
    W[0, 0] = [[0, cy, 0], [cx, 1 - 2 * cx - 2 * cy - cz, cx], [0, cy, 0]]
    W[0, 1, 1, 1] = c
    T0, P = synth.heat2d_init(3, 13, 17)
    x = np.stack([T0, P]).astype(np.float64)
    out = oracle.sg_conv3x3(W, np.array([cz * Tamb]), x)[0]
    ref = oracle.heat2d(T0, P, 1, c=c, Rx=Rx, Ry=Ry, Rz=Rz, Tamb=Tamb)
    assert np.max(np.abs(out - ref)) < 1e-12


def test_forward_chain_of_gelus_closed_form():
    # Weights that pass the normalised T through every layer's channel 0:
    # y = gelu(gelu(gelu(t))) per pixel, with t = (T0-333)/10 (no rounding).
    w = np.zeros(NW)
    for l, ci in ((1, 2), (2, 32), (3, 32)):
        W = np.zeros((32, ci, 3, 3))
        W[0, 0, 1, 1] = 1.0
        put(w, f"W{l}", W)
    W4 = np.zeros((1, 32, 3, 3))
    W4[0, 0, 1, 1] = 1.0
    put(w, "W4", W4)
    T0, P = synth.heat2d_init(4, 6, 7)
    y = oracle.sg_forward(w, T0, P, round_bf16=False)
    g = lambda v: 0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0)))
    ref = np.vectorize(lambda t: g(g(g(t))))((T0.astype(np.float64) - 333.0) / 10.0)
    assert np.max(np.abs(y - ref)) < 1e-14
    # the power channel enters through W1[:, 1]
    put(w, "W1", np.zeros((32, 2, 3, 3)))
    W1 = np.zeros((32, 2, 3, 3))
    W1[0, 1, 1, 1] = 1.0
    put(w, "W1", W1)
    y = oracle.sg_forward(w, T0, P, round_bf16=False)
    ref = np.vectorize(lambda p: g(g(g(p))))((P.astype(np.float64) - 0.5) / 0.29)
    assert np.max(np.abs(y - ref)) < 1e-14


def test_gradient_matches_central_differences():
    w = random_weights(5)
    T0, P = synth.heat2d_init(6, 5, 6)
    target = np.sin(np.arange(30)).reshape(5, 6) * 0.3
    loss, g = oracle.sg_loss_grad(w, T0, P, target, round_bf16=False)
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(np.arange(a, a + int(np.prod(s))), min(6, int(np.prod(s))), replace=False)
                          for a, s in OFF.values()])
    h = 1e-5
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        lp = np.mean((oracle.sg_forward(wp, T0, P, round_bf16=False) - target) ** 2)
        lm = np.mean((oracle.sg_forward(wm, T0, P, round_bf16=False) - target) ** 2)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, g[i])
    assert abs(loss - np.mean((oracle.sg_forward(w, T0, P, round_bf16=False) - target) ** 2)) < 1e-15


def test_gradient_edge_pixels_adjoint():
    # <conv(W, x), g> = <x, conv^T(W, g)> is exercised through the loss
    # gradient of a one-pixel-wide image, where every tap clamps.
    w = random_weights(8)
    for shape in ((1, 1), (1, 4), (3, 1)):
        T0, P = synth.heat2d_init(9, *shape)
        target = np.zeros(shape)
        loss, g = oracle.sg_loss_grad(w, T0, P, target, round_bf16=False)
        i = OFF["W2"][0] + 7
        h = 1e-5
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (np.mean(oracle.sg_forward(wp, T0, P, round_bf16=False) ** 2)
              - np.mean(oracle.sg_forward(wm, T0, P, round_bf16=False) ** 2)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-4, abs(fd))


def test_rounded_forward_close_to_exact():
    # bf16 operands move the output by about 2^-8 relative per layer.
    w = random_weights(10)
    T0, P = synth.heat2d_init(11, 16, 16)
    a = oracle.sg_forward(w, T0, P, round_bf16=True)
    b = oracle.sg_forward(w, T0, P, round_bf16=False)
    assert 0 < np.max(np.abs(a - b)) < 0.05 * np.max(np.abs(b))


def test_adam_constant_gradient_closed_form():
    # With a constant gradient the bias-corrected moments equal g and g^2,
    # so every step moves w by lr * g / (|g| + eps).
    n, lr, eps = 5, 1e-3, 1e-8
    g = np.array([0.5, -2.0, 1e-3, 3.0, -0.25])
    w = np.zeros(n)
    m = np.zeros(n)
    v = np.zeros(n)
    for t in range(1, 11):
        oracle.adam(w, g, m, v, t, lr=lr, eps=eps)
    ref = -10 * lr * g / (np.abs(g) + eps)
    assert np.max(np.abs(w - ref)) < 1e-15
