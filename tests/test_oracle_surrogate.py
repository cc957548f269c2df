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


# ---------------------------------------------------------------------------
# Rounding points of the bf16 path (round_bf16=True).  Each case is a single
# path through channel 0 of every layer (centre taps only, other weights
# zero) on a uniform field, with every pre-activation of channel 0 >= 16,
# where erf(z/sqrt 2) is exactly 1 in double: GELU is then exactly the
# identity and GELU' exactly 1, so the output is known by hand.  In each
# case exactly one operand class is not bf16-representable -- the input, one
# layer's weight, one hidden activation, or the gradient entering a product
# -- and the expected value is the one that rounds at that point; the value
# an oracle gets when it skips that rounding (or rounds a bias) is listed
# beside it and differs.  Biases (layer 2 or 3 here) are not rounded; they
# move an activation into a finer binade so that a skipped rounding is not
# masked by the next layer's rounding.
# ---------------------------------------------------------------------------
def single_path(w1, w2, w3, w4, b=(0.0, 0.0, 0.0, 0.0)):
    w = np.zeros(NW)
    for l, (wl, ci) in enumerate(((w1, 2), (w2, 32), (w3, 32), (w4, 32))):
        W = np.zeros((32 if l < 3 else 1, ci, 3, 3))
        W[0, 0, 1, 1] = wl
        put(w, f"W{l + 1}", W)
        bias = np.zeros(32 if l < 3 else 1)
        bias[0] = b[l]
        put(w, f"b{l + 1}", bias)
    return w


def uniform_field(T, shape=(2, 3)):
    return np.full(shape, T, np.float32), np.full(shape, 0.5, np.float32)   # P = 0.5: p input exactly 0


@pytest.mark.parametrize("case,T,ws,b,expected,skipped", [
    # the input t = (336-333)/10 = 0.3 -> 0.30078125; 96 t = 28.875
    ("input", 336.0, (96.0, 1.0, 1.0, 2.0 ** -5), (0, 0, 0, 0), 0.90234375, 0.8984375),
    # t = 0.75 exact; W1 = 32.09 -> 32 (unrounded: 24.0675 -> 24.125)
    ("weight 1", 340.5, (32.09, 1.0, 1.0, 2.0 ** -5), (0, 0, 0, 0), 0.75, 0.75390625),
    ("weight 2", 340.5, (32.0, 1.003, 1.0, 2.0 ** -5), (0, 0, 0, 0), 0.75, 0.75390625),
    ("weight 3", 340.5, (32.0, 1.0, 1.003, 2.0 ** -5), (0, 0, 0, 0), 0.75, 0.75390625),
    # last layer: 0.0157 -> 129 * 2^-13; y = 32 * that (no activation after it)
    ("weight 4", 338.0, (64.0, 1.0, 1.0, 0.0157), (0, 0, 0, 0), 0.50390625, 32 * 0.0157),
    # activation 1: 96.5 * 0.75 = 72.375 -> 72.5; minus 48.5 -> 24 (unrounded 23.875)
    ("activation 1", 340.5, (96.5, 1.0, 1.0, 2.0 ** -5), (0, -48.5, 0, 0), 0.75, 0.74609375),
    # activation 2: 24 * 193/64 = 72.375 -> 72.5; minus 48.5 -> 24
    ("activation 2", 340.5, (32.0, 193 / 64, 1.0, 2.0 ** -5), (0, 0, -48.5, 0), 0.75, 0.74609375),
    # activation 3: 72.375 -> 72.5 straight into the last layer
    ("activation 3", 340.5, (32.0, 1.0, 193 / 64, 2.0 ** -7), (0, 0, 0, 0), 0.56640625, 72.375 / 128),
    # the last bias is not rounded: 0.3 stays 0.3 (rounded it would be 0.30078125)
    ("bias", 338.0, (64.0, 1.0, 1.0, 0.0157), (0, 0, 0, 0.3), 0.50390625 + 0.3, 0.50390625 + 0.30078125),
])
def test_rounded_forward_rounding_points(case, T, ws, b, expected, skipped):
    assert expected != skipped
    T0, P = uniform_field(T)
    y = oracle.sg_forward(single_path(*ws, b=b), T0, P, round_bf16=True)
    assert np.all(np.abs(y - expected) <= 1e-15 * abs(expected)), (case, y[0, 0], expected)
    # the unrounded evaluation gives the exact path value (no rounding anywhere)
    exact = oracle.sg_forward(single_path(*ws, b=b), T0, P, round_bf16=False)
    t = (np.float64(T) - 333.0) / 10.0
    z = ws[0] * t + b[0]
    z = ws[1] * z + b[1]
    z = ws[2] * z + b[2]
    assert np.allclose(exact, ws[3] * z + b[3], rtol=1e-14, atol=0)


def test_rounded_gradient_rounding_points():
    """One pixel (every tap clamps onto it), loss (y - target)^2.  Path:
    t = 0.75, W1 = 32 (a1 = 24), W2 = 1 (a2 = 24), W3 = 5 (a3 = 120),
    W4 = 7/128 (y = 6.5625); target 6.4125, so dL/dy = 0.3 (not bf16).
    Hand-computed, with r() = bf16 rounding and GELU' = 1 on the path:
      g4 = r(0.3) = 77/256                  dW4 = g4 * 120 = 36.09375 (all 9 taps)
      db4 = 0.3 (unrounded)
      gb3 = 7/128 * g4 = 539/2^15           db3 = 539/2^15 (unrounded)
      g3 = r(gb3) = 540/2^15                dW3 = g3 * 24 = 0.3955078125
      gb2 = 5 * g3 = 2700/2^15              db2 = 2700/2^15
      g2 = r(gb2) = 2704/2^15               dW2 = g2 * 24 = 1.98046875
      gb1 = g2 (exact)                      db1 = 2704/2^15, dW1[.,t] = g2 * 0.75
    Skipping a rounding gives: dW4 21.6*120/72 = 36.0, db4 0.30078125 if the
    bias took the rounded g, g3 536/2^15 if dgrad took the unrounded g4,
    dW3 539*24/2^15, g2 2688/2^15 if dgrad took the unrounded g3."""
    w = single_path(32.0, 1.0, 5.0, 7.0 / 128.0)
    T0, P = uniform_field(340.5, (1, 1))
    target = np.array([[6.4125]])
    dy = 2.0 * (6.5625 - 6.4125)
    loss, g = oracle.sg_loss_grad(w, T0, P, target, round_bf16=True)
    assert abs(loss - (6.5625 - 6.4125) ** 2) < 1e-15

    def grad(name):
        o, shape = OFF[name]
        return g[o:o + int(np.prod(shape))].reshape(shape)

    S = 2.0 ** -15
    cases = [  # (array, index, expected, what an oracle that skips the rounding gets)
        ("W4", (0, 0), 77 / 256 * 120, dy * 120),
        ("b4", (0,), dy, 77 / 256),
        ("W3", (0, 0), 540 * S * 24, 539 * S * 24),
        ("b3", (0,), 539 * S, 540 * S),
        ("W2", (0, 0), 2704 * S * 24, 2688 * S * 24),
        ("b2", (0,), 2700 * S, 2704 * S),
        ("W1", (0, 0), 2704 * S * 0.75, 2688 * S * 0.75),
        ("b1", (0,), 2704 * S, 2688 * S),
    ]
    for name, idx, want, skipped in cases:
        got = grad(name)[idx]
        assert want != skipped
        if got.ndim:                       # a 3x3 weight block: every tap reads the one pixel
            assert np.all(np.abs(got - want) <= 1e-15 * abs(want)), (name, got, want)
        else:
            assert abs(got - want) <= 1e-15 * abs(want), (name, got, want)
    # nothing reaches the other channels or the power input (p = 0)
    assert np.all(grad("W1")[0, 1] == 0) and np.all(grad("W1")[1:] == 0)
    for name in ("W2", "W3"):
        G = grad(name).copy()
        G[0, 0] = 0
        assert np.all(G == 0), name
    assert np.all(grad("W4")[0, 1:] == 0)
    # the unrounded gradient is the plain chain rule on the same path
    _, g0 = oracle.sg_loss_grad(w, T0, P, target, round_bf16=False)
    o, _ = OFF["W1"]
    assert abs(g0[o + 4] - dy * (7 / 128) * 5 * 0.75) < 1e-15


def test_conv_adjoints_are_adjoint():
    """<conv(W, x), g> = <x, adjoint_input(W, g)> and the weight adjoint
    equals the derivative of <conv(W, x), g> in W (it is linear in W), on
    a small field where every tap clamps somewhere."""
    rng = np.random.default_rng(3)
    W = rng.standard_normal((5, 3, 3, 3))
    x = rng.standard_normal((3, 4, 6))
    g = rng.standard_normal((5, 4, 6))
    lhs = np.sum(oracle.sg_conv3x3(W, None, x) * g)
    assert abs(lhs - np.sum(x * oracle.sg_conv3x3_adjoint_input(W, g))) < 1e-12 * np.sum(np.abs(g))
    dW, db = oracle.sg_conv3x3_adjoint_weights(x, g)
    assert abs(lhs - np.sum(dW * W)) < 1e-12 * np.sum(np.abs(g))
    assert np.allclose(db, g.sum(axis=(1, 2)), rtol=1e-14, atol=1e-14)


def test_oracle_threads_do_not_change_bits():
    T0, P = synth.heat2d_init(12, 40, 70)
    w = random_weights(13)
    with oracle.threads(1):
        a = oracle.heat2d(T0, P, 30, dtype=np.float32)
        ya = oracle.sg_forward(w, T0, P)
        la, ga = oracle.sg_loss_grad(w, T0, P, np.zeros((40, 70)))
    with oracle.threads(4):
        b = oracle.heat2d(T0, P, 30, dtype=np.float32)
        yb = oracle.sg_forward(w, T0, P)
        lb, gb = oracle.sg_loss_grad(w, T0, P, np.zeros((40, 70)))
    assert np.array_equal(a, b) and np.array_equal(ya, yb) and la == lb and np.array_equal(ga, gb)


def test_gelu_relative_accuracy_in_the_negative_tail():
    """GELU(x) = x Phi(x) and GELU'(x) = Phi(x) + x phi(x) with Phi the normal
    distribution function: against scipy's ndtr (a library routine, not the
    oracle's formula) over [-30, 8], where the form (1 + erf(x/sqrt 2))/2
    loses every digit below x = -8, to 1e-14 (1 + x^2) relative (x^2: the
    condition number of Phi in the tail).  Two table values as well:
    Phi(-5) = 2.866515718791939e-7 and Phi(-10) = 7.619853024160527e-24."""
    from scipy.special import ndtr
    x = np.linspace(-30.0, 8.0, 3801)
    g, dg = oracle.sg_gelu(x)
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    ref_g = x * ndtr(x)
    ref_dg = ndtr(x) + x * phi
    nz = ref_g != 0
    assert np.all(np.abs(g[nz] / ref_g[nz] - 1.0) < 1e-14 * (1.0 + x[nz] ** 2))
    ok = np.abs(ref_dg) > 1e-300
    # GELU' changes sign near x = -0.75: relative there to its two terms
    scale = np.abs(ndtr(x)) + np.abs(x * phi)
    assert np.all(np.abs(dg[ok] - ref_dg[ok]) <= 1e-14 * (1.0 + x[ok] ** 2) * scale[ok])
    g5, _ = oracle.sg_gelu(np.array([-5.0, -10.0]))
    assert abs(g5[0] / (-5.0 * 2.866515718791939e-7) - 1.0) < 1e-13
    assert abs(g5[1] / (-10.0 * 7.619853024160527e-24) - 1.0) < 1e-13
