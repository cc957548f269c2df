"""GPU parity of the learned surrogate through the C ABI.

* forward: the network output matches the float64 oracle evaluated on the
  same bf16-rounded operands, within float32-accumulation and occasional
  bf16-rounding-flip error;
* gradient: kb_sg_loss_grad matches the oracle's loss gradient (itself
  pinned by central differences) per layer;
* training: Adam steps lower the loss;
* fallback: an untrained (zero) network fails the residual check on every
  block, and the predicated plain fallback makes the result bit-identical
  to the plain stencil; with the check disabled it is pure persistence;
* graph replay of surrogate blocks is bit-identical to per-launch.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu, rel_maxnorm

pytestmark = pytest.mark.gpu

HEAT = (1e-3, 1.0, 1.0, 10.0, 300.0)
S = 0.8


@pytest.fixture(scope="module")
def kb():
    need_gpu()
    import paper_2501_09398_amd as kb
    kb.lib()
    return kb


def random_weights(seed):
    w = synth.surrogate_init(seed).astype(np.float32)
    w[19104:19104 + 288] = synth.uniform_f32(seed + 1, 9, 288, -0.06, 0.06)
    w[19392] = 0.01
    return w


def run_block(kb, T0, P, w, steps, threshold, b=0, variant=0):
    ny, nx = T0.shape
    with kb.Problem(kb.HEAT2D_SURROGATE, (ny, nx), HEAT + (S, threshold, 16), 0) as p:
        if variant:
            p.set_option(kb.OPT_TILE, variant)
        p.write(kb.F_T, T0)
        p.write(kb.F_P, P)
        p.write(kb.F_W, w)
        p.run(steps, b)
        return p.read(kb.F_T), p.read(kb.F_SGSTATS), p.read(kb.F_RESID)


@pytest.mark.parametrize("seed,shape", [(0, (512, 512)), (20250116, (512, 512)), (7, (96, 130)), (900011, (37, 64))])
def test_initial_state_hot_spots_match_generator(kb, seed, shape):
    """kb_create draws the surrogate workload's inputs on the device: T0
    from stream 1 and the hot-spot power map (uniform stream 2 plus 1-4
    Gaussian spots from stream 7) bit for bit as the host generator."""
    announce(f"surrogate initial state seed {seed} {shape}")
    with kb.Problem(kb.HEAT2D_SURROGATE, shape, HEAT, seed) as p:
        T0, P = p.read(kb.F_T), p.read(kb.F_P)
    T0_ref, _ = synth.heat2d_init(seed, *shape)
    P_ref = synth.hot_spot_power(seed, *shape)
    assert np.array_equal(T0, T0_ref)
    diff = P != P_ref
    print(f"hot spots: {int(diff.sum())} cells differ, max |P| {P.max():.3f}")
    assert not diff.any()


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("shape", [(64, 96), (40, 33), (35, 70)])
def test_forward_matches_oracle(kb, shape, variant):
    """variant 1: fused network (tiles of 16x32, ragged at both edges for
    (40, 33) and (35, 70)); variant 2: one kernel per layer."""
    announce(f"surrogate forward {shape} variant {variant}")
    T0, _ = synth.heat2d_init(40, *shape)
    P = synth.hot_spot_power(41, *shape)
    w = random_weights(42)
    T16, stats, _ = run_block(kb, T0, P, w, 16, 1e30, variant=variant)
    assert stats[0] == 1 and stats[1] == 0
    y_gpu = (T16.astype(np.float64) - T0.astype(np.float64)) / S
    y_ref = oracle.sg_forward(w, T0, P, round_bf16=True)
    err = np.abs(y_gpu - y_ref)
    scale = np.max(np.abs(y_ref))
    print(f"forward {shape}: max |dy| {err.max():.3e} mean {err.mean():.3e} (max|y| {scale:.3e})")
    # bf16 activations: a rounding flip moves one activation by 2^-8 relative;
    # measured 1.2e-3 (max) and 2e-5 (mean) of max|y|.
    assert err.max() <= 5e-3 * scale
    assert err.mean() <= 2e-4 * scale


def make_fields(kb, nf, H, W, seed):
    import torch
    T0s, Ps, T16s = [], [], []
    for f in range(nf):
        T0, _ = synth.heat2d_init(seed + f, H, W)
        P = synth.hot_spot_power(seed + f, H, W)
        T16 = oracle.heat2d(T0, P, 16).astype(np.float32)
        T0s.append(T0)
        Ps.append(P)
        T16s.append(T16)
    dev = lambda a: torch.from_numpy(np.stack(a)).cuda().contiguous()
    return (np.stack(T0s), np.stack(Ps), np.stack(T16s)), (dev(T0s), dev(Ps), dev(T16s))


def test_gradient_matches_oracle(kb):
    announce("surrogate gradient 2 crops of 64^2")
    (T0, P, T16), (dT0, dP, dT16) = make_fields(kb, 2, 96, 128, 50)
    crops = np.array([[0, 10, 64], [1, 32, 0]], np.int32)
    w = random_weights(51)
    C = 64
    with kb.Problem(kb.HEAT2D_SURROGATE, (64, 64, 2 * C * C), HEAT, 0) as p:
        p.write(kb.F_W, w)
        loss, g = p.sg_loss_grad(dT0, dP, dT16, crops, C)
        loss2, g2 = p.sg_loss_grad(dT0, dP, dT16, crops, C)
    assert loss == loss2 and np.array_equal(g, g2)          # deterministic
    norm = crops.shape[0] * C * C
    lref, gref = 0.0, np.zeros(oracle.SG_NW)
    for f, y0, x0 in crops:
        t0 = T0[f, y0:y0 + C, x0:x0 + C]
        pp = P[f, y0:y0 + C, x0:x0 + C]
        tgt = (T16[f, y0:y0 + C, x0:x0 + C].astype(np.float32) - t0).astype(np.float32) / np.float32(S)
        l, gg = oracle.sg_loss_grad(w, t0, pp, tgt.astype(np.float64), norm=norm, round_bf16=True)
        lref += l
        gref += gg
    print(f"loss gpu {loss:.6e} oracle {lref:.6e}")
    assert abs(loss - lref) <= 1e-2 * lref
    bounds = [0, 576, 608, 9824, 9856, 19072, 19104, 19392, 19393]
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    for nm, a, b in zip(names, bounds[:-1], bounds[1:]):
        e = rel_maxnorm(g[a:b], gref[a:b])
        print(f"grad {nm}: rel max err {e:.3e}")
        assert e < 5e-3, nm     # measured <= 2e-4 (float32 sums of bf16 products)


def test_gradient_matches_oracle_training_batch(kb):
    """The training batch (16 crops of 128^2, the split-K weight gradient at
    its full size) end to end against the oracle's own forward and
    backward on each crop.  End to end a hidden activation within float32
    accumulation error of a bf16 tie can round the other way on one side,
    so this is a report with a loose bound; each layer's products are
    checked on the GPU's own operands at float32-summation tolerance in
    test_gpu_surrogate_layers.py."""
    announce("surrogate gradient 16 crops of 128^2")
    (T0, P, T16), (dT0, dP, dT16) = make_fields(kb, 4, 256, 256, 52)
    rng = np.random.default_rng(53)
    crops = np.array([[rng.integers(0, 4), rng.integers(0, 129), rng.integers(0, 129)] for _ in range(12)]
                     + [[0, 0, 0], [1, 128, 128], [2, 0, 128], [3, 128, 0]], np.int32)
    w = random_weights(54)
    C = 128
    with kb.Problem(kb.HEAT2D_SURROGATE, (64, 64, 16 * C * C), HEAT, 0) as p:
        p.write(kb.F_W, w)
        loss, g = p.sg_loss_grad(dT0, dP, dT16, crops, C)
    norm = crops.shape[0] * C * C
    lref, gref = 0.0, np.zeros(oracle.SG_NW)
    for f, y0, x0 in crops:
        t0 = T0[f, y0:y0 + C, x0:x0 + C]
        pp = P[f, y0:y0 + C, x0:x0 + C]
        tgt = (T16[f, y0:y0 + C, x0:x0 + C].astype(np.float32) - t0).astype(np.float32) / np.float32(S)
        l, gg = oracle.sg_loss_grad(w, t0, pp, tgt.astype(np.float64), norm=norm, round_bf16=True)
        lref += l
        gref += gg
    print(f"loss gpu {loss:.6e} oracle {lref:.6e}")
    assert abs(loss - lref) <= 1e-2 * lref
    bounds = [0, 576, 608, 9824, 9856, 19072, 19104, 19392, 19393]
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    for nm, a, b in zip(names, bounds[:-1], bounds[1:]):
        e = rel_maxnorm(g[a:b], gref[a:b])
        print(f"grad {nm}: rel max err {e:.3e}")
        assert e < 5e-3, nm


def test_training_lowers_loss(kb):
    announce("surrogate training steps")
    import torch
    (_, _, _), (dT0, dP, dT16) = make_fields(kb, 2, 128, 128, 60)
    crops = np.array([[0, 0, 0], [1, 64, 64], [0, 64, 0], [1, 0, 64]], np.int32)
    with kb.Problem(kb.HEAT2D_SURROGATE, (64, 64, 4 * 64 * 64), HEAT, 0) as p:
        p.write(kb.F_W, synth.surrogate_init(61))
        losses = [p.sg_train_step(dT0, dP, dT16, crops, 64, 1e-3) for _ in range(60)]
    print("losses", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]
    torch.cuda.synchronize()


def test_untrained_network_falls_back_to_plain_stencil(kb):
    announce("surrogate fallback")
    shape = (64, 80)
    T0, _ = synth.heat2d_init(70, *shape)
    P = synth.hot_spot_power(70, *shape)
    zero = np.zeros(oracle.SG_NW, np.float32)
    got, stats, resid = run_block(kb, T0, P, zero, 48, 1e-3)
    assert stats[0] == 3 and stats[1] == 3
    assert np.all(resid[:3] > 1e-3)
    with kb.Problem(kb.HEAT2D, shape, HEAT, 0) as q:
        q.write(kb.F_T, T0)
        q.write(kb.F_P, P)
        q.run(48, 0)
        assert np.array_equal(got, q.read(kb.F_T))
    # check disabled: the zero network is persistence
    got, stats, _ = run_block(kb, T0, P, zero, 32, 1e30)
    assert stats[0] == 2 and stats[1] == 0
    assert np.array_equal(got, T0)


@pytest.mark.parametrize("variant", [1, 2])
def test_graph_replay_bitwise_and_peeling(kb, variant):
    announce(f"surrogate graph variant {variant}")
    shape = (64, 64)
    T0, _ = synth.heat2d_init(80, *shape)
    P = synth.hot_spot_power(80, *shape)
    w = random_weights(81)
    a = run_block(kb, T0, P, w, 16 * 5 + 7, 1e-3, b=0, variant=variant)
    b = run_block(kb, T0, P, w, 16 * 5 + 7, 1e-3, b=2, variant=variant)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert a[1][0] == 5


def host_residual(kb, T0, P, Tnew, seed, k=16):
    """The residual check recomputed on the host: r_tile against k plain
    steps of the GPU's plain stencil (the check runs the same fused update;
    the plain path is pinned to the oracle by the heat tests) on the four
    seeded 32x32 tiles (stream 10), r_mean from the mean's closed form with
    the float32-rounded coefficients, sums in float64."""
    ny, nx = T0.shape
    with kb.Problem(kb.HEAT2D, (ny, nx), HEAT, 0) as q:
        q.set_option(kb.OPT_TILE, 1)
        q.write(kb.F_T, T0)
        q.write(kb.F_P, P)
        q.run(k, 0)
        plain = q.read(kb.F_T)
    scale = float(np.max(np.abs(Tnew)))
    r_tile = 0.0
    for t in range(4):
        y0 = int(synth.randint(seed, 10, 2 * t, ny - 31))
        x0 = int(synth.randint(seed, 10, 2 * t + 1, nx - 31))
        d = np.abs(Tnew[y0:y0 + 32, x0:x0 + 32].astype(np.float64) - plain[y0:y0 + 32, x0:x0 + 32])
        r_tile = max(r_tile, float(d.max()))
    c, Rz, Tamb = HEAT[0], HEAT[3], HEAT[4]
    cP, cz = float(np.float32(c)), float(np.float32(c / Rz))
    n = ny * nx
    A = float(np.float32(Tamb)) + cP * (math.fsum(P.astype(np.float64).ravel()) / n) / cz
    mk = A + (math.fsum(T0.astype(np.float64).ravel()) / n - A) * (1.0 - cz) ** k
    r_mean = abs(math.fsum(Tnew.astype(np.float64).ravel()) / n - mk)
    return max(r_mean, r_tile) / scale, r_mean / scale, r_tile / scale


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("shape,wseed", [((40, 33), 95), ((512, 512), 96), ((64, 80), None)])
def test_residual_check_matches_host(kb, shape, wseed, variant):
    """The device residual r of one block equals the host recomputation
    (float64 sums in another order: agreement to 1e-9 relative); wseed None
    is the zero network (persistence)."""
    announce(f"surrogate residual {shape} variant {variant}")
    seed = 7
    T0, _ = synth.heat2d_init(97, *shape)
    P = synth.hot_spot_power(97, *shape)
    w = np.zeros(oracle.SG_NW, np.float32) if wseed is None else random_weights(wseed)
    ny, nx = shape
    with kb.Problem(kb.HEAT2D_SURROGATE, (ny, nx), HEAT + (S, 1e30, 16), seed) as p:
        p.set_option(kb.OPT_TILE, variant)
        p.write(kb.F_T, T0)
        p.write(kb.F_P, P)
        p.write(kb.F_W, w)
        p.run(16, 0)
        Tnew = p.read(kb.F_T)
        r_dev = float(p.read(kb.F_RESID)[0])
    r, r_mean, r_tile = host_residual(kb, T0, P, Tnew, seed)
    print(f"r device {r_dev:.9e} host {r:.9e} (mean {r_mean:.3e}, tile {r_tile:.3e})")
    assert abs(r_dev - r) <= 1e-9 * r + 1e-15


def test_fused_and_per_layer_agree_at_full_size(kb):
    """512 x 512 (the trained workload's size): the fused network and the
    per-layer kernels differ only in the float32 order of the last layer's
    nine tap sums, and both are deterministic run to run."""
    announce("surrogate fused vs per-layer 512^2")
    T0, _ = synth.heat2d_init(90, 512, 512)
    P = synth.hot_spot_power(90, 512, 512)
    w = random_weights(91)
    f1 = run_block(kb, T0, P, w, 16, 1e30, variant=1)[0]
    f2 = run_block(kb, T0, P, w, 16, 1e30, variant=1)[0]
    l1 = run_block(kb, T0, P, w, 16, 1e30, variant=2)[0]
    assert np.array_equal(f1, f2)
    # y differs by float32 rounding (~1e-7); T = T0 + s*y may then round
    # to the neighbouring float32: at most one or two ulps of T
    d = np.abs(f1.astype(np.float64) - l1)
    ulp = float(np.spacing(np.float32(np.abs(l1).max())))
    print(f"fused vs per-layer: max |dT| {d.max():.3e} ({d.max() / ulp:.1f} ulp), differing cells {np.mean(d > 0):.2e}")
    assert d.max() <= 2 * ulp
    # sampled oracle rows: the top edge, an interior band and the bottom edge.
    # bf16 activations: where a hidden activation lies within float32
    # accumulation error of a bf16 rounding tie the two sides round it to
    # neighbouring bf16 values; for a large activation (measured: 3.5 vs
    # 3.515625 in layer 2) that moves y by about 1e-3 over the 5x5 patch it
    # feeds.  Such flips are rare: the bound is on the max (1e-2 of the
    # field's max |y|) and on the share of cells off by more than 1e-3 of it.
    yscale = np.abs((f1.astype(np.float64) - T0) / S).max()
    for y0 in (0, 250, 508):
        sl = slice(max(y0 - 4, 0), min(y0 + 8, 512))
        ref = oracle.sg_forward(w, T0[sl], P[sl], round_bf16=True)
        # rows further than 4 from a cut edge see the same receptive field
        lo = 0 if y0 == 0 else 4
        hi = ref.shape[0] if y0 == 508 else ref.shape[0] - 4
        y = (f1[sl].astype(np.float64) - T0[sl].astype(np.float64)) / S
        err = np.abs(y[lo:hi] - ref[lo:hi])
        print(f"rows {y0}..: max |dy| {err.max():.3e}, share > 1e-3 max|y| {np.mean(err > 1e-3 * yscale):.2e} "
              f"(field max |y| {yscale:.3e})")
        assert err.max() <= 1e-2 * yscale, y0
        assert np.mean(err > 1e-3 * yscale) <= 1e-2, y0


@pytest.mark.parametrize("seed", [900011, 900012])
def test_shipped_weights_accuracy_vs_float64(kb, seed):
    """The shipped network on a held-out 512^2 field, one block of 16 steps
    with the residual check at 1e-3: T within the 1e-3 relative max-norm bar
    of the float64 oracle.  The increment error (T16 - T0 against the exact
    increment) is reported beside persistence (T16 = T0) and one explicit
    step of 16*c, measured 12-16% vs 5% for the explicit step: on this
    stencil the network is not more accurate than a plain step of 16*c."""
    from paper_2501_09398_amd import sg_train
    announce(f"shipped surrogate weights seed {seed}")
    w = sg_train.load_weights()
    T0, _ = synth.heat2d_init(seed, 512, 512)
    P = synth.hot_spot_power(seed, 512, 512)
    T16, stats, resid = run_block(kb, T0, P, w, 16, 1e-3)
    ref = oracle.heat2d(T0, P, 16)
    inc = ref - T0
    euler = oracle.heat2d(T0, P, 1, c=16e-3)

    def err(a):
        a = a.astype(np.float64)
        return (np.max(np.abs(a - ref)) / np.max(np.abs(ref)),
                np.max(np.abs((a - T0) - inc)) / np.max(np.abs(inc)))
    (eT, eI), (pT, pI), (uT, uI) = err(T16), err(T0), err(euler)
    print(f"surrogate T {eT:.2e} inc {eI:.3f} | persistence T {pT:.2e} inc {pI:.3f} | big Euler T {uT:.2e} "
          f"inc {uI:.3f} | residual {resid[0]:.2e} fallbacks {stats[1]}")
    assert stats[0] == 1
    assert stats[1] == 0                # the network's own output was kept (no fallback)
    assert eT <= 1e-3
    # what the network gains over the methods without it: against doing
    # nothing it gains (persistence misses the whole increment); against the
    # cheapest plain alternative, one explicit step of 16*c, it loses on the
    # increment (measured 12-18% vs 5%, printed above), and the 16 plain
    # steps it replaces are exact -- the loss is the recorded result
    assert eT < pT and eI < 0.5 * pI
