"""Seeded synthetic inputs shared by the oracle side and the tests.

This module holds no arithmetic of the solvers or of the batching method:
it only turns (seed, tag, index) into numbers with the distributions that
the workloads use.  The GPU library draws the same numbers on the device
from its own implementation of the same published generator, so tests can
check that both sides start from identical bits.

Generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used in counter mode.
Draw ``idx`` of stream ``tag`` under ``seed`` is output ``idx+1`` of a
SplitMix64 sequence whose state starts at ``seed XOR (tag << 48)``:

    state = (seed ^ (tag << 48)) + (idx + 1) * 0x9E3779B97F4A7C15   (mod 2^64)
    z = (state ^ (state >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

A uniform on [0, 1) keeps the top 24 bits: ``u = (z >> 40) * 2**-24``.
A value on [lo, hi) is ``float32(lo + (hi - lo) * u)`` evaluated in
float64 (one multiply, one add, no fused multiply-add), then rounded once
to float32.  An integer on [0, m) is ``((z >> 40) * m) >> 24``.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

# Stream tags (one per kind of drawn quantity).
TAG_T0 = 1        # initial temperature
TAG_P = 2         # power map
TAG_X0 = 3        # skeleton vector
TAG_A = 4         # skeleton multipliers a_k
TAG_B = 5         # skeleton offsets b_k
TAG_SRC = 6       # FDTD source cell
TAG_HOT = 7       # surrogate hot spots
TAG_SIDES = 8     # multi-grid side lengths

# Distributions of the workloads.
T0_RANGE = (323.0, 343.0)
P_RANGE = (0.0, 1.0)
X0_RANGE = (-1.0, 1.0)
A_RANGE = (0.9, 1.0)
B_RANGE = (-0.01, 0.01)


def raw64(seed: int, tag: int, idx) -> np.ndarray:
    """SplitMix64 outputs for the given counter indices (uint64 array)."""
    idx = np.asarray(idx, dtype=np.uint64)
    base = np.uint64((int(seed) ^ (int(tag) << 48)) & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        z = base + (idx + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def top24(seed: int, tag: int, idx) -> np.ndarray:
    return (raw64(seed, tag, idx) >> np.uint64(40)).astype(np.int64)


def uniform01(seed: int, tag: int, idx) -> np.ndarray:
    """Float64 uniforms on [0, 1) with 24 significant bits."""
    return top24(seed, tag, idx).astype(np.float64) * (2.0 ** -24)


def uniform_f32(seed: int, tag: int, count: int, lo: float, hi: float,
                offset: int = 0) -> np.ndarray:
    """``count`` float32 draws on [lo, hi) from indices offset..offset+count-1."""
    u = uniform01(seed, tag, np.arange(offset, offset + count, dtype=np.uint64))
    return (lo + (hi - lo) * u).astype(np.float32)


def randint(seed: int, tag: int, idx, m: int) -> np.ndarray:
    """Integers on [0, m) (m < 2**39) from the top 24 bits."""
    return (top24(seed, tag, idx) * int(m)) >> 24


# ----------------------------------------------------------------------------
# Workload recipes.  Each returns plain arrays; nothing here advances a solver.
# ----------------------------------------------------------------------------

def heat2d_init(seed: int, ny: int, nx: int):
    """T0 ~ U[323,343) and P ~ U[0,1), row-major [ny][nx], float32."""
    n = ny * nx
    T0 = uniform_f32(seed, TAG_T0, n, *T0_RANGE).reshape(ny, nx)
    P = uniform_f32(seed, TAG_P, n, *P_RANGE).reshape(ny, nx)
    return T0, P


def heat3d_init(seed: int, nz: int, ny: int, nx: int):
    """T0 ~ U[323,343) on every cell; P ~ U[0,1) on layer z=0 only.

    Returns T0 as [nz][ny][nx] and the power plane P as [ny][nx]; the
    power of layers z>0 is zero.
    """
    T0 = uniform_f32(seed, TAG_T0, nz * ny * nx, *T0_RANGE).reshape(nz, ny, nx)
    P = uniform_f32(seed, TAG_P, ny * nx, *P_RANGE).reshape(ny, nx)
    return T0, P


def skeleton_init(seed: int, n: int, K: int = 4):
    """x0 ~ U[-1,1), a_k ~ U[0.9,1.0), b_k ~ U[-0.01,0.01)."""
    x0 = uniform_f32(seed, TAG_X0, n, *X0_RANGE)
    a = uniform_f32(seed, TAG_A, K, *A_RANGE)
    b = uniform_f32(seed, TAG_B, K, *B_RANGE)
    return x0, a, b


def fdtd_source_cell(seed: int, N: int):
    """Ez node (i, j, k) of the soft source, at least one cell from every wall.

    Ez sits at (i, j, k+1/2); its interior nodes have 1 <= i, j <= N-1.
    The source is drawn with 2 <= i, j <= N-2 and 1 <= k <= N-2.
    """
    i = 2 + int(randint(seed, TAG_SRC, 0, N - 3))
    j = 2 + int(randint(seed, TAG_SRC, 1, N - 3))
    k = 1 + int(randint(seed, TAG_SRC, 2, N - 2))
    return i, j, k


def multigrid_sides(seed: int, count: int = 64, lo: int = 64, hi: int = 1024):
    """Square grid sides, log-uniform on [lo, hi]: round(lo * (hi/lo)**u)."""
    u = uniform01(seed, TAG_SIDES, np.arange(count, dtype=np.uint64))
    return [int(v) for v in np.rint(lo * np.power(hi / lo, u)).astype(np.int64)]


def multigrid_init(seed: int, sides):
    """Concatenated T0 and P over square grids of the given sides.

    Grid g occupies flat indices [off_g, off_g + s_g^2) of one stream per
    tag, so each grid's values are a contiguous slice of the same draws.
    """
    T0s, Ps, off = [], [], 0
    for s in sides:
        n = s * s
        T0s.append(uniform_f32(seed, TAG_T0, n, *T0_RANGE, offset=off).reshape(s, s))
        Ps.append(uniform_f32(seed, TAG_P, n, *P_RANGE, offset=off).reshape(s, s))
        off += n
    return T0s, Ps


def hot_spot_power(seed: int, ny: int, nx: int, offset: int = 0):
    """Power map P ~ U[0,1) plus 1-4 Gaussian hot spots of amplitude
    U[1,4) and width sigma U[4,32) cells at uniform centres (tag 7 draws:
    count, then per spot centre y, centre x, amplitude, sigma).  The
    Gaussians are evaluated in float64 and the sum rounded once to float32."""
    base = uniform01(seed, TAG_P, np.arange(offset, offset + ny * nx, dtype=np.uint64)).reshape(ny, nx)
    P = base.copy()
    k0 = offset * 8
    count = 1 + int(randint(seed, TAG_HOT, k0, 4))
    yy = np.arange(ny)[:, None]
    xx = np.arange(nx)[None, :]
    for h in range(count):
        u = uniform01(seed, TAG_HOT, np.arange(k0 + 1 + 4 * h, k0 + 5 + 4 * h, dtype=np.uint64))
        cy, cx, amp, sig = u[0] * ny, u[1] * nx, 1.0 + 3.0 * u[2], 4.0 + 28.0 * u[3]
        P += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * sig * sig))
    return P.astype(np.float32)


def surrogate_init(seed: int):
    """Initial weights of the 4-layer surrogate (19393 float32, canonical
    order W1, b1, W2, b2, W3, b3, W4, b4): weights and biases of layer l
    uniform on [-1/sqrt(fan_in), 1/sqrt(fan_in)) with fan_in = 9*cin, except
    the last layer, which starts at zero (the untrained network predicts no
    change)."""
    cin, cout = (2, 32, 32, 32), (32, 32, 32, 1)
    parts, off = [], 0
    for l in range(4):
        nw, nb = cout[l] * cin[l] * 9, cout[l]
        bound = 1.0 / np.sqrt(9.0 * cin[l])
        if l == 3:
            parts.append(np.zeros(nw + nb, np.float32))
        else:
            parts.append(uniform_f32(seed, 9, nw + nb, -bound, bound, offset=off))
        off += nw + nb
    return np.concatenate(parts)
